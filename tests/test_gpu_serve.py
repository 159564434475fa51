"""GPU tests of the served form: continuous batching gives every request the
result it gets alone (bitwise), every result agrees with the FP64 oracle,
admission respects the HBM budget and the slots, and a request completes once
its Fourier error is below its tolerance.

Requests span the pattern sizes of the served mixed load (N = 64, 128, 256)
with few positions, so the oracle reruns each of them in seconds.  A request
of one iteration is held to the single-step gate (1e-5) from its float32
start; a longer one to the linearised trajectory bound.
"""
import numpy as np
import pytest

from gpu_helpers import rel_l2, PERTURB, STEP_GATE, trajectory_bound
from oracle import pty_oracle as po
from ptysynth import make_scan
from ptysynth.scans import small_config

pytestmark = pytest.mark.gpu

# (n, raster, step, algorithm, param, arrival, max_iter, noise-free start from the truth)
SPECS = [
    (64, 3, 24, "RAAR", 0.75, 0.0, 20, False),
    (128, 3, 40, "DR", 0.0, 0.0, 20, False),
    (256, 2, 80, "RRR", 0.5, 0.0, 10, False),
    (64, 3, 24, "DC", 0.0, 0.01, 30, True),     # completes by tolerance at its first check
    (128, 2, 40, "SF", 0.0, 0.02, 1, False),    # one iteration: single-step gate
    (256, 2, 80, "AR", 0.0, 0.03, 1, False),
    (64, 2, 24, "TLAMBDA", 0.5, 0.04, 1, False),
]
TOL_EF = 1e-6
_CACHE = {}


def _scans():
    if "scans" not in _CACHE:
        out = []
        for i, (n, ras, step, algo, prm, t, it, truth) in enumerate(SPECS):
            cfg = small_config(f"r{i}", n, ras, step, jitter=1, photons=None if truth else 1e5, seed=70 + 3 * i)
            out.append(make_scan(cfg))
        _CACHE["scans"] = out
    return _CACHE["scans"]


def _requests():
    from paper_2311_11466_amd.serve import request_from_scan
    reqs = []
    for i, (sc, spec) in enumerate(zip(_scans(), SPECS)):
        n, ras, step, algo, prm, t, it, truth = spec
        r = request_from_scan(i, sc, algo, prm, arrival=t, max_iter=it, tol=TOL_EF if truth else 1e-12)
        if truth:
            r.obj0 = sc.obj_true.astype(np.complex64)
            r.probe0 = sc.probe_true.astype(np.complex64)
        reqs.append(r)
    return reqs


def _oracle(req, n_iter, eps=0.0, seed=0):
    """The oracle's run of a request from its float32 start (optionally with the
    exit waves perturbed by a relative eps)."""
    amp = np.sqrt(req.intensity.astype(np.float32).astype(np.float64))
    st = po.init_state(req.obj0.astype(np.complex128), req.probe0.astype(np.complex128), req.pos)
    if eps:
        rng = np.random.default_rng(seed)
        st.x = st.x * (1 + eps * rng.standard_normal(st.x.shape))
    return po.run(st, amp, req.pos, *po.preset(req.algorithm, req.param), n_iter, blind=True)


def _covered(req):
    m = np.zeros(req.obj0.shape, bool)
    for p, q in req.pos:
        m[p:p + req.n, q:q + req.n] = True
    return m


@pytest.fixture(scope="module")
def served():
    from paper_2311_11466_amd.serve import Server
    reqs = _requests()
    print("case: served mix of", len(reqs), "requests, N =", [r.n for r in reqs], flush=True)
    mix = Server(max_slots=3, chunk=10).run(reqs)
    return reqs, mix


def test_mix_equals_alone_bitwise(served):
    from paper_2311_11466_amd.serve import Server
    reqs, mix = served
    assert len(mix.results) == len(reqs)
    assert mix.peak_active <= 3
    for r in reqs:
        print("  alone", r.rid, flush=True)
        alone = Server(max_slots=1, chunk=10).run([r]).results[0]
        got = mix.results[r.rid]
        assert got.iterations == alone.iterations
        assert np.array_equal(got.obj.view(np.uint32), alone.obj.view(np.uint32)), r.rid
        assert np.array_equal(got.probe.view(np.uint32), alone.probe.view(np.uint32)), r.rid
    s = mix.summary()
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0 and s["projections_per_s"] > 0


def test_served_results_match_oracle(served):
    reqs, mix = served
    for r in reqs:
        got = mix.results[r.rid]
        truth_start = SPECS[r.rid][7]
        if truth_start:
            # noise-free data from the true state: E_F is at rounding level, so
            # the request completes at its first check, before its limit
            assert got.iterations == 10 < r.max_iter, got.iterations
            assert got.fourier_err < TOL_EF
        else:
            assert got.iterations == r.max_iter
        ref = _oracle(r, got.iterations)
        cov = _covered(r)
        errs = np.array([rel_l2(got.obj, ref.obj, cov), rel_l2(got.probe, ref.probe)])
        if got.iterations == 1:
            bound = np.array([STEP_GATE, STEP_GATE])
        else:
            drift = np.zeros(2)
            for sd in (1, 2):
                q = _oracle(r, got.iterations, PERTURB, sd)
                drift = np.maximum(drift, [rel_l2(q.obj, ref.obj, cov), rel_l2(q.probe, ref.probe)])
            bound = trajectory_bound(drift, got.iterations)
        ef_o = ref.history[-1]["fourier_err"]
        print(f"  request {r.rid} N={r.n} {r.algorithm} {got.iterations} it: obj/probe {errs} bound {bound}; "
              f"E_F gpu {got.fourier_err:.4e} oracle {ef_o:.4e}", flush=True)
        assert np.all(errs <= bound), (r.rid, errs, bound)
        if got.iterations == 1:
            assert abs(got.fourier_err - ef_o) <= 1e-4 * ef_o, (r.rid, got.fourier_err, ef_o)


def test_admission_by_budget():
    from paper_2311_11466_amd.serve import Server
    reqs = _requests()
    sizes = sorted(r.workspace() for r in reqs)
    budget = sizes[-1] + sizes[-2]            # at most two of the largest at once
    st = Server(budget_bytes=budget, max_slots=16, chunk=10).run(reqs)
    assert len(st.results) == len(reqs)
    assert st.peak_bytes <= budget
    with pytest.raises(ValueError):
        Server(budget_bytes=sizes[0] - 1).run(reqs[:1])


def test_iterate_many_matches_iterate():
    import torch
    import paper_2311_11466_amd as pk
    reqs = _requests()[:3]
    dev = torch.device("cuda", 0)

    def mk(r, stream):
        with torch.cuda.stream(stream):
            g = pk.Scan(torch.as_tensor(r.pos).to(dev), torch.as_tensor(r.intensity).to(dev),
                        torch.as_tensor(r.obj0).to(dev), torch.as_tensor(r.probe0).to(dev), stream=stream)
        g.set_algorithm_named(r.algorithm, r.param)
        return g
    streams = [torch.cuda.Stream() for _ in reqs]
    many = [mk(r, s) for r, s in zip(reqs, streams)]
    pk.iterate_many(many, 7)
    one = [mk(r, s) for r, s in zip(reqs, streams)]
    for g in one:
        g.iterate(7)
    for a, b in zip(many, one):
        for ta, tb in zip(a.get_state(), b.get_state()):
            assert torch.equal(ta.view(torch.int64) if ta.dtype == torch.complex64 else ta,
                               tb.view(torch.int64) if tb.dtype == torch.complex64 else tb)
        a.close()
        b.close()


def test_grouped_launches_match_iterate_bitwise():
    """pty_iterate_many on scans that share a stream runs grouped launches (one
    launch per kernel class for up to eight scans of one pattern size, storage
    and prologue mode); every scan's state must equal that of pty_iterate on
    it alone, bitwise.  The mix covers every grouping branch: N = 32 ... 256,
    float32 and float16 storage, the blend and x forms, the prologue modes of
    DC, SF, RAAR and the full metrics, a known probe, two concur sweeps, ten
    scans of one size (two chunks), and scans whose state was read in between
    (their next iteration starts from a materialised x)."""
    import torch
    import paper_2311_11466_amd as pk
    dev = torch.device("cuda", 0)
    # (n, raster, step, algorithm, param, storage, full_metrics, blind, sweeps)
    specs = ([(64, 3, 24, a, p, "fp32", False, True, 1) for a, p in
              [("RAAR", 0.75), ("DC", 0.0), ("SF", 0.0), ("DR", 0.0), ("RRR", 0.5), ("AR", 0.0),
               ("TLAMBDA", 0.5), ("RAAR", 0.9), ("DC", 0.0), ("RAAR", 0.6)]]
             + [(32, 4, 12, "TLAMBDA", 0.5, "fp32", True, True, 1),
                (128, 2, 40, "RAAR", 0.75, "fp32", False, True, 1),
                (128, 2, 40, "DR", 0.0, "fp16", False, True, 1),
                (128, 2, 40, "DC", 0.0, "fp32", True, False, 1),
                (256, 2, 80, "RRR", 0.5, "fp32", False, True, 1),
                (256, 2, 80, "AR", 0.0, "fp16", True, True, 1),
                (64, 3, 24, "RAAR", 0.75, "fp16", False, True, 2)])
    scans = []
    for i, (n, ras, step, *_rest) in enumerate(specs):
        scans.append(make_scan(small_config(f"g{i}", n, ras, step, jitter=1, photons=1e6, seed=300 + 7 * i)))
    shared = torch.cuda.Stream()

    def mk(sc, spec, stream):
        n, ras, step, algo, prm, storage, full, blind, sweeps = spec
        with torch.cuda.stream(stream):
            g = pk.Scan(torch.as_tensor(sc.pos.astype(np.int32)).to(dev),
                        torch.as_tensor(sc.intensity.astype(np.float32)).to(dev),
                        torch.as_tensor(sc.obj0.astype(np.complex64)).to(dev),
                        torch.as_tensor(sc.probe0.astype(np.complex64)).to(dev),
                        storage=storage, full_metrics=full, blind=blind, stream=stream)
        g.set_algorithm_named(algo, prm)
        g.set_concur_sweeps(sweeps)
        return g
    print("case: grouped launches,", len(specs), "scans", flush=True)
    many = [mk(sc, sp, shared) for sc, sp in zip(scans, specs)]
    pk.iterate_many(many, 4)
    # a change of algorithm in the middle (switches some scans' form and mode)
    many[0].set_algorithm_named("DC")
    many[11].set_algorithm_named("SF")
    pk.iterate_many(many, 3)
    # reading the state materialises x: the next iteration of these scans runs
    # the materialised-x prologue (alone at N = 256) beside grouped scans
    read_mid = (11, 14, 15)
    for i in read_mid:
        many[i].get_state()
    pk.iterate_many(many, 2)
    shared.synchronize()
    for i, (sc, sp) in enumerate(zip(scans, specs)):
        alone = mk(sc, sp, torch.cuda.current_stream())
        alone.iterate(4)
        if i == 0:
            alone.set_algorithm_named("DC")
        if i == 11:
            alone.set_algorithm_named("SF")
        alone.iterate(3)
        if i in read_mid:
            alone.get_state()
        alone.iterate(2)
        for name, ta, tb in zip("xyop", many[i].get_state(), alone.get_state()):
            assert torch.equal(ta.view(torch.int64), tb.view(torch.int64)), (i, sp, name)
        ha, hb = many[i].metric_history(), alone.metric_history()
        assert len(ha) == len(hb) == 9
        for ma, mb in zip(ha, hb):
            for key in ("fourier_err", "consistency_err", "change"):
                va, vb = ma[key], mb[key]
                assert (np.isnan(va) and np.isnan(vb)) or va == vb, (i, key, va, vb)
        alone.close()
    for g in many:
        g.close()
