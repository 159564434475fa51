// Host engine and C ABI: argument validation, workspace layout, the per-scan
// state machine (pending update, metric bookkeeping) and the launch sequence
// of one iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "ptyabc.h"
#include "params.hpp"

using namespace pty;

namespace {

thread_local std::string g_last_error;

pty_status fail(pty_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

constexpr size_t kAlign = 256;
constexpr int kTileW = 64, kTileH = 16;
constexpr int kDefaultCap = 4096;
constexpr double kDefaultTau = 1e-10;
constexpr int kMaxSweeps = 64;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// exit-wave state of the next divide prologue
// State of the exit-wave buffers between iterations:
//   MODE_INIT       nothing stored; x_0 = P S_j O
//   MODE_MATERIAL   x holds x_k
//   MODE_PENDING    x, y hold x_{k-1}, y_{k-1}; x_k = pa P S_j O + pb y + pg x
//   MODE_PENDING_W  x holds the blend w_{k-1} = pg x_{k-1} + pb y_{k-1},
//                   y holds y_{k-1}; x_k = pa P S_j O + w
enum Mode { MODE_INIT = 0, MODE_MATERIAL = 1, MODE_PENDING = 2, MODE_PENDING_W = 3 };

struct Layout {
  size_t amp, x, y, tmp, obj, probe, pos, tile_off, tile_list, part, met, met2, ring, tile_max, pmax, tw, flag, eval, sp_list,
      sp_omax,
      total;
  int tiles_x, tiles_y, n_tiles, max_list, G, chunk, npb, nslot, cap;
  size_t elem_bytes;
};

bool desc_shape_ok(const pty_scan_desc* d, std::string* why) {
  if (!d) { *why = "desc is NULL"; return false; }
  if (!divide_supported(d->n)) { *why = "n must be 32, 64, 128 or 256"; return false; }
  if (d->n_pos < 1) { *why = "n_pos must be >= 1"; return false; }
  if (d->obj_h < d->n || d->obj_w < d->n) { *why = "object must be at least N x N"; return false; }
  if (int64_t(d->obj_h) * d->obj_w > (int64_t(1) << 31)) { *why = "object too large"; return false; }
  {
    // the tile lists are indexed with int: every (position, tile) pair must fit
    const int64_t per_pos = ((d->n + kTileH - 2) / kTileH + 1) * ((d->n + kTileW - 2) / kTileW + 1);
    if (int64_t(d->n_pos) * per_pos > int64_t(INT32_MAX)) { *why = "too many positions"; return false; }
  }
  if (d->storage != PTY_STORE_FP32 && d->storage != PTY_STORE_FP16) { *why = "storage must be 0 or 1"; return false; }
  if (d->blind != 0 && d->blind != 1) { *why = "blind must be 0 or 1"; return false; }
  if (d->probe_update_start < 0) { *why = "probe_update_start must be >= 0"; return false; }
  if (d->full_metrics != 0 && d->full_metrics != 1) { *why = "full_metrics must be 0 or 1"; return false; }
  if (d->metric_capacity < 0) { *why = "metric_capacity must be >= 0"; return false; }
  if (!(d->tau >= 0.0) || !std::isfinite(d->tau)) { *why = "tau must be finite and >= 0"; return false; }
  if (d->inputs_on_device != 0 && d->inputs_on_device != 1) { *why = "inputs_on_device must be 0 or 1"; return false; }
  return true;
}

Layout make_layout(const pty_scan_desc* d) {
  Layout L{};
  const size_t N = size_t(d->n), J = size_t(d->n_pos), H = size_t(d->obj_h), W = size_t(d->obj_w);
  const size_t nn = N * N;
  L.elem_bytes = d->storage == PTY_STORE_FP16 ? 4 : 8;
  L.tiles_x = int((W + kTileW - 1) / kTileW);
  L.tiles_y = int((H + kTileH - 1) / kTileH);
  L.n_tiles = L.tiles_x * L.tiles_y;
  // a window of N pixels meets at most ceil((N-1)/T)+1 tiles along an axis
  const int per_pos = ((d->n + kTileH - 2) / kTileH + 1) * ((d->n + kTileW - 2) / kTileW + 1);
  L.max_list = int(J) * per_pos;
  L.npb = int((nn + 255) / 256);
  // position chunks of the probe reduction: about 1024 work-groups in all
  int G = std::max(1, (1024 + L.npb - 1) / L.npb);
  G = std::min<int>(G, int(J));
  L.chunk = int((J + G - 1) / G);
  L.G = int((J + L.chunk - 1) / L.chunk);
  L.nslot = divide_slots(d->n);
  L.cap = d->metric_capacity > 0 ? d->metric_capacity : kDefaultCap;

  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align_up(bytes); return o; };
  L.amp = take(J * nn * 4);
  L.x = take(J * nn * L.elem_bytes);
  L.y = take(J * nn * L.elem_bytes);
  L.tmp = (d->n == 256 && d->storage == PTY_STORE_FP16) ? take(J * nn * 8) : size_t(-1);
  L.obj = take(H * W * 8);
  L.probe = take(nn * 8);
  L.pos = take(J * 8);
  L.tile_off = take((size_t(L.n_tiles) + 1) * 4);
  L.tile_list = take(size_t(L.max_list) * 16);
  L.part = take(3 * size_t(L.G) * nn * 8);
  L.met = take(J * size_t(L.nslot) * MF_COUNT * 8);
  L.met2 = take(size_t(std::max(L.n_tiles, 64)) * MF_COUNT * 8);
  L.ring = take(size_t(L.cap) * kRingFields * 8);
  L.tile_max = take(size_t(L.n_tiles) * 4);
  L.pmax = take(size_t(L.npb) * 4);
  L.tw = take(N * 8);
  L.flag = take(64);
  L.eval = take(size_t(object_error_blocks((long long)H * W) + 1) * 4 * 8);   // object-error partial sums, result
  L.sp_list = take(J * 4);                            // batch member lists of sequential projections
  L.sp_omax = d->n == 256 ? take(J * 16 * 4) : size_t(-1);   // N = 256 SP: row-block maxima of |S_j O|^2
  L.total = off;
  return L;
}

}  // namespace

struct pty_scan {
  int N = 0, J = 0, H = 0, W = 0;
  int fp16 = 0, blind = 0, probe_update_start = 0, full_metrics = 1;
  double tau = kDefaultTau;
  hipStream_t stream = nullptr;
  int device = 0;
  char* ws = nullptr;
  Layout L{};
  float scale = 1.0f, inv_scale = 1.0f;
  double a = 1.0, b = 1.0, c = 1.0;
  int64_t k = 0;
  int mode = MODE_INIT;
  int sweeps = 1;                          // concur (object, probe) sweeps per iteration
  std::vector<int> hpos;                   // positions (row, col) on the host
  std::vector<int> sp_members;             // batch member lists of the last sequential-projection call
  int sp_batches_last = 0;                 // batches of the last sequential-projection call
  float pa = 1.0f, pb = 0.0f, pg = 0.0f;  // pending prologue coefficients
  bool x_valid = false, y_valid = false;
  bool prev_metrics_done = true;          // metrics of iteration k-1 already finalised
  bool failed = false;
  // per-kernel event timing
  bool prof = false;
  int prof_every = 1;               // time the launches of every prof_every-th iteration
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_class;        // class of each (start, end) pair queued
  size_t ev_used = 0;               // events handed out from ev_pool
  double prof_ms[PTY_K_COUNT] = {0};
  int64_t prof_n[PTY_K_COUNT] = {0};

  template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  float2* tmp_ptr() const { return L.tmp == size_t(-1) ? at<float2>(L.y) : at<float2>(L.tmp); }
};

namespace {

pty_status device_fail(pty_scan* s, hipError_t e, const char* what) {
  if (s) s->failed = true;
  return fail(PTY_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define PTY_HIP(s, call, what)                          \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return device_fail(s, e_, what); \
  } while (0)

pty_status check_usable(const pty_scan* s) {
  if (!s) return fail(PTY_ERR_INVALID_ARG, "scan is NULL");
  if (s->failed) return fail(PTY_ERR_BAD_STATE, "scan had a device error; only pty_destroy_scan is allowed");
  return PTY_OK;
}

// Record an event pair around one launch when timing is on.
template <class F>
hipError_t timed(pty_scan* s, int cls, F&& launch) {
  if (!s->prof || s->k % s->prof_every != 0) return launch();
  auto next = [&](hipEvent_t* e) -> hipError_t {
    if (s->ev_used == s->ev_pool.size()) {
      hipEvent_t ne;
      hipError_t r = hipEventCreate(&ne);
      if (r != hipSuccess) return r;
      s->ev_pool.push_back(ne);
    }
    *e = s->ev_pool[s->ev_used++];
    return hipSuccess;
  };
  hipEvent_t a, b;
  hipError_t r = next(&a);
  if (r == hipSuccess) r = next(&b);
  if (r == hipSuccess) r = hipEventRecord(a, s->stream);
  if (r == hipSuccess) r = launch();
  if (r == hipSuccess) r = hipEventRecord(b, s->stream);
  if (r == hipSuccess) s->ev_class.push_back(cls);
  return r;
}

// fold the queued event pairs into the totals (synchronises the stream)
hipError_t drain_profile(pty_scan* s) {
  if (s->ev_class.empty()) return hipSuccess;
  hipError_t r = hipStreamSynchronize(s->stream);
  if (r != hipSuccess) return r;
  for (size_t i = 0; i < s->ev_class.size(); ++i) {
    float ms = 0.f;
    r = hipEventElapsedTime(&ms, s->ev_pool[2 * i], s->ev_pool[2 * i + 1]);
    if (r != hipSuccess) return r;
    s->prof_ms[s->ev_class[i]] += ms;
    s->prof_n[s->ev_class[i]] += 1;
  }
  s->ev_class.clear();
  s->ev_used = 0;
  return hipSuccess;
}

MetricParams metric_params(const pty_scan* s, int slices) {
  MetricParams m{};
  m.met = s->at<double>(s->L.met);
  m.J = s->J;
  m.nslot = s->L.nslot;
  m.part2 = s->at<double>(s->L.met2);
  m.slices = slices;
  m.ring = s->at<double>(s->L.ring);
  m.cap = s->L.cap;
  m.k_cur = -1;
  m.k_prev = -1;
  return m;
}

FinalParams final_params(const pty_scan* s, const MetricParams& mp) {
  FinalParams f{};
  f.part = s->at<double>(s->L.part);
  f.probe = s->at<float2>(s->L.probe);
  f.pmax_part = s->at<float>(s->L.pmax);
  f.tile_max = s->at<float>(s->L.tile_max);
  f.n_tiles = object_blocks(s->N, s->L.n_tiles);   // tile_max entries the object launch wrote
  f.N = s->N;
  f.G = s->L.G;
  f.npb = s->L.npb;
  f.tau = s->tau;
  f.mp = mp;
  return f;
}

// One iteration: divide (with the pending update), object (+ metrics), [probe].
pty_status flush(pty_scan* s, bool materialise);

DivideParams divide_params(const pty_scan* s) {
  DivideParams p{};
  p.obj = s->at<float2>(s->L.obj);
  p.probe = s->at<float2>(s->L.probe);
  p.pos = s->at<int2>(s->L.pos);
  p.amp = s->at<float>(s->L.amp);
  p.tw = s->at<float2>(s->L.tw);
  p.x = s->ws + s->L.x;
  p.y = s->ws + s->L.y;
  p.tmp = s->tmp_ptr();
  p.obj_w = s->W;
  p.j_begin = 0;
  p.scale = s->scale;
  p.inv_scale = s->inv_scale;
  p.met = s->at<double>(s->L.met);
  p.nslot = s->L.nslot;
  return p;
}

// The divide over every pattern: one launch per stage (the N = 256 passes
// each span all patterns).
pty_status launch_divide(pty_scan* s, const DivideParams& p, bool timed_launch) {
  for (int stage = 0; stage < divide_stages(s->N); ++stage) {
    auto fn = [&] { return launch_divide_stage(s->N, s->fp16, p, s->J, stage, s->stream); };
    PTY_HIP(s, timed_launch ? timed(s, PTY_K_DIVIDE + stage, fn) : fn(), "divide launch");
  }
  return PTY_OK;
}

// The concur of the y buffer into the scan's object and probe: s->sweeps
// (object, probe) sweeps when the probe is updated, one object step
// otherwise.  Every sweep's object launch writes the same metric slices and
// every finalise the same ring entries (from mp), so repeating them is
// harmless.
// Parameter blocks of the concur launches of one scan.
void concur_params(const pty_scan* s, const MetricParams& mp, ObjParams* po, ProbeParams* pq) {
  ObjParams o{};
  o.y = s->ws + s->L.y;
  o.inv_scale = s->inv_scale;
  o.probe = s->at<float2>(s->L.probe);
  o.pos = s->at<int2>(s->L.pos);
  o.tile_off = s->at<int>(s->L.tile_off);
  o.tile_ent = s->at<int4>(s->L.tile_list);
  o.obj = s->at<float2>(s->L.obj);
  o.H = s->H; o.W = s->W; o.N = s->N;
  o.tiles_x = s->L.tiles_x;
  o.n_tiles = s->L.n_tiles;
  o.tile_max = s->at<float>(s->L.tile_max);
  o.pmax_part = s->at<float>(s->L.pmax);
  o.npb = s->L.npb;
  o.tau = s->tau;
  o.mp = mp;
  ProbeParams q{};
  q.y = o.y;
  q.inv_scale = s->inv_scale;
  q.obj = o.obj;
  q.pos = o.pos;
  q.N = s->N; q.W = s->W; q.J = s->J;
  q.chunk = s->L.chunk;
  q.G = s->L.G;
  q.part = s->at<double>(s->L.part);
  *po = o;
  *pq = q;
}

pty_status launch_concur(pty_scan* s, const MetricParams& mp, bool update_probe, bool timed_launch) {
  const hipStream_t st = s->stream;
  ObjParams o;
  ProbeParams q;
  concur_params(s, mp, &o, &q);
  const FinalParams f = final_params(s, mp);
  const int n_sweeps = update_probe ? s->sweeps : 1;
  auto run = [&](int cls, auto&& fn) { return timed_launch ? timed(s, cls, fn) : fn(); };
  for (int sw = 0; sw < n_sweeps; ++sw) {
    PTY_HIP(s, run(PTY_K_OBJECT, [&] { return launch_object_update(s->fp16, o, st); }), "object launch");
    if (update_probe)
      PTY_HIP(s, run(PTY_K_PROBE, [&] { return launch_probe_partial(s->fp16, q, st); }), "probe launch");
    PTY_HIP(s, run(PTY_K_FINAL, [&] { return launch_probe_final(f, update_probe, st); }), "finalise launch");
  }
  return PTY_OK;
}

// Blend form (x buffer holds w, see MODE_PENDING_W): it saves the y read of
// the next prologue when x and y are both needed, i.e. a != 1 and b != 1.
// It leaves no x_k for the change metric, so it is used only without
// full_metrics.  It keeps x_k in registers through the transforms; at
// N = 128 that rules out the two patterns per CU of the x form's split
// exchanges, which measured faster, so it is used for N <= 64.
bool use_blend(const pty_scan* s) {
  return !s->full_metrics && s->N <= 64 && float(1.0 - s->a) != 0.f && float(s->a * (1.0 - s->b)) != 0.f;
}

// One iteration of a scan, planned on the host: its divide parameters, the
// metric bookkeeping of its concur launches, and the state it leaves.
struct IterPlan {
  DivideParams dp;
  MetricParams mp;
  bool update_probe;
  bool wf;
  bool write_x;
};

// Plan the next iteration (a change of state form first materialises x, which
// launches the flush kernel on the scan's stream).
pty_status plan_iteration(pty_scan* s, IterPlan* L) {
  const bool wf = use_blend(s);
  if ((wf && s->mode == MODE_PENDING) || (!wf && s->mode == MODE_PENDING_W)) {
    // a change of form passes through a materialised x
    const pty_status fs = flush(s, true);
    if (fs != PTY_OK) return fs;
  }
  DivideParams p = divide_params(s);
  float al = 1.f, be = 0.f, ga = 0.f;
  if (s->mode == MODE_MATERIAL) { al = 0.f; be = 0.f; ga = 1.f; }
  if (s->mode == MODE_PENDING) { al = s->pa; be = s->pb; ga = s->pg; }
  p.alpha = al; p.beta = be; p.gamma = ga;
  const bool pending = s->mode == MODE_PENDING;
  const bool need_y = pending && be != 0.f;
  const bool need_x = (pending && ga != 0.f) || s->mode == MODE_MATERIAL;
  const bool want_prev = pending && !s->prev_metrics_done;
  p.prev_ec = want_prev && s->y_valid && (need_y || s->full_metrics);
  p.prev_dx = want_prev && s->x_valid && (need_x || s->full_metrics);
  p.read_y = need_y || p.prev_ec;
  p.read_x = need_x || p.prev_dx;
  bool write_x = (1.0 - s->a) != 0.0 || s->full_metrics;
  if (wf) {
    p.wform = 1;
    if (s->mode == MODE_INIT) { p.alpha = 1.f; p.read_x = 0; }
    else if (s->mode == MODE_MATERIAL) { p.alpha = 0.f; p.read_x = 1; }
    else { p.alpha = s->pa; p.read_x = s->x_valid; }
    p.beta = 0.f; p.gamma = 0.f;
    p.read_y = 0; p.prev_ec = 0; p.prev_dx = 0;
    p.next_beta = float(s->a * (1.0 - s->b));
    p.next_gamma = float(1.0 - s->a);
    write_x = true;
  }
  p.write_x = write_x;
  p.c = float(s->c);
  L->dp = p;
  L->update_probe = s->blind && s->k >= s->probe_update_start;
  MetricParams mp = metric_params(s, metric_slices(s->N, s->L.n_tiles));
  mp.k_cur = s->k;
  mp.k_prev = (p.prev_ec || p.prev_dx) ? s->k - 1 : -1;
  mp.ec_ok = p.prev_ec;
  mp.dx_ok = p.prev_dx;
  L->mp = mp;
  L->wf = wf;
  L->write_x = write_x;
  return PTY_OK;
}

// The state after the planned iteration's launches: pending with its (a, b).
void commit_iteration(pty_scan* s, const IterPlan& L) {
  s->mode = L.wf ? MODE_PENDING_W : MODE_PENDING;
  s->pa = float(s->a * s->b);
  s->pb = float(s->a * (1.0 - s->b));
  s->pg = float(1.0 - s->a);
  s->x_valid = L.write_x;
  s->y_valid = true;
  s->prev_metrics_done = L.wf;   // the blend form has no consistency / change metrics
  s->k += 1;
}

pty_status launch_iteration(pty_scan* s) {
  IterPlan L;
  pty_status st = plan_iteration(s, &L);
  if (st != PTY_OK) return st;
  if (s->prof && s->ev_class.size() > 4096) PTY_HIP(s, drain_profile(s), "profile drain");
  st = launch_divide(s, L.dp, true);
  if (st != PTY_OK) return st;
  st = launch_concur(s, L.mp, L.update_probe, true);
  if (st != PTY_OK) return st;
  commit_iteration(s, L);
  return PTY_OK;
}

// One iteration of several scans on one stream with grouped launches: every
// kernel class runs once per group of up to kGroupMax scans of the same
// pattern size and storage (and, for the divide, the same prologue mode)
// instead of once per scan.  Each scan's kernels see exactly the parameters
// of its own launch, so its results are bitwise those of pty_iterate.
static pty_status launch_iteration_grouped_body(pty_scan* const* scans, int count, std::vector<IterPlan>& plans);

// One iteration of every scan with grouped launches.  Once launches have
// started, a failure leaves every scan of the call with device buffers that
// its host state no longer describes, so all of them are marked failed.
pty_status launch_iteration_grouped(pty_scan* const* scans, int count) {
  std::vector<IterPlan> plans(count);
  for (int i = 0; i < count; ++i) {
    const pty_status st = plan_iteration(scans[i], &plans[i]);
    if (st != PTY_OK) return st;
  }
  const pty_status st = launch_iteration_grouped_body(scans, count, plans);
  if (st != PTY_OK) {
    for (int i = 0; i < count; ++i) scans[i]->failed = true;
    return st;
  }
  for (int i = 0; i < count; ++i) commit_iteration(scans[i], plans[i]);
  return PTY_OK;
}

static pty_status launch_iteration_grouped_body(pty_scan* const* scans, int count, std::vector<IterPlan>& plans) {
  const hipStream_t stream = scans[0]->stream;
  // a failed grouped launch carried the work of every scan of its chunk
  auto group_fail = [&](const int* m, int n, hipError_t e, const char* what) {
    for (int q = 1; q < n; ++q) scans[m[q]]->failed = true;
    return device_fail(scans[m[0]], e, what);
  };
  // scans in call order, grouped by key; groups are launched in order of
  // their first scan, each in chunks of kGroupMax
  auto run_groups = [&](auto key_of, auto launch_chunk) -> pty_status {
    std::vector<char> done(count, 0);
    for (int i = 0; i < count; ++i) {
      if (done[i]) continue;
      const auto key = key_of(i);
      std::vector<int> members;
      for (int q = i; q < count; ++q)
        if (!done[q] && key_of(q) == key) { members.push_back(q); done[q] = 1; }
      for (size_t c = 0; c < members.size(); c += kGroupMax) {
        const int n = int(std::min<size_t>(kGroupMax, members.size() - c));
        const pty_status st = launch_chunk(members.data() + c, n);
        if (st != PTY_OK) return st;
      }
    }
    return PTY_OK;
  };
  // divide
  for (int stage = 0; stage < 3; ++stage) {
    auto key = [&](int i) {
      const pty_scan* s = scans[i];
      if (stage >= divide_stages(s->N)) return -1;                 // no such stage for this scan
      if (!divide_groupable(s->N, plans[i].dp)) return -2 - i;     // alone
      return ((s->N * 2 + s->fp16) * 64) + divide_mode(plans[i].dp);   // one prologue mode per group
    };
    const pty_status st = run_groups(key, [&](const int* m, int n) -> pty_status {
      if (key(m[0]) == -1) return PTY_OK;
      pty_scan* s0 = scans[m[0]];
      if (key(m[0]) < -1) {
        const hipError_t e = launch_divide_stage(s0->N, s0->fp16, plans[m[0]].dp, s0->J, stage, stream);
        return e == hipSuccess ? PTY_OK : device_fail(s0, e, "divide launch");
      }
      DivideParams ps[kGroupMax];
      int np[kGroupMax];
      for (int q = 0; q < n; ++q) { ps[q] = plans[m[q]].dp; np[q] = scans[m[q]]->J; }
      const hipError_t e = launch_divide_stage_group(s0->N, s0->fp16, ps, np, n, stage, stream);
      return e == hipSuccess ? PTY_OK : group_fail(m, n, e, "grouped divide launch");
    });
    if (st != PTY_OK) return st;
  }
  // concur: object steps, probe sums (scans whose probe is updated), finalise;
  // a scan with several concur sweeps runs its own launches
  auto swept = [&](int i) { return plans[i].update_probe && scans[i]->sweeps > 1; };
  pty_status st = run_groups([&](int i) { return swept(i) ? -1 - i : scans[i]->N * 2 + scans[i]->fp16; },
                             [&](const int* m, int n) -> pty_status {
    pty_scan* s0 = scans[m[0]];
    if (swept(m[0])) return launch_concur(s0, plans[m[0]].mp, true, false);
    ObjParams os[kGroupMax];
    for (int q = 0; q < n; ++q) {
      ProbeParams unused;
      concur_params(scans[m[q]], plans[m[q]].mp, &os[q], &unused);
    }
    const hipError_t e = launch_object_update_group(s0->fp16, os, n, stream);
    return e == hipSuccess ? PTY_OK : group_fail(m, n, e, "grouped object launch");
  });
  if (st != PTY_OK) return st;
  st = run_groups([&](int i) { return (swept(i) || !plans[i].update_probe) ? -1 : scans[i]->N * 2 + scans[i]->fp16; },
                  [&](const int* m, int n) -> pty_status {
    if (swept(m[0]) || !plans[m[0]].update_probe) return PTY_OK;
    ProbeParams qs[kGroupMax];
    for (int q = 0; q < n; ++q) {
      ObjParams unused;
      concur_params(scans[m[q]], plans[m[q]].mp, &unused, &qs[q]);
    }
    const hipError_t e = launch_probe_partial_group(scans[m[0]]->fp16, qs, n, stream);
    return e == hipSuccess ? PTY_OK : group_fail(m, n, e, "grouped probe launch");
  });
  if (st != PTY_OK) return st;
  st = run_groups([&](int i) { return swept(i) ? -1 : 0; }, [&](const int* m, int n) -> pty_status {
    if (swept(m[0])) return PTY_OK;
    FinalParams fs[kGroupMax];
    int up[kGroupMax];
    for (int q = 0; q < n; ++q) {
      fs[q] = final_params(scans[m[q]], plans[m[q]].mp);
      up[q] = plans[m[q]].update_probe ? 1 : 0;
    }
    const hipError_t e = launch_probe_final_group(fs, up, n, stream);
    return e == hipSuccess ? PTY_OK : group_fail(m, n, e, "grouped finalise launch");
  });
  return st;
}

// Finalise the metrics of iteration k-1 and/or materialise x_k.
pty_status flush(pty_scan* s, bool materialise) {
  const bool pending = s->mode == MODE_PENDING;
  const bool want_metrics = pending && !s->prev_metrics_done;
  if (!want_metrics && !(materialise && s->mode != MODE_MATERIAL)) return PTY_OK;
  FlushParams fp{};
  fp.obj = s->at<float2>(s->L.obj);
  fp.probe = s->at<float2>(s->L.probe);
  fp.pos = s->at<int2>(s->L.pos);
  fp.x = s->ws + s->L.x;
  fp.y = s->ws + s->L.y;
  fp.N = s->N;
  fp.obj_w = s->W;
  if (s->mode == MODE_INIT) { fp.alpha = 1.f; fp.beta = 0.f; fp.gamma = 0.f; }
  else if (s->mode == MODE_MATERIAL) { fp.alpha = 0.f; fp.beta = 0.f; fp.gamma = 1.f; }
  else { fp.alpha = s->pa; fp.beta = s->pb; fp.gamma = s->pg; }
  fp.read_x = (s->x_valid && (fp.gamma != 0.f || want_metrics)) ? 1 : 0;
  fp.read_y = (s->y_valid && (fp.beta != 0.f || want_metrics)) ? 1 : 0;
  if (s->mode == MODE_PENDING_W) {
    fp.wform = 1;
    fp.beta = 0.f; fp.gamma = 0.f;
    fp.read_x = s->x_valid ? 1 : 0;
    fp.read_y = 0;
  }
  fp.scale = s->scale;
  fp.inv_scale = s->inv_scale;
  fp.write_x = materialise && s->mode != MODE_MATERIAL;
  fp.met = s->at<double>(s->L.met);
  fp.nslot = s->L.nslot;
  PTY_HIP(s, launch_flush(s->fp16, fp, s->J, s->stream), "flush launch");
  if (want_metrics) {
    MetricParams m = metric_params(s, 1);
    m.k_prev = s->k - 1;
    m.ec_ok = fp.read_y;
    m.dx_ok = fp.read_x;
    PTY_HIP(s, launch_metric_slices(m, s->stream), "metrics launch");
    PTY_HIP(s, launch_probe_final(final_params(s, m), 0, s->stream), "metrics launch");
    s->prev_metrics_done = true;
  }
  if (fp.write_x) {
    s->mode = MODE_MATERIAL;
    s->x_valid = true;
  }
  return PTY_OK;
}

pty_status refresh_probe_max(pty_scan* s) {
  PTY_HIP(s, launch_max_abs2_parts(s->at<float2>(s->L.probe), size_t(s->N) * s->N, s->at<float>(s->L.pmax),
                                   s->L.npb, s->stream),
          "probe max");
  return PTY_OK;
}

hipMemcpyKind kind(int src_dev, int dst_dev) {
  if (src_dev && dst_dev) return hipMemcpyDeviceToDevice;
  if (src_dev) return hipMemcpyDeviceToHost;
  if (dst_dev) return hipMemcpyHostToDevice;
  return hipMemcpyHostToHost;
}

// copy an exit-wave stack between the library's storage and float32 complex
pty_status copy_waves_out(pty_scan* s, size_t off, float* dst, int on_device) {
  const size_t count = size_t(s->J) * s->N * s->N;
  if (!s->fp16) {
    PTY_HIP(s, hipMemcpyAsync(dst, s->ws + off, count * 8, kind(1, on_device), s->stream), "copy out");
    return PTY_OK;
  }
  if (on_device) {
    PTY_HIP(s, launch_convert_state(1, 0, nullptr, nullptr, s->ws + off, reinterpret_cast<float2*>(dst), count,
                                    s->scale, s->inv_scale, s->stream),
            "convert out");
    return PTY_OK;
  }
  std::vector<_Float16> h(count * 2);
  PTY_HIP(s, hipMemcpyAsync(h.data(), s->ws + off, count * 4, hipMemcpyDeviceToHost, s->stream), "copy out");
  PTY_HIP(s, hipStreamSynchronize(s->stream), "sync");
  for (size_t i = 0; i < count * 2; ++i) dst[i] = float(h[i]) * s->inv_scale;
  return PTY_OK;
}

pty_status copy_waves_in(pty_scan* s, size_t off, const float* src, int on_device) {
  const size_t count = size_t(s->J) * s->N * s->N;
  if (!s->fp16) {
    PTY_HIP(s, hipMemcpyAsync(s->ws + off, src, count * 8, kind(on_device, 1), s->stream), "copy in");
    return PTY_OK;
  }
  if (on_device) {
    PTY_HIP(s, launch_convert_state(1, 1, reinterpret_cast<const float2*>(src), s->ws + off, nullptr, nullptr, count,
                                    s->scale, s->inv_scale, s->stream),
            "convert in");
    return PTY_OK;
  }
  std::vector<_Float16> h(count * 2);
  for (size_t i = 0; i < count * 2; ++i) h[i] = _Float16(src[i] * s->scale);
  PTY_HIP(s, hipMemcpyAsync(s->ws + off, h.data(), count * 4, hipMemcpyHostToDevice, s->stream), "copy in");
  PTY_HIP(s, hipStreamSynchronize(s->stream), "sync");
  return PTY_OK;
}

bool finite_abc(double a, double b, double c) { return std::isfinite(a) && std::isfinite(b) && std::isfinite(c); }

pty_status named_abc(int32_t algo, double prm, double* a, double* b, double* c) {
  switch (algo) {
    case PTY_DC: *a = 1; *b = 1; *c = 1; return PTY_OK;
    case PTY_AR: *a = 1; *b = 1; *c = 2; return PTY_OK;
    case PTY_DR: *a = 0.5; *b = 2; *c = 2; return PTY_OK;
    case PTY_SF: *a = 1; *b = 2; *c = 1; return PTY_OK;
    case PTY_RAAR: *a = 0.5; *b = 2 * prm; *c = 2; return PTY_OK;
    case PTY_RRR: *a = prm / 2; *b = 2; *c = 2; return PTY_OK;
    case PTY_TLAMBDA: *a = 1 / (1 + prm); *b = 1 + prm; *c = 1 + prm; return PTY_OK;
    default: return fail(PTY_ERR_INVALID_ARG, "unknown algorithm");
  }
}

pty_status create_impl(const pty_scan_desc* d, void* d_ws, size_t ws_bytes, void* stream, pty_scan** out) {
  if (!out) return fail(PTY_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!desc_shape_ok(d, &why)) return fail(PTY_ERR_INVALID_ARG, why);
  if (!d->pos || !d->intensity || !d->init_object || !d->init_probe)
    return fail(PTY_ERR_INVALID_ARG, "pos, intensity, init_object and init_probe must be non-NULL");
  if (!d_ws) return fail(PTY_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign != 0) return fail(PTY_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(PTY_ERR_OUT_OF_MEMORY, "workspace too small: need " + std::to_string(L.total) + " bytes");

  const int N = d->n, J = d->n_pos, H = d->obj_h, W = d->obj_w;
  // positions: validate on the host
  std::vector<int32_t> pos(size_t(J) * 2);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (d->inputs_on_device) {
    hipError_t e = hipMemcpyAsync(pos.data(), d->pos, pos.size() * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_fail(nullptr, e, "reading positions");
  } else {
    std::memcpy(pos.data(), d->pos, pos.size() * 4);
  }
  for (int j = 0; j < J; ++j) {
    const int r = pos[2 * j], c = pos[2 * j + 1];
    if (r < 0 || c < 0 || r > H - N || c > W - N)
      return fail(PTY_ERR_INVALID_ARG, "position " + std::to_string(j) + " puts the window outside the object");
  }
  // tile lists (ascending j)
  std::vector<int> cnt(size_t(L.n_tiles) + 1, 0);
  for (int j = 0; j < J; ++j) {
    const int r = pos[2 * j], c = pos[2 * j + 1];
    for (int ty = r / kTileH; ty <= (r + N - 1) / kTileH; ++ty)
      for (int tx = c / kTileW; tx <= (c + N - 1) / kTileW; ++tx) cnt[size_t(ty) * L.tiles_x + tx + 1]++;
  }
  for (int t = 0; t < L.n_tiles; ++t) cnt[t + 1] += cnt[t];
  // entries (j, row, col, 0): the concur kernel needs no second lookup of the position
  std::vector<int> list(4 * size_t(std::max(1, cnt[L.n_tiles])), 0);
  std::vector<int> fillp(cnt.begin(), cnt.end() - 1);
  for (int j = 0; j < J; ++j) {
    const int r = pos[2 * j], c = pos[2 * j + 1];
    for (int ty = r / kTileH; ty <= (r + N - 1) / kTileH; ++ty)
      for (int tx = c / kTileW; tx <= (c + N - 1) / kTileW; ++tx) {
        int* e = &list[4 * size_t(fillp[size_t(ty) * L.tiles_x + tx]++)];
        e[0] = j; e[1] = r; e[2] = c;
      }
  }
  if (cnt[L.n_tiles] > L.max_list) return fail(PTY_ERR_INVALID_ARG, "internal: tile list bound exceeded");

  pty_scan* s = new (std::nothrow) pty_scan();
  if (!s) return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->N = N; s->J = J; s->H = H; s->W = W;
  s->fp16 = d->storage == PTY_STORE_FP16;
  s->blind = d->blind;
  s->probe_update_start = d->probe_update_start;
  s->full_metrics = d->full_metrics;
  s->tau = d->tau > 0 ? d->tau : kDefaultTau;
  s->stream = st;
  s->ws = reinterpret_cast<char*>(d_ws);
  s->L = L;
  s->hpos = pos;
  if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;

  auto bail = [&](pty_status r) { delete s; return r; };
  const size_t nn = size_t(N) * N;
  const int dev = d->inputs_on_device;
#define CK(call, what)                                               \
  do {                                                               \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) return bail(device_fail(nullptr, e_, what)); \
  } while (0)
  CK(hipMemsetAsync(s->ws, 0, L.total, st), "clear workspace");
  CK(hipMemcpyAsync(s->ws + L.pos, pos.data(), pos.size() * 4, hipMemcpyHostToDevice, st), "positions");
  CK(hipMemcpyAsync(s->ws + L.tile_off, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice, st), "tile offsets");
  CK(hipMemcpyAsync(s->ws + L.tile_list, list.data(), size_t(cnt[L.n_tiles]) * 16, hipMemcpyHostToDevice, st),
     "tile lists");
  std::vector<float2> tw(N);
  for (int m = 0; m < N; ++m) {
    const double ang = -2.0 * 3.14159265358979323846 * double(m) / double(N);
    tw[m] = make_float2(float(std::cos(ang)), float(std::sin(ang)));
  }
  CK(hipMemcpyAsync(s->ws + L.tw, tw.data(), size_t(N) * 8, hipMemcpyHostToDevice, st), "twiddles");
  CK(hipMemcpyAsync(s->ws + L.obj, d->init_object, size_t(H) * W * 8, kind(dev, 1), st), "object");
  CK(hipMemcpyAsync(s->ws + L.probe, d->init_probe, nn * 8, kind(dev, 1), st), "probe");
  // intensities: stage host data in the x buffer (at least 4 bytes per value)
  const float* isrc = d->intensity;
  if (!dev) {
    CK(hipMemcpyAsync(s->ws + L.x, d->intensity, size_t(J) * nn * 4, hipMemcpyHostToDevice, st), "intensity");
    isrc = s->at<float>(L.x);
  }
  int* bad = s->at<int>(L.flag);
  CK(launch_amp_prepare(N, isrc, s->at<float>(L.amp), J, bad, st), "amplitudes");
  CK(hipMemsetAsync(s->ws + L.x, 0, size_t(J) * nn * L.elem_bytes, st), "clear x");
  CK(launch_max_abs2_parts(s->at<float2>(L.probe), nn, s->at<float>(L.pmax), L.npb, st), "probe max");
  // float16 scale: max |x| = max|P| max|O| brought to about 2^8
  // object maxima go to the tile-max buffer, one part per tile at most
  const int onp = std::min(256, L.n_tiles);
  std::vector<float> omax(onp), pmax(L.npb);
  CK(launch_max_abs2_parts(s->at<float2>(L.obj), size_t(H) * W, s->at<float>(L.tile_max), onp, st), "object max");
  int nbad = 0;
  CK(hipMemcpyAsync(&nbad, bad, 4, hipMemcpyDeviceToHost, st), "flag");
  CK(hipMemcpyAsync(omax.data(), s->ws + L.tile_max, size_t(onp) * 4, hipMemcpyDeviceToHost, st), "object max");
  CK(hipMemcpyAsync(pmax.data(), s->ws + L.pmax, size_t(L.npb) * 4, hipMemcpyDeviceToHost, st), "probe max");
  CK(hipStreamSynchronize(st), "create");
#undef CK
  if (nbad > 0) return bail(fail(PTY_ERR_INVALID_ARG, "intensity has negative or non-finite values"));
  const double om = std::sqrt(double(*std::max_element(omax.begin(), omax.end())));
  const double pm = std::sqrt(double(*std::max_element(pmax.begin(), pmax.end())));
  if (!std::isfinite(om) || !std::isfinite(pm)) return bail(fail(PTY_ERR_INVALID_ARG, "object or probe not finite"));
  if (s->fp16) {
    const double xm = om * pm;
    int e = 0;
    if (xm > 0) e = 8 - int(std::ceil(std::log2(xm)));
    e = std::max(-100, std::min(100, e));
    s->scale = float(std::ldexp(1.0, e));
    s->inv_scale = float(std::ldexp(1.0, -e));
  }
  s->mode = MODE_INIT;
  *out = s;
  return PTY_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t pty_workspace_bytes(const pty_scan_desc* desc) {
  try {
    std::string why;
    if (!desc_shape_ok(desc, &why)) {
      g_last_error = why;
      return 0;
    }
    return make_layout(desc).total;
  } catch (...) {
    return 0;
  }
}

pty_status pty_create_scan(const pty_scan_desc* desc, void* d_workspace, size_t ws_bytes, void* stream,
                           pty_scan** out) {
  try {
    return create_impl(desc, d_workspace, ws_bytes, stream, out);
  } catch (const std::exception& e) {
    return fail(PTY_ERR_OUT_OF_MEMORY, e.what());
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unknown error in pty_create_scan");
  }
}

pty_status pty_set_algorithm(pty_scan* scan, double a, double b, double c) {
  pty_status st = check_usable(scan);
  if (st != PTY_OK) return st;
  if (!finite_abc(a, b, c)) return fail(PTY_ERR_INVALID_ARG, "a, b, c must be finite");
  if (a == 0.0) return fail(PTY_ERR_INVALID_ARG, "a must be nonzero");
  scan->a = a;
  scan->b = b;
  scan->c = c;
  return PTY_OK;
}

pty_status pty_set_algorithm_named(pty_scan* scan, int32_t algorithm, double param) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (!std::isfinite(param)) return fail(PTY_ERR_INVALID_ARG, "param must be finite");
    double a, b, c;
    st = named_abc(algorithm, param, &a, &b, &c);
    if (st != PTY_OK) return st;
    return pty_set_algorithm(scan, a, b, c);
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_algorithm_abc(int32_t algorithm, double param, double* abc) {
  if (!abc) return fail(PTY_ERR_INVALID_ARG, "abc is NULL");
  if (!std::isfinite(param)) return fail(PTY_ERR_INVALID_ARG, "param must be finite");
  double a, b, c;
  const pty_status st = named_abc(algorithm, param, &a, &b, &c);
  if (st != PTY_OK) return st;
  abc[0] = a;
  abc[1] = b;
  abc[2] = c;
  return PTY_OK;
}

int32_t pty_state_form(const pty_scan* scan) {
  if (!scan) return -1;
  return use_blend(scan) ? 1 : 0;
}

pty_status pty_iterate(pty_scan* scan, int32_t n) {
  pty_status st = check_usable(scan);
  if (st != PTY_OK) return st;
  if (n < 0) return fail(PTY_ERR_INVALID_ARG, "n must be >= 0");
  try {
    for (int32_t i = 0; i < n; ++i) {
      st = launch_iteration(scan);
      if (st != PTY_OK) return st;
    }
  } catch (...) {
    scan->failed = true;
    return fail(PTY_ERR_DEVICE, "exception during iterate");
  }
  return PTY_OK;
}

pty_status pty_iterate_many(pty_scan* const* scans, int32_t count, int32_t n) {
  if (count < 0 || (count > 0 && !scans)) return fail(PTY_ERR_INVALID_ARG, "bad scans/count");
  if (n < 0) return fail(PTY_ERR_INVALID_ARG, "n must be >= 0");
  for (int32_t i = 0; i < count; ++i) {
    pty_status st = check_usable(scans[i]);
    if (st != PTY_OK) return st;
    for (int32_t q = 0; q < i; ++q)
      if (scans[q] == scans[i]) return fail(PTY_ERR_INVALID_ARG, "a scan is listed twice");
  }
  bool grouped = count > 1;
  for (int32_t i = 0; i < count && grouped; ++i)
    grouped = scans[i]->stream == scans[0]->stream && !scans[i]->prof;
  try {
    for (int32_t it = 0; it < n; ++it) {
      if (grouped) {
        const pty_status st = launch_iteration_grouped(scans, count);
        if (st != PTY_OK) return st;
        continue;
      }
      for (int32_t i = 0; i < count; ++i) {
        pty_status st = launch_iteration(scans[i]);
        if (st != PTY_OK) return st;
      }
    }
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "exception during iterate_many");
  }
  return PTY_OK;
}

pty_status pty_iterate_schedule(pty_scan* scan, const double* abc, int32_t n) {
  pty_status st = check_usable(scan);
  if (st != PTY_OK) return st;
  if (n < 0 || (n > 0 && !abc)) return fail(PTY_ERR_INVALID_ARG, "bad abc/n");
  for (int32_t i = 0; i < n; ++i) {
    if (!finite_abc(abc[3 * i], abc[3 * i + 1], abc[3 * i + 2]))
      return fail(PTY_ERR_INVALID_ARG, "schedule entry " + std::to_string(i) + ": a, b, c must be finite");
    if (abc[3 * i] == 0.0) return fail(PTY_ERR_INVALID_ARG, "schedule entry " + std::to_string(i) + ": a is zero");
  }
  try {
    for (int32_t i = 0; i < n; ++i) {
      scan->a = abc[3 * i];
      scan->b = abc[3 * i + 1];
      scan->c = abc[3 * i + 2];
      st = launch_iteration(scan);
      if (st != PTY_OK) return st;
    }
  } catch (...) {
    scan->failed = true;
    return fail(PTY_ERR_DEVICE, "exception during iterate_schedule");
  }
  return PTY_OK;
}

pty_status pty_set_concur_sweeps(pty_scan* scan, int32_t sweeps) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (sweeps < 1 || sweeps > kMaxSweeps) return fail(PTY_ERR_INVALID_ARG, "sweeps must be in [1, 64]");
    scan->sweeps = sweeps;
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_shadow(pty_scan* scan, float* obj_out, float* probe_out) {
  pty_status st = check_usable(scan);
  if (st != PTY_OK) return st;
  if (!obj_out || !probe_out) return fail(PTY_ERR_INVALID_ARG, "obj_out and probe_out must be device buffers");
  try {
    st = flush(scan, true);                    // x_k materialised
    if (st != PTY_OK) return st;
    const hipStream_t s = scan->stream;
    // unrelaxed divide of x_k into the y buffer (x is rewritten unchanged)
    DivideParams p = divide_params(scan);
    p.alpha = 0.f; p.beta = 0.f; p.gamma = 1.f;
    p.read_x = 1; p.read_y = 0; p.write_x = 1;
    p.c = 1.0f;
    st = launch_divide(scan, p, false);
    if (st != PTY_OK) return st;
    scan->y_valid = false;
    // the consensus runs in place; the outputs first receive the current
    // (O, P) and are swapped with the result afterwards
    float2* O = scan->at<float2>(scan->L.obj);
    float2* P = scan->at<float2>(scan->L.probe);
    const size_t no = size_t(scan->H) * scan->W, np = size_t(scan->N) * scan->N;
    PTY_HIP(scan, hipMemcpyAsync(obj_out, O, no * 8, hipMemcpyDeviceToDevice, s), "shadow copy");
    PTY_HIP(scan, hipMemcpyAsync(probe_out, P, np * 8, hipMemcpyDeviceToDevice, s), "shadow copy");
    MetricParams mp = metric_params(scan, metric_slices(scan->N, scan->L.n_tiles));   // writes no ring entry
    st = launch_concur(scan, mp, scan->blind && scan->k >= scan->probe_update_start, false);
    if (st != PTY_OK) return st;
    PTY_HIP(scan, launch_swap(O, reinterpret_cast<float2*>(obj_out), no, s), "shadow swap");
    PTY_HIP(scan, launch_swap(P, reinterpret_cast<float2*>(probe_out), np, s), "shadow swap");
    st = refresh_probe_max(scan);
    if (st != PTY_OK) return st;
  } catch (...) {
    scan->failed = true;
    return fail(PTY_ERR_DEVICE, "exception during shadow");
  }
  return PTY_OK;
}

// Batches of pairwise disjoint windows by dependency level: position j goes
// to the batch after the last one holding an overlapping position placed
// before it (further on while batches are full), so every overlapping pair
// keeps the order.
static std::vector<std::vector<int>> sp_batches(const std::vector<int>& pos, const std::vector<int>& order, int n,
                                                int max_batch) {
  std::vector<std::vector<int>> batches;
  std::vector<int> where(order.size(), -1);
  std::vector<int> placed;
  placed.reserve(order.size());
  for (int j : order) {
    int last = -1;
    for (int i : placed) {
      if (where[i] > last && std::abs(pos[2 * i] - pos[2 * j]) < n && std::abs(pos[2 * i + 1] - pos[2 * j + 1]) < n)
        last = where[i];
    }
    int b = last + 1;
    while (max_batch > 0 && b < int(batches.size()) && int(batches[b].size()) >= max_batch) ++b;
    if (b == int(batches.size())) batches.emplace_back();
    batches[b].push_back(j);
    where[j] = b;
    placed.push_back(j);
  }
  return batches;
}

pty_status pty_sp_iterate(pty_scan* scan, const int32_t* order, int32_t max_batch, double alpha, double beta) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(PTY_ERR_INVALID_ARG, "alpha, beta must be finite");
    if (max_batch < 0) return fail(PTY_ERR_INVALID_ARG, "max_batch must be >= 0");
    const int J = scan->J, N = scan->N;
    // the probe steps of a batch (up to J of N^2 complex float32) live in the
    // exit-wave buffers x and y, which are adjacent
    if (size_t(J) * N * N * 8 > scan->L.y + size_t(J) * N * N * scan->L.elem_bytes - scan->L.x)
      return fail(PTY_ERR_DEVICE, "internal: exit-wave buffers too small for the probe steps");
    std::vector<int> ord(J);
    if (order) {
      std::vector<char> seen(J, 0);
      for (int i = 0; i < J; ++i) {
        const int j = order[i];
        if (j < 0 || j >= J || seen[j]) return fail(PTY_ERR_INVALID_ARG, "order must be a permutation of 0..J-1");
        seen[j] = 1;
        ord[i] = j;
      }
    } else {
      for (int i = 0; i < J; ++i) ord[i] = i;
    }
    try {
      st = flush(scan, false);                  // metrics of the previous iteration, if pending
      if (st != PTY_OK) return st;
      const auto batches = sp_batches(scan->hpos, ord, N, max_batch);
      scan->sp_members.clear();
      for (const auto& b : batches) scan->sp_members.insert(scan->sp_members.end(), b.begin(), b.end());
      const hipStream_t s = scan->stream;
      int* d_list = scan->at<int>(scan->L.sp_list);
      PTY_HIP(scan, hipMemcpyAsync(d_list, scan->sp_members.data(), size_t(J) * 4, hipMemcpyHostToDevice, s),
              "batch lists");
      const bool blind = scan->blind && scan->k >= scan->probe_update_start;
      DivideParams p = divide_params(scan);
      p.alpha = 1.f;                            // psi = P S_j O
      p.c = 1.0f;
      p.obj_out = scan->at<float2>(scan->L.obj);
      p.contrib = scan->at<float2>(scan->L.x);  // x and y hold no state during sequential projections
      p.pmax_part = scan->at<float>(scan->L.pmax);
      p.npb = scan->L.npb;
      p.sp_alpha = float(alpha);
      p.sp_beta = float(beta);
      p.sp_blind = blind;
      p.sp_omax = N == 256 ? scan->at<float>(scan->L.sp_omax) : nullptr;
      SpProbeParams q{};
      q.probe = scan->at<float2>(scan->L.probe);
      q.contrib = p.contrib;
      q.N = N;
      q.pmax_part = scan->at<float>(scan->L.pmax);
      int off = 0;
      for (const auto& b : batches) {
        p.batch = d_list + off;
        PTY_HIP(scan, timed(scan, PTY_K_DIVIDE, [&] { return launch_sp_batch(N, p, int(b.size()), s); }),
                "sequential projection launch");
        if (blind) {
          q.count = int(b.size());
          PTY_HIP(scan, timed(scan, PTY_K_PROBE, [&] { return launch_sp_probe(q, s); }), "probe step launch");
        }
        off += int(b.size());
      }
      MetricParams m = metric_params(scan, 1);
      m.k_cur = scan->k;
      PTY_HIP(scan, launch_metric_slices(m, s), "metrics launch");
      PTY_HIP(scan, launch_probe_final(final_params(scan, m), 0, s), "metrics launch");
      scan->sp_batches_last = int(batches.size());
      scan->k += 1;
      scan->mode = MODE_INIT;                   // the next generalised iteration starts from x = P S_j O
      scan->x_valid = scan->y_valid = false;
      scan->prev_metrics_done = true;
    } catch (...) {
      scan->failed = true;
      return fail(PTY_ERR_DEVICE, "exception during sequential projections");
    }
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

int32_t pty_sp_last_batches(const pty_scan* scan) { return scan ? scan->sp_batches_last : -1; }

pty_status pty_object_error(pty_scan* scan, const float* truth, int32_t r0, int32_t c0, int32_t h, int32_t w,
                            double* err) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (!truth || !err) return fail(PTY_ERR_INVALID_ARG, "truth and err must be given");
    if (h < 1 || w < 1 || r0 < 0 || c0 < 0 || r0 + h > scan->H || c0 + w > scan->W)
      return fail(PTY_ERR_INVALID_ARG, "the box must lie inside the object");
    double* part = scan->at<double>(scan->L.eval);
    const int blocks = object_error_blocks((long long)h * w);
    PTY_HIP(scan, launch_object_error(scan->at<float2>(scan->L.obj), scan->W, reinterpret_cast<const float2*>(truth),
                                      r0, c0, h, w, part, blocks, part + 4 * blocks, scan->stream),
            "object error");
    double out = 0.0;
    PTY_HIP(scan, hipMemcpyAsync(&out, part + 4 * blocks, 8, hipMemcpyDeviceToHost, scan->stream), "copy");
    PTY_HIP(scan, hipStreamSynchronize(scan->stream), "synchronize");
    *err = out;
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_object_error_noalloc(const float* obj, int32_t obj_h, int32_t obj_w, const float* truth, int32_t r0,
                                    int32_t c0, int32_t h, int32_t w, double* err, void* stream) {
  try {
    if (!obj || !truth || !err) return fail(PTY_ERR_INVALID_ARG, "obj, truth and err must be device pointers");
    if (obj_h < 1 || obj_w < 1 || int64_t(obj_h) * obj_w > (int64_t(1) << 31))
      return fail(PTY_ERR_INVALID_ARG, "object size out of range");
    if (h < 1 || w < 1 || r0 < 0 || c0 < 0 || int64_t(r0) + h > obj_h || int64_t(c0) + w > obj_w)
      return fail(PTY_ERR_INVALID_ARG, "the box must lie inside the object");
    const long long pixels = (long long)h * w;
    if (object_error_blocks(pixels) > kErrScratchBlocks)
      return fail(PTY_ERR_INVALID_ARG, "box of " + std::to_string(pixels) + " pixels exceeds the static scratch of " +
                                           std::to_string((long long)kErrScratchBlocks * kErrPixelsPerBlock) +
                                           " pixels");
    const hipError_t e = object_error_static(reinterpret_cast<const float2*>(obj), obj_w,
                                             reinterpret_cast<const float2*>(truth), r0, c0, h, w, err,
                                             reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_fail(nullptr, e, "object error (static scratch)");
    return PTY_OK;
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_synchronize(pty_scan* scan) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    PTY_HIP(scan, hipStreamSynchronize(scan->stream), "synchronize");
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

static pty_status get_array(pty_scan* scan, size_t off, size_t floats, float* dst, size_t n_floats, int on_dev) {
  pty_status st = check_usable(scan);
  if (st != PTY_OK) return st;
  if (!dst) return fail(PTY_ERR_INVALID_ARG, "dst is NULL");
  if (n_floats < floats) return fail(PTY_ERR_INVALID_ARG, "dst too small: need " + std::to_string(floats) + " floats");
  PTY_HIP(scan, hipMemcpyAsync(dst, scan->ws + off, floats * 4, kind(1, on_dev ? 1 : 0), scan->stream), "copy");
  PTY_HIP(scan, hipStreamSynchronize(scan->stream), "synchronize");
  return PTY_OK;
}

pty_status pty_get_object(pty_scan* scan, float* dst, size_t n_floats, int32_t dst_on_device) {
  try {
    if (!scan) return fail(PTY_ERR_INVALID_ARG, "scan is NULL");
    return get_array(scan, scan->L.obj, size_t(scan->H) * scan->W * 2, dst, n_floats, dst_on_device);
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_get_probe(pty_scan* scan, float* dst, size_t n_floats, int32_t dst_on_device) {
  try {
    if (!scan) return fail(PTY_ERR_INVALID_ARG, "scan is NULL");
    return get_array(scan, scan->L.probe, size_t(scan->N) * scan->N * 2, dst, n_floats, dst_on_device);
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

static pty_status read_ring(pty_scan* scan, std::vector<double>& ring) {
  ring.resize(size_t(scan->L.cap) * kRingFields);
  PTY_HIP(scan, hipMemcpyAsync(ring.data(), scan->ws + scan->L.ring, ring.size() * 8, hipMemcpyDeviceToHost,
                               scan->stream),
          "metrics copy");
  PTY_HIP(scan, hipStreamSynchronize(scan->stream), "synchronize");
  return PTY_OK;
}

pty_status pty_get_metrics(pty_scan* scan, pty_metrics* out) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (!out) return fail(PTY_ERR_INVALID_ARG, "out is NULL");
    if (scan->k == 0) return fail(PTY_ERR_BAD_STATE, "no iteration has run");
    st = flush(scan, false);
    if (st != PTY_OK) return st;
    std::vector<double> ring;
    st = read_ring(scan, ring);
    if (st != PTY_OK) return st;
    const int64_t k = scan->k - 1;
    const double* e = ring.data() + (k % scan->L.cap) * kRingFields;
    out->iteration = k;
    out->fourier_err = e[1];
    out->consistency_err = e[2];
    out->change = e[3];
    // NaN in the consistency or change slot marks a metric that was not formed
    // (blend form, sequential projections); divergence shows in the Fourier
    // error, which every iteration forms, or as an infinite metric
    if (!std::isfinite(e[1]) || std::isinf(e[2]) || std::isinf(e[3]))
      return fail(PTY_ERR_DIVERGED, "a metric of the last iteration is not finite");
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_get_metric_history(pty_scan* scan, pty_metrics* dst, int32_t cap, int32_t* n_out) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (!n_out || (cap > 0 && !dst) || cap < 0) return fail(PTY_ERR_INVALID_ARG, "bad dst/cap/n_out");
    st = flush(scan, false);
    if (st != PTY_OK) return st;
    std::vector<double> ring;
    st = read_ring(scan, ring);
    if (st != PTY_OK) return st;
    const int64_t avail = std::min<int64_t>(scan->k, scan->L.cap);
    const int64_t n = std::min<int64_t>(avail, cap);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t k = scan->k - n + i;
      const double* e = ring.data() + (k % scan->L.cap) * kRingFields;
      dst[i].iteration = k;
      dst[i].fourier_err = e[1];
      dst[i].consistency_err = e[2];
      dst[i].change = e[3];
    }
    *n_out = int32_t(n);
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

int64_t pty_get_iteration(const pty_scan* scan) { return scan ? scan->k : -1; }

pty_status pty_get_state(pty_scan* scan, float* x, float* y, float* obj, float* probe, int32_t on_device) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (on_device != 0 && on_device != 1) return fail(PTY_ERR_INVALID_ARG, "on_device must be 0 or 1");
    if (x) {
      st = flush(scan, true);
      if (st != PTY_OK) return st;
      st = copy_waves_out(scan, scan->L.x, x, on_device);
      if (st != PTY_OK) return st;
    }
    if (y) {
      st = copy_waves_out(scan, scan->L.y, y, on_device);
      if (st != PTY_OK) return st;
    }
    if (obj) PTY_HIP(scan, hipMemcpyAsync(obj, scan->ws + scan->L.obj, size_t(scan->H) * scan->W * 8,
                                          kind(1, on_device), scan->stream), "copy object");
    if (probe) PTY_HIP(scan, hipMemcpyAsync(probe, scan->ws + scan->L.probe, size_t(scan->N) * scan->N * 8,
                                            kind(1, on_device), scan->stream), "copy probe");
    PTY_HIP(scan, hipStreamSynchronize(scan->stream), "synchronize");
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_set_state(pty_scan* scan, const float* x, const float* y, const float* obj, const float* probe,
                         int32_t on_device) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (!x) return fail(PTY_ERR_INVALID_ARG, "x must be given");
    if (on_device != 0 && on_device != 1) return fail(PTY_ERR_INVALID_ARG, "on_device must be 0 or 1");
    st = copy_waves_in(scan, scan->L.x, x, on_device);
    if (st != PTY_OK) return st;
    if (y) {
      st = copy_waves_in(scan, scan->L.y, y, on_device);
      if (st != PTY_OK) return st;
    } else {
      PTY_HIP(scan, hipMemsetAsync(scan->ws + scan->L.y, 0, size_t(scan->J) * scan->N * scan->N * scan->L.elem_bytes,
                                   scan->stream), "clear y");
    }
    if (obj) PTY_HIP(scan, hipMemcpyAsync(scan->ws + scan->L.obj, obj, size_t(scan->H) * scan->W * 8,
                                          kind(on_device, 1), scan->stream), "copy object");
    if (probe) {
      PTY_HIP(scan, hipMemcpyAsync(scan->ws + scan->L.probe, probe, size_t(scan->N) * scan->N * 8,
                                   kind(on_device, 1), scan->stream), "copy probe");
      st = refresh_probe_max(scan);
      if (st != PTY_OK) return st;
    }
    PTY_HIP(scan, hipStreamSynchronize(scan->stream), "synchronize");
    scan->mode = MODE_MATERIAL;
    scan->x_valid = true;
    scan->y_valid = y != nullptr;
    scan->prev_metrics_done = true;
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_profile(pty_scan* scan, int32_t enable) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (enable < 0) return fail(PTY_ERR_INVALID_ARG, "enable must be >= 0");
    PTY_HIP(scan, drain_profile(scan), "profile drain");
    if (enable) {
      for (int i = 0; i < PTY_K_COUNT; ++i) {
        scan->prof_ms[i] = 0.0;
        scan->prof_n[i] = 0;
      }
    }
    scan->prof = enable != 0;
    scan->prof_every = enable > 0 ? enable : 1;
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

pty_status pty_profile_read(pty_scan* scan, double* ms, int64_t* launches, int32_t n) {
  try {
    pty_status st = check_usable(scan);
    if (st != PTY_OK) return st;
    if (n < 0 || (n > 0 && (!ms || !launches))) return fail(PTY_ERR_INVALID_ARG, "bad ms/launches/n");
    PTY_HIP(scan, drain_profile(scan), "profile drain");
    for (int i = 0; i < n; ++i) {
      ms[i] = i < PTY_K_COUNT ? scan->prof_ms[i] : 0.0;
      launches[i] = i < PTY_K_COUNT ? scan->prof_n[i] : 0;
    }
    return PTY_OK;
  } catch (const std::bad_alloc&) {
    return fail(PTY_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PTY_ERR_DEVICE, "unexpected exception");
  }
}

void pty_destroy_scan(pty_scan* scan) {
  if (!scan) return;
  if (!scan->failed) (void)hipStreamSynchronize(scan->stream);
  for (hipEvent_t e : scan->ev_pool) (void)hipEventDestroy(e);
  delete scan;
}

const char* pty_status_string(int32_t status) {
  switch (status) {
    case PTY_OK: return "ok";
    case PTY_ERR_INVALID_ARG: return "invalid argument";
    case PTY_ERR_OUT_OF_MEMORY: return "out of memory";
    case PTY_ERR_DEVICE: return "device error";
    case PTY_ERR_BAD_STATE: return "bad state";
    case PTY_ERR_DIVERGED: return "diverged";
    case PTY_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* pty_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
