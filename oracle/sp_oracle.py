"""FP64 CPU oracle of Sequential Projections (SP) for blind ptychography.

TEST INFRASTRUCTURE ONLY (like pty_oracle): imported by the test-suite and
nothing on the product path; it shares no code with the GPU implementation.

The paper contrasts its product-space method with sequential projections: the
constraint sets are visited one after another, in a fixed order or in an
order shuffled between iterations, and the relaxation of each projection may
vary (Introduction).  In ptychography the sets are the per-position modulus
sets S_j = {(O, P) : |F(P S_j O)| = sqrt(I_j)}.  Reading taken here (listed
with the other readings in the design notes):

* one step onto S_j: psi = P S_j O, psi' = the Fourier-modulus projection of
  psi (the divide's rules: unnormalised F, phase 0 where F psi = 0),
  d = psi' - psi, then
      O <- O + alpha S_j^T[conj(P) d] / max |P|^2
      P <- P + beta conj(S_j O) d / max |S_j O|^2        (blind; S_j O before
                                                          this step's update)
  For a probe of constant modulus and alpha = 1 the object step is the exact
  projection (the new exit wave equals psi'); in general the factor
  |P|^2 / max |P|^2 <= 1 is a per-pixel under-relaxation that stays stable
  where the probe is weak.
* a schedule of batches: positions in one batch have pairwise disjoint
  windows and all start from the (O, P) at the start of the batch; object
  steps touch disjoint pixels, probe steps are summed in batch order and
  applied after the batch.  With a known probe a batch schedule built by
  dependency level from an order is exactly sequential SP in that order; with
  an updated probe, one position per batch is the strictly sequential
  algorithm and larger batches its mini-batch form.
"""
from __future__ import annotations

import numpy as np

from .pty_oracle import modulus_projection, fourier_error_terms


def windows_overlap(p, q, n):
    """Whether the n x n windows at top-left corners p and q share a pixel."""
    return abs(int(p[0]) - int(q[0])) < n and abs(int(p[1]) - int(q[1])) < n


def batches_by_level(pos, order, n, max_batch=0):
    """Batches of pairwise disjoint windows that keep every overlapping pair in
    the given order: position j goes to the batch after the last one holding
    an overlapping position placed before it (a later batch when that one is
    full, max_batch > 0)."""
    batches = []
    for j in order:
        last = -1
        for b, members in enumerate(batches):
            if any(windows_overlap(pos[j], pos[i], n) for i in members):
                last = b
        b = last + 1
        while max_batch > 0 and b < len(batches) and len(batches[b]) >= max_batch:
            b += 1
        if b == len(batches):
            batches.append([])
        batches[b].append(int(j))
    return batches


def sp_iteration(obj, probe, pos, amp, batches, alpha=1.0, beta=1.0, blind=True):
    """One SP iteration over the given batches.  Returns (O, P, E_F) with E_F
    the Fourier error of the exit waves met along the way."""
    obj = np.array(obj, dtype=np.complex128)
    probe = np.array(probe, dtype=np.complex128)
    amp = np.asarray(amp, dtype=np.float64)
    n = probe.shape[0]
    ef_num = ef_den = 0.0
    for members in batches:
        pmax = float(np.max(np.abs(probe) ** 2))
        dprobe = np.zeros_like(probe)
        new_obj = obj.copy()
        for j in members:
            p, q = int(pos[j][0]), int(pos[j][1])
            o_win = obj[p:p + n, q:q + n]
            psi = probe * o_win
            a, b = fourier_error_terms(psi[None], amp[j][None])
            ef_num += a
            ef_den += b
            d = modulus_projection(psi[None], amp[j][None])[0] - psi
            if pmax > 0:
                new_obj[p:p + n, q:q + n] = o_win + alpha * np.conj(probe) * d / pmax
            if blind:
                omax = float(np.max(np.abs(o_win) ** 2))
                if omax > 0:
                    dprobe += beta * np.conj(o_win) * d / omax
        obj = new_obj
        probe = probe + dprobe
    return obj, probe, (ef_num / ef_den if ef_den > 0 else float("nan"))


def sp_run(obj, probe, pos, amp, n_iter, orders=None, max_batch=0, alpha=1.0, beta=1.0, blind=True):
    """n_iter SP iterations; orders[i] is iteration i's order (ascending if None)."""
    n = np.asarray(probe).shape[0]
    efs = []
    for i in range(n_iter):
        order = range(len(pos)) if orders is None else orders[i]
        obj, probe, ef = sp_iteration(obj, probe, pos, amp, batches_by_level(pos, order, n, max_batch),
                                      alpha, beta, blind)
        efs.append(ef)
    return obj, probe, efs
