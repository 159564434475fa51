// Divide step P^c_D of the generalised iteration, fused with the pending
// update of the previous iteration (see the formula in the header).
//
// For N <= 128 one work-group owns one diffraction pattern end to end:
//   prologue   x_k = alpha P S_j O + beta y_{k-1} + gamma x_{k-1}   (registers)
//   forward    2-D DFT of x_k  (three register stages, two LDS exchanges)
//   Fourier    y^ = (c A / |X| + 1 - c) X / N^2   -- the relaxed modulus
//              projection; since F is linear, c P_D x + (1 - c) x is formed
//              on the spectrum and needs no copy of x_k
//   inverse    2-D inverse DFT (mirror of the forward, two exchanges)
//   epilogue   store y_k (blend form: also w_k from the x_k kept in
//              registers; sequential projections: the object step into the
//              window and the probe step of the batch slot instead)
//
// The 2-D DFT of N = 4 M points per axis is split, for both axes, as
//   r = r2 + M r1,  k = k1 + 4 k2:
//   stage A: 4 x 4 DFT over (r1, c1), twiddle W_N^(r2 kr1 + c2 kc1)
//   stage B: M-point DFT over r2 -> kr2
//   stage C: M-point DFT over c2 -> kc2
// so the spectrum element (kr1 + 4 kr2, kc1 + 4 kc2) sits in registers of the
// stage-C thread; the amplitudes are stored in exactly that order at scan
// creation, which makes every HBM access of the kernel contiguous across a
// wavefront.
//
// For N = 256 (512 KiB per pattern, more than one CU's LDS) the divide runs as
// three passes (divide.hip): rows forward (with the prologue), columns
// forward + Fourier + columns inverse, rows inverse (with the epilogue).
//
// This header holds the fused kernel (N <= 128); each size is instantiated in
// its own translation unit (divide_n32/64/128.hip) so the sizes compile in
// parallel.
#pragma once

#include "divide_ops.hpp"

namespace pty {

// Which exit-wave buffers the divide prologue touches.  The common cases are
// compile-time so no load sits behind a per-element branch.  The PRO_W_*
// modes are the blend form: PRO_W_PENDING reads w and gathers P S_j O,
// PRO_W_MATERIAL reads a materialised x (alpha = 0), PRO_W_ZERO gathers only
// (w = 0: the first iteration, or a blend with beta' = gamma' = 0).
enum ProMode {
  PRO_GENERAL = 0, PRO_UPDATE = 1, PRO_MATERIAL = 2, PRO_INIT = 3, PRO_FLAGS = 4,
  PRO_W_PENDING = 5, PRO_W_MATERIAL = 6, PRO_W_ZERO = 7, PRO_SP = 8,
  PRO_Z = 9, PRO_Y_EC = 10, PRO_Y = 11, PRO_COUNT = 12
};

// Buffers and metrics of each x-form mode: read x, read y, write x, consistency
// and change partials.  PRO_Z / PRO_Y / PRO_Y_EC are the Fourier-only forms of
// DC and AR (x = P S_j O, nothing read or kept) and SF (x = P S_j O + beta y).
struct ModeBits {
  bool rx, ry, wx, ec, dx;
};
constexpr ModeBits kModeBits[PRO_COUNT] = {
    {true, true, true, true, true},     // GENERAL
    {true, true, true, false, false},   // UPDATE
    {true, false, true, false, false},  // MATERIAL
    {false, false, true, false, false}, // INIT
    {false, false, false, false, false},// FLAGS (runtime)
    {true, false, false, false, false}, // W_PENDING
    {true, false, false, false, false}, // W_MATERIAL
    {false, false, false, false, false},// W_ZERO
    {false, false, false, false, false},// SP
    {false, false, false, false, false},// Z
    {false, true, false, true, false},  // Y_EC
    {false, true, false, false, false}, // Y
};

template <int MODE>
struct Pro {
  static constexpr bool sp = MODE == PRO_SP;          // sequential projections (psi kept like x_k)
  static constexpr bool wf = MODE >= PRO_W_PENDING && MODE <= PRO_SP;
  static constexpr bool gather = MODE != PRO_W_MATERIAL;
  static constexpr bool rx(const DivideParams& p) { return MODE == PRO_FLAGS ? p.read_x : kModeBits[MODE].rx; }
  static constexpr bool ry(const DivideParams& p) { return MODE == PRO_FLAGS ? p.read_y : kModeBits[MODE].ry; }
  static constexpr bool wx(const DivideParams& p) { return MODE == PRO_FLAGS ? p.write_x : kModeBits[MODE].wx; }
  static constexpr bool ec(const DivideParams& p) { return MODE == PRO_FLAGS ? p.prev_ec : kModeBits[MODE].ec; }
  static constexpr bool dx(const DivideParams& p) { return MODE == PRO_FLAGS ? p.prev_dx : kModeBits[MODE].dx; }
};

inline int prologue_mode(const DivideParams& p) {
  if (p.wform) return p.read_x ? (p.alpha != 0.f ? PRO_W_PENDING : PRO_W_MATERIAL) : PRO_W_ZERO;
  const bool rx = p.read_x, ry = p.read_y, wx = p.write_x, ec = p.prev_ec, dx = p.prev_dx;
  for (int m : {PRO_GENERAL, PRO_UPDATE, PRO_MATERIAL, PRO_INIT, PRO_Z, PRO_Y_EC, PRO_Y}) {
    const ModeBits b = kModeBits[m];
    if (b.rx == rx && b.ry == ry && b.wx == wx && b.ec == ec && b.dx == dx) return m;
  }
  return PRO_FLAGS;
}

// Register/LDS geometry of the fused kernel.  Task orders:
//   stage A  qa = r2 * M + c2            (coalesced HBM access: c2 fastest)
//   stage B  qb = c2 * 16 + kk           (kk = 4 kr1 + kc1; holds r2 -> kr2)
//   stage C  qc = kr2 * 16 + kk          (holds c2 -> kc2)
// LDS entries are padded so the strided side of every exchange spreads over
// the banks.
template <int N, int T>
struct DivGeom {
  static constexpr int M = N / 4;
  static constexpr int E = N * N / T;      // complex values per thread
  static constexpr int SA = E / 16;        // stage-A tasks per thread
  static constexpr int SB = E / M;         // stage-B / C tasks per thread
  static constexpr int PA = M * 17;        // A <-> B plane (r2): entry c2 * 17 + kk
  static constexpr int PB = 16 * M + 16;   // B <-> C plane (c2): entry kr2 * 16 + kk, padded
  static constexpr int LDS = M * (PA > PB ? PA : PB);   // N = 128: 136 KiB, one pattern per CU
  // Split exchanges (N = 128): each runs in two passes over half the data, so
  // the work-group needs 68 KiB of LDS and two patterns share a CU, one's
  // transforms overlapping the other's memory traffic.  A <-> B passes take
  // the planes r2 of one stage-A set.  B <-> C is, for each kk, a transpose of
  // M rows (the threads) by M values; in pass h the thread of row r moves the
  // half u xor h of its values, u = r / (M/2): a symmetric choice, so every
  // thread receives exactly into the registers it has just sent.  Threads
  // with u = 1 (a uniform half of the work-group) hold their stage-B spectrum
  // and their stage-C sequence with the two halves swapped, so that every
  // thread sends and receives registers [h M/2, (h+1) M/2) in pass h: negating
  // the odd inputs of an M-point DFT swaps the halves of its output, and a
  // half-swapped input multiplies the output by (-1)^k.  Both are exact (the
  // butterflies are symmetric under a change of sign), and the modulus
  // projection commutes with the sign except where it sets the phase to zero.
  static constexpr int PB2 = (M / 2) * 16 + 16;   // B <-> C plane of one pass: entry (k % (M/2)) * 16 + kk
  static constexpr int LDS_SPLIT = (M / 2) * PA > M * PB2 ? (M / 2) * PA : M * PB2;
  // prologue elements whose loads are issued together: 4 (8 spilled 3
  // registers in the float32 general mode and 7 in float16 once x_k is
  // rounded to storage form; 4 spills none in the compile-time modes:
  // 125 -> 123 us float32, 90.7 -> 84.6 us float16 on the 1024-pattern scan,
  // same bits; 16 spilled 29 and was 13 % slower.  The rare runtime-flag
  // form spills about 60 either way.)
  static constexpr int GP = 4;
  static_assert(SA >= 1 && SB >= 1 && SA * 16 == E && SB * M == E, "geometry");
};

// Modes that run with split exchanges: N = 128, x form (the blend and SP
// forms keep x_k in registers and cannot share a CU anyway), compile-time
// buffer flags.
template <int N, int MODE>
constexpr bool split_exchange() {
  return N == 128 && MODE != PRO_FLAGS && !Pro<MODE>::wf;
}

// The divide of one pattern by one work-group; blk is the work-group's index
// within its scan's launch (the batch slot for sequential projections).
template <int N, int T, class St, int MODE>
__device__ __forceinline__ void divide_fused_body(const DivideParams& p, const int blk) {
  using G = DivGeom<N, T>;
  using PR = Pro<MODE>;
  constexpr int M = G::M, E = G::E, SA = G::SA, SB = G::SB, PA = G::PA, PB = G::PB, PB2 = G::PB2;
  constexpr bool SPLIT = split_exchange<N, MODE>();
  static_assert(!SPLIT || (SA == 2 && SB == 1 && T / M == M / 2), "split exchange geometry");
  __shared__ float2 lds[SPLIT ? G::LDS_SPLIT : G::LDS];
  __shared__ double red[MF_COUNT * (T / 64)];

  const unsigned tid = threadIdx.x;
  const int j = PR::sp ? p.batch[blk] : p.j_begin + blk;
  const size_t base = size_t(j) * (N * N);
  const int2 pj = p.pos[j];
  using elem = typename St::elem;
  elem* __restrict__ xb = reinterpret_cast<elem*>(p.x) + base;
  elem* __restrict__ yb = reinterpret_cast<elem*>(p.y) + base;
  const float* __restrict__ ab = p.amp + base;
  const float2* __restrict__ ob = p.obj + (size_t(pj.x) * p.obj_w + pj.y);
  const float2* __restrict__ pb = p.probe;
  const float2* __restrict__ tw = p.tw;
  const unsigned ow = p.obj_w;
  const bool rx = PR::rx(p), ry = PR::ry(p), wx = PR::wx(p), mec = PR::ec(p), mdx = PR::dx(p);
  const bool wx_blend = PR::wf && p.write_x;   // wave-uniform

  float2 v[E];
  float2 xk[PR::wf ? E : 1];   // blend form: x_k, kept for w_k (registers are not the limit: LDS is)
  float om = 0.0f;             // sequential projections: max |S_j O|^2 over the window
  float sp_ka = 0.f, sp_kb = 0.f;
  float2* ob_out = nullptr;   // the same window as ob (sequential projections write it)
  float ec_n = 0.f, ec_d = 0.f, dx_n = 0.f, dx_d = 0.f, ef_n = 0.f, ef_d = 0.f;

  // ---- prologue and stage A, set by set -----------------------------------
  // x_k = alpha P S_j O + beta y + gamma x in the stage-A layout; loads go out
  // GP elements at a time.  Then the 4x4 DFT over (r1, c1) and the twiddles
  // W_N^(r2 kr1 + c2 kc1).
  auto prologue_and_stage_a = [&](auto s) {
    const unsigned qa = tid + T * s.value;
    const unsigned r2 = qa / M, c2 = qa % M;
    static_for<0, 16, G::GP>([&](auto g0) {
      float2 zp[G::GP], zo[G::GP], xo[G::GP], yo[G::GP];
      static_for<0, G::GP>([&](auto q) {
        constexpr int e = g0.value + q.value;
        constexpr int r1 = e / 4, c1 = e % 4;
        const unsigned r = r2 + M * r1, c = c2 + M * c1;
        const unsigned idx = r * N + c;
        zp[q.value] = PR::gather ? pb[idx] : make_float2(0.f, 0.f);
        zo[q.value] = PR::gather ? ob[r * ow + c] : make_float2(0.f, 0.f);
        xo[q.value] = rx ? St::load(xb, idx, p.inv_scale) : make_float2(0.f, 0.f);
        yo[q.value] = ry ? St::load(yb, idx, p.inv_scale) : make_float2(0.f, 0.f);
      });
      static_for<0, G::GP>([&](auto q) {
        constexpr int e = g0.value + q.value;
        constexpr int r1 = e / 4, c1 = e % 4;
        const unsigned idx = (r2 + M * r1) * N + (c2 + M * c1);
        const float2 z = PR::gather ? cmul(zp[q.value], zo[q.value]) : make_float2(0.f, 0.f);
        // x_k as the storage keeps it (float16: rounded), so that a run
        // that stores x_k and reads it back continues with the same bits
        const float2 xf = PR::wf ? blend_x(z, xo[q.value], p.alpha)
                                 : update_x(z, yo[q.value], xo[q.value], p.alpha, p.beta, p.gamma);
        const typename St::elem xe = St::pack(xf, p.scale);
        if (wx) St::store_packed(xb, idx, xe);
        const float2 xn = PR::sp ? xf : St::unpack(xe, p.inv_scale);
        if constexpr (PR::sp) om = fmaxf(om, cnorm(zo[q.value]));
        if (mec) {
          const float dr = z.x - yo[q.value].x, di = z.y - yo[q.value].y;
          ec_n = fmaf(dr, dr, fmaf(di, di, ec_n));
          ec_d = fmaf(yo[q.value].x, yo[q.value].x, fmaf(yo[q.value].y, yo[q.value].y, ec_d));
        }
        if (mdx) {
          const float dr = xn.x - xo[q.value].x, di = xn.y - xo[q.value].y;
          dx_n = fmaf(dr, dr, fmaf(di, di, dx_n));
          dx_d = fmaf(xo[q.value].x, xo[q.value].x, fmaf(xo[q.value].y, xo[q.value].y, dx_d));
        }
        if constexpr (PR::wf) xk[s.value * 16 + e] = xn;
        v[s.value * 16 + e] = xn;
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    dft4x4_reg<false, s.value * 16>(v);
    const float2 wr1 = tw[r2], wr2 = tw[2 * r2], wr3 = tw[3 * r2];
    const float2 wc1 = tw[c2], wc2 = tw[2 * c2], wc3 = tw[3 * c2];
    static_for<0, 16>([&](auto e) {
      constexpr int kr1 = e.value / 4, kc1 = e.value % 4;
      float2 t = v[s.value * 16 + e.value];
      if constexpr (kr1 == 1) t = cmul(t, wr1);
      if constexpr (kr1 == 2) t = cmul(t, wr2);
      if constexpr (kr1 == 3) t = cmul(t, wr3);
      if constexpr (kc1 == 1) t = cmul(t, wc1);
      if constexpr (kc1 == 2) t = cmul(t, wc2);
      if constexpr (kc1 == 3) t = cmul(t, wc3);
      v[s.value * 16 + e.value] = t;
    });
    __builtin_amdgcn_sched_barrier(0);
  };
  // ---- exchange A -> B: element (r2, kk, c2) at plane r2, entry c2*17 + kk --
  static_for<0, SA>([&](auto s) { prologue_and_stage_a(s); });
  if constexpr (SPLIT) {
    // pass h: set h holds the planes r2 in [h M/2, (h+1) M/2); the values read
    // land in v[h M/2 ...], which held set h, sent before the barrier
    static_for<0, 2>([&](auto h) {
      const unsigned qa = tid + T * h.value;
      const unsigned r2 = qa / M - h.value * (M / 2), c2 = qa % M;
      static_for<0, 16>([&](auto kk) { lds[r2 * PA + c2 * 17 + kk.value] = v[h.value * 16 + kk.value]; });
      __syncthreads();
      const unsigned o = (tid / 16) * 17 + tid % 16;
      static_for<0, M / 2>([&](auto r) { v[h.value * (M / 2) + r.value] = lds[r.value * PA + o]; });
      __syncthreads();
    });
  } else {
    static_for<0, SA>([&](auto s) {
      const unsigned qa = tid + T * s.value;
      const unsigned r2 = qa / M, c2 = qa % M;
      static_for<0, 16>([&](auto kk) { lds[r2 * PA + c2 * 17 + kk.value] = v[s.value * 16 + kk.value]; });
    });
    __syncthreads();
    static_for<0, SB>([&](auto s) {
      const unsigned qb = tid + T * s.value;
      const unsigned o = (qb / 16) * 17 + qb % 16;
      static_for<0, M>([&](auto r2) { v[s.value * M + r2.value] = lds[r2.value * PA + o]; });
    });
    __syncthreads();
  }
  __builtin_amdgcn_sched_barrier(0);
  // ---- stage B forward: DFT over r2 -> kr2 --------------------------------
  // split exchanges: the upper half of the work-group negates its odd inputs,
  // so its spectrum comes out with the halves swapped
  const unsigned hi_half = __builtin_amdgcn_readfirstlane(tid / (T / 2));
  const float hs = (SPLIT && hi_half != 0) ? -1.0f : 1.0f;
  if constexpr (SPLIT) {
    static_for<1, M, 2>([&](auto r) { v[r.value] = make_float2(v[r.value].x * hs, v[r.value].y * hs); });
  }
  static_for<0, SB>([&](auto s) { dft_reg<M, false, 1, s.value * M>(v); });
  __builtin_amdgcn_sched_barrier(0);

  // ---- exchange B -> C: element (c2, kk, kr2) at plane c2, entry kr2*16 + kk
  if constexpr (SPLIT) {
    // pass h: row c2 sends registers [h M/2, (h+1) M/2) (its half u xor h of
    // the spectrum) to plane c2; row kr2 receives the same registers from the
    // planes c of its half u xor h
    const unsigned kk = tid % 16, row = tid / 16, rl = row % (M / 2);
    static_for<0, 2>([&](auto h) {
      constexpr int b = h.value * (M / 2);
      const unsigned c0 = (hi_half ^ h.value) * (M / 2);
      static_for<0, M / 2>([&](auto i) { lds[row * PB2 + i.value * 16 + kk] = v[b + i.value]; });
      __syncthreads();
      static_for<0, M / 2>([&](auto i) { v[b + i.value] = lds[(c0 + i.value) * PB2 + rl * 16 + kk]; });
      __syncthreads();
    });
  } else {
    static_for<0, SB>([&](auto s) {
      const unsigned qb = tid + T * s.value;
      const unsigned c2 = qb / 16, kk = qb % 16;
      static_for<0, M>([&](auto k) { lds[c2 * PB + k.value * 16 + kk] = v[s.value * M + k.value]; });
    });
    __syncthreads();
    static_for<0, SB>([&](auto s) {
      const unsigned qc = tid + T * s.value;
      static_for<0, M>([&](auto c) { v[s.value * M + c.value] = lds[c.value * PB + qc]; });
    });
    __syncthreads();
  }
  __builtin_amdgcn_sched_barrier(0);

  // ---- stage C forward, Fourier-space relaxed projection, stage C inverse --
  const float c = p.c, omc = 1.0f - p.c, inv_n2 = 1.0f / float(N * N);
  static_for<0, SB>([&](auto s) {
    dft_reg<M, false, 1, s.value * M>(v);
    const unsigned qc = tid + T * s.value;
    static_for<0, M>([&](auto kc2) {
      const float A = ab[kc2.value * (4 * N) + qc];
      v[s.value * M + kc2.value] = fourier_op(v[s.value * M + kc2.value], A, c, omc, inv_n2, ef_n, ef_d,
                                              (kc2.value & 1) ? hs : 1.0f);
    });
    dft_reg<M, true, 1, s.value * M>(v);
  });
  __builtin_amdgcn_sched_barrier(0);

  // ---- exchange C -> B, mirror of B -> C ------------------------------------
  if constexpr (SPLIT) {
    // mirror: row kr2 sends registers [h M/2, (h+1) M/2) to the planes c of
    // its half u xor h; row c2 receives them (its half u xor h of the spectrum)
    const unsigned kk = tid % 16, row = tid / 16, rl = row % (M / 2);
    static_for<0, 2>([&](auto h) {
      constexpr int b = h.value * (M / 2);
      const unsigned c0 = (hi_half ^ h.value) * (M / 2);
      static_for<0, M / 2>([&](auto i) { lds[(c0 + i.value) * PB2 + rl * 16 + kk] = v[b + i.value]; });
      __syncthreads();
      static_for<0, M / 2>([&](auto i) { v[b + i.value] = lds[row * PB2 + i.value * 16 + kk]; });
      __syncthreads();
    });
  } else {
    static_for<0, SB>([&](auto s) {
      const unsigned qc = tid + T * s.value;
      static_for<0, M>([&](auto c) { lds[c.value * PB + qc] = v[s.value * M + c.value]; });
    });
    __syncthreads();
    static_for<0, SB>([&](auto s) {
      const unsigned qb = tid + T * s.value;
      const unsigned c2 = qb / 16, kk = qb % 16;
      static_for<0, M>([&](auto k) { v[s.value * M + k.value] = lds[c2 * PB + k.value * 16 + kk]; });
    });
    __syncthreads();
  }
  __builtin_amdgcn_sched_barrier(0);
  // ---- stage B inverse -----------------------------------------------------
  // (a half-swapped spectrum gives (-1)^r2 times the sequence: undone here)
  static_for<0, SB>([&](auto s) { dft_reg<M, true, 1, s.value * M>(v); });
  if constexpr (SPLIT) {
    static_for<1, M, 2>([&](auto r) { v[r.value] = make_float2(v[r.value].x * hs, v[r.value].y * hs); });
  }
  __builtin_amdgcn_sched_barrier(0);

  // ---- exchange B -> A, mirror of A -> B; then per set the conjugate
  // twiddles, the 4x4 inverse DFT and the store of y --------------------------
  auto finish_set = [&](auto s) {
    // recompute the element offsets instead of keeping the prologue's alive
    // through the whole transform
    unsigned qa = tid + T * s.value;
    asm volatile("" : "+v"(qa));
    const unsigned r2 = qa / M, c2 = qa % M;
    const float2 wr1 = tw[r2], wr2 = tw[2 * r2], wr3 = tw[3 * r2];
    const float2 wc1 = tw[c2], wc2 = tw[2 * c2], wc3 = tw[3 * c2];
    static_for<0, 16>([&](auto e) {
      constexpr int kr1 = e.value / 4, kc1 = e.value % 4;
      float2 t = v[s.value * 16 + e.value];
      if constexpr (kr1 == 1) t = cmulc(t, wr1);
      if constexpr (kr1 == 2) t = cmulc(t, wr2);
      if constexpr (kr1 == 3) t = cmulc(t, wr3);
      if constexpr (kc1 == 1) t = cmulc(t, wc1);
      if constexpr (kc1 == 2) t = cmulc(t, wc2);
      if constexpr (kc1 == 3) t = cmulc(t, wc3);
      v[s.value * 16 + e.value] = t;
    });
    dft4x4_reg<true, s.value * 16>(v);
    if constexpr (PR::sp) {
      // d = psi' - psi; object step into the window, probe step to this slot
      static_for<0, 16, G::GP>([&](auto g0) {
        float2 pp[G::GP], oo[G::GP];
        static_for<0, G::GP>([&](auto q) {
          constexpr int e = g0.value + q.value;
          constexpr int r1 = e / 4, c1 = e % 4;
          const unsigned r = r2 + M * r1, c = c2 + M * c1;
          pp[q.value] = pb[r * N + c];
          oo[q.value] = ob_out[r * ow + c];
        });
        static_for<0, G::GP>([&](auto q) {
          constexpr int e = g0.value + q.value;
          constexpr int r1 = e / 4, c1 = e % 4;
          const unsigned r = r2 + M * r1, c = c2 + M * c1;
          const float2 d = csub(v[s.value * 16 + e], xk[s.value * 16 + e]);
          const float2 po = cmulc(d, pp[q.value]);       // conj(P) d
          ob_out[r * ow + c] = make_float2(fmaf(sp_ka, po.x, oo[q.value].x), fmaf(sp_ka, po.y, oo[q.value].y));
          if (p.sp_blind) {
            const float2 oc = cmulc(d, oo[q.value]);     // conj(S_j O) d
            p.contrib[size_t(blk) * (N * N) + r * N + c] = make_float2(sp_kb * oc.x, sp_kb * oc.y);
          }
        });
        __builtin_amdgcn_sched_barrier(0);
      });
    } else if (PR::wf && wx_blend) {
      // blend form: w_k from the x_k kept in registers since the prologue
      static_for<0, 16>([&](auto e) {
        constexpr int r1 = e.value / 4, c1 = e.value % 4;
        const unsigned idx = (r2 + M * r1) * N + (c2 + M * c1);
        const float2 yk = v[s.value * 16 + e.value];
        St::store(yb, idx, yk, p.scale);
        St::store(xb, idx, blend_w(xk[PR::wf ? s.value * 16 + e.value : 0], yk, p.next_beta, p.next_gamma),
                  p.scale);
      });
    } else {
      static_for<0, 16>([&](auto e) {
        constexpr int r1 = e.value / 4, c1 = e.value % 4;
        St::store(yb, (r2 + M * r1) * N + (c2 + M * c1), v[s.value * 16 + e.value], p.scale);
      });
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  if constexpr (SPLIT) {
    static_for<0, 2>([&](auto h) {
      const unsigned o = (tid / 16) * 17 + tid % 16;
      static_for<0, M / 2>([&](auto r) { lds[r.value * PA + o] = v[h.value * (M / 2) + r.value]; });
      __syncthreads();
      const unsigned qa = tid + T * h.value;
      const unsigned r2 = qa / M - h.value * (M / 2), c2 = qa % M;
      static_for<0, 16>([&](auto kk) { v[h.value * 16 + kk.value] = lds[r2 * PA + c2 * 17 + kk.value]; });
      if constexpr (h.value == 0) __syncthreads();
    });
  } else {
    static_for<0, SB>([&](auto s) {
      const unsigned qb = tid + T * s.value;
      const unsigned o = (qb / 16) * 17 + qb % 16;
      static_for<0, M>([&](auto r2) { lds[r2.value * PA + o] = v[s.value * M + r2.value]; });
    });
    __syncthreads();
    static_for<0, SA>([&](auto s) {
      const unsigned qa = tid + T * s.value;
      const unsigned r2 = qa / M, c2 = qa % M;
      static_for<0, 16>([&](auto kk) { v[s.value * 16 + kk.value] = lds[r2 * PA + c2 * 17 + kk.value]; });
    });
  }
  if constexpr (PR::sp) {
    // step sizes alpha / max|P|^2 and beta / max|S_j O|^2 (zero when the maximum is zero)
    __shared__ float fred[T / 64];
    float pm = 0.f;
    for (int i = 0; i < p.npb; ++i) pm = fmaxf(pm, p.pmax_part[i]);
    const float omx = block_max<T>(om, fred);
    sp_ka = pm > 0.f ? p.sp_alpha / pm : 0.f;
    sp_kb = omx > 0.f ? p.sp_beta / omx : 0.f;
    ob_out = p.obj_out + (size_t(pj.x) * p.obj_w + pj.y);
  }
  static_for<0, SA>([&](auto s) { finish_set(s); });

  // ---- per-pattern metric partials (float64 block sums) ----------------------
  double acc[MF_COUNT] = {ef_n, ef_d, ec_n, ec_d, dx_n, dx_d};
  block_sum<MF_COUNT, T>(acc, red);
  if (tid < MF_COUNT) p.met[size_t(j) * p.nslot * MF_COUNT + tid] = acc[tid];
}

template <int N, int T, class St, int MODE>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(split_exchange<N, MODE>() ? 4 : 2)))
void divide_fused_kernel(DivideParams p) {
  divide_fused_body<N, T, St, MODE>(p, int(blockIdx.x));
}

// Several scans in one launch (the served form): the same per-pattern work.
template <int N, int T, class St, int MODE>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(split_exchange<N, MODE>() ? 4 : 2)))
void divide_fused_group_kernel(Group<DivideParams> g) {
  const int b = int(blockIdx.x);
  const int sc = group_scan(g, b);
  divide_fused_body<N, T, St, MODE>(g.p[sc], b - g.first[sc]);
}

template <int N, int T, class St, int MODE>
static void launch_fused_mode(const DivideParams& p, int n_patterns, hipStream_t s) {
  // plain order: consecutive patterns round-robin over the XCDs measured faster
  // here than XCD-contiguous ranges (xcd_block)
  hipLaunchKernelGGL((divide_fused_kernel<N, T, St, MODE>), dim3(n_patterns), dim3(T), 0, s, p);
}

template <int N, int T, class St>
static hipError_t launch_fused(const DivideParams& p, int n_patterns, hipStream_t s) {
  switch (prologue_mode(p)) {
    case PRO_GENERAL: launch_fused_mode<N, T, St, PRO_GENERAL>(p, n_patterns, s); break;
    case PRO_UPDATE: launch_fused_mode<N, T, St, PRO_UPDATE>(p, n_patterns, s); break;
    case PRO_MATERIAL: launch_fused_mode<N, T, St, PRO_MATERIAL>(p, n_patterns, s); break;
    case PRO_INIT: launch_fused_mode<N, T, St, PRO_INIT>(p, n_patterns, s); break;
    case PRO_W_PENDING: launch_fused_mode<N, T, St, PRO_W_PENDING>(p, n_patterns, s); break;
    case PRO_W_MATERIAL: launch_fused_mode<N, T, St, PRO_W_MATERIAL>(p, n_patterns, s); break;
    case PRO_W_ZERO: launch_fused_mode<N, T, St, PRO_W_ZERO>(p, n_patterns, s); break;
    case PRO_Z: launch_fused_mode<N, T, St, PRO_Z>(p, n_patterns, s); break;
    case PRO_Y_EC: launch_fused_mode<N, T, St, PRO_Y_EC>(p, n_patterns, s); break;
    case PRO_Y: launch_fused_mode<N, T, St, PRO_Y>(p, n_patterns, s); break;
    default: launch_fused_mode<N, T, St, PRO_FLAGS>(p, n_patterns, s); break;
  }
  return hipGetLastError();
}

template <int N, int T, class St, int MODE>
static void launch_fused_group_mode(const Group<DivideParams>& g, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((divide_fused_group_kernel<N, T, St, MODE>), dim3(blocks), dim3(T), 0, s, g);
}

// Grouped launches exist for the compile-time modes of the iteration's steady
// state and first step; others return hipErrorInvalidValue (the host launches
// such scans one by one).
template <int N, int T, class St>
static hipError_t launch_fused_group(const Group<DivideParams>& g, int blocks, hipStream_t s) {
  switch (prologue_mode(g.p[0])) {
    case PRO_GENERAL: launch_fused_group_mode<N, T, St, PRO_GENERAL>(g, blocks, s); break;
    case PRO_UPDATE: launch_fused_group_mode<N, T, St, PRO_UPDATE>(g, blocks, s); break;
    case PRO_INIT: launch_fused_group_mode<N, T, St, PRO_INIT>(g, blocks, s); break;
    case PRO_W_PENDING: launch_fused_group_mode<N, T, St, PRO_W_PENDING>(g, blocks, s); break;
    case PRO_W_ZERO: launch_fused_group_mode<N, T, St, PRO_W_ZERO>(g, blocks, s); break;
    case PRO_Z: launch_fused_group_mode<N, T, St, PRO_Z>(g, blocks, s); break;
    case PRO_Y_EC: launch_fused_group_mode<N, T, St, PRO_Y_EC>(g, blocks, s); break;
    case PRO_Y: launch_fused_group_mode<N, T, St, PRO_Y>(g, blocks, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Entry points of one size: the divide in every prologue mode (alone and
// grouped), and the sequential-projection batch kernel.
#define PTY_DEFINE_FUSED(NN, TT)                                                            \
  hipError_t launch_fused_n##NN(int fp16, const DivideParams& p, int n_patterns, hipStream_t s) { \
    return fp16 ? launch_fused<NN, TT, StoreF16>(p, n_patterns, s)                          \
                : launch_fused<NN, TT, StoreF32>(p, n_patterns, s);                         \
  }                                                                                         \
  hipError_t launch_fused_group_n##NN(int fp16, const Group<DivideParams>& g, int blocks, hipStream_t s) { \
    return fp16 ? launch_fused_group<NN, TT, StoreF16>(g, blocks, s)                        \
                : launch_fused_group<NN, TT, StoreF32>(g, blocks, s);                       \
  }                                                                                         \
  hipError_t launch_sp_n##NN(const DivideParams& p, int count, hipStream_t s) {             \
    launch_fused_mode<NN, TT, StoreF32, PRO_SP>(p, count, s);                               \
    return hipGetLastError();                                                               \
  }

}  // namespace pty
