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
//   epilogue   store y_k
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
// three passes: rows forward (with the prologue), columns forward + Fourier +
// columns inverse, rows inverse (with the epilogue).
#include <algorithm>

#include "common.hpp"
#include "params.hpp"

namespace pty {

__device__ __forceinline__ float2 update_x(float2 z, float2 yo, float2 xo, float al, float be, float ga) {
  // x_k = alpha z + beta y + gamma x, evaluated in one fixed order everywhere
  float2 r;
  r.x = fmaf(ga, xo.x, fmaf(be, yo.x, al * z.x));
  r.y = fmaf(ga, xo.y, fmaf(be, yo.y, al * z.y));
  return r;
}

// Blend form: x_k = alpha z + w, one fused multiply-add per component.
__device__ __forceinline__ float2 blend_x(float2 z, float2 w, float al) {
  return make_float2(fmaf(al, z.x, w.x), fmaf(al, z.y, w.y));
}

// Blend form: w_k = gamma x_k + beta y_k.
__device__ __forceinline__ float2 blend_w(float2 x, float2 y, float be, float ga) {
  return make_float2(fmaf(ga, x.x, be * y.x), fmaf(ga, x.y, be * y.y));
}

// Relaxed modulus projection of one spectrum value, already scaled by 1/N^2
// for the inverse transform: X (c A / |X| + 1 - c) / N^2, and c A / N^2 (phase
// 0) where X = 0.  |X|^2 below the smallest normal float counts as zero.
// Branch-free (per-component selects, hardware reciprocal square root).
// Accumulates (|X| - A)^2 and A^2 in float32 per thread.
__device__ __forceinline__ float2 fourier_op(float2 X, float A, float c, float one_minus_c, float inv_n2,
                                             float& ef_num, float& ef_den) {
  const float m2 = fmaf(X.x, X.x, X.y * X.y);
  const bool nz = m2 >= 1.17549435e-38f;
  const float r = __builtin_amdgcn_rsqf(nz ? m2 : 1.0f);
  const float mag = nz ? m2 * r : 0.0f;
  const float d = mag - A;
  ef_num = fmaf(d, d, ef_num);
  ef_den = fmaf(A, A, ef_den);
  const float cA = c * A;
  const float f = fmaf(cA, r, one_minus_c) * inv_n2;
  float2 out;
  out.x = nz ? X.x * f : cA * inv_n2;
  out.y = nz ? X.y * f : 0.0f;
  return out;
}

// Which exit-wave buffers the divide prologue touches.  The common cases are
// compile-time so no load sits behind a per-element branch.  The PRO_W_*
// modes are the blend form: PRO_W_PENDING reads w and gathers P S_j O,
// PRO_W_MATERIAL reads a materialised x (alpha = 0), PRO_W_ZERO gathers only
// (w = 0: the first iteration, or a blend with beta' = gamma' = 0).
enum ProMode {
  PRO_GENERAL = 0, PRO_UPDATE = 1, PRO_MATERIAL = 2, PRO_INIT = 3, PRO_FLAGS = 4,
  PRO_W_PENDING = 5, PRO_W_MATERIAL = 6, PRO_W_ZERO = 7, PRO_SP = 8
};

template <int MODE>
struct Pro {
  static constexpr bool sp = MODE == PRO_SP;          // sequential projections (psi kept like x_k)
  static constexpr bool wf = MODE >= PRO_W_PENDING;
  static constexpr bool gather = MODE != PRO_W_MATERIAL;
  static constexpr bool rx(const DivideParams& p) {
    return MODE == PRO_FLAGS ? p.read_x : (MODE != PRO_INIT && MODE != PRO_W_ZERO && MODE != PRO_SP);
  }
  static constexpr bool ry(const DivideParams& p) {
    return MODE == PRO_FLAGS ? p.read_y : (MODE == PRO_GENERAL || MODE == PRO_UPDATE);
  }
  static constexpr bool wx(const DivideParams& p) { return MODE == PRO_FLAGS ? p.write_x : !wf; }
  static constexpr bool ec(const DivideParams& p) { return MODE == PRO_FLAGS ? p.prev_ec : MODE == PRO_GENERAL; }
  static constexpr bool dx(const DivideParams& p) { return MODE == PRO_FLAGS ? p.prev_dx : MODE == PRO_GENERAL; }
};

int prologue_mode(const DivideParams& p) {
  if (p.wform) return p.read_x ? (p.alpha != 0.f ? PRO_W_PENDING : PRO_W_MATERIAL) : PRO_W_ZERO;
  const bool met = p.prev_ec || p.prev_dx;
  if (p.read_x && p.read_y && p.write_x && p.prev_ec && p.prev_dx) return PRO_GENERAL;
  if (p.read_x && p.read_y && p.write_x && !met) return PRO_UPDATE;
  if (p.read_x && !p.read_y && p.write_x && !met) return PRO_MATERIAL;
  if (!p.read_x && !p.read_y && p.write_x && !met) return PRO_INIT;
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
#ifndef PTY_PROLOGUE_GROUP
#define PTY_PROLOGUE_GROUP 8
#endif
  static constexpr int GP = PTY_PROLOGUE_GROUP;  // prologue elements whose loads are issued together
  static_assert(SA >= 1 && SB >= 1 && SA * 16 == E && SB * M == E, "geometry");
};

template <int N, int T, class St, int MODE>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(2)))
void divide_fused_kernel(DivideParams p) {
  using G = DivGeom<N, T>;
  using PR = Pro<MODE>;
  constexpr int M = G::M, E = G::E, SA = G::SA, SB = G::SB, PA = G::PA, PB = G::PB;
  __shared__ float2 lds[G::LDS];
  __shared__ double red[MF_COUNT * (T / 64)];

  const unsigned tid = threadIdx.x;
  const int j = PR::sp ? p.batch[blockIdx.x] : p.j_begin + int(blockIdx.x);
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
        const float2 xn = PR::wf ? blend_x(z, xo[q.value], p.alpha)
                                 : update_x(z, yo[q.value], xo[q.value], p.alpha, p.beta, p.gamma);
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
        if (wx) St::store(xb, idx, xn, p.scale);
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
  __builtin_amdgcn_sched_barrier(0);
  // ---- stage B forward: DFT over r2 -> kr2 --------------------------------
  static_for<0, SB>([&](auto s) { dft_reg<M, false, 1, s.value * M>(v); });
  __builtin_amdgcn_sched_barrier(0);

  // ---- exchange B -> C: element (c2, kk, kr2) at plane c2, entry kr2*16 + kk
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
  __builtin_amdgcn_sched_barrier(0);

  // ---- stage C forward, Fourier-space relaxed projection, stage C inverse --
  const float c = p.c, omc = 1.0f - p.c, inv_n2 = 1.0f / float(N * N);
  static_for<0, SB>([&](auto s) {
    dft_reg<M, false, 1, s.value * M>(v);
    const unsigned qc = tid + T * s.value;
    static_for<0, M>([&](auto kc2) {
      const float A = ab[kc2.value * (4 * N) + qc];
      v[s.value * M + kc2.value] = fourier_op(v[s.value * M + kc2.value], A, c, omc, inv_n2, ef_n, ef_d);
    });
    dft_reg<M, true, 1, s.value * M>(v);
  });
  __builtin_amdgcn_sched_barrier(0);

  // ---- exchange C -> B, mirror of B -> C ------------------------------------
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
  __builtin_amdgcn_sched_barrier(0);
  // ---- stage B inverse -----------------------------------------------------
  static_for<0, SB>([&](auto s) { dft_reg<M, true, 1, s.value * M>(v); });
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
            p.contrib[size_t(blockIdx.x) * (N * N) + r * N + c] = make_float2(sp_kb * oc.x, sp_kb * oc.y);
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

// ---------------------------------------------------------------------------
// N = 256: three passes.  A work-group handles 16 rows (or 16 columns) of one
// pattern, 16 threads per line, 16 values per thread; a line's 256-point DFT
// is 16 x 16 with one LDS exchange inside the group.  The column pass keeps
// its exchange tiles interleaved by column ([a][b][column]), so a wave's 16
// columns touch consecutive LDS words rather than one bank.
// ---------------------------------------------------------------------------
constexpr int L256 = 256;
constexpr int LP = 17;                 // padded pitch of a 16 x 16 exchange tile
constexpr int LT = 16 * LP;            // one line's exchange tile

template <class St>
__global__ __launch_bounds__(256) void rows256_fwd_kernel(DivideParams p) {
  __shared__ float2 lds[16 * LT];
  __shared__ double red[MF_COUNT * 4];
  const int tid = threadIdx.x;
  const int t = tid & 15, rl = tid >> 4;
  const int r = blockIdx.x * 16 + rl;
  const int j = p.j_begin + blockIdx.y;
  const size_t base = size_t(j) * L256 * L256;
  const int2 pj = p.pos[j];
  using elem = typename St::elem;
  elem* __restrict__ xs = reinterpret_cast<elem*>(p.x);
  const elem* ys = reinterpret_cast<const elem*>(p.y);  // may alias p.tmp
  float2 v[16];
  double acc[MF_COUNT];
#pragma unroll
  for (int q = 0; q < MF_COUNT; ++q) acc[q] = 0.0;

  // prologue: column c = t + 16 c1
  static_for<0, 16>([&](auto c1) {
    const int c = t + 16 * c1.value;
    const int idx = r * L256 + c;
    const float2 z = cmul(p.probe[idx], p.obj[size_t(pj.x + r) * p.obj_w + (pj.y + c)]);
    float2 xo = make_float2(0.f, 0.f), yo = make_float2(0.f, 0.f);
    if (p.read_x) xo = St::load(xs, base + idx, p.inv_scale);
    if (p.read_y) yo = St::load(ys, base + idx, p.inv_scale);
    const float2 xn = update_x(z, yo, xo, p.alpha, p.beta, p.gamma);
    if (p.prev_ec) {
      const double dr = double(z.x) - double(yo.x), di = double(z.y) - double(yo.y);
      acc[MF_EC_NUM] += dr * dr + di * di;
      acc[MF_EC_DEN] += double(yo.x) * yo.x + double(yo.y) * yo.y;
    }
    if (p.prev_dx) {
      const double dr = double(xn.x) - double(xo.x), di = double(xn.y) - double(xo.y);
      acc[MF_DX_NUM] += dr * dr + di * di;
      acc[MF_DX_DEN] += double(xo.x) * xo.x + double(xo.y) * xo.y;
    }
    if (p.write_x) St::store(xs, base + idx, xn, p.scale);
    v[c1.value] = xn;
  });
  dft_reg<16, false>(v);                                  // over c1 -> kc1
  static_for<1, 16>([&](auto k) { v[k.value] = cmul(v[k.value], p.tw[t * k.value]); });
  static_for<0, 16>([&](auto k) { lds[rl * LT + k.value * LP + t] = v[k.value]; });
  __syncthreads();
  static_for<0, 16>([&](auto c2) { v[c2.value] = lds[rl * LT + t * LP + c2.value]; });
  dft_reg<16, false>(v);                                  // over c2 -> kc2; thread t = kc1
  static_for<0, 16>([&](auto k2) { p.tmp[base + r * L256 + t + 16 * k2.value] = v[k2.value]; });

  block_sum<MF_COUNT, 256>(acc, red);
  if (tid >= MF_EC_NUM && tid < MF_COUNT)
    p.met[(size_t(j) * p.nslot + blockIdx.x) * MF_COUNT + tid] = acc[tid];
}

__global__ __launch_bounds__(256) void cols256_kernel(DivideParams p) {
  __shared__ float2 lds[16 * LT];
  __shared__ double red[2 * 4];
  const int tid = threadIdx.x;
  const int cl = tid & 15, t = tid >> 4;
  const int col = blockIdx.x * 16 + cl;
  const int j = p.j_begin + blockIdx.y;
  const size_t base = size_t(j) * L256 * L256;
  float2 v[16];
  // rows r = t + 16 r1
  static_for<0, 16>([&](auto r1) { v[r1.value] = p.tmp[base + (t + 16 * r1.value) * L256 + col]; });
  dft_reg<16, false>(v);                                  // over r1 -> kr1
  static_for<1, 16>([&](auto k) { v[k.value] = cmul(v[k.value], p.tw[t * k.value]); });
  static_for<0, 16>([&](auto k) { lds[(k.value * LP + t) * 16 + cl] = v[k.value]; });
  __syncthreads();
  static_for<0, 16>([&](auto r2) { v[r2.value] = lds[(t * LP + r2.value) * 16 + cl]; });
  dft_reg<16, false>(v);                                  // over r2 -> kr2; thread t = kr1
  float ef_n = 0.f, ef_d = 0.f;
  const float c = p.c, omc = 1.0f - p.c, inv_n2 = 1.0f / float(L256 * L256);
  static_for<0, 16>([&](auto k2) {
    const int kr = t + 16 * k2.value;
    const float A = p.amp[base + size_t(kr) * L256 + col];
    v[k2.value] = fourier_op(v[k2.value], A, c, omc, inv_n2, ef_n, ef_d);
  });
  double acc[2] = {ef_n, ef_d};
  dft_reg<16, true>(v);                                   // over kr2 -> r2
  __syncthreads();
  static_for<0, 16>([&](auto r2) { lds[(t * LP + r2.value) * 16 + cl] = v[r2.value]; });
  __syncthreads();
  static_for<0, 16>([&](auto k) { v[k.value] = lds[(k.value * LP + t) * 16 + cl]; });  // thread t = r2
  static_for<1, 16>([&](auto k) { v[k.value] = cmulc(v[k.value], p.tw[t * k.value]); });
  dft_reg<16, true>(v);                                   // over kr1 -> r1
  static_for<0, 16>([&](auto r1) { p.tmp[base + (t + 16 * r1.value) * L256 + col] = v[r1.value]; });

  block_sum<2, 256>(acc, red);
  if (tid < 2) p.met[(size_t(j) * p.nslot + blockIdx.x) * MF_COUNT + tid] = acc[tid];
}

template <class St>
__global__ __launch_bounds__(256) void rows256_inv_kernel(DivideParams p) {
  __shared__ float2 lds[16 * LT];
  const int tid = threadIdx.x;
  const int t = tid & 15, rl = tid >> 4;
  const int r = blockIdx.x * 16 + rl;
  const int j = p.j_begin + blockIdx.y;
  const size_t base = size_t(j) * L256 * L256;
  using elem = typename St::elem;
  elem* __restrict__ ys = reinterpret_cast<elem*>(p.y);
  float2 v[16];
  // thread t = kc1 holds kc2
  static_for<0, 16>([&](auto k2) { v[k2.value] = p.tmp[base + r * L256 + t + 16 * k2.value]; });
  dft_reg<16, true>(v);                                   // over kc2 -> c2
  static_for<0, 16>([&](auto c2) { lds[rl * LT + c2.value * LP + t] = v[c2.value]; });
  __syncthreads();
  static_for<0, 16>([&](auto k1) { v[k1.value] = lds[rl * LT + t * LP + k1.value]; });  // thread t = c2
  static_for<1, 16>([&](auto k) { v[k.value] = cmulc(v[k.value], p.tw[t * k.value]); });
  dft_reg<16, true>(v);                                   // over kc1 -> c1
  static_for<0, 16>([&](auto c1) {
    St::store(ys, base + r * L256 + t + 16 * c1.value, v[c1.value], p.scale);
  });
}

// ---------------------------------------------------------------------------
// Materialise the pending update and/or the previous iteration's metrics:
// x_k = alpha P S_j O + beta y_{k-1} + gamma x_{k-1} (same arithmetic as the
// divide prologue).  One block per pattern; slot 0 gets the sums and the other
// slots are cleared.
// ---------------------------------------------------------------------------
template <class St>
__global__ __launch_bounds__(256) void flush_kernel(FlushParams p) {
  __shared__ double red[4 * 4];
  const int j = blockIdx.x;
  const int N = p.N;
  const size_t base = size_t(j) * N * N;
  const int2 pj = p.pos[j];
  using elem = typename St::elem;
  elem* xs = reinterpret_cast<elem*>(p.x);
  const elem* ys = reinterpret_cast<const elem*>(p.y);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int idx = threadIdx.x; idx < N * N; idx += 256) {
    const int r = idx / N, c = idx % N;
    const float2 z = cmul(p.probe[idx], p.obj[size_t(pj.x + r) * p.obj_w + (pj.y + c)]);
    float2 xo = make_float2(0.f, 0.f), yo = make_float2(0.f, 0.f);
    if (p.read_x) xo = St::load(xs, base + idx, p.inv_scale);
    if (p.read_y) yo = St::load(ys, base + idx, p.inv_scale);
    const float2 xn = p.wform ? blend_x(z, xo, p.alpha) : update_x(z, yo, xo, p.alpha, p.beta, p.gamma);
    double dr = double(z.x) - double(yo.x), di = double(z.y) - double(yo.y);
    acc[0] += dr * dr + di * di;
    acc[1] += double(yo.x) * yo.x + double(yo.y) * yo.y;
    dr = double(xn.x) - double(xo.x);
    di = double(xn.y) - double(xo.y);
    acc[2] += dr * dr + di * di;
    acc[3] += double(xo.x) * xo.x + double(xo.y) * xo.y;
    if (p.write_x) St::store(xs, base + idx, xn, p.scale);
  }
  block_sum<4, 256>(acc, red);
  for (int q = threadIdx.x; q < p.nslot * MF_COUNT; q += 256) {
    const int slot = q / MF_COUNT, f = q % MF_COUNT;
    double v = 0.0;
    if (slot == 0 && f >= MF_EC_NUM) v = acc[f - MF_EC_NUM];
    p.met[size_t(j) * p.nslot * MF_COUNT + q] = v;
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
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
    default: launch_fused_mode<N, T, St, PRO_FLAGS>(p, n_patterns, s); break;
  }
  return hipGetLastError();
}

template <class St>
static hipError_t launch_256(const DivideParams& p, int n_patterns, hipStream_t s) {
  const dim3 grid(16, n_patterns);
  hipLaunchKernelGGL((rows256_fwd_kernel<St>), grid, dim3(256), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cols256_kernel, grid, dim3(256), 0, s, p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((rows256_inv_kernel<St>), grid, dim3(256), 0, s, p);
  return hipGetLastError();
}

template <class St>
static hipError_t launch_divide_t(int n, const DivideParams& p, int n_patterns, hipStream_t s) {
  switch (n) {
    case 32: return launch_fused<32, 64, St>(p, n_patterns, s);
    case 64: return launch_fused<64, 256, St>(p, n_patterns, s);
    case 128: return launch_fused<128, 512, St>(p, n_patterns, s);
    case 256: return launch_256<St>(p, n_patterns, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sp_batch(int n, const DivideParams& p, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  switch (n) {
    case 32: launch_fused_mode<32, 64, StoreF32, PRO_SP>(p, count, s); break;
    case 64: launch_fused_mode<64, 256, StoreF32, PRO_SP>(p, count, s); break;
    case 128: launch_fused_mode<128, 512, StoreF32, PRO_SP>(p, count, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void sp_probe_kernel(SpProbeParams p) {
  __shared__ float red[4];
  const int NN = p.N * p.N;
  const int u = blockIdx.x * 256 + threadIdx.x;
  float m = 0.f;
  if (u < NN) {
    double ax = 0.0, ay = 0.0;
    for (int k = 0; k < p.count; ++k) {
      const float2 c = p.contrib[size_t(k) * NN + u];
      ax += c.x;
      ay += c.y;
    }
    const float2 o = p.probe[u];
    const float2 nv = make_float2(float(double(o.x) + ax), float(double(o.y) + ay));
    p.probe[u] = nv;
    m = cnorm(nv);
  }
  m = block_max<256>(m, red);
  if (threadIdx.x == 0) p.pmax_part[blockIdx.x] = m;
}

hipError_t launch_sp_probe(const SpProbeParams& p, hipStream_t s) {
  hipLaunchKernelGGL(sp_probe_kernel, dim3((p.N * p.N + 255) / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_divide(int n, int fp16, const DivideParams& p, int n_patterns, hipStream_t s) {
  if (n_patterns <= 0) return hipSuccess;
  return fp16 ? launch_divide_t<StoreF16>(n, p, n_patterns, s) : launch_divide_t<StoreF32>(n, p, n_patterns, s);
}

hipError_t launch_flush(int fp16, const FlushParams& p, int J, hipStream_t s) {
  if (J <= 0) return hipSuccess;
  if (fp16) hipLaunchKernelGGL(flush_kernel<StoreF16>, dim3(J), dim3(256), 0, s, p);
  else hipLaunchKernelGGL(flush_kernel<StoreF32>, dim3(J), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <class St>
static hipError_t launch_stage_t(int n, const DivideParams& p, int n_patterns, int stage, hipStream_t s) {
  if (n != 256) {
    if (stage != 0) return hipErrorInvalidValue;
    return launch_divide_t<St>(n, p, n_patterns, s);
  }
  if (p.wform) return hipErrorInvalidValue;   // the three-pass form keeps x
  const dim3 grid(16, n_patterns);
  switch (stage) {
    case 0: hipLaunchKernelGGL((rows256_fwd_kernel<St>), grid, dim3(256), 0, s, p); break;
    case 1: hipLaunchKernelGGL(cols256_kernel, grid, dim3(256), 0, s, p); break;
    case 2: hipLaunchKernelGGL((rows256_inv_kernel<St>), grid, dim3(256), 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_divide_stage(int n, int fp16, const DivideParams& p, int n_patterns, int stage, hipStream_t s) {
  if (n_patterns <= 0) return hipSuccess;
  return fp16 ? launch_stage_t<StoreF16>(n, p, n_patterns, stage, s) : launch_stage_t<StoreF32>(n, p, n_patterns, stage, s);
}

int divide_stages(int n) { return n == 256 ? 3 : 1; }

int divide_slots(int n) { return n == 256 ? 16 : 1; }
bool divide_supported(int n) { return n == 32 || n == 64 || n == 128 || n == 256; }

// Amplitudes sqrt(I) in the order the divide kernel reads them.  N <= 128:
// amp[j][kc2][qc] with qc = kr2*16 + kr1*4 + kc1 for the spectrum element
// (kr1 + 4 kr2, kc1 + 4 kc2); N = 256: natural order.  Values that are not
// finite or are negative are counted in *bad.
__global__ void amp_prepare_kernel(const float* __restrict__ I, float* __restrict__ amp, int n, int J,
                                   int* bad) {
  const size_t nn = size_t(n) * n;
  const size_t total = nn * J;
  for (size_t g = blockIdx.x * size_t(blockDim.x) + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const size_t j = g / nn;
    const int rem = int(g % nn);
    size_t src;
    if (n == 256) {
      src = g;
    } else {
      const int kc2 = rem / (4 * n), qc = rem % (4 * n);
      const int kr2 = qc / 16, kk = qc % 16;  // spectral order of the fused kernel's stage C
      const int kr = kk / 4 + 4 * kr2, kc = kk % 4 + 4 * kc2;
      src = j * nn + size_t(kr) * n + kc;
    }
    const float iv = I[src];
    if (!(iv >= 0.0f) || !isfinite(iv)) {
      atomicAdd(bad, 1);
      amp[g] = 0.0f;
    } else {
      amp[g] = float(sqrt(double(iv)));
    }
  }
}

hipError_t launch_amp_prepare(int n, const float* intensity, float* amp, int J, int* bad, hipStream_t s) {
  const size_t total = size_t(n) * n * J;
  const int blocks = int(std::min<size_t>((total + 255) / 256, 65536));
  hipLaunchKernelGGL(amp_prepare_kernel, dim3(blocks), dim3(256), 0, s, intensity, amp, n, J, bad);
  return hipGetLastError();
}

}  // namespace pty
