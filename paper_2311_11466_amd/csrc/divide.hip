// Divide step, N = 256 three-pass form, flush, amplitude preparation and the
// dispatch to the fused kernels (divide_fused.hpp, one translation unit per
// size).
// No implicit contraction of a * b + c: the kernels of this file exist in
// one instantiation per prologue mode, and each must round every value the
// same way (the products that should fuse are written as fused multiply-adds).
#pragma clang fp contract(off)
#include <algorithm>

#include "divide_fused.hpp"

namespace pty {

// ---------------------------------------------------------------------------
// N = 256: three passes.  A work-group handles 16 rows (or 16 columns) of one
// pattern, 16 threads per line, 16 values per thread; a line's 256-point DFT
// is 16 x 16 with a transpose of the line's 16 x 16 block between its
// threads.  In the row passes a row's 16 threads are lanes of one wave, so
// the transpose needs no work-group barrier; it runs in two halves through a
// buffer of 8 values per thread, and the twiddles come from a 16 x 16 table
// in LDS.  The forward row pass is bound by the memory requests it keeps in
// flight: its prologue issues eight elements' loads at a time (compile-time
// buffer modes), which costs registers (four waves per SIMD) but moves more
// bytes than seven waves each waiting on one element.  The column pass, whose 16 threads
// of a column sit in four waves, exchanges all values at once (the same
// halving measured 5 % slower there); it keeps its exchange tiles interleaved
// by column ([a][b][column]), so a wave's 16 columns touch consecutive LDS
// words rather than one bank.  Its twiddles come from the same LDS table:
// read from the global table they took 30 loads and about 30 registers per
// thread (127 -> 97 VGPRs; 1030 -> 943 us on the 4096-pattern scan, same
// bits).  Issuing the amplitude loads at the start instead of in the Fourier
// step is slower with the table (969 us: 9 more registers).
// ---------------------------------------------------------------------------
constexpr int L256 = 256;
constexpr int LP = 17;                 // padded pitch of an exchange tile
constexpr int LT = 16 * LP;            // one column's exchange tile (column pass)
constexpr int LTH = 8 * LP;            // one row's half exchange tile (row passes)
// Patterns per launch of a pass: the grid's second dimension holds the
// pattern, and the device allows at most 65536 there.
constexpr int kMaxPatternsPerLaunch = 65535;

// Ordering of LDS accesses between the lanes of one wave: the hardware keeps
// a wave's LDS operations in order, so only the compiler must not move them.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Transpose of a row's 16 x 16 block: on return thread t of the row holds in
// v[c] what thread c held in v[t].  buf: the row's LTH entries, private to
// the wave; round h moves values 8h .. 8h+7 and serves threads 8h .. 8h+7.
__device__ __forceinline__ void row_transpose(float2 (&v)[16], float2* buf, int t) {
  float2 w[16];
  static_for<0, 2>([&](auto h) {
    static_for<0, 8>([&](auto kk) { buf[kk.value * LP + t] = v[8 * h.value + kk.value]; });
    wave_lds_order();
    if ((t >> 3) == h.value) {
      static_for<0, 16>([&](auto c) { w[c.value] = buf[(t - 8 * h.value) * LP + c.value]; });
    }
    wave_lds_order();
  });
  static_for<0, 16>([&](auto c) { v[c.value] = w[c.value]; });
}


// The float32 intermediate of the N = 256 passes is streamed once by each
// pass: non-temporal accesses keep it from displacing the object and probe
// lines that the gathers reuse.
__device__ __forceinline__ float2 tmp_load(const float2* p, size_t i) {
  const f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p) + i);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void tmp_store(float2* p, size_t i, float2 v) {
  f32x2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<f32x2*>(p) + i);
}

// rb: the work-group's block of 16 rows, jl: its pattern within the launch
// (SP: its slot in the batch of sequential projections, whose pattern is
// batch[jl]; the prologue is psi = P S_j O, and the block's maximum of
// |S_j O|^2 goes to sp_omax for the inverse row pass)
// MODE: the prologue's buffers and metrics as in the fused kernel (Pro<MODE>;
// compile-time except PRO_FLAGS), so the loads of GP elements go out together:
// with the buffers chosen by runtime tests every element's loads waited for
// the previous element (at most 4 loads in flight per wave; 1613 -> 1517 us
// float32, 1553 -> 1192 us float16 on the 4096-pattern scan, same bits).
template <class St, int MODE, bool SP = false>
__device__ __forceinline__ void rows256_fwd_body(const DivideParams& p, const int rb, const int jl) {
  __shared__ float2 lds[16 * LTH];
  __shared__ float2 twt[16 * 16];      // twt[16 a + b] = tw[a b]
  __shared__ double red[MF_COUNT * 4];
  __shared__ float fred[4];
  const int tid = threadIdx.x;
  const int t = tid & 15, rl = tid >> 4;
  twt[tid] = p.tw[(tid >> 4) * (tid & 15)];
  const int r = rb * 16 + rl;
  const int j = SP ? p.batch[jl] : p.j_begin + jl;
  const size_t base = size_t(j) * L256 * L256;
  const int2 pj = p.pos[j];
  using elem = typename St::elem;
  elem* __restrict__ xs = reinterpret_cast<elem*>(p.x);
  const elem* ys = reinterpret_cast<const elem*>(p.y);  // may alias p.tmp
  float2 v[16];
  double acc[MF_COUNT];
#pragma unroll
  for (int q = 0; q < MF_COUNT; ++q) acc[q] = 0.0;
  float om = 0.0f;                     // SP: max |S_j O|^2 of the thread's pixels

  // prologue: column c = t + 16 c1, GP elements' loads at a time
  using PR = Pro<MODE>;
  const bool rx = PR::rx(p), ry = PR::ry(p), wx = PR::wx(p), mec = PR::ec(p), mdx = PR::dx(p);
  constexpr int GP = 8;
  const float2* __restrict__ orow = p.obj + size_t(pj.x + r) * p.obj_w + pj.y;
  static_for<0, 16, GP>([&](auto g0) {
    float2 zp[GP], zo[GP], xo[GP], yo[GP];
    static_for<0, GP>([&](auto q) {
      const int c = t + 16 * (g0.value + q.value);
      const int idx = r * L256 + c;
      zp[q.value] = p.probe[idx];
      zo[q.value] = orow[c];
      xo[q.value] = rx ? St::load(xs, base + idx, p.inv_scale) : make_float2(0.f, 0.f);
      yo[q.value] = ry ? St::load(ys, base + idx, p.inv_scale) : make_float2(0.f, 0.f);
    });
    static_for<0, GP>([&](auto q) {
      constexpr int c1 = g0.value + q.value;
      const int idx = r * L256 + t + 16 * c1;
      const float2 z = cmul(zp[q.value], zo[q.value]);
      if constexpr (SP) {
        om = fmaxf(om, cnorm(zo[q.value]));
        v[c1] = z;
      } else {
        // x_k as the storage keeps it (float16: rounded; see the fused kernel)
        const elem xe = St::pack(update_x(z, yo[q.value], xo[q.value], p.alpha, p.beta, p.gamma), p.scale);
        const float2 xn = St::unpack(xe, p.inv_scale);
        if (mec) {
          const double dr = double(z.x) - double(yo[q.value].x), di = double(z.y) - double(yo[q.value].y);
          acc[MF_EC_NUM] += fma(dr, dr, di * di);
          acc[MF_EC_DEN] += fma(double(yo[q.value].x), double(yo[q.value].x), double(yo[q.value].y) * yo[q.value].y);
        }
        if (mdx) {
          const double dr = double(xn.x) - double(xo[q.value].x), di = double(xn.y) - double(xo[q.value].y);
          acc[MF_DX_NUM] += fma(dr, dr, di * di);
          acc[MF_DX_DEN] += fma(double(xo[q.value].x), double(xo[q.value].x), double(xo[q.value].y) * xo[q.value].y);
        }
        if (wx) St::store_packed(xs, base + idx, xe);
        v[c1] = xn;
      }
    });
    // the group's metric terms are summed before the next group's loads:
    // without this the compiler forms every element's float64 terms first and
    // holds them (205 instead of 72 registers, two waves per SIMD)
    if constexpr (!SP) {
#pragma unroll
      for (int q = 0; q < MF_COUNT; ++q) asm volatile("" : "+v"(acc[q]));
    }
    __builtin_amdgcn_sched_barrier(0);
  });
  dft_reg<16, false>(v);                                  // over c1 -> kc1
  __syncthreads();                                        // twt is complete
  static_for<1, 16>([&](auto k) { v[k.value] = cmul(v[k.value], twt[16 * t + k.value]); });
  row_transpose(v, lds + rl * LTH, t);                    // thread t = kc1, v over c2
  dft_reg<16, false>(v);                                  // over c2 -> kc2; thread t = kc1
  static_for<0, 16>([&](auto k2) { tmp_store(p.tmp, base + r * L256 + t + 16 * k2.value, v[k2.value]); });

  if constexpr (SP) {
    om = block_max<256>(om, fred);
    if (tid == 0) p.sp_omax[jl * 16 + rb] = om;
  }
  block_sum<MF_COUNT, 256>(acc, red);   // SP: zeros (no consistency or change partials)
  if (tid >= MF_EC_NUM && tid < MF_COUNT)
    p.met[(size_t(j) * p.nslot + rb) * MF_COUNT + tid] = acc[tid];
}

template <bool SP = false>
__device__ __forceinline__ void cols256_body(const DivideParams& p, const int cb, const int jl) {
  __shared__ float2 lds[16 * LT];
  __shared__ float2 twt[16 * 16];      // twt[16 a + b] = tw[a b]
  __shared__ double red[2 * 4];
  const int tid = threadIdx.x;
  const int cl = tid & 15, t = tid >> 4;
  twt[tid] = p.tw[(tid >> 4) * (tid & 15)];
  const int col = cb * 16 + cl;
  const int j = SP ? p.batch[jl] : p.j_begin + jl;
  const size_t base = size_t(j) * L256 * L256;
  float2 v[16];
  // rows r = t + 16 r1
  static_for<0, 16>([&](auto r1) { v[r1.value] = tmp_load(p.tmp, base + (t + 16 * r1.value) * L256 + col); });
  dft_reg<16, false>(v);                                  // over r1 -> kr1
  __syncthreads();                                        // twt is complete
  static_for<1, 16>([&](auto k) { v[k.value] = cmul(v[k.value], twt[16 * t + k.value]); });
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
  static_for<1, 16>([&](auto k) { v[k.value] = cmulc(v[k.value], twt[16 * t + k.value]); });
  dft_reg<16, true>(v);                                   // over kr1 -> r1
  static_for<0, 16>([&](auto r1) { tmp_store(p.tmp, base + (t + 16 * r1.value) * L256 + col, v[r1.value]); });

  block_sum<2, 256>(acc, red);
  if (tid < 2) p.met[(size_t(j) * p.nslot + cb) * MF_COUNT + tid] = acc[tid];
}

// SP: the epilogue is the step of a sequential projection instead of the
// store of y (see the fused kernel): with psi = P S_j O formed again from the
// window (no other member of the batch touches it) and d = P_D psi - psi, the
// object window gets O + alpha conj(P) d / max|P|^2 and the batch slot's
// probe step beta conj(S_j O) d / max|S_j O|^2 (blind).
template <class St, bool SP = false>
__device__ __forceinline__ void rows256_inv_body(const DivideParams& p, const int rb, const int jl) {
  __shared__ float2 lds[16 * LTH];
  __shared__ float2 twt[16 * 16];      // twt[16 a + b] = tw[a b]
  __shared__ float fred[4];
  const int tid = threadIdx.x;
  const int t = tid & 15, rl = tid >> 4;
  twt[tid] = p.tw[(tid >> 4) * (tid & 15)];
  const int r = rb * 16 + rl;
  const int j = SP ? p.batch[jl] : p.j_begin + jl;
  const size_t base = size_t(j) * L256 * L256;
  using elem = typename St::elem;
  elem* __restrict__ ys = reinterpret_cast<elem*>(p.y);
  float2 v[16];
  // thread t = kc1 holds kc2
  static_for<0, 16>([&](auto k2) { v[k2.value] = tmp_load(p.tmp, base + r * L256 + t + 16 * k2.value); });
  dft_reg<16, true>(v);                                   // over kc2 -> c2
  row_transpose(v, lds + rl * LTH, t);                    // thread t = c2, v over kc1
  __syncthreads();                                        // twt is complete
  static_for<1, 16>([&](auto k) { v[k.value] = cmulc(v[k.value], twt[16 * t + k.value]); });
  dft_reg<16, true>(v);                                   // over kc1 -> c1
  if constexpr (SP) {
    // step sizes alpha / max|P|^2 and beta / max|S_j O|^2 (zero where the
    // maximum is zero); |P|^2 partial maxima: one per thread (npb <= 256)
    float pm = tid < p.npb ? p.pmax_part[tid] : 0.0f;
    float om = tid < 16 ? p.sp_omax[jl * 16 + tid] : 0.0f;
    pm = block_max<256>(pm, fred);
    om = block_max<256>(om, fred);
    const float ka = pm > 0.f ? p.sp_alpha / pm : 0.f;
    const float kb = om > 0.f ? p.sp_beta / om : 0.f;
    const int2 pj = p.pos[j];
    float2* __restrict__ orow = p.obj_out + size_t(pj.x + r) * p.obj_w + pj.y;
    float2* __restrict__ crow = p.contrib + size_t(jl) * (L256 * L256) + r * L256;
    static_for<0, 16>([&](auto c1) {
      const int c = t + 16 * c1.value;
      const float2 pp = p.probe[r * L256 + c];
      const float2 oo = orow[c];
      const float2 d = csub(v[c1.value], cmul(pp, oo));
      const float2 po = cmulc(d, pp);                  // conj(P) d
      orow[c] = make_float2(fmaf(ka, po.x, oo.x), fmaf(ka, po.y, oo.y));
      if (p.sp_blind) {
        const float2 oc = cmulc(d, oo);                // conj(S_j O) d
        crow[c] = make_float2(kb * oc.x, kb * oc.y);
      }
    });
    return;
  }
  static_for<0, 16>([&](auto c1) {
    St::store(ys, base + r * L256 + t + 16 * c1.value, v[c1.value], p.scale);
  });
}

// Sequential projections at N = 256: the three passes for one batch, grid
// (16, batch size); the pattern of slot s is batch[s].  The exit-wave storage
// is not touched (the intermediate and the probe steps are float32).
__global__ __launch_bounds__(256) void sp256_rows_fwd_kernel(DivideParams p) {
  rows256_fwd_body<StoreF32, PRO_Z, true>(p, int(blockIdx.x), int(blockIdx.y));
}
__global__ __launch_bounds__(256) void sp256_rows_inv_kernel(DivideParams p) {
  rows256_inv_body<StoreF32, true>(p, int(blockIdx.x), int(blockIdx.y));
}

// Column block of the column pass's work-group b (0..15 within its pattern).
// The amplitudes of 16 columns are 64 bytes per row, half a cache line, which
// blocks 2m and 2m + 1 share; work-group b runs on XCD b mod 8, so both go to
// XCD m and the second read of a line hits that XCD's L2 (in plain order the
// pass fetched every amplitude line twice).
__device__ __forceinline__ int col_block(int b) { return 2 * (b & 7) + ((b >> 3) & 1); }

// One scan: grid (16, patterns).  Grouped (the served form): a flat grid, 16
// consecutive work-groups per pattern.
template <class St, int MODE>
__global__ __launch_bounds__(256) void rows256_fwd_kernel(DivideParams p) {
  rows256_fwd_body<St, MODE>(p, int(blockIdx.x), int(blockIdx.y));
}
__global__ __launch_bounds__(256) void cols256_kernel(DivideParams p) {
  cols256_body(p, col_block(int(blockIdx.x)), int(blockIdx.y));
}
__global__ __launch_bounds__(256) void sp256_cols_kernel(DivideParams p) {
  cols256_body<true>(p, col_block(int(blockIdx.x)), int(blockIdx.y));
}
template <class St>
__global__ __launch_bounds__(256) void rows256_inv_kernel(DivideParams p) {
  rows256_inv_body<St>(p, int(blockIdx.x), int(blockIdx.y));
}
// MODE: the prologue mode every scan of the group shares (stage 0 only)
template <class St, int STAGE, int MODE = PRO_GENERAL>
__global__ __launch_bounds__(256) void pass256_group_kernel(Group<DivideParams> g) {
  const int b = int(blockIdx.x);
  const int sc = group_scan(g, b);
  const int l = b - g.first[sc];
  if constexpr (STAGE == 0) rows256_fwd_body<St, MODE>(g.p[sc], l & 15, l >> 4);
  if constexpr (STAGE == 1) cols256_body(g.p[sc], col_block(l & 15), l >> 4);
  if constexpr (STAGE == 2) rows256_inv_body<St>(g.p[sc], l & 15, l >> 4);
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
    // x_k as the divide's prologue forms it (in storage form)
    const elem xe = St::pack(p.wform ? blend_x(z, xo, p.alpha) : update_x(z, yo, xo, p.alpha, p.beta, p.gamma),
                             p.scale);
    const float2 xn = St::unpack(xe, p.inv_scale);
    double dr = double(z.x) - double(yo.x), di = double(z.y) - double(yo.y);
    acc[0] += fma(dr, dr, di * di);
    acc[1] += fma(double(yo.x), double(yo.x), double(yo.y) * yo.y);
    dr = double(xn.x) - double(xo.x);
    di = double(xn.y) - double(xo.y);
    acc[2] += fma(dr, dr, di * di);
    acc[3] += fma(double(xo.x), double(xo.x), double(xo.y) * xo.y);
    if (p.write_x) St::store_packed(xs, base + idx, xe);
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

// the fused divide (N <= 128)
static hipError_t launch_fused_any(int n, int fp16, const DivideParams& p, int n_patterns, hipStream_t s) {
  switch (n) {
    case 32: return launch_fused_n32(fp16, p, n_patterns, s);
    case 64: return launch_fused_n64(fp16, p, n_patterns, s);
    case 128: return launch_fused_n128(fp16, p, n_patterns, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sp_batch(int n, const DivideParams& p, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  switch (n) {
    case 32: return launch_sp_n32(p, count, s);
    case 64: return launch_sp_n64(p, count, s);
    case 128: return launch_sp_n128(p, count, s);
    case 256: {
      // batch slots in launches of at most kMaxPatternsPerLaunch: a chunk's
      // slot c reads batch[c0 + c] and its maxima and probe-step slots
      for (int c0 = 0; c0 < count; c0 += kMaxPatternsPerLaunch) {
        DivideParams q = p;
        q.batch = p.batch + c0;
        q.sp_omax = p.sp_omax + size_t(c0) * 16;
        q.contrib = p.contrib + size_t(c0) * L256 * L256;
        const dim3 grid(16, std::min(kMaxPatternsPerLaunch, count - c0));
        hipLaunchKernelGGL(sp256_rows_fwd_kernel, grid, dim3(256), 0, s, q);
        hipLaunchKernelGGL(sp256_cols_kernel, grid, dim3(256), 0, s, q);
        hipLaunchKernelGGL(sp256_rows_inv_kernel, grid, dim3(256), 0, s, q);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
    default: return hipErrorInvalidValue;
  }
}

// Probe step of one sequential-projection batch: P += the batch's probe
// contributions, summed in float64.  A work-group owns 256 probe pixels; its
// four quarters sum four consecutive ranges of batch slots (each in slot
// order, four loads in flight), and the quarters are added in order, so the
// result does not depend on timing.  Also writes the group's max |P|^2.
__global__ __launch_bounds__(1024) void sp_probe_kernel(SpProbeParams p) {
  __shared__ double part[2][3][256];
  __shared__ float red[16];
  const int NN = p.N * p.N;
  const int lt = threadIdx.x & 255, q = threadIdx.x >> 8;
  const int u = blockIdx.x * 256 + lt;
  const int per = (p.count + 3) / 4;
  const int k0 = min(p.count, q * per), k1 = min(p.count, k0 + per);
  double ax = 0.0, ay = 0.0;
  if (u < NN) {
    int k = k0;
    for (; k + 4 <= k1; k += 4) {
      float2 c[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = p.contrib[size_t(k + i) * NN + u];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ax += c[i].x;
        ay += c[i].y;
      }
    }
    for (; k < k1; ++k) {
      const float2 c = p.contrib[size_t(k) * NN + u];
      ax += c.x;
      ay += c.y;
    }
  }
  if (q > 0) {
    part[0][q - 1][lt] = ax;
    part[1][q - 1][lt] = ay;
  }
  __syncthreads();
  float m = 0.f;
  if (q == 0 && u < NN) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ax += part[0][i][lt];
      ay += part[1][i][lt];
    }
    const float2 o = p.probe[u];
    const float2 nv = make_float2(float(double(o.x) + ax), float(double(o.y) + ay));
    p.probe[u] = nv;
    m = cnorm(nv);
  }
  m = block_max<1024>(m, red);
  if (threadIdx.x == 0) p.pmax_part[blockIdx.x] = m;
}

hipError_t launch_sp_probe(const SpProbeParams& p, hipStream_t s) {
  hipLaunchKernelGGL(sp_probe_kernel, dim3((p.N * p.N + 255) / 256), dim3(1024), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_flush(int fp16, const FlushParams& p, int J, hipStream_t s) {
  if (J <= 0) return hipSuccess;
  if (fp16) hipLaunchKernelGGL(flush_kernel<StoreF16>, dim3(J), dim3(256), 0, s, p);
  else hipLaunchKernelGGL(flush_kernel<StoreF32>, dim3(J), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <class St, int MODE>
static void launch_256_fwd(const DivideParams& p, const dim3 grid, hipStream_t s) {
  hipLaunchKernelGGL((rows256_fwd_kernel<St, MODE>), grid, dim3(256), 0, s, p);
}

template <class St>
static hipError_t launch_256_chunk(const DivideParams& p, int n_patterns, int stage, hipStream_t s) {
  const dim3 grid(16, n_patterns);
  switch (stage) {
    case 0:
      switch (prologue_mode(p)) {
        case PRO_GENERAL: launch_256_fwd<St, PRO_GENERAL>(p, grid, s); break;
        case PRO_UPDATE: launch_256_fwd<St, PRO_UPDATE>(p, grid, s); break;
        case PRO_MATERIAL: launch_256_fwd<St, PRO_MATERIAL>(p, grid, s); break;
        case PRO_INIT: launch_256_fwd<St, PRO_INIT>(p, grid, s); break;
        case PRO_Z: launch_256_fwd<St, PRO_Z>(p, grid, s); break;
        case PRO_Y_EC: launch_256_fwd<St, PRO_Y_EC>(p, grid, s); break;
        case PRO_Y: launch_256_fwd<St, PRO_Y>(p, grid, s); break;
        default: launch_256_fwd<St, PRO_FLAGS>(p, grid, s); break;
      }
      break;
    case 1: hipLaunchKernelGGL(cols256_kernel, grid, dim3(256), 0, s, p); break;
    case 2: hipLaunchKernelGGL((rows256_inv_kernel<St>), grid, dim3(256), 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// One pass over all patterns, in launches of at most kMaxPatternsPerLaunch
// (each takes its patterns from j_begin on; a pattern's work does not depend
// on the launch it is in)
template <class St>
static hipError_t launch_256_stage(const DivideParams& p, int n_patterns, int stage, hipStream_t s) {
  if (p.wform) return hipErrorInvalidValue;   // the three-pass form keeps x
  for (int c0 = 0; c0 < n_patterns; c0 += kMaxPatternsPerLaunch) {
    DivideParams q = p;
    q.j_begin = p.j_begin + c0;
    const hipError_t e = launch_256_chunk<St>(q, std::min(kMaxPatternsPerLaunch, n_patterns - c0), stage, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <class St, int MODE>
static void launch_256_fwd_group(const Group<DivideParams>& g, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((pass256_group_kernel<St, 0, MODE>), dim3(blocks), dim3(256), 0, s, g);
}

// Grouped forward row passes exist for the compile-time modes of the
// iteration's steady state and first step (every scan of g in the mode of
// g.p[0]); others return hipErrorInvalidValue (the host launches such scans
// one by one).
template <class St>
static hipError_t launch_256_stage_group(const Group<DivideParams>& g, int blocks, int stage, hipStream_t s) {
  if (g.p[0].wform) return hipErrorInvalidValue;
  switch (stage) {
    case 0:
      switch (prologue_mode(g.p[0])) {
        case PRO_GENERAL: launch_256_fwd_group<St, PRO_GENERAL>(g, blocks, s); break;
        case PRO_UPDATE: launch_256_fwd_group<St, PRO_UPDATE>(g, blocks, s); break;
        case PRO_INIT: launch_256_fwd_group<St, PRO_INIT>(g, blocks, s); break;
        case PRO_Z: launch_256_fwd_group<St, PRO_Z>(g, blocks, s); break;
        case PRO_Y_EC: launch_256_fwd_group<St, PRO_Y_EC>(g, blocks, s); break;
        case PRO_Y: launch_256_fwd_group<St, PRO_Y>(g, blocks, s); break;
        default: return hipErrorInvalidValue;
      }
      break;
    case 1: hipLaunchKernelGGL((pass256_group_kernel<St, 1>), dim3(blocks), dim3(256), 0, s, g); break;
    case 2: hipLaunchKernelGGL((pass256_group_kernel<St, 2>), dim3(blocks), dim3(256), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_divide_stage_group(int n, int fp16, const DivideParams* ps, const int* n_patterns, int count,
                                     int stage, hipStream_t s) {
  if (count < 1 || count > kGroupMax) return hipErrorInvalidValue;
  Group<DivideParams> g{};
  const int per_pattern = n == 256 ? 16 : 1;     // work-groups per pattern
  int blocks = 0;
  for (int i = 0; i < count; ++i) {
    g.p[i] = ps[i];
    g.first[i] = blocks;
    blocks += per_pattern * n_patterns[i];
  }
  g.first[count] = blocks;
  g.count = count;
  if (blocks <= 0) return hipSuccess;
  if (n == 256) return fp16 ? launch_256_stage_group<StoreF16>(g, blocks, stage, s)
                            : launch_256_stage_group<StoreF32>(g, blocks, stage, s);
  if (stage != 0) return hipErrorInvalidValue;
  switch (n) {
    case 32: return launch_fused_group_n32(fp16, g, blocks, s);
    case 64: return launch_fused_group_n64(fp16, g, blocks, s);
    case 128: return launch_fused_group_n128(fp16, g, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_divide_stage(int n, int fp16, const DivideParams& p, int n_patterns, int stage, hipStream_t s) {
  if (n_patterns <= 0) return hipSuccess;
  if (n != 256) return stage == 0 ? launch_fused_any(n, fp16, p, n_patterns, s) : hipErrorInvalidValue;
  return fp16 ? launch_256_stage<StoreF16>(p, n_patterns, stage, s) : launch_256_stage<StoreF32>(p, n_patterns, stage, s);
}

int divide_stages(int n) { return n == 256 ? 3 : 1; }

int divide_mode(const DivideParams& p) { return prologue_mode(p); }

bool divide_groupable(int n, const DivideParams& p) {
  if (n == 256 && p.wform) return false;
  switch (prologue_mode(p)) {
    case PRO_GENERAL: case PRO_UPDATE: case PRO_INIT: case PRO_W_PENDING: case PRO_W_ZERO:
    case PRO_Z: case PRO_Y_EC: case PRO_Y:
      return true;
    default:
      return false;
  }
}

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
