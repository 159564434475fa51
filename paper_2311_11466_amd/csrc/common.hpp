// Device building blocks shared by the gfx950 kernels: complex arithmetic,
// compile-time DFT twiddles, fully unrolled in-register DFTs and the exit-wave
// storage formats.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <utility>

namespace pty {

// ---------------------------------------------------------------------------
// complex float helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// Products are written with explicit fused multiply-adds so every kernel that
// forms the same product (e.g. an exit wave P * O) rounds it identically,
// whatever contraction the compiler would otherwise choose.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
__device__ __forceinline__ float cnorm(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// ---------------------------------------------------------------------------
// compile-time cos / sin of 2*pi*k/L, from the Taylor series on [0, pi/2) and
// quadrant symmetry (exact 0 and +-1 on the axes)
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// returns cos(2 pi k / L) (want_sin = false) or sin(2 pi k / L)
constexpr double trig2pi(long k, long L, bool want_sin) {
  k = ((k % L) + L) % L;
  const long q = (4 * k) / L;            // quadrant
  const long r = 4 * k - q * L;          // remainder, angle = pi/2 * r / L
  const double t = 0.5 * kPi * double(r) / double(L);
  const double c = (r == 0) ? 1.0 : taylor_cos(t);
  const double s = (r == 0) ? 0.0 : taylor_sin(t);
  double cc = 0, ss = 0;
  switch (q) {
    case 0: cc = c; ss = s; break;
    case 1: cc = -s; ss = c; break;
    case 2: cc = -c; ss = -s; break;
    default: cc = s; ss = -c; break;
  }
  return want_sin ? ss : cc;
}

// d * exp(-2 pi i K / L) (forward) or d * exp(+2 pi i K / L) (inverse), with the
// trivial angles special-cased at compile time.
template <int L, int K, bool INV>
__device__ __forceinline__ float2 twiddle_const(float2 d) {
  constexpr int k = ((K % L) + L) % L;
  if constexpr (k == 0) {
    return d;
  } else if constexpr (2 * k == L) {
    return make_float2(-d.x, -d.y);
  } else if constexpr (4 * k == L) {
    // forward: * (-i); inverse: * (+i)
    return INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
  } else if constexpr (4 * k == 3 * L) {
    return INV ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
  } else {
    constexpr float c = float(trig2pi(k, L, false));
    constexpr float s = float(trig2pi(k, L, true));
    // W = c - i s (forward), c + i s (inverse); explicit fused multiply-adds
    // (a sum of two products left to the compiler is contracted differently
    // in different instantiations of one kernel, and their results would then
    // differ in the last bit).  Where |c| = |s| (odd multiples of pi/4) both
    // components share one product: three operations instead of four.
    if constexpr (c == s) {
      if constexpr (!INV) { const float m = d.y * c; return make_float2(fmaf(d.x, c, m), fmaf(-d.x, c, m)); }
      else { const float m = d.x * c; return make_float2(fmaf(-d.y, c, m), fmaf(d.y, c, m)); }
    } else if constexpr (c == -s) {
      if constexpr (!INV) { const float m = d.x * c; return make_float2(fmaf(d.y, s, m), fmaf(d.y, c, m)); }
      else { const float m = d.y * c; return make_float2(fmaf(d.x, c, m), fmaf(d.x, s, m)); }
    } else if constexpr (!INV) {
      return make_float2(fmaf(d.x, c, d.y * s), fmaf(d.y, c, -(d.x * s)));
    } else {
      return make_float2(fmaf(d.x, c, -(d.y * s)), fmaf(d.y, c, d.x * s));
    }
  }
}

// ---------------------------------------------------------------------------
// compile-time loops
// ---------------------------------------------------------------------------
template <int B, int E, int S = 1, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + S, E, S>(std::forward<F>(f));
  }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}

// ---------------------------------------------------------------------------
// In-register DFT of M = 2^m points held at v[OFF + STRIDE * i], i < M.
// Radix-2 decimation in frequency, then a compile-time relabelling so that on
// return v[OFF + STRIDE * k] holds the k-th frequency (natural order).
// Forward: X_k = sum_n x_n exp(-2 pi i n k / M); inverse: exp(+...), unscaled.
// ---------------------------------------------------------------------------
template <int M, bool INV, int STRIDE = 1, int OFF = 0, int NV>
__device__ __forceinline__ void dft_reg(float2 (&v)[NV]) {
  static_assert((M & (M - 1)) == 0, "power of two");
  if constexpr (M == 1) {
    return;
  } else {
    static_for<0, ilog2(M)>([&](auto st) {
      constexpr int half = M >> (st.value + 1);
      constexpr int span = 2 * half;
      static_for<0, M, span>([&](auto blk) {
        static_for<0, half>([&](auto i) {
          constexpr int ia = OFF + STRIDE * (blk.value + i.value);
          constexpr int ib = OFF + STRIDE * (blk.value + i.value + half);
          const float2 a = v[ia];
          const float2 b = v[ib];
          v[ia] = cadd(a, b);
          v[ib] = twiddle_const<span, i.value, INV>(csub(a, b));
        });
      });
    });
    // output of DIF is in bit-reversed order: relabel
    float2 t[M];
    static_for<0, M>([&](auto k) { t[k.value] = v[OFF + STRIDE * bitrev(k.value, ilog2(M))]; });
    static_for<0, M>([&](auto k) { v[OFF + STRIDE * k.value] = t[k.value]; });
  }
}

// 4 x 4 two-dimensional DFT on v[OFF + 4*r + c] (r: slow axis, c: fast axis).
template <bool INV, int OFF, int NV>
__device__ __forceinline__ void dft4x4_reg(float2 (&v)[NV]) {
  static_for<0, 4>([&](auto r) { dft_reg<4, INV, 1, OFF + 4 * r.value>(v); });
  static_for<0, 4>([&](auto c) { dft_reg<4, INV, 4, OFF + c.value>(v); });
}

// ---------------------------------------------------------------------------
// exit-wave storage formats
// ---------------------------------------------------------------------------
// Raw buffer resource over `bytes` bytes from p (gfx9 family: stride 0, word 3
// = 0x00020000).  A load through it at a byte offset at or past `bytes`
// returns zero and makes no memory request; kOutside is such an offset.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kOutside = 0x7fffffff;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ float2 buffer_load_f2(__amdgpu_buffer_rsrc_t r, int byte_off) {
  const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
  return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}

// Cache policy of the exit-wave accesses, chosen per storage type from timing
// the whole iteration on the 1024-pattern N = 128 scan: float32 exit waves are
// streamed with non-temporal loads and stores (the object and probe gathers
// then stay in L2; -4.9 % per iteration in the x form, -7.9 % in the blend
// form), float16 exit waves (half the bytes) are fastest with plain accesses.
// load_stream is the load of the probe sums, the last reader in an iteration.
typedef float f32x2 __attribute__((ext_vector_type(2)));
constexpr bool kNtStoreF32 = true, kNtLoadF32 = true, kNtProbeF32 = true;
constexpr bool kNtStoreF16 = false, kNtLoadF16 = false, kNtProbeF16 = false;

struct StoreF32 {
  using elem = float2;
  static constexpr int kFormat = 0;
  __device__ __forceinline__ static float2 load_nt(const elem* p, size_t i) {
    const f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p) + i);
    return make_float2(v.x, v.y);
  }
  __device__ __forceinline__ static float2 load(const elem* p, size_t i, float /*inv_scale*/) {
    return kNtLoadF32 ? load_nt(p, i) : p[i];
  }
  __device__ __forceinline__ static float2 load_stream(const elem* p, size_t i, float /*inv_scale*/) {
    return kNtProbeF32 ? load_nt(p, i) : p[i];
  }
  // a value in storage form and back (float32: itself), and the store of a
  // value already in storage form
  __device__ __forceinline__ static elem pack(float2 v, float /*scale*/) { return v; }
  __device__ __forceinline__ static float2 unpack(elem e, float /*inv_scale*/) { return e; }
  __device__ __forceinline__ static void store_packed(elem* p, size_t i, elem e) { store(p, i, e, 1.0f); }
  __device__ __forceinline__ static void store(elem* p, size_t i, float2 v, float /*scale*/) {
    if constexpr (kNtStoreF32) {
      f32x2 w;
      w.x = v.x;
      w.y = v.y;
      __builtin_nontemporal_store(w, reinterpret_cast<f32x2*>(p) + i);
    } else {
      p[i] = v;
    }
  }
  // the object step's exit-wave loads use the default policy: non-temporal
  // ones measured slower (N = 256: 722 vs 675 us) and leave the probe step's
  // second read of y without the memory-side cache (N = 128: 37.8 vs 25.4 us).
  // The value as stored (no storage scale), through a buffer resource.
  __device__ __forceinline__ static float2 load_buf_unscaled(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return buffer_load_f2(r, byte_off);
  }
};

// complex float16 times a power-of-two scale (round to nearest even)
struct StoreF16 {
  using elem = __half2;
  static constexpr int kFormat = 1;
  __device__ __forceinline__ static float2 cvt(unsigned u, float inv_scale) {
    __half2 h;
    __builtin_memcpy(&h, &u, 4);
    const float2 f = __half22float2(h);
    return make_float2(f.x * inv_scale, f.y * inv_scale);
  }
  __device__ __forceinline__ static float2 load(const elem* p, size_t i, float inv_scale) {
    if constexpr (kNtLoadF16) return cvt(__builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p) + i), inv_scale);
    const float2 f = __half22float2(p[i]);
    return make_float2(f.x * inv_scale, f.y * inv_scale);
  }
  __device__ __forceinline__ static float2 load_stream(const elem* p, size_t i, float inv_scale) {
    if constexpr (kNtProbeF16) return cvt(__builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p) + i), inv_scale);
    return load(p, i, inv_scale);
  }
  // storage form: v 2^s rounded to float16; unpack(pack(v)) is what load
  // returns after store (both factors are powers of two)
  __device__ __forceinline__ static elem pack(float2 v, float scale) {
    return __float22half2_rn(make_float2(v.x * scale, v.y * scale));
  }
  __device__ __forceinline__ static float2 unpack(elem h, float inv_scale) {
    const float2 f = __half22float2(h);
    return make_float2(f.x * inv_scale, f.y * inv_scale);
  }
  __device__ __forceinline__ static void store(elem* p, size_t i, float2 v, float scale) {
    store_packed(p, i, pack(v, scale));
  }
  __device__ __forceinline__ static void store_packed(elem* p, size_t i, elem h) {
    if constexpr (kNtStoreF16) {
      unsigned u;
      __builtin_memcpy(&u, &h, 4);
      __builtin_nontemporal_store(u, reinterpret_cast<unsigned*>(p) + i);
    } else {
      p[i] = h;
    }
  }
  // the stored value times 2^s (the caller applies the power-of-two scale
  // to its sums, which is exact)
  __device__ __forceinline__ static float2 load_buf_unscaled(__amdgpu_buffer_rsrc_t r, int byte_off) {
    const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
    __half2 h;
    __builtin_memcpy(&h, &v, 4);
    return __half22float2(h);
  }
};

// ---------------------------------------------------------------------------
// block-wide float64 sum of NV values per thread, in a fixed order
// (wave butterfly, then waves in ascending order).  red must hold
// NV * (blockDim / 64) doubles.  All threads receive the sums.
// ---------------------------------------------------------------------------
template <int NV, int NT>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  static_assert(NT % 64 == 0, "whole waves");
  constexpr int NW = NT / 64;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q * NW + wave] = v[q];
  }
  __syncthreads();
  // one value at a time for many waves (NV * NW loads in flight would spill)
  constexpr int kUnrollQ = NW > 4 ? 1 : NV;
#pragma unroll kUnrollQ
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[q * NW + w];
    v[q] = s;
  }
  __syncthreads();
}

// Work-groups of one launch go to the 8 XCDs (each with its own L2) in
// round-robin order of their id.  xcd_block maps the id so that every XCD
// runs a contiguous range of logical blocks: neighbouring blocks, which read
// overlapping object pixels, then share an L2.  The grid is padded to a
// multiple of 8 (xcd_pad); logical ids beyond the real count exit at once.
constexpr int kXcds = 8;
__host__ __device__ constexpr int xcd_pad(int n) { return (n + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_block(int b, int padded) {
  return (b % kXcds) * (padded / kXcds) + b / kXcds;
}

template <int NT>
__device__ __forceinline__ float block_max(float v, float* red) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  float m = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) m = fmaxf(m, red[w]);
  __syncthreads();
  return m;
}

}  // namespace pty
