// Per-element operations of the divide step shared by the fused kernel
// (N <= 128), the three-pass N = 256 kernels and the flush kernel.
#pragma once

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
// Accumulates (|X| - A)^2 and A^2 in float32 per thread.  zsign (+1 or -1)
// multiplies the value set where X = 0, for a caller that holds -X.
__device__ __forceinline__ float2 fourier_op(float2 X, float A, float c, float one_minus_c, float inv_n2,
                                             float& ef_num, float& ef_den, float zsign = 1.0f) {
  const float m2 = fmaf(X.x, X.x, X.y * X.y);
  const bool nz = m2 >= 1.17549435e-38f;
  const float r = __builtin_amdgcn_rsqf(nz ? m2 : 1.0f);
  const float d = nz ? fmaf(m2, r, -A) : -A;            // |X| - A
  ef_num = fmaf(d, d, ef_num);
  ef_den = fmaf(A, A, ef_den);
  const float cA = c * A;
  const float f = fmaf(cA, r, one_minus_c) * inv_n2;
  float2 out;
  out.x = nz ? X.x * f : cA * inv_n2 * zsign;
  out.y = nz ? X.y * f : 0.0f * zsign;
  return out;
}

}  // namespace pty
