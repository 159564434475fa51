// Concur step P_C: deterministic overlap consensus in float64.
//
//   object  O(r) = sum_j [S_j^T conj(P) y_j](r) / sum_j [S_j^T |P|^2](r)
//   probe   P(u) = sum_j conj(S_j O)(u) y_j(u) / sum_j |S_j O(u)|^2    (blind)
//
// Object: the object is cut into 64 x 16 tiles; each tile has the ascending
// list of scan positions whose window meets it (built on the host).  One
// work-group owns one tile, one thread a column of four pixels, and sums over
// its list in list order: every exit-wave pixel is read exactly once, no
// atomics, and the result does not depend on launch order.
// Probe: a grid of (256-pixel block) x (position chunk) writes float64
// partial sums; a finalise kernel adds the chunks in ascending order.  The
// object launch also sums slices of the metric partials, which the finalise
// kernel's last block adds up.
#include "common.hpp"
#include "params.hpp"

namespace pty {

constexpr int kTileW = 64;
constexpr int kTileH = 16;

// Slice `b` of the metric partials, summed in a fixed order into part2[b].
__device__ void metric_slice(const MetricParams& p, int b, double* red) {
  double acc[MF_COUNT];
#pragma unroll
  for (int q = 0; q < MF_COUNT; ++q) acc[q] = 0.0;
  const int total = p.J * p.nslot;
  const int per = (total + p.slices - 1) / p.slices;
  const int i0 = b * per, i1 = min(total, i0 + per);
  for (int i = i0 + int(threadIdx.x); i < i1; i += 256) {
#pragma unroll
    for (int q = 0; q < MF_COUNT; ++q) acc[q] += p.met[size_t(i) * MF_COUNT + q];
  }
  block_sum<MF_COUNT, 256>(acc, red);
  if (threadIdx.x < MF_COUNT) p.part2[size_t(b) * MF_COUNT + threadIdx.x] = acc[threadIdx.x];
}

// Add the slice sums in order and write the history ring (one work-group).
__device__ void metric_finish(const MetricParams& p, double* red) {
  double acc[MF_COUNT];
#pragma unroll
  for (int q = 0; q < MF_COUNT; ++q) acc[q] = 0.0;
  for (int i = threadIdx.x; i < p.slices; i += 256) {
#pragma unroll
    for (int q = 0; q < MF_COUNT; ++q) acc[q] += p.part2[size_t(i) * MF_COUNT + q];
  }
  block_sum<MF_COUNT, 256>(acc, red);
  if (threadIdx.x == 0) {
    const double nan = __builtin_nan("");
    if (p.k_cur >= 0) {
      double* e = p.ring + (p.k_cur % p.cap) * kRingFields;
      e[0] = double(p.k_cur);
      e[1] = acc[MF_EF_DEN] > 0 ? acc[MF_EF_NUM] / acc[MF_EF_DEN] : nan;
      e[2] = nan;
      e[3] = nan;
    }
    if (p.k_prev >= 0) {
      double* e = p.ring + (p.k_prev % p.cap) * kRingFields;
      e[2] = (p.ec_ok && acc[MF_EC_DEN] > 0) ? acc[MF_EC_NUM] / acc[MF_EC_DEN] : nan;
      e[3] = (p.dx_ok && acc[MF_DX_DEN] > 0) ? sqrt(acc[MF_DX_NUM] / acc[MF_DX_DEN]) : nan;
    }
  }
}

__global__ __launch_bounds__(256) void metric_slice_kernel(MetricParams p) {
  __shared__ double red[MF_COUNT * 4];
  metric_slice(p, blockIdx.x, red);
}

// One work-group per 64 x 16 object tile; a thread owns one column and four
// rows (row0 + 4 i).  The tile's list of overlapping positions is staged in
// LDS (in chunks of kListChunk), then consumed kUnroll entries at a time so
// that each thread keeps 4 * kUnroll exit-wave loads in flight.
constexpr int kListChunk = 256;
constexpr int kUnroll = 4;

template <class St>
__global__ __launch_bounds__(256) void object_update_kernel(ObjParams p) {
  __shared__ float red[4];
  __shared__ int4 ent[kListChunk];     // (scan index, row offset, col offset, unused)
  const int tile = blockIdx.x;
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = tx * kTileW + lane;
  const int row0 = ty * kTileH + wave;
  const int N = p.N;
  const size_t NN = size_t(N) * N;
  using elem = typename St::elem;
  const elem* ys = reinterpret_cast<const elem*>(p.y);

  float pm = 0.0f;
  for (int i = threadIdx.x; i < p.npb; i += 256) pm = fmaxf(pm, p.pmax_part[i]);
  pm = block_max<256>(pm, red);
  const double thr = p.tau * double(pm);

  double nr[4] = {0, 0, 0, 0}, ni[4] = {0, 0, 0, 0}, dd[4] = {0, 0, 0, 0};
  const int e0 = p.tile_off[tile], e1 = p.tile_off[tile + 1];
  for (int c0 = e0; c0 < e1; c0 += kListChunk) {
    const int cn = min(kListChunk, e1 - c0);
    __syncthreads();
    for (int i = threadIdx.x; i < cn; i += 256) {
      const int j = p.tile_list[c0 + i];
      const int2 pj = p.pos[j];
      ent[i] = make_int4(j, pj.x, pj.y, 0);
    }
    __syncthreads();
    // Branch-free: indices are clamped into the window (valid addresses, the
    // same rows and lines the in-window lanes fetch) and masked values are
    // zeroed, so a group of loads issues back to back.
    int e = 0;
    for (; e < cn; e += kUnroll) {
      float2 pv[kUnroll][4], yv[kUnroll][4];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int4 en = ent[min(e + q, cn - 1)];
        const bool live = e + q < cn;
        const int u1 = col - en.z;
        const bool cin = live && (unsigned)u1 < (unsigned)N;
        const int u1c = min(max(u1, 0), N - 1);
        const elem* yj = ys + size_t(en.x) * NN;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int u0 = row0 + 4 * i - en.y;
          const bool ok = cin && (unsigned)u0 < (unsigned)N;
          const int u = min(max(u0, 0), N - 1) * N + u1c;
          const float2 a = p.probe[u];
          const float2 b = St::load(yj, u, p.inv_scale);
          pv[q][i] = make_float2(ok ? a.x : 0.f, ok ? a.y : 0.f);
          yv[q][i] = make_float2(ok ? b.x : 0.f, ok ? b.y : 0.f);
        }
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double px = pv[q][i].x, py = pv[q][i].y, yx = yv[q][i].x, yy = yv[q][i].y;
          nr[i] += px * yx + py * yy;
          ni[i] += px * yy - py * yx;
          dd[i] += px * px + py * py;
        }
      }
    }
  }
  float m = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = row0 + 4 * i;
    if (row < p.H && col < p.W) {
      const size_t idx = size_t(row) * p.W + col;
      float2 o = p.obj[idx];
      if (dd[i] > thr) {
        o = make_float2(float(nr[i] / dd[i]), float(ni[i] / dd[i]));
        p.obj[idx] = o;
      }
      m = fmaxf(m, cnorm(o));
    }
  }
  m = block_max<256>(m, red);
  if (threadIdx.x == 0) p.tile_max[tile] = m;
  __shared__ double mred[MF_COUNT * 4];
  metric_slice(p.mp, tile, mred);
}

constexpr int kProbeUnroll = 8;

template <class St>
__global__ __launch_bounds__(256) void probe_partial_kernel(ProbeParams p) {
  const int N = p.N;
  const int NN = N * N;
  const int u = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  const int j0 = g * p.chunk;
  const int j1 = min(p.J, j0 + p.chunk);
  const int uu = min(u, NN - 1);
  const int u0 = uu / N, u1 = uu % N;
  using elem = typename St::elem;
  const elem* ys = reinterpret_cast<const elem*>(p.y);
  double nr = 0.0, ni = 0.0, dd = 0.0;
  // kProbeUnroll positions per step: 2 * kProbeUnroll loads in flight
  for (int j = j0; j < j1; j += kProbeUnroll) {
    float2 ov[kProbeUnroll], yv[kProbeUnroll];
#pragma unroll
    for (int q = 0; q < kProbeUnroll; ++q) {
      const int jj = min(j + q, j1 - 1);
      const int2 pj = p.pos[jj];
      ov[q] = p.obj[size_t(pj.x + u0) * p.W + (pj.y + u1)];
      yv[q] = St::load(ys, size_t(jj) * NN + uu, p.inv_scale);
    }
#pragma unroll
    for (int q = 0; q < kProbeUnroll; ++q) {
      if (j + q < j1) {
        const double ox = ov[q].x, oy = ov[q].y, yx = yv[q].x, yy = yv[q].y;
        nr += ox * yx + oy * yy;
        ni += ox * yy - oy * yx;
        dd += ox * ox + oy * oy;
      }
    }
  }
  if (u < NN) {
    const size_t plane = size_t(p.G) * NN;
    const size_t o = size_t(g) * NN + u;
    p.part[o] = nr;
    p.part[plane + o] = ni;
    p.part[2 * plane + o] = dd;
  }
}

__global__ __launch_bounds__(256) void probe_final_kernel(FinalParams p) {
  __shared__ double dred[MF_COUNT * 4];
  __shared__ float fred[4];
  const int b = blockIdx.x + p.first_block;
  if (b == p.npb) {
    metric_finish(p.mp, dred);
    return;
  }
  const int NN = p.N * p.N;
  const int u = b * 256 + threadIdx.x;
  float om = 0.0f;
  for (int i = threadIdx.x; i < p.n_tiles; i += 256) om = fmaxf(om, p.tile_max[i]);
  om = block_max<256>(om, fred);
  const double thr = p.tau * double(om);
  float m = 0.0f;
  if (u < NN) {
    const size_t plane = size_t(p.G) * NN;
    double nr = 0.0, ni = 0.0, dd = 0.0;
    int g = 0;
    for (; g + 4 <= p.G; g += 4) {
      double a[4], c[4], d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const size_t o = size_t(g + q) * NN + u;
        a[q] = p.part[o];
        c[q] = p.part[plane + o];
        d[q] = p.part[2 * plane + o];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        nr += a[q];
        ni += c[q];
        dd += d[q];
      }
    }
    for (; g < p.G; ++g) {
      const size_t o = size_t(g) * NN + u;
      nr += p.part[o];
      ni += p.part[plane + o];
      dd += p.part[2 * plane + o];
    }
    float2 pv = p.probe[u];
    if (dd > thr) {
      pv = make_float2(float(nr / dd), float(ni / dd));
      p.probe[u] = pv;
    }
    m = cnorm(pv);
  }
  m = block_max<256>(m, fred);
  if (threadIdx.x == 0) p.pmax_part[b] = m;
}

__global__ __launch_bounds__(256) void max_abs2_parts_kernel(const float2* a, size_t count, float* parts) {
  __shared__ float red[4];
  float m = 0.0f;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) {
    m = fmaxf(m, cnorm(a[i]));
  }
  m = block_max<256>(m, red);
  if (threadIdx.x == 0) parts[blockIdx.x] = m;
}

template <class St>
__global__ void convert_kernel(int to_store, const float2* src, typename St::elem* dst_store,
                               const typename St::elem* src_store, float2* dst, size_t count, float scale,
                               float inv_scale) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < count; i += size_t(gridDim.x) * blockDim.x) {
    if (to_store) St::store(dst_store, i, src[i], scale);
    else dst[i] = St::load(src_store, i, inv_scale);
  }
}

// ---------------------------------------------------------------------------
hipError_t launch_object_update(int fp16, const ObjParams& p, hipStream_t s) {
  if (fp16) hipLaunchKernelGGL(object_update_kernel<StoreF16>, dim3(p.n_tiles), dim3(256), 0, s, p);
  else hipLaunchKernelGGL(object_update_kernel<StoreF32>, dim3(p.n_tiles), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_probe_partial(int fp16, const ProbeParams& p, hipStream_t s) {
  const dim3 grid((p.N * p.N + 255) / 256, p.G);
  if (fp16) hipLaunchKernelGGL(probe_partial_kernel<StoreF16>, grid, dim3(256), 0, s, p);
  else hipLaunchKernelGGL(probe_partial_kernel<StoreF32>, grid, dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_probe_final(const FinalParams& p, int update_probe, hipStream_t s) {
  FinalParams q = p;
  q.first_block = update_probe ? 0 : p.npb;
  const int blocks = update_probe ? p.npb + 1 : 1;
  hipLaunchKernelGGL(probe_final_kernel, dim3(blocks), dim3(256), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_metric_slices(const MetricParams& p, hipStream_t s) {
  hipLaunchKernelGGL(metric_slice_kernel, dim3(p.slices), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_max_abs2_parts(const float2* a, size_t count, float* parts, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(max_abs2_parts_kernel, dim3(nparts), dim3(256), 0, s, a, count, parts);
  return hipGetLastError();
}

hipError_t launch_convert_state(int fp16, int to_store, const float2* src, void* dst_store, const void* src_store,
                                float2* dst, size_t count, float scale, float inv_scale, hipStream_t s) {
  const int blocks = int(std::min<size_t>((count + 255) / 256, 16384));
  if (blocks <= 0) return hipSuccess;
  if (fp16) {
    hipLaunchKernelGGL(convert_kernel<StoreF16>, dim3(blocks), dim3(256), 0, s, to_store, src,
                       reinterpret_cast<__half2*>(dst_store), reinterpret_cast<const __half2*>(src_store), dst,
                       count, scale, inv_scale);
  } else {
    hipLaunchKernelGGL(convert_kernel<StoreF32>, dim3(blocks), dim3(256), 0, s, to_store, src,
                       reinterpret_cast<float2*>(dst_store), reinterpret_cast<const float2*>(src_store), dst,
                       count, scale, inv_scale);
  }
  return hipGetLastError();
}

}  // namespace pty
