// Concur step P_C: deterministic overlap consensus in float64.
//
//   object  O(r) = sum_j [S_j^T conj(P) y_j](r) / sum_j [S_j^T |P|^2](r)
//   probe   P(u) = sum_j conj(S_j O)(u) y_j(u) / sum_j |S_j O(u)|^2    (blind)
//
// Object: the object is cut into 64 x 16 tiles; each tile has the ascending
// list of scan positions whose window meets it (built on the host).  256
// threads own one tile, one thread a column of four pixels, and sum over the
// list in list order: every exit-wave pixel is read exactly once, no atomics,
// and the result does not depend on launch order.  For N <= 128 a work-group
// of 1024 threads owns four neighbouring tiles and keeps the probe in LDS.
// Probe: (position chunk) x (256-pixel block) work-groups write float64
// partial sums; a finalise kernel adds the chunks in ascending order.  The
// probe launch and the N <= 128 object launch place neighbouring work on one
// XCD (xcd_block), so the object pixels a chunk or tile row gathers stay in
// one L2; the N = 256 object launch keeps plain order (measured faster: its
// concurrent work-groups then read neighbouring exit waves).  The object launch also
// sums slices of the metric partials, which the finalise kernel's last block
// adds up.
#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "params.hpp"

namespace pty {

constexpr int kTileW = 64;
constexpr int kTileH = 16;

// Slice `b` of the metric partials, summed in a fixed order into part2[b]
// by a work-group of NT threads.
template <int NT = 256>
__device__ void metric_slice(const MetricParams& p, int b, double* red) {
  double acc[MF_COUNT];
#pragma unroll
  for (int q = 0; q < MF_COUNT; ++q) acc[q] = 0.0;
  const int total = p.J * p.nslot;
  const int per = (total + p.slices - 1) / p.slices;
  const int i0 = b * per, i1 = min(total, i0 + per);
  for (int i = i0 + int(threadIdx.x); i < i1; i += NT) {
#pragma unroll
    for (int q = 0; q < MF_COUNT; ++q) acc[q] += p.met[size_t(i) * MF_COUNT + q];
  }
  block_sum<MF_COUNT, NT>(acc, red);
  if (threadIdx.x < MF_COUNT) p.part2[size_t(b) * MF_COUNT + threadIdx.x] = acc[threadIdx.x];
}

// Add the slice sums in order and write the history ring (one work-group).
__device__ void metric_finish(const MetricParams& p, double* red) {
  double acc[MF_COUNT];
#pragma unroll
  for (int q = 0; q < MF_COUNT; ++q) acc[q] = 0.0;
  // (unrolled so that several slices' loads are in flight; the additions
  // keep their order)
#pragma unroll 8
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
  metric_slice<256>(p, blockIdx.x, red);
}

// One work-group per 64 x 16 object tile (N = 256, whose probe does not fit
// in LDS); a thread owns one column and four rows (row0 + 4 i).  The tile's
// list entries are staged in LDS (in chunks of kListChunk).  Exit waves and
// probe are read through buffer resources covering one pattern and the
// probe: a pixel outside the window gets an out-of-range offset, which reads
// zero without a memory request, so it adds exactly zero.  The next entry's
// requests are in flight while the current one is accumulated.
constexpr int kListChunk = 256;
static_assert(kListChunk == 256, "a tile's 256 threads stage one list entry each");

// blk, grid: the work-group's index and the (multiple of 8) work-group count
// of its scan's launch
template <class St>
__device__ __forceinline__ void object_update_body(const ObjParams& p, const int blk, const int grid) {
  __shared__ float red[4];
  __shared__ int4 ent[kListChunk];     // (scan index, row offset, col offset, unused)
  __shared__ double mred[MF_COUNT * 4];
  // tiles in plain order: consecutive work-groups, on different XCDs, then
  // read exit waves of neighbouring positions at the same time (XCD-contiguous
  // tile ranges measured 678 vs 668 us on the 4096-pattern scan, same bits)
  (void)grid;
  const int tile = blk;
  if (tile >= p.n_tiles) return;
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = tx * kTileW + lane;
  const int row0 = ty * kTileH + wave;
  const int N = p.N;
  const int NN = N * N;
  using elem = typename St::elem;
  const elem* ys = reinterpret_cast<const elem*>(p.y);

  if (tile < p.mp.slices) metric_slice<256>(p.mp, tile, mred);   // uniform in the work-group
  const int e0 = p.tile_off[tile], e1 = p.tile_off[tile + 1];
  float pm = 0.0f;
  for (int i = threadIdx.x; i < p.npb; i += 256) pm = fmaxf(pm, p.pmax_part[i]);
  float2 oldo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = row0 + 4 * i;
    oldo[i] = (row < p.H && col < p.W) ? p.obj[size_t(row) * p.W + col] : make_float2(0.f, 0.f);
  }
  pm = block_max<256>(pm, red);
  const double thr = p.tau * double(pm);
  // the exit waves are summed as stored: float16 storage holds y 2^s, and
  // scaling the float64 sums by 2^-s afterwards is exact (the same bits as
  // scaling every load)
  const double ysc = St::kFormat ? double(p.inv_scale) : 1.0;

  double nr[4] = {0, 0, 0, 0}, ni[4] = {0, 0, 0, 0}, dd[4] = {0, 0, 0, 0};
  const __amdgpu_buffer_rsrc_t prs = buffer_rsrc(p.probe, NN * 8);
  auto issue = [&](int e, int cn, float2 (&pv)[4], float2 (&yv)[4]) {
    const int4 en = ent[min(e, cn - 1)];
    const int du = col - en.z;
    const int dr = row0 - en.y;
    const bool cin = e < cn && (unsigned)du < (unsigned)N;
    const int base = dr * N + du;
    const int j = __builtin_amdgcn_readfirstlane(en.x);       // one entry per wave
    const __amdgpu_buffer_rsrc_t yrs = buffer_rsrc(ys + size_t(j) * NN, NN * int(sizeof(elem)));
    // byte offsets of the lane's pixel 0 (probe, exit wave), kOutside where
    // its column is outside the window; a row outside the window needs no
    // test: in unsigned arithmetic its offset is at or above N^2 elements
    // (or, below row 0, at or above 2^31), outside the buffer, so it reads
    // zero without a request like the out-of-window columns
    const unsigned op = cin ? unsigned(base) * 8u : unsigned(kOutside);
    const unsigned oy = cin ? unsigned(base) * unsigned(sizeof(elem)) : unsigned(kOutside);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      pv[i] = buffer_load_f2(prs, int(op + 32u * unsigned(N) * i));
      yv[i] = St::load_buf_unscaled(yrs, int(oy + 4u * unsigned(N) * unsigned(sizeof(elem)) * i));
    }
  };
  auto accumulate = [&](const float2 (&pv)[4], const float2 (&yv)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double px = pv[i].x, py = pv[i].y, yx = yv[i].x, yy = yv[i].y;
      nr[i] = fma(px, yx, fma(py, yy, nr[i]));
      ni[i] = fma(px, yy, fma(-py, yx, ni[i]));
      dd[i] = fma(px, px, fma(py, py, dd[i]));
    }
  };
  for (int c0 = e0; c0 < e1; c0 += kListChunk) {
    const int cn = min(kListChunk, e1 - c0);
    __syncthreads();
    if (int(threadIdx.x) < cn) ent[threadIdx.x] = p.tile_ent[c0 + threadIdx.x];   // one entry per thread
    __syncthreads();
    // (The conditional request of entry e + 2 makes the compiler wait for
    // every load before the second accumulation; issuing it unconditionally,
    // as the N <= 128 kernel does, measured slower here: 697 vs 675 us
    // float32, 533 vs 516 us float16 on the 4096-pattern scan.)
    float2 pa[4], ya[4], pb[4], yb[4];
    issue(0, cn, pa, ya);
    for (int e = 0; e < cn; e += 2) {
      issue(e + 1, cn, pb, yb);
      accumulate(pa, ya);
      if (e + 2 < cn) issue(e + 2, cn, pa, ya);
      accumulate(pb, yb);
    }
  }
  float m = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = row0 + 4 * i;
    if (row < p.H && col < p.W) {
      float2 o = oldo[i];
      if (dd[i] > thr) {
        o = make_float2(float(nr[i] * ysc / dd[i]), float(ni[i] * ysc / dd[i]));
        p.obj[size_t(row) * p.W + col] = o;
      }
      m = fmaxf(m, cnorm(o));
    }
  }
  m = block_max<256>(m, red);
  if (threadIdx.x == 0) p.tile_max[tile] = m;
}

// N <= 128: the probe (at most 128 KiB) is staged in LDS once per work-group
// and the work-group of 1024 threads owns kGroupTiles tiles, one per 256
// threads, summing in the same list order as above.  A pixel outside the
// window takes its probe factor from a zero entry after the probe in LDS and
// its exit wave through an out-of-range buffer offset (zero, no memory
// request), so it adds exactly zero.  Tile maxima and metric slices are per
// work-group.
constexpr int kGroupTiles = 4;
// list entries in flight per wave (3 and 4 measured the same, 6 and 8 slower:
// the loop waits on memory latency with the registers that two sets leave)
constexpr int kObjRing = 2;

template <class St, int N>
__device__ __forceinline__ void object_lds_body(const ObjParams& p, const int blk_id, const int grid) {
  constexpr int NN = N * N;
  constexpr int kZero = NN;            // index of the zero probe entry
  __shared__ float2 pl[NN + 1];
  __shared__ int4 ent[kGroupTiles][kListChunk];
  __shared__ float red[16];
  __shared__ int cnt[kGroupTiles];
  const int blk = xcd_block(blk_id, grid);   // neighbouring tiles on one XCD
  if (blk >= (p.n_tiles + kGroupTiles - 1) / kGroupTiles) return;
  const int g = threadIdx.x >> 8, lt = threadIdx.x & 255;
  const int tile = blk * kGroupTiles + g;
  const bool tile_ok = tile < p.n_tiles;
  const int tc = tile_ok ? tile : p.n_tiles - 1;
  const int tx = tc % p.tiles_x, ty = tc / p.tiles_x;
  const int lane = lt & 63, wave = lt >> 6;
  const int col = tx * kTileW + lane;
  const int row0 = ty * kTileH + wave;
  using elem = typename St::elem;
  const elem* ys = reinterpret_cast<const elem*>(p.y);

  // ---- the block's independent reads, requested together: metric slice,
  // list bounds, probe, probe maxima, the old object values -----------------
  // The metric slice (a few entries per block) is summed by the first wave
  // alone, without a barrier, so its reads go out with the others.
  const MetricParams& mp = p.mp;
  const int mtotal = mp.J * mp.nslot;
  const int mper = (mtotal + mp.slices - 1) / mp.slices;
  const int mi0 = blk * mper, mi1 = min(mtotal, mi0 + mper);
  double macc[MF_COUNT];
#pragma unroll
  for (int q = 0; q < MF_COUNT; ++q)
    macc[q] = (threadIdx.x < 64 && mi0 + int(threadIdx.x) < mi1)
                  ? mp.met[size_t(mi0 + threadIdx.x) * MF_COUNT + q] : 0.0;
  const int e0 = p.tile_off[tc];
  const int len = tile_ok ? p.tile_off[tc + 1] - e0 : 0;
  float2 pst[NN / 1024];
#pragma unroll
  for (int k = 0; k < NN / 1024; ++k) pst[k] = p.probe[threadIdx.x + 1024 * k];
  float pm = 0.0f;
  for (int i = threadIdx.x; i < p.npb; i += 1024) pm = fmaxf(pm, p.pmax_part[i]);
  float2 oldo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = row0 + 4 * i;
    const bool in = tile_ok && row < p.H && col < p.W;
    oldo[i] = in ? p.obj[size_t(row) * p.W + col] : make_float2(0.f, 0.f);
  }
  if (lt == 0) cnt[g] = len;
#pragma unroll
  for (int k = 0; k < NN / 1024; ++k) pl[threadIdx.x + 1024 * k] = pst[k];
  if (threadIdx.x == 0) pl[kZero] = make_float2(0.f, 0.f);
  if (threadIdx.x < 64) {
    for (int i = mi0 + 64 + int(threadIdx.x); i < mi1; i += 64) {
#pragma unroll
      for (int q = 0; q < MF_COUNT; ++q) macc[q] += mp.met[size_t(i) * MF_COUNT + q];
    }
#pragma unroll
    for (int q = 0; q < MF_COUNT; ++q) {
      for (int off = 32; off >= 1; off >>= 1) macc[q] += __shfl_xor(macc[q], off, 64);
    }
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < MF_COUNT; ++q) mp.part2[size_t(blk) * MF_COUNT + q] = macc[q];
    }
  }
  pm = block_max<1024>(pm, red);      // its barriers also publish pl and cnt
  const double thr = p.tau * double(pm);
  const double ysc = St::kFormat ? double(p.inv_scale) : 1.0;   // as in object_update_body
  int maxlen = cnt[0];
#pragma unroll
  for (int q = 1; q < kGroupTiles; ++q) maxlen = max(maxlen, cnt[q]);

  double nr[4] = {0, 0, 0, 0}, ni[4] = {0, 0, 0, 0}, dd[4] = {0, 0, 0, 0};
  // requests for entry e (past the end of the list: the last entry with a
  // zero probe): exit waves from memory, probe factors from LDS
  auto issue = [&](int e, int cn, float2 (&pv)[4], float2 (&yv)[4]) {
    const int4 en = ent[g][min(e, cn - 1)];
    const int du = col - en.z;                 // column in the window
    // row in the window of pixel 0: the same for the whole wave (one entry,
    // one row0 per wave), so the row tests below are scalar
    const int dr = __builtin_amdgcn_readfirstlane(row0 - en.y);
    const bool cin = e < cn && (unsigned)du < (unsigned)N;
    const int base = dr * N + du;
    const int j = __builtin_amdgcn_readfirstlane(en.x);       // one entry per wave
    const __amdgpu_buffer_rsrc_t yrs = buffer_rsrc(ys + size_t(j) * NN, NN * int(sizeof(elem)));
    // exit-wave byte offset of the lane's pixel 0, kOutside where its column
    // is outside the window; rows outside the window fall outside the buffer
    // by themselves (unsigned offsets at or above N^2 elements, or at or
    // above 2^31 below row 0) and read zero without a request.  The probe in
    // LDS has no such check: its index takes the zero entry explicitly.
    const unsigned oy = cin ? unsigned(base) * unsigned(sizeof(elem)) : unsigned(kOutside);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool ok = cin && (unsigned)(dr + 4 * i) < (unsigned)N;
      const int u = base + 4 * N * i;
      pv[i] = pl[ok ? u : kZero];
      yv[i] = St::load_buf_unscaled(yrs, int(oy + 4u * unsigned(N) * unsigned(sizeof(elem)) * i));
    }
  };
  auto accumulate = [&](const float2 (&pv)[4], const float2 (&yv)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double px = pv[i].x, py = pv[i].y, yx = yv[i].x, yy = yv[i].y;
      nr[i] = fma(px, yx, fma(py, yy, nr[i]));
      ni[i] = fma(px, yy, fma(-py, yx, ni[i]));
      dd[i] = fma(px, px, fma(py, py, dd[i]));
    }
  };
  for (int c0 = 0; c0 < maxlen; c0 += kListChunk) {   // same trip count in every group
    const int cn = min(kListChunk, len - c0);
    __syncthreads();
    if (lt < cn) ent[g][lt] = p.tile_ent[e0 + c0 + lt];   // one entry per thread
    __syncthreads();
    if (cn <= 0) continue;
    // a ring of kObjRing register sets: the following entries' requests are
    // in flight while one is accumulated, in list order; requests past the
    // end of the list are issued too (zero, no memory request, adding exactly
    // zero), since a conditional request makes the compiler's wait counts
    // assume it absent and wait for every load
    float2 pr[kObjRing][4], yr[kObjRing][4];
    static_for<0, kObjRing>([&](auto q) { issue(q.value, cn, pr[q.value], yr[q.value]); });
    for (int e = 0; e < cn; e += kObjRing) {
      static_for<0, kObjRing>([&](auto q) {
        accumulate(pr[q.value], yr[q.value]);
        issue(e + kObjRing + q.value, cn, pr[q.value], yr[q.value]);
      });
    }
  }
  float m = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = row0 + 4 * i;
    if (tile_ok && row < p.H && col < p.W) {
      float2 o = oldo[i];
      if (dd[i] > thr) {
        o = make_float2(float(nr[i] * ysc / dd[i]), float(ni[i] * ysc / dd[i]));
        p.obj[size_t(row) * p.W + col] = o;
      }
      m = fmaxf(m, cnorm(o));
    }
  }
  m = block_max<1024>(m, red);
  if (threadIdx.x == 0) p.tile_max[blk] = m;
}

constexpr int kProbeUnroll = 8;

template <class St>
__device__ __forceinline__ void probe_partial_body(const ProbeParams& p, const int blk, const int grid) {
  const int N = p.N;
  const int NN = N * N;
  // logical block = chunk-major (g, pixel block); each XCD runs whole chunks,
  // whose object gathers then stay in its L2
  const int npb = (NN + 255) / 256;
  const int l = xcd_block(blk, grid);
  if (l >= npb * p.G) return;
  const int g = l / npb;
  const int u = (l % npb) * 256 + threadIdx.x;
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
      yv[q] = St::load_stream(ys, size_t(jj) * NN + uu, p.inv_scale);
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

__device__ __forceinline__ void probe_final_body(const FinalParams& p, const int blk) {
  __shared__ double dred[MF_COUNT * 4];
  __shared__ float fred[4];
  const int b = blk + p.first_block;
  if (b == p.npb) {
    metric_finish(p.mp, dred);
    return;
  }
  const int NN = p.N * p.N;
  const int u = b * 256 + threadIdx.x;
  // the chunk sums first (they do not depend on the object maximum), so their
  // loads overlap those of the tile maxima and the block reduction
  double nr = 0.0, ni = 0.0, dd = 0.0;
  float2 pv = make_float2(0.f, 0.f);
  if (u < NN) {
    const size_t plane = size_t(p.G) * NN;
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
    pv = p.probe[u];
  }
  float om = 0.0f;
#pragma unroll 8
  for (int i = threadIdx.x; i < p.n_tiles; i += 256) om = fmaxf(om, p.tile_max[i]);
  om = block_max<256>(om, fred);
  const double thr = p.tau * double(om);
  float m = 0.0f;
  if (u < NN) {
    if (dd > thr) {
      pv = make_float2(float(nr / dd), float(ni / dd));
      p.probe[u] = pv;
    }
    m = cnorm(pv);
  }
  m = block_max<256>(m, fred);
  if (threadIdx.x == 0) p.pmax_part[b] = m;
}

// Kernels: one scan, or a group of scans in one launch (the served form),
// with the same per-work-group work.
template <class St>
__global__ __launch_bounds__(256) void object_update_kernel(ObjParams p) {
  object_update_body<St>(p, int(blockIdx.x), int(gridDim.x));
}
template <class St>
__global__ __launch_bounds__(256) void object_update_group_kernel(Group<ObjParams> g) {
  const int b = int(blockIdx.x);
  const int sc = group_scan(g, b);
  object_update_body<St>(g.p[sc], b - g.first[sc], g.first[sc + 1] - g.first[sc]);
}
template <class St, int N>
__global__ __launch_bounds__(1024) void object_lds_kernel(ObjParams p) {
  object_lds_body<St, N>(p, int(blockIdx.x), int(gridDim.x));
}
template <class St, int N>
__global__ __launch_bounds__(1024) void object_lds_group_kernel(Group<ObjParams> g) {
  const int b = int(blockIdx.x);
  const int sc = group_scan(g, b);
  object_lds_body<St, N>(g.p[sc], b - g.first[sc], g.first[sc + 1] - g.first[sc]);
}
template <class St>
__global__ __launch_bounds__(256) void probe_partial_kernel(ProbeParams p) {
  probe_partial_body<St>(p, int(blockIdx.x), int(gridDim.x));
}
template <class St>
__global__ __launch_bounds__(256) void probe_partial_group_kernel(Group<ProbeParams> g) {
  const int b = int(blockIdx.x);
  const int sc = group_scan(g, b);
  probe_partial_body<St>(g.p[sc], b - g.first[sc], g.first[sc + 1] - g.first[sc]);
}
__global__ __launch_bounds__(256) void probe_final_kernel(FinalParams p) { probe_final_body(p, int(blockIdx.x)); }
__global__ __launch_bounds__(256) void probe_final_group_kernel(Group<FinalParams> g) {
  const int b = int(blockIdx.x);
  const int sc = group_scan(g, b);
  probe_final_body(g.p[sc], b - g.first[sc]);
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
int object_blocks(int n, int n_tiles) {
  return n <= 128 ? (n_tiles + kGroupTiles - 1) / kGroupTiles : n_tiles;
}

// Metric slices: one per object work-group, at N = 256 at most
// kMaxMetricSlices (its 16384 tiles at the 4096-pattern scan gave slices of
// four entries, which the finalise block then added 64 after one another:
// 24 us for the whole finalise launch).
constexpr int kMaxMetricSlices = 256;
int metric_slices(int n, int n_tiles) {
  const int b = object_blocks(n, n_tiles);
  return n <= 128 ? b : (b < kMaxMetricSlices ? b : kMaxMetricSlices);
}

template <class St>
static void launch_object_t(const ObjParams& p, hipStream_t s) {
  const dim3 grid(xcd_pad(object_blocks(p.N, p.n_tiles)));
  switch (p.N) {
    case 32: hipLaunchKernelGGL((object_lds_kernel<St, 32>), grid, dim3(1024), 0, s, p); break;
    case 64: hipLaunchKernelGGL((object_lds_kernel<St, 64>), grid, dim3(1024), 0, s, p); break;
    case 128: hipLaunchKernelGGL((object_lds_kernel<St, 128>), grid, dim3(1024), 0, s, p); break;
    default: hipLaunchKernelGGL(object_update_kernel<St>, grid, dim3(256), 0, s, p); break;
  }
}

hipError_t launch_object_update(int fp16, const ObjParams& p, hipStream_t s) {
  if (fp16) launch_object_t<StoreF16>(p, s);
  else launch_object_t<StoreF32>(p, s);
  return hipGetLastError();
}

hipError_t launch_probe_partial(int fp16, const ProbeParams& p, hipStream_t s) {
  const dim3 grid(xcd_pad((p.N * p.N + 255) / 256 * p.G));
  if (fp16) hipLaunchKernelGGL(probe_partial_kernel<StoreF16>, grid, dim3(256), 0, s, p);
  else hipLaunchKernelGGL(probe_partial_kernel<StoreF32>, grid, dim3(256), 0, s, p);
  return hipGetLastError();
}

// Grouped launchers: every scan's range of work-groups is the count its own
// launch would use (a multiple of 8 where the work-groups are mapped to
// XCD-contiguous ranges), one after the other.
hipError_t launch_object_update_group(int fp16, const ObjParams* ps, int count, hipStream_t s) {
  if (count < 1 || count > kGroupMax) return hipErrorInvalidValue;
  Group<ObjParams> g{};
  int blocks = 0;
  for (int i = 0; i < count; ++i) {
    if (ps[i].N != ps[0].N) return hipErrorInvalidValue;
    g.p[i] = ps[i];
    g.first[i] = blocks;
    blocks += xcd_pad(object_blocks(ps[i].N, ps[i].n_tiles));
  }
  g.first[count] = blocks;
  g.count = count;
  const int N = ps[0].N;
  const dim3 grid(blocks);
  if (fp16) {
    switch (N) {
      case 32: hipLaunchKernelGGL((object_lds_group_kernel<StoreF16, 32>), grid, dim3(1024), 0, s, g); break;
      case 64: hipLaunchKernelGGL((object_lds_group_kernel<StoreF16, 64>), grid, dim3(1024), 0, s, g); break;
      case 128: hipLaunchKernelGGL((object_lds_group_kernel<StoreF16, 128>), grid, dim3(1024), 0, s, g); break;
      default: hipLaunchKernelGGL(object_update_group_kernel<StoreF16>, grid, dim3(256), 0, s, g); break;
    }
  } else {
    switch (N) {
      case 32: hipLaunchKernelGGL((object_lds_group_kernel<StoreF32, 32>), grid, dim3(1024), 0, s, g); break;
      case 64: hipLaunchKernelGGL((object_lds_group_kernel<StoreF32, 64>), grid, dim3(1024), 0, s, g); break;
      case 128: hipLaunchKernelGGL((object_lds_group_kernel<StoreF32, 128>), grid, dim3(1024), 0, s, g); break;
      default: hipLaunchKernelGGL(object_update_group_kernel<StoreF32>, grid, dim3(256), 0, s, g); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_probe_partial_group(int fp16, const ProbeParams* ps, int count, hipStream_t s) {
  if (count < 1 || count > kGroupMax) return hipErrorInvalidValue;
  Group<ProbeParams> g{};
  int blocks = 0;
  for (int i = 0; i < count; ++i) {
    g.p[i] = ps[i];
    g.first[i] = blocks;
    blocks += xcd_pad((ps[i].N * ps[i].N + 255) / 256 * ps[i].G);
  }
  g.first[count] = blocks;
  g.count = count;
  if (fp16) hipLaunchKernelGGL(probe_partial_group_kernel<StoreF16>, dim3(blocks), dim3(256), 0, s, g);
  else hipLaunchKernelGGL(probe_partial_group_kernel<StoreF32>, dim3(blocks), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_probe_final_group(const FinalParams* ps, const int* update_probe, int count, hipStream_t s) {
  if (count < 1 || count > kGroupMax) return hipErrorInvalidValue;
  Group<FinalParams> g{};
  int blocks = 0;
  for (int i = 0; i < count; ++i) {
    g.p[i] = ps[i];
    g.p[i].first_block = update_probe[i] ? 0 : ps[i].npb;
    g.first[i] = blocks;
    blocks += update_probe[i] ? ps[i].npb + 1 : 1;
  }
  g.first[count] = blocks;
  g.count = count;
  hipLaunchKernelGGL(probe_final_group_kernel, dim3(blocks), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_probe_final(const FinalParams& p, int update_probe, hipStream_t s) {
  FinalParams q = p;
  q.first_block = update_probe ? 0 : p.npb;
  const int blocks = update_probe ? p.npb + 1 : 1;
  hipLaunchKernelGGL(probe_final_kernel, dim3(blocks), dim3(256), 0, s, q);
  return hipGetLastError();
}

// Exchange two complex arrays element by element (no temporary buffer).
__global__ void swap_kernel(float2* __restrict__ a, float2* __restrict__ b, size_t count) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < count; i += size_t(gridDim.x) * blockDim.x) {
    const float2 t = a[i];
    a[i] = b[i];
    b[i] = t;
  }
}

hipError_t launch_swap(float2* a, float2* b, size_t count, hipStream_t s) {
  const int blocks = int(std::min<size_t>((count + 255) / 256, 8192));
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(swap_kernel, dim3(blocks), dim3(256), 0, s, a, b, count);
  return hipGetLastError();
}

// Object error against ground truth with the global complex scale removed:
// with S_tt = sum |t|^2, S_oo = sum |o|^2, S_ot = sum conj(o) t over the box,
// min_g sum |t - g o|^2 = S_tt - |S_ot|^2 / S_oo (g = S_ot / S_oo).  Rows are
// split over the blocks in order; float64 sums in a fixed order.
__global__ __launch_bounds__(256) void object_error_part_kernel(const float2* __restrict__ o, int ow,
                                                                const float2* __restrict__ t, int r0, int c0,
                                                                int h, int w, double* part) {
  __shared__ double red[4 * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const size_t total = size_t(h) * w;
  const size_t per = (total + gridDim.x - 1) / gridDim.x;
  const size_t i0 = blockIdx.x * per, i1 = min(total, i0 + per);
  for (size_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const int r = int(i / w), c = int(i % w);
    const float2 a = o[size_t(r0 + r) * ow + (c0 + c)];
    const float2 b = t[i];
    const double ox = a.x, oy = a.y, tx = b.x, ty = b.y;
    acc[0] += tx * tx + ty * ty;
    acc[1] += ox * ox + oy * oy;
    acc[2] += ox * tx + oy * ty;     // Re conj(o) t
    acc[3] += ox * ty - oy * tx;     // Im conj(o) t
  }
  block_sum<4, 256>(acc, red);
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = acc[threadIdx.x];
}

__global__ void object_error_finish_kernel(const double* part, int blocks, double* result) {
  if (threadIdx.x != 0) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < blocks; ++b)
    for (int q = 0; q < 4; ++q) s[q] += part[b * 4 + q];
  double e = __builtin_nan("");
  if (s[0] > 0.0) e = s[1] > 0.0 ? (s[0] - (s[2] * s[2] + s[3] * s[3]) / s[1]) / s[0] : 1.0;
  *result = e;
}

hipError_t launch_object_error(const float2* o, int ow, const float2* t, int r0, int c0, int h, int w, double* part,
                               int blocks, double* result, hipStream_t s) {
  hipLaunchKernelGGL(object_error_part_kernel, dim3(blocks), dim3(256), 0, s, o, ow, t, r0, c0, h, w, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(object_error_finish_kernel, dim3(1), dim3(64), 0, s, part, blocks, result);
  return hipGetLastError();
}

// Partial sums of the allocation-free object error: every work-group writes
// its four sums before the finishing kernel reads them, so nothing needs
// clearing; all calls on one GPU share this array, so calls that overlap on
// that GPU (different streams, or threads) race.
static __device__ __align__(256) double scratch[4 * kErrScratchBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};   // each device's address of `scratch`, looked up once
}  // namespace

hipError_t object_error_static(const float2* o, int ow, const float2* t, int r0, int c0, int h, int w,
                               double* result, hipStream_t s) {
  const int blocks = object_error_blocks((long long)h * w);
  if (blocks > kErrScratchBlocks) return hipErrorInvalidValue;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
      // with this device current: the array's address on this device
      e = hipGetSymbolAddress(&g_scratch_addr[dev], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        g_scratch_addr[dev] = nullptr;
        return e;
      }
    }
    ptr = g_scratch_addr[dev];
  }
  return launch_object_error(o, ow, t, r0, c0, h, w, static_cast<double*>(ptr), blocks, result, s);
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
