// Kernel parameter blocks (plain structs, passed by value) and launcher
// declarations shared by the host engine and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pty {

// per-slot metric partials, float64:
enum MetricField { MF_EF_NUM = 0, MF_EF_DEN, MF_EC_NUM, MF_EC_DEN, MF_DX_NUM, MF_DX_DEN, MF_COUNT };
// ring entry: iteration, fourier_err, consistency_err, change
constexpr int kRingFields = 4;

struct DivideParams {
  const float2* obj;      // [H][W]
  const float2* probe;    // [N][N]
  const int2* pos;        // [J] (row, col)
  const float* amp;       // sqrt(I) in the layout of the consuming kernel
  const float2* tw;       // tw[m] = exp(-2 pi i m / N), m < N
  void* x;                // exit waves, storage format of the kernel
  void* y;
  float2* tmp;            // N = 256: float32 intermediate (may alias y)
  int obj_w;
  int j_begin;
  // prologue: x_k = alpha * P S_j O + beta * y_{k-1} + gamma * x_{k-1}
  float alpha, beta, gamma;
  float c;                // divide relaxation
  float scale, inv_scale; // float16 storage scale and its inverse
  int read_x, read_y, write_x;
  int prev_ec, prev_dx;   // accumulate consistency / change partials of the previous iteration
  double* met;            // [J][nslot][MF_COUNT]
  int nslot;
  // Blend form (fused kernel only).  The x buffer holds the blend
  //   w_{k-1} = gamma' x_{k-1} + beta' y_{k-1}
  // of the previous iteration, the prologue forms x_k = alpha * P S_j O + w_{k-1}
  // (read_x = 0: w is zero), and the epilogue forms x_k again the same way and
  // stores w_k = next_gamma * x_k + next_beta * y_k (if write_x) beside y_k.
  int wform;
  float next_beta, next_gamma;
  // Sequential projections (one launch per batch of disjoint windows): the
  // work-group of slot s handles pattern batch[s]; the prologue forms
  // psi = P S_j O, the Fourier step is the unrelaxed modulus projection, the
  // epilogue adds sp_alpha conj(P) d / max|P|^2 to the object window and
  // writes sp_beta conj(S_j O) d / max|S_j O|^2 to contrib[s] (d = psi' - psi).
  const int* batch;
  float2* obj_out;          // the object, written in place (windows of a batch are disjoint)
  float2* contrib;          // [batch size][N][N] probe steps (blind)
  const float* pmax_part;   // [npb] partial maxima of |P|^2
  int npb;
  float sp_alpha, sp_beta;
  int sp_blind;
  float* sp_omax;           // N = 256: [batch slot][16] row-block maxima of |S_j O|^2
};

// Probe update after a batch of sequential projections: P += sum over the
// batch's slots (in order) of contrib, float64 sums; then the partial maxima.
struct SpProbeParams {
  float2* probe;
  const float2* contrib;
  int count, N;
  float* pmax_part;
};

// Metric finalisation of one iteration: a fixed-order two-level float64
// reduction of the per-pattern partials into the history ring.  The object
// launch sums one slice per work-group into part2; after that kernel has
// finished, one work-group of the finalise launch adds the slice sums in
// order (a kernel boundary, not a device-wide fence, publishes part2).
struct MetricParams {
  const double* met;      // [J][nslot][MF_COUNT]
  int J, nslot;
  double* part2;          // [slices][MF_COUNT]
  int slices;
  double* ring;           // [cap][kRingFields]
  int cap;
  long long k_cur;        // iteration whose Fourier error is in met (-1: none)
  long long k_prev;       // iteration whose consistency / change are in met (-1: none)
  int ec_ok, dx_ok;
};

struct ObjParams {
  const void* y;
  float inv_scale;
  const float2* probe;
  const int2* pos;
  const int* tile_off;    // [n_tiles + 1]
  const int4* tile_ent;   // per tile, ascending j: (j, row, col, 0) of each overlapping window
  float2* obj;
  int H, W, N, tiles_x, n_tiles;
  float* tile_max;        // [object_blocks] max |O_new|^2 of each work-group's tiles
  const float* pmax_part; // [npb] partial maxima of |P|^2
  int npb;
  double tau;
  MetricParams mp;        // the object launch also finalises the metrics
};

// Probe partial sums over position chunks (one work-group per 256-pixel
// block and chunk).
struct ProbeParams {
  const void* y;
  float inv_scale;
  const float2* obj;
  const int2* pos;
  int N, W, J, chunk, G;
  double* part;           // [3][G][N*N]: Re N_P, Im N_P, D_P
};

// Finalise: probe blocks add the chunks in ascending order, apply the guard
// and write the probe and its per-block maxima; the metrics block (index
// npb) finishes the metric reduction.
struct FinalParams {
  const double* part;
  float2* probe;
  float* pmax_part;       // [npb]
  const float* tile_max;  // [n_tiles]
  int n_tiles, N, G, npb;
  double tau;
  int first_block;        // npb: run the metrics block only
  MetricParams mp;
};

struct FlushParams {
  const float2* obj;
  const float2* probe;
  const int2* pos;
  void* x;
  const void* y;
  int N, obj_w;
  float alpha, beta, gamma;
  float scale, inv_scale;
  int read_x, read_y;     // a buffer not read counts as zero
  int write_x;
  double* met;
  int nslot;
  int wform;              // x holds the blend w: x = alpha * P S_j O + w, no metrics
};

// Grouped launch: one launch runs the same kernel for up to kGroupMax scans
// (same pattern size, storage and prologue mode); scan s owns the launch's
// work-groups [first[s], first[s+1]).  Work-group b runs on XCD b mod 8.  The
// object and probe launches pad each scan's range to a multiple of 8, so a
// block's XCD (and xcd_block's mapping) is the one of its scan's launch alone;
// the N = 256 passes take 16 blocks per pattern, so their pairing of column
// blocks on one XCD holds too.  The fused divide's ranges are not padded: its
// per-pattern work does not depend on where it runs.
constexpr int kGroupMax = 8;
template <class P>
struct Group {
  P p[kGroupMax];
  int first[kGroupMax + 1];
  int count;
};
// The scan of work-group b in a grouped launch: the last s with first[s] <= b
// (a few scalar comparisons; first[] is in the kernel arguments).
template <class P>
__device__ __forceinline__ int group_scan(const Group<P>& g, int b) {
  int s = 0;
#pragma unroll
  for (int i = 1; i < kGroupMax; ++i) s += (i < g.count && b >= g.first[i]) ? 1 : 0;
  return s;
}

// ---- launchers (return hipGetLastError() of the launch) ----
// one kernel of the divide: stage 0 (fused, or N = 256 rows forward), 1 (N = 256 columns), 2 (N = 256 rows inverse)
hipError_t launch_divide_stage(int n, int fp16, const DivideParams& p, int n_patterns, int stage, hipStream_t s);
// the same stage for count <= kGroupMax scans in one launch (ps[i] with n_patterns[i]
// patterns; every ps[i] has the prologue mode of ps[0])
hipError_t launch_divide_stage_group(int n, int fp16, const DivideParams* ps, const int* n_patterns, int count,
                                     int stage, hipStream_t s);
int divide_stages(int n);
// the prologue mode a divide launch with these parameters runs (scans are
// grouped only with scans of the same mode)
int divide_mode(const DivideParams& p);
// whether a divide launch with these parameters has a grouped form
bool divide_groupable(int n, const DivideParams& p);
hipError_t launch_object_update(int fp16, const ObjParams& p, hipStream_t s);
hipError_t launch_object_update_group(int fp16, const ObjParams* ps, int count, hipStream_t s);
// work-groups of the object launch: each writes one tile_max entry; the first
// metric_slices of them also sum one metric slice each
int object_blocks(int n, int n_tiles);
int metric_slices(int n, int n_tiles);
hipError_t launch_probe_partial(int fp16, const ProbeParams& p, hipStream_t s);
hipError_t launch_probe_partial_group(int fp16, const ProbeParams* ps, int count, hipStream_t s);
hipError_t launch_flush(int fp16, const FlushParams& p, int J, hipStream_t s);
hipError_t launch_probe_final(const FinalParams& p, int update_probe, hipStream_t s);
hipError_t launch_probe_final_group(const FinalParams* ps, const int* update_probe, int count, hipStream_t s);
hipError_t launch_metric_slices(const MetricParams& p, hipStream_t s);
hipError_t launch_swap(float2* a, float2* b, size_t count, hipStream_t s);
hipError_t launch_sp_batch(int n, const DivideParams& p, int count, hipStream_t s);
// the fused divide and the sequential-projection batch kernel per size (divide_n*.hip)
hipError_t launch_fused_n32(int fp16, const DivideParams& p, int n_patterns, hipStream_t s);
hipError_t launch_fused_n64(int fp16, const DivideParams& p, int n_patterns, hipStream_t s);
hipError_t launch_fused_n128(int fp16, const DivideParams& p, int n_patterns, hipStream_t s);
hipError_t launch_fused_group_n32(int fp16, const Group<DivideParams>& g, int blocks, hipStream_t s);
hipError_t launch_fused_group_n64(int fp16, const Group<DivideParams>& g, int blocks, hipStream_t s);
hipError_t launch_fused_group_n128(int fp16, const Group<DivideParams>& g, int blocks, hipStream_t s);
hipError_t launch_sp_n32(const DivideParams& p, int count, hipStream_t s);
hipError_t launch_sp_n64(const DivideParams& p, int count, hipStream_t s);
hipError_t launch_sp_n128(const DivideParams& p, int count, hipStream_t s);
hipError_t launch_sp_probe(const SpProbeParams& p, hipStream_t s);
// min over complex g of sum |t - g o|^2 / sum |t|^2 over the box [r0, r0+h) x [c0, c0+w)
// of o (row pitch ow) against t ([h][w]); part holds 4 blocks doubles (one set of
// float64 partial sums per work-group), the result lands in *result
hipError_t launch_object_error(const float2* o, int ow, const float2* t, int r0, int c0, int h, int w, double* part,
                               int blocks, double* result, hipStream_t s);
// work-groups of the object error: one per kErrPixelsPerBlock box pixels
constexpr long long kErrPixelsPerBlock = 16384;
inline int object_error_blocks(long long pixels) {
  return int(pixels < 1 ? 1 : (pixels + kErrPixelsPerBlock - 1) / kErrPixelsPerBlock);
}
// The allocation-free object error keeps its partial sums in a static device
// array of this many work-groups' sums (boxes of at most
// kErrScratchBlocks * kErrPixelsPerBlock = 4096^2 pixels).
constexpr int kErrScratchBlocks = 1024;
hipError_t object_error_static(const float2* o, int ow, const float2* t, int r0, int c0, int h, int w,
                               double* result, hipStream_t s);
hipError_t launch_amp_prepare(int n, const float* intensity, float* amp, int J, int* bad, hipStream_t s);
hipError_t launch_max_abs2_parts(const float2* a, size_t count, float* parts, int nparts, hipStream_t s);
hipError_t launch_convert_state(int fp16, int to_store, const float2* src, void* dst_store,
                                const void* src_store, float2* dst, size_t count, float scale,
                                float inv_scale, hipStream_t s);

// divide-kernel geometry helpers for the host
int divide_slots(int n);                 // metric slots per pattern
bool divide_supported(int n);

}  // namespace pty
