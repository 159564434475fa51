/*
 * ptyabc.h -- C ABI of the MI355X (gfx950) library for the generalised 'abc'
 * set-projection iteration of blind ptychography
 * (Mei & Maiden, "Set projection algorithms for blind ptychographic phase
 * retrieval").
 *
 * One call of pty_iterate(scan, n) runs n iterations of
 *
 *     x_{k+1} = a P^b_C P^c_D x_k + (1 - a) x_k                  (Introduction,
 *                                                    the generalised formula)
 *
 * over the product space of exit waves x = [x_0 .. x_{J-1}], one N x N wave
 * per scan position (the product-space construction of divide and concur),
 * with the relaxed projection P^a_S = a P_S + (1 - a) I (Introduction).
 *
 *   P_D  divide: per exit wave, F^-1 [ sqrt(I_j) F x_j / |F x_j| ]; where
 *        F x_j = 0 the phase is taken as 0.  F is the unnormalised 2-D DFT
 *        with the zero frequency at index [0][0] (no shift).
 *   P_C  concur: the least-squares consensus of the exit waves with one object
 *        O (H x W) and one probe P (N x N).  The flow of the 'abc' method forms
 *        exit waves from the current probe and object, projects, and updates
 *        both.  Object step: O = sum_j S_j^T(conj(P) y_j) / sum_j S_j^T |P|^2;
 *        then, when the probe is being reconstructed, probe step
 *        P = sum_j conj(S_j O) y_j / sum_j |S_j O|^2 with the new object.
 *        A pixel whose denominator is not above tau * max|P|^2 (object) or
 *        tau * max|O|^2 (probe) keeps its previous value.  Both sums are
 *        accumulated in float64 in a fixed order, so results are
 *        bit-reproducible.  P_C y is z_j = P S_j O.
 *
 * Data layout (all row-major, complex = interleaved (re, im) float32):
 *   object  [H][W] complex      probe [N][N] complex
 *   exit waves x, y [J][N][N] complex      intensities [J][N][N] float32
 *   positions [J][2] int32: (row, col) of the top-left corner of patch j,
 *             0 <= row <= H - N, 0 <= col <= W - N.
 *
 * Errors: every call returns a pty_status; no exception crosses the ABI.  An
 * invalid argument leaves the scan unchanged.  After PTY_ERR_DEVICE a scan
 * accepts only pty_destroy_scan.  pty_last_error() gives a thread-local
 * message for the last failing call on this thread.
 *
 * Concurrency: a scan must not be used from two threads at once; distinct
 * scans may be.  pty_iterate is asynchronous on the scan's stream; getters
 * synchronise that stream.
 */
#ifndef PTYABC_H
#define PTYABC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pty_scan pty_scan; /* opaque; created and destroyed by the library */

typedef enum {
  PTY_OK = 0,
  PTY_ERR_INVALID_ARG = 1,   /* bad pointer, size, value or range            */
  PTY_ERR_OUT_OF_MEMORY = 2, /* workspace too small                          */
  PTY_ERR_DEVICE = 3,        /* a HIP call failed; the scan is now unusable  */
  PTY_ERR_BAD_STATE = 4,     /* call not valid in the scan's current state   */
  PTY_ERR_DIVERGED = 5,      /* the last iteration's Fourier error is not finite
                                (or another metric is infinite)               */
  PTY_ERR_UNSUPPORTED = 6    /* valid request the library does not implement */
} pty_status;

typedef enum {
  PTY_STORE_FP32 = 0, /* exit waves x, y kept as complex float32              */
  PTY_STORE_FP16 = 1  /* kept as complex float16 times a power-of-two scale;
                         transforms and projections still run in float32 and
                         the overlap sums in float64.  The iterate x_k is its
                         stored (rounded) value wherever it is formed, so
                         pty_get_state / pty_set_state in between iterations
                         leave the results unchanged, as with float32       */
} pty_storage;

/* Named algorithms (Introduction lists them; the paper gives (1,1,1) for
 * divide and concur).  (a, b, c) used for each:
 *   DC (1,1,1)   AR (1,1,2)   DR (1/2,2,2)   SF (1,2,1)
 *   RAAR(beta) (1/2, 2 beta, 2)   RRR(beta) (beta/2, 2, 2)
 *   T_lambda (1/(1+lambda), 1+lambda, 1+lambda)                              */
typedef enum {
  PTY_DC = 0, PTY_AR = 1, PTY_DR = 2, PTY_SF = 3,
  PTY_RAAR = 4, PTY_RRR = 5, PTY_TLAMBDA = 6
} pty_algorithm;

typedef struct {
  int32_t n;                  /* N: 32, 64, 128 or 256                          */
  int32_t n_pos;              /* J >= 1                                          */
  int32_t obj_h, obj_w;       /* H, W >= N                                       */
  const int32_t *pos;         /* [J][2] (row, col), see above                    */
  const float *intensity;     /* [J][N][N], finite and >= 0, unshifted          */
  const float *init_object;   /* [H][W] complex                                  */
  const float *init_probe;    /* [N][N] complex                                  */
  int32_t inputs_on_device;   /* 0: the four arrays are host memory, 1: device   */
  int32_t storage;            /* pty_storage                                     */
  int32_t blind;              /* 0: probe known (never updated), 1: updated      */
  int32_t probe_update_start; /* blind: probe updated from this iteration on     */
  int32_t full_metrics;       /* 1: compute all three metrics every iteration
                                 (forces x and y to be kept even where (a,b,c)
                                 would not need them); 0: the Fourier error
                                 every iteration, the other two only where
                                 their inputs are read anyway (else NaN).
                                 With 0, N <= 64 and a != 1, b != 1 the
                                 library keeps w = (1-a) x + a(1-b) y in place
                                 of x between iterations (one read fewer per
                                 pixel); consistency and change are then NaN.
                                 pty_get_state still returns x.               */
  int32_t metric_capacity;    /* entries of the metric history ring; 0: 4096    */
  double tau;                 /* division guard; 0 selects 1e-10                 */
} pty_scan_desc;

/* Metrics of one iteration k (from x_k), the quantities behind the error
 * lines of the simulation figures (Figs. 7 and 8; the paper plots them
 * without a formula, so these definitions are this library's reading):
 *   fourier_err     sum (|F x_k| - sqrt(I))^2 / sum I
 *   consistency_err sum |z - y|^2 / sum |y|^2,  y = P^c_D x_k, z = P_C y
 *   change          ||x_{k+1} - x_k|| / ||x_k||
 * Sums run over all patterns and pixels, in float64.                        */
typedef struct {
  int64_t iteration;
  double fourier_err;
  double consistency_err;
  double change;
} pty_metrics;

/* Exact device-workspace size for desc, in bytes; 0 if desc is invalid. */
size_t pty_workspace_bytes(const pty_scan_desc *desc);

/* Create a scan.  d_workspace: device memory of at least
 * pty_workspace_bytes(desc) bytes, 256-byte aligned, owned by the caller, kept
 * alive and unmoved until pty_destroy_scan.  stream: a hipStream_t (NULL: the
 * default stream) on which all of the scan's work is queued.  The input arrays
 * are copied; the caller may free them on return.  The first iteration starts
 * from x_0 = P_0 S_j O_0 (the flow's first step). */
pty_status pty_create_scan(const pty_scan_desc *desc, void *d_workspace, size_t ws_bytes,
                           void *stream, pty_scan **out);

/* Select (a, b, c) for subsequent iterations.  All three must be finite and a
 * must be nonzero; any other values (under- or over-relaxation) are allowed. */
pty_status pty_set_algorithm(pty_scan *scan, double a, double b, double c);

/* Select a named algorithm; param is beta (RAAR, RRR) or lambda (T_lambda)
 * and is ignored otherwise. */
pty_status pty_set_algorithm_named(pty_scan *scan, int32_t algorithm, double param);

/* (a, b, c) of a named algorithm (the table above; param is beta or lambda),
 * written to abc[0..2].  PTY_ERR_INVALID_ARG for an unknown algorithm, a
 * non-finite param or abc == NULL.  Needs no scan and no device. */
pty_status pty_algorithm_abc(int32_t algorithm, double param, double *abc);

/* Which exit-wave state the scan's next iteration keeps between iterations
 * with its current (a, b, c) and metric setting: 0 the iterate x (52 bytes
 * per pattern pixel in the blind float32 form), 1 the blend
 * w = (1-a) x + a(1-b) y (44 bytes; only without full_metrics, for N <= 64,
 * and when 1-a and a(1-b) are both nonzero in float32).  -1 for NULL. */
int32_t pty_state_form(const pty_scan *scan);

/* Queue n >= 0 iterations on the scan's stream and return. */
pty_status pty_iterate(pty_scan *scan, int32_t n);

/* Queue n iterations of each of count scans.  The scans' kernels are launched
 * interleaved, iteration by iteration, so that scans on different streams
 * overlap on the device.  Each scan's result is identical to pty_iterate on
 * it alone. */
pty_status pty_iterate_many(pty_scan *const *scans, int32_t count, int32_t n);

/* Iteration-dependent relaxation (Introduction: the relaxation of a
 * projection may change as the iteration proceeds).  Runs n iterations,
 * iteration i with (a, b, c) = (abc[3i], abc[3i+1], abc[3i+2]); abc is a host
 * array of 3n doubles.  Every entry is checked (finite, a != 0) before any
 * work is queued: PTY_ERR_INVALID_ARG leaves the scan unchanged.  The last
 * entry stays the scan's (a, b, c) afterwards.  Asynchronous like
 * pty_iterate. */
pty_status pty_iterate_schedule(pty_scan *scan, const double *abc, int32_t n);

/* Number of (object, probe) sweeps of the concur step per iteration (1 to
 * 64; default 1).  The blind concur is a least-squares consensus over two
 * bilinear factors; with K sweeps the object step (from the current probe)
 * and the probe step (from the new object) are repeated K times on the same
 * divided exit waves, each sweep starting from the previous one.  Without
 * probe updates one object step is exact and K is ignored. */
pty_status pty_set_concur_sweeps(pty_scan *scan, int32_t sweeps);

/* Shadow estimate P_C(P_D x_k) of the current iterate: the unrelaxed divide
 * of x_k followed by the consensus (with the scan's sweeps, the probe updated
 * as in the next iteration would update it), warm started from the scan's
 * (O, P).  At a fixed point of the Douglas-Rachford family the solution is
 * P_D x*, so this is the estimate to report there (Conclusion's comparison of
 * those algorithms).  obj_out ([H][W] complex) and probe_out ([N][N]
 * complex) are device buffers; results are there once the scan's stream
 * reaches this point.  The scan's x, object, probe, iteration count and
 * metrics are unchanged; x is materialised first, and the exit-wave buffer
 * pty_get_state returns as y then holds P_D x_k. */
pty_status pty_shadow(pty_scan *scan, float *obj_out, float *probe_out);

/* One iteration of sequential projections (Introduction: the constraint sets
 * visited one after another, in a fixed or shuffled order, with relaxed
 * projections), for every supported N (N = 256 runs each batch as the three
 * passes of the divide: rows forward, columns with the modulus projection,
 * rows inverse with the step).  The sets are
 * the per-position modulus sets; the step onto set j, with psi = P S_j O,
 * psi' its Fourier-modulus projection and d = psi' - psi, is
 *   O <- O + alpha S_j^T[conj(P) d] / max|P|^2
 *   P <- P + beta conj(S_j O) d / max|S_j O|^2      (probe updated: blind and
 *                                                     iteration >= probe_update_start)
 * taken at the (O, P) of the start of the position's batch.  Batches: the
 * positions of `order` (host array, a permutation of 0..J-1; NULL: ascending)
 * are placed by dependency level into batches of pairwise disjoint windows,
 * each overlapping pair keeping its order; max_batch > 0 caps a batch's size
 * (1: strictly sequential).  A batch's object steps touch disjoint pixels; its
 * probe steps are summed in batch order after it.  With a known probe every
 * batch schedule equals the sequential order.  The Fourier error of the exit
 * waves visited goes to the metric history (the other two metrics are NaN).
 * The generalised iteration's exit waves are discarded: a following
 * pty_iterate starts again from x = P S_j O.  A batch sums its probe steps,
 * so a batch of m windows moves the probe by up to m single steps: with
 * batched orders beta of about 1 / (mean batch size) keeps the probe update
 * stable (beta = 1 with batches of tens of windows diverges, in the FP64
 * reference too); beta = 1 suits max_batch = 1. */
pty_status pty_sp_iterate(pty_scan *scan, const int32_t *order, int32_t max_batch, double alpha, double beta);

/* Number of batches of the last pty_sp_iterate call (-1 for NULL). */
int32_t pty_sp_last_batches(const pty_scan *scan);

/* Object error against a ground truth with the global complex scale removed
 * (the object is determined only up to one complex factor in blind
 * ptychography; the paper's error lines of Figs. 7-8 are measured inside a
 * box of the object, Fig. 5): min over complex g of
 *   sum |t - g O|^2 / sum |t|^2
 * over the box rows [r0, r0+h), columns [c0, c0+w) of the scan's current
 * object.  truth: device buffer, [h][w] complex, row-major.  Sums in
 * float64 in a fixed order.  Synchronises the scan's stream; *err is NaN for
 * an all-zero truth and 1 for an all-zero object. */
pty_status pty_object_error(pty_scan *scan, const float *truth, int32_t r0, int32_t c0, int32_t h, int32_t w,
                            double *err);

/* The object error above without a scan, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops that forbid
 * allocation): min over complex g of sum |t - g o|^2 / sum |t|^2 over the box
 * rows [r0, r0+h), columns [c0, c0+w) of obj ([obj_h][obj_w] complex,
 * row-major, device memory) against truth ([h][w] complex, device memory).
 * The result (NaN for an all-zero truth, 1 for an all-zero object box) is
 * written to err, a device double, asynchronously on stream (a hipStream_t;
 * NULL: the default stream); nothing is synchronised.  The float64 partial
 * sums live in a static device array of the library (32 KiB per GPU, kept
 * until the process ends), not in allocated memory: the box may hold at most
 * 16777216 (4096^2) pixels, larger boxes are rejected with
 * PTY_ERR_INVALID_ARG before any device work.  All calls on one GPU share that
 * array, so calls that overlap on one GPU (other streams, other threads)
 * race.  Same kernels and summation order as pty_object_error, so the two
 * give bitwise-equal results.  Calls no allocating routine. */
pty_status pty_object_error_noalloc(const float *obj, int32_t obj_h, int32_t obj_w, const float *truth,
                                    int32_t r0, int32_t c0, int32_t h, int32_t w, double *err, void *stream);

/* Wait for all queued work of the scan. */
pty_status pty_synchronize(pty_scan *scan);

/* Copy the current object O ([H][W] complex, 2*H*W floats) or probe P
 * ([N][N] complex, 2*N*N floats) into dst (host or device memory): the pair
 * that the last concur step P_C formed (Introduction, the flow of the 'abc'
 * method), or the initial pair before the first iteration.  n_floats is
 * dst's capacity in floats; PTY_ERR_INVALID_ARG if it is too small.
 * Synchronises the scan's stream.  The object and probe hold the values of
 * a completed iteration only: a pending x update of the last step does not
 * change them. */
pty_status pty_get_object(pty_scan *scan, float *dst, size_t n_floats, int32_t dst_on_device);
pty_status pty_get_probe(pty_scan *scan, float *dst, size_t n_floats, int32_t dst_on_device);

/* Metrics of the last completed iteration (the error-line quantities
 * defined at pty_metrics).  PTY_ERR_BAD_STATE before the
 * first iteration; PTY_ERR_DIVERGED (with *out filled) if the Fourier error is
 * not finite or another metric is infinite.  A NaN consistency or change
 * error marks a metric that iteration did not form (blend form, sequential
 * projections), not divergence. */
pty_status pty_get_metrics(pty_scan *scan, pty_metrics *out);

/* Up to cap most recent entries, oldest first; *n_out receives the count. */
pty_status pty_get_metric_history(pty_scan *scan, pty_metrics *dst, int32_t cap, int32_t *n_out);

/* Number of completed iterations. */
int64_t pty_get_iteration(const pty_scan *scan);

/* Read the state: x = x_k (the iterate the next iteration starts from),
 * y = P^c_D x_{k-1} of the last iteration, object, probe.  Each pointer may be
 * NULL to skip it; sizes are those of the layout above (complex float32,
 * also under FP16 storage). */
pty_status pty_get_state(pty_scan *scan, float *x, float *y, float *obj, float *probe,
                         int32_t on_device);

/* Replace the state (checkpoint restore, parity tests).  x must be given; y
 * may be NULL (then it is zeroed); obj and probe may be NULL to keep the
 * current ones.  The iteration counter is left unchanged. */
pty_status pty_set_state(pty_scan *scan, const float *x, const float *y, const float *obj,
                         const float *probe, int32_t on_device);

/* Release the scan (not the caller's workspace).  NULL is a no-op. */
void pty_destroy_scan(pty_scan *scan);

/* Kernel classes for the per-kernel timing below. */
typedef enum {
  PTY_K_DIVIDE = 0,          /* divide, fused (N <= 128) or row forward pass (N = 256) */
  PTY_K_DIVIDE_COLS = 1,     /* N = 256: column pass with the Fourier-space projection  */
  PTY_K_DIVIDE_ROWS_INV = 2, /* N = 256: row inverse pass                                */
  PTY_K_OBJECT = 3,          /* concur, object (and the sums of metric slices)           */
  PTY_K_PROBE = 4,           /* concur, probe partial sums                               */
  PTY_K_FINAL = 5,           /* probe finalisation and the metric history entry          */
  PTY_K_COUNT = 6
} pty_kernel_class;

/* Per-kernel timing with HIP events recorded on the scan's stream around the
 * launches of pty_iterate / pty_iterate_many (and the other iterating calls).
 * enable = m > 0 starts timing and clears the totals: the launches of every
 * m-th iteration (iteration count divisible by m) are timed, so m = 1 times
 * every launch; 0 stops it.  Timing adds two event records per timed launch
 * and nothing else; each pair costs a few microseconds of device time, which
 * sampling (m > 1) spreads thin. */
pty_status pty_profile(pty_scan *scan, int32_t enable);

/* Synchronise, then give per class the total milliseconds and the number of
 * launches timed since timing was last started (pty_profile with m > 0).  ms and launches hold n entries;
 * n may be smaller than PTY_K_COUNT. */
pty_status pty_profile_read(pty_scan *scan, double *ms, int64_t *launches, int32_t n);

const char *pty_status_string(int32_t status);
const char *pty_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PTYABC_H */
