/*
 * pftpie.h -- C ABI of the MI355X (gfx950) batched 2-D partial Fourier
 * transform and the PIE sweep built on it.
 *
 * Method: Parada, Wu Fung, Osher, "Fast Partial Fourier Transforms for
 * Large-Scale Ptychography" (arXiv 2408.03532).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Complex data are interleaved complex64: {float re, float im}, the memory
 *    of torch.complex64.  Arrays are dense, row-major (C order).
 *  - Window: a transform of an n x n patch keeps m coefficients per axis,
 *    the frequencies t_c = c - floor(m/2), c = 0..m-1, stored in that
 *    centred order, row-major [c1][c2] (axis 0 = rows).  This is the centred
 *    m x m crop of an fftshift-ed 2-D DFT (the paper's Fig. 2 and the data
 *    cropping of Algorithm 3).  Spatial indices run 0..n-1 from the patch's
 *    top-left corner.
 *  - Pointers named *_dev / data pointers are device pointers; host_* are
 *    host pointers.  The caller owns every data buffer and workspace; the
 *    library owns plans and scans (device twiddle tables, positions).
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL = the default stream) and never synchronises with the host except
 *    plan / scan creation and destruction.  No call other than plan / scan
 *    creation allocates device memory.
 *  - Errors: arguments are validated on the host before anything is
 *    enqueued; a non-OK status means nothing was enqueued and no output was
 *    touched.  pftpie_last_error() gives a thread-local message for the last
 *    failure.  A device fault surfaces as PFTPIE_E_DEVICE from a later call
 *    or at the caller's synchronisation.  Nothing throws across the ABI.
 *  - Plans and scans are immutable after creation and may be shared between
 *    streams; workspaces may not.  Plans and scans belong to the device that
 *    was current when they were created.
 */
#ifndef PFTPIE_H
#define PFTPIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PFTPIE_OK = 0,
  PFTPIE_E_INVALID = 1,      /* bad argument: shape, pointer, range, alias */
  PFTPIE_E_UNSUPPORTED = 2,  /* valid request this build does not implement */
  PFTPIE_E_NOMEM = 3,        /* device or host allocation failed (creation) */
  PFTPIE_E_DEVICE = 4        /* HIP runtime error */
} pftpie_status;

/* Arithmetic of the contractions.  FP32: float operands and accumulation.
 * SPLIT_BF16 / SPLIT_FP16: each operand x is split into hi = RNE(x) and
 * lo = RNE(x - hi) in the 16-bit type; products are hi*hi + hi*lo + lo*hi,
 * accumulated in float.  Twiddles are generated in double in every mode. */
typedef enum {
  PFTPIE_FP32 = 0,
  PFTPIE_SPLIT_BF16 = 1,
  PFTPIE_SPLIT_FP16 = 2
} pftpie_precision;

/* How a plan computes its transform.  DENSE: the contraction F_m psi F_m^T
 * on matrix cores, in the plan's precision.  FFT: for the full window
 * m = n in {16, 32, 64, 128} only (the second, full-resolution phase of the
 * hybrid method, Algorithm 3, Sec. 3.2), a fast 2-D transform held in LDS,
 * in FP32 whatever the plan's precision; results are the same transform
 * (centred window order) to float rounding.  AUTO: FFT where it applies,
 * otherwise DENSE. */
typedef enum {
  PFTPIE_METHOD_AUTO = 0,
  PFTPIE_METHOD_DENSE = 1,
  PFTPIE_METHOD_FFT = 2
} pftpie_method;

typedef struct pftpie_plan_s* pftpie_plan;
typedef struct pftpie_poly_s* pftpie_poly;
typedef struct pie_scan_s* pie_scan;

const char* pftpie_status_string(pftpie_status s);
const char* pftpie_last_error(void);

/* ------------------------------------------------------------------------ */
/* Partial transform of n x n patches to their m x m low-frequency window.
 * The exact DFT restricted to the window (Appendix A, 2-D DFT; Sec. 3.1.1,
 * 1-D DFT): the quantity the paper's PFT approximates (Sec. 3.1, Fig. 2).
 *
 * pftpie_plan_create: 1 <= m <= n <= 8192.  Builds the partial DFT matrix
 *   F_m[c][k] = exp(-2 pi i ((t_c k) mod n) / n) in double (integer
 *   reduction of the phase first), rounds it to the plan's precision and
 *   uploads it in the kernels' tile order.  Allocates device memory on the
 *   current device; synchronous.  *out is NULL on failure. */
pftpie_status pftpie_plan_create(int32_t n, int32_t m, pftpie_precision prec,
                                 pftpie_plan* out);
/* As pftpie_plan_create with an explicit method (pftpie_plan_create uses
 * AUTO).  FFT for sizes it does not cover returns PFTPIE_E_UNSUPPORTED; an
 * unknown method value returns PFTPIE_E_INVALID.  The method applies to
 * pft2d_forward / pft2d_adjoint and to pie_sweep over scans of this plan;
 * uneven batches (pftpie_group_*) always use the dense contraction. */
pftpie_status pftpie_plan_create_method(int32_t n, int32_t m, pftpie_precision prec,
                                        pftpie_method method, pftpie_plan* out);
/* The method a plan resolved to (DENSE or FFT). */
pftpie_status pftpie_plan_method(pftpie_plan plan, pftpie_method* method);
/* Masked larger field (Sec. 4.1.3: an n x n illuminated window inside a
 * period x period field, every other pixel zero): the plan's transform uses
 * DFT length `period` (n <= period <= 2^20),
 *   F_m[c][k] = exp(-2 pi i ((t_c k) mod period) / period),  k < n,
 * so pft2d_forward returns the kept coefficients of the whole field for a
 * window at the field's origin.  A window whose corner sits at (s1, s2)
 * has them times exp(-2 pi i ((t_c1 s1 + t_c2 s2) mod period) / period)
 * (shift theorem); the caller applies that phase where it needs the
 * field's coefficients themselves.  pie_sweep and the amplitude loss use
 * magnitudes only and need no phase (the adjoint of the phase cancels it);
 * pie_sweep normalises its correction by 1/period^2 (the inverse
 * period-point DFT of the band change) and Phi by J period^2.  The FFT
 * method needs period == n.  pftpie_plan_create is period = n. */
pftpie_status pftpie_plan_create_period(int32_t n, int32_t m, int32_t period, pftpie_precision prec,
                                        pftpie_method method, pftpie_plan* out);
pftpie_status pftpie_plan_period(pftpie_plan plan, int32_t* period);
pftpie_status pftpie_plan_destroy(pftpie_plan plan);
/* Query a plan's sizes and precision (any output pointer may be NULL). */
pftpie_status pftpie_plan_info(pftpie_plan plan, int32_t* n, int32_t* m,
                               pftpie_precision* prec);

/* Autotuner: times the plan's candidate launch choices on a scratch batch of
 * `sample` patches filled with random values (uniform in [-1, 1)) and keeps
 * the fastest: forward column tiles per wave and an LDS-resident or
 * L2-resident twiddle table; adjoint LDS or L2 table, a whole patch or one
 * column tile per wave, and (FP32) row tiles per step and workgroup size.
 * Allocates and frees scratch memory and synchronises the device; call it
 * before the plan is used from other threads or streams (it changes the
 * plan's launch choices, never its results' definition).  best_ms (may be
 * NULL) receives the best forward + adjoint time per call in milliseconds.
 * The environment variable PFTPIE_TUNE_CACHE names a text file in which
 * results are looked up and recorded (keyed by device name, n, m and
 * precision).  The candidates are those of the dense contraction (which
 * uneven batches use for every plan); best_ms times the dense form. */
pftpie_status pftpie_plan_autotune(pftpie_plan plan, int64_t sample, double* best_ms);

/* ------------------------------------------------------------------------ */
/* The paper's polynomial PFT (Sec. 3.1, Algorithms 1-2; Appendix A,
 * Algorithms 4-5), kept beside the exact transform for comparison of error
 * and speed.  With n = p q, each q x q block of the window is contracted
 * with B[j][l] = w_l (1 - 2j/q)^l on both axes, the p x p grid of each
 * (l1, l2) plane is transformed (fast transform in LDS), and the kept
 * coefficients t_c = c - floor(m/2) are the sums over (l1, l2) of the
 * planes at (t1 mod p, t2 mod p) weighted by W[t][l] = (t/p)^l
 * exp(-pi i t / p) per axis.  w: the interpolant of exp(i pi x) at the r
 * Chebyshev points of [-xi, xi], xi(eps, r) the largest scope within eps
 * (bisection in double), r the least with xi(eps, r) >= floor(m/2) / p
 * (Algorithm 1); each coefficient is within (2 eps + eps^2) * sum |psi| of
 * the exact one (plus FP32 rounding).
 *
 * pftpie_poly_create: p in {16, 32, 64, 128}, p | n, n / p <= 32,
 *   1 <= m <= min(n, 128), 0 < eps < 1; PFTPIE_E_UNSUPPORTED when no
 *   r <= 25 reaches eps.  Synchronous; allocates device tables.
 * pftpie_poly_info: the chosen r and xi (either pointer may be NULL).
 * pftpie_poly_workspace_size: bytes of device workspace for `batch`
 *   patches (2 batch r^2 p^2 complex64: the expanded and transformed
 *   planes); the caller owns it.
 * pft2d_poly_forward: psi device complex64 [batch][n][n] -> y [batch][m][m]
 *   (centred order, as pft2d_forward); psi, y and ws 8-byte aligned, psi
 *   and y disjoint; enqueued on `stream`. */
pftpie_status pftpie_poly_create(int32_t n, int32_t m, int32_t p, double eps, pftpie_poly* out);
pftpie_status pftpie_poly_destroy(pftpie_poly poly);
pftpie_status pftpie_poly_info(pftpie_poly poly, int32_t* r, double* xi);
pftpie_status pftpie_poly_workspace_size(pftpie_poly poly, int64_t batch, size_t* bytes);
pftpie_status pft2d_poly_forward(pftpie_poly poly, const void* psi, void* y, int64_t batch, void* ws,
                                 size_t ws_bytes, void* stream);

/* Forward: y_b = F_m psi_b F_m^T for b < batch.
 *   psi: device complex64 [batch][n][n]; y: device complex64 [batch][m][m].
 *   batch >= 0 (0 enqueues nothing).  psi and y must not overlap and must be
 *   8-byte aligned (16-byte alignment enables the vector-load path). */
pftpie_status pft2d_forward(pftpie_plan plan, const void* psi, void* y,
                            int64_t batch, void* stream);

/* Adjoint: psi_b = F_m^H y_b conj(F_m) (no 1/n^2 factor), the exact adjoint
 * of pft2d_forward, so <F x, y> = <x, F^H y>, and F_m F_m^H = n^2 I.
 *   y: device complex64 [batch][m][m]; psi: device complex64 [batch][n][n]. */
pftpie_status pft2d_adjoint(pftpie_plan plan, const void* y, void* psi,
                            int64_t batch, void* stream);

/* ------------------------------------------------------------------------ */
/* Uneven batch: many patches of different sizes in one persistent launch
 * (the partial transform of each patch, Sec. 3.1 / Appendix A, with the
 * per-axis window sizes left free as the paper leaves them).
 * Descriptor i: patch side n, window m, and element offsets (complex
 * elements) of its input and output inside the packed `in` / `out` arrays.
 * Forward: in holds n*n, out holds m*m elements per descriptor; adjoint the
 * reverse.  At most 8 distinct (n, m) classes; output blocks must not
 * overlap.  Work items (column-tile groups of a patch) are ordered longest
 * first and pulled by the waves of one persistent kernel from a device
 * counter; every wave leaves once the counter passes the item count.
 *
 * Two forms share that kernel.
 *
 * Per call, over host descriptors and a caller workspace:
 * pft2d_grouped_workspace_size: bytes of workspace for these descriptors
 *   (an upper bound valid for any launch choices of the plans).
 * pft2d_forward_grouped / pft2d_adjoint_grouped: the transforms of every
 *   descriptor.  Each (n, m) present needs a live plan of precision `prec`
 *   (and DFT length n) created on the current device, whose twiddle tables
 *   are used; a missing one is PFTPIE_E_INVALID.  in / out: device
 *   complex64 packed arrays, 16-byte aligned, disjoint; their extents are
 *   those the descriptors reach.  workspace: device memory, 256-byte
 *   aligned, at least pft2d_grouped_workspace_size bytes, disjoint from the
 *   data (it receives the work list and the counter).  The descriptors are
 *   validated and the work list built on the host, then copied to the
 *   workspace on `stream` (the copy takes the host data before the call
 *   returns); nothing is allocated.  A workspace must not be shared by
 *   calls that may run at the same time.
 *
 * Group object, for repeated runs of one descriptor set:
 * pftpie_group_create: validates the descriptors (sizes in range, blocks
 *   inside the packed arrays of in_len / out_len complex elements, outputs
 *   disjoint), uploads the work list and instantiates a hipGraph (a counter
 *   reset node, then the persistent kernel node).  Synchronous, allocates.
 * pft2d_group_run: replays that graph on `stream` (its buffers are updated
 *   when in / out differ from the previous run's); allocates nothing. */
typedef struct {
  int32_t n, m;
  int64_t in_offset, out_offset;
} pft2d_desc;
typedef struct pft2d_group_s* pft2d_group;

pftpie_status pft2d_grouped_workspace_size(const pft2d_desc* host_desc, int64_t count, int32_t adjoint,
                                           size_t* bytes);
pftpie_status pft2d_forward_grouped(const pft2d_desc* host_desc, int64_t count, const void* in, void* out,
                                    pftpie_precision prec, void* workspace, size_t ws_bytes, void* stream);
pftpie_status pft2d_adjoint_grouped(const pft2d_desc* host_desc, int64_t count, const void* in, void* out,
                                    pftpie_precision prec, void* workspace, size_t ws_bytes, void* stream);

pftpie_status pftpie_group_create(const pftpie_plan* plans, int32_t nplans,
                                  const pft2d_desc* host_desc, int64_t count,
                                  int64_t in_len, int64_t out_len, int32_t adjoint,
                                  pft2d_group* out);
pftpie_status pftpie_group_destroy(pft2d_group group);
/* Run the whole uneven batch (all plans share one precision).  in / out:
 * device complex64 packed arrays. */
pftpie_status pft2d_group_run(pft2d_group group, const void* in, void* out, void* stream);
/* Autotuner of the group's own launch choices, timed on its real
 * descriptor mix with random inputs (uniform in [-1, 1)): per (n, m) class,
 * largest work first, the forward column tiles per wave (1 or 2) or the
 * adjoint column tiles per work item (1, 2, 4 or 8), then the workgroups
 * per compute unit (1..4); each choice is kept when it lowers the batch
 * time.  Rebuilds the work list and the graph with the result; allocates
 * and frees scratch and synchronises the device.  best_ms (may be NULL):
 * the best batch time.  Results keep their definition (only the order of
 * float sums changes). */
pftpie_status pftpie_group_autotune(pft2d_group group, double* best_ms);

/* ------------------------------------------------------------------------ */
/* PIE / ePIE sweep (Sec. 2.1: projection eq. (3), objective eq. (4), object
 * and probe iterates eqs. (5)-(6); data cropping of Algorithm 3).
 *
 * pie_scan_create: positions host_pos int32 [J][2] = top-left (row, col) of
 *   each n x n window inside an H x W object; 0 <= row <= H-n and
 *   0 <= col <= W-n are required (no wrap-around).  Uploads the positions.
 *   The plan (its n, m, precision) is referenced, not copied: keep it alive. */
pftpie_status pie_scan_create(pftpie_plan plan, const int32_t* host_pos, int32_t J,
                              int32_t H, int32_t W, pie_scan* out);
pftpie_status pie_scan_destroy(pie_scan scan);

typedef struct {
  int32_t batch;  /* positions per accumulate-and-apply chunk: 1 = the
                     sequential iterate of eq. (5); J = fully batched */
  int32_t norm;   /* 0: O += beta * sum conj(P) dpsi (eq. (5));
                     1: divided by sum |P|^2 + alpha * max (overlap-normalised) */
  float beta;     /* object step */
  float gamma;    /* probe step; 0 = probe fixed (non-blind PIE) */
  float alpha;    /* denominator regulariser relative to the max (norm == 1) */
  int32_t probe_update; /* probe step of eq. (6), gamma > 0: 0 = evaluated with
                     the object and residual of the object step; 1 = as
                     printed, at the updated object with the exit wave and
                     projection formed again (a second transform pair per
                     position; needs batch == 1 and norm == 0) */
} pie_params;

/* Bytes of device workspace pie_sweep needs for these parameters. */
pftpie_status pie_workspace_size(pie_scan scan, const pie_params* p, size_t* bytes);

/* One sweep over all J positions, in chunks of p->batch of the order
 * order_dev (device int32 [J]: a permutation of [0, J), or NULL for scan
 * order).  An entry outside [0, J) names no position: it keeps its place in
 * its chunk and contributes nothing.  A position listed more than once is
 * not supported (the result is then unspecified; the device holds the
 * order, so the host cannot check it).
 * For each position j of a chunk, against the object and probe as they
 * were at the chunk start:
 *   psi = P * O[window j];  u = F_m psi F_m^T;
 *   u' = amp_j * u / |u|  (amp_j where u == 0);
 *   dpsi = F_m^H (u' - u) conj(F_m) / n^2     (pseudo-inverse correction);
 * then O += beta * sum_j conj(P) dpsi (norm 0) or that sum divided by
 * sum_j |P|^2 + alpha max (norm 1); with gamma > 0 likewise
 * P += gamma * sum_j conj(O_j) dpsi (divided by sum |O_j|^2 + alpha max).
 *   object: device complex64 [H][W], updated in place.
 *   probe:  device complex64 [n][n], updated in place when gamma > 0.
 *   amp:    device float32 [J][m][m], the square roots of the centred m x m
 *           crop of the measured intensities (indexed by position j).
 *   stats_dev: device double[4] or NULL, written with
 *           {Phi, ||O_after - O_before||^2, ||O_before||^2, n_nonfinite},
 *           Phi = sum_j sum (|u_j| - amp_j)^2 / (J n^2) (eq. (4)).
 *   workspace: device memory of at least pie_workspace_size bytes,
 *           256-byte aligned. */
pftpie_status pie_sweep(pie_scan scan, void* object, void* probe, const float* amp,
                        const int32_t* order_dev, const pie_params* p,
                        void* workspace, size_t ws_bytes, double* stats_dev,
                        void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sweep
 * of pie_sweep with the library's own fixed device scratch in place of the
 * caller's workspace.  Same arguments, semantics and results as pie_sweep
 * (the same kernels run); no call allocates.  The scratch is a static
 * device array of PFTPIE_NOALLOC_SCRATCH_MIB MiB that every GPU the library
 * runs on holds until the process ends; its address is looked up once per
 * device on the first call there.  A sweep whose pie_workspace_size exceeds
 * it returns PFTPIE_E_INVALID (use a smaller batch, or pie_sweep).  Every
 * call on one GPU shares that GPU's scratch: calls that may overlap in time
 * on one GPU (different streams, threads) race and must not be issued;
 * calls in one stream are ordered and safe.  The scratch keeps the last
 * call's contents; each sweep clears what it needs itself. */
#define PFTPIE_NOALLOC_SCRATCH_MIB 160
pftpie_status pie_sweep_noalloc(pie_scan scan, void* object, void* probe, const float* amp,
                                const int32_t* order_dev, const pie_params* p, double* stats_dev,
                                void* stream);

/* Data cropping of Algorithm 3 (Sec. 3.2): amp[j] = sqrt(centred m x m crop
 * of intensity[j]).  intensity: device float32 [J][n][n] in fftshift layout
 * (zero frequency at (floor(n/2), floor(n/2))), non-negative; amp: device
 * float32 [J][m][m], the layout pie_sweep and the loss calls take.  Rows and
 * columns floor(n/2) - floor(m/2) .. + m - 1 are kept.  1 <= m <= n. */
pftpie_status pie_crop_amplitudes(const float* intensity, int32_t J, int32_t n, int32_t m,
                                  float* amp, void* stream);

/* ------------------------------------------------------------------------ */
/* Amplitude loss L = sum_j || |F_m (P * O_j) F_m^T| - amp_j ||^2 and its
 * gradient (the derivative through the partial transform that the paper's
 * gradient view of PIE needs, Sec. 1.1 and the remark after eq. (6)).
 * Gradients use grad = dL/dRe + i dL/dIm; the subgradient of |u| at 0 is 0.
 *
 * amp_loss_forward: loss_dev device double[1] receives L.  saved_u: device
 *   complex64 [J][m][m] receiving u_j, or NULL.
 * amp_loss_backward: grad_object device complex64 [H][W] (overwritten with
 *   scale * dL/dO), grad_probe device complex64 [n][n] (overwritten with
 *   scale * dL/dP) or NULL, where scale = *grad_scale_dev (device double) or
 *   1 when grad_scale_dev is NULL.  saved_u: the u_j written by
 *   amp_loss_forward, or NULL to recompute them (one more forward
 *   transform).  The exit waves themselves are never stored; the workspace
 *   (amp_loss_workspace_size, 256-byte aligned) holds the back-projected
 *   residuals R_j [J][n][n] that the object and probe gradients are gathered
 *   from (no atomics, deterministic summation order). */
pftpie_status amp_loss_workspace_size(pie_scan scan, size_t* bytes);
pftpie_status amp_loss_forward(pie_scan scan, const void* object, const void* probe,
                               const float* amp, double* loss_dev, void* saved_u,
                               void* workspace, size_t ws_bytes, void* stream);
pftpie_status amp_loss_backward(pie_scan scan, const void* object, const void* probe,
                                const float* amp, const void* saved_u, const double* grad_scale_dev,
                                void* grad_object, void* grad_probe,
                                void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Measurement aid (not part of the method): the matrix-core rate the device
 * delivers, in TFLOP/s, from a loop of independent MFMA products on random
 * register operands over 8 waves per SIMD (v_mfma_f32_16x16x4_f32 for
 * FP32, v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation), so that
 * roofline fractions can be given against measured as well as published
 * peaks.  Synchronous; allocates and frees a small output buffer; runs on
 * the current device. */
pftpie_status pftpie_measure_mfma_peaks(double* fp32_tflops, double* bf16_tflops, double* fp16_tflops);

#ifdef __cplusplus
}
#endif

#endif /* PFTPIE_H */
