/*
 * sgwls.h -- C ABI of the MI355X (gfx950) SG-WLS filtering library.
 *
 * Semi-Global Weighted Least Squares (SG-WLS): W. Liu, X. Chen, C. Shen,
 * Z. Liu, J. Yang, "Semi-Global Weighted Least Squares in Image Filtering",
 * ICCV 2017, arXiv 1705.01674.
 *
 * The filter approximates the weighted-least-squares smoothing of Eq. (1),
 * min_U sum (U-F)^2 + lambda sum w_ij (U_i-U_j)^2 with guidance weights of
 * Eq. (2), by many one-dimensional WLS subsystems (Sec. 2.1-2.3):
 *   - for every strip of 2r+1 columns centred at k = r, r+tau, ... (and the
 *     last centre N-1-r), the strip's rows are concatenated head to end with
 *     every second row reversed (Sec. 2.1), giving a vector of s = (2r+1)M
 *     pixels;
 *   - its subsystem A_s u = f (Eq. 5), A_s = I + lambda*L over pairs at most r
 *     apart on the vector, weights of Eq. (2) with |i-j| the distance along
 *     the vector, is solved exactly (Sec. 2.2; the library uses an exact
 *     partitioned banded LDL^T, not the paper's r-band LU);
 *   - solutions are scattered back and pixels covered by several strips are
 *     averaged with equal weights (Sec. 2.3);
 *   - a column pass and then a row pass (the same on the transposed image)
 *     make one iteration; T iterations are run (Sec. 2.3).
 *
 * Conventions for every entry point:
 *   - images are planar C x M x N float32, contiguous, row-major (CHW); a
 *     batch of such images is N C H W.  The guidance g is one M x N float32
 *     plane shared by all C channels.
 *   - every image, workspace and gradient pointer is a DEVICE pointer owned
 *     by the caller.  Parameter structs and image tables are HOST memory.
 *     The library allocates no device memory in any entry point.
 *   - `stream` is a hipStream_t passed as an opaque pointer (NULL = the
 *     default stream).  Work is enqueued asynchronously on it; results are
 *     ready when the stream is synchronised.
 *   - all arguments are validated on the host before anything is enqueued;
 *     on any error nothing is enqueued and outputs are untouched.  HIP launch
 *     errors are reported as SGWLS_E_HIP.  No entry point aborts or exits.
 *   - lambda_dev (where accepted) is a device float that overrides p->lambda
 *     without a host synchronisation.  The kernels clamp a negative device
 *     lambda to 0 (A_s = I + lambda L is only positive definite for
 *     lambda >= 0); a NaN device lambda propagates to every output.
 *   - NaN or Inf in f propagate to the outputs of the strips that read them;
 *     NaN or Inf in g make the affected weights NaN (not trapped).  Guidance
 *     values must stay below 1e28 in magnitude: the kernels pad the image
 *     with a guidance of 1e30 and give every edge whose guidance difference
 *     reaches 1e29 a weight of 0.
 */
#ifndef SGWLS_H
#define SGWLS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGWLS_OK = 0,
  SGWLS_E_ARG = 1,          /* a parameter is out of range, or a required pointer is NULL */
  SGWLS_E_SHAPE = 2,        /* C < 1, M or N < 2r+1 or > 65536, or C*M*N >= 2^31 */
  SGWLS_E_WORKSPACE = 3,    /* the workspace is NULL or smaller than required */
  SGWLS_E_UNSUPPORTED = 4,  /* a valid request this build does not implement (e.g. r > 4) */
  SGWLS_E_HIP = 5           /* a HIP runtime call or kernel launch failed */
} sgwls_status;

/* Guidance weight of Eq. (2). */
typedef enum {
  SGWLS_W_EXP = 0,   /* exp(-d^2/(2 sigma_s^2)) * exp(-(G_i-G_j)^2/(2 sigma_r^2)) */
  SGWLS_W_FRAC = 1   /* 1/(d^alpha_s + eps) * 1/(|G_i-G_j|^alpha_r + eps) */
} sgwls_weight;

/* Arithmetic of the elimination (not in the paper).  FP32: all arithmetic in
 * float32.  FP64_PIVOT: weights are computed in float32, but the diagonal
 * sums, the pivots, the elimination and the running recurrences are carried
 * in float64 (for large lambda*w, where float32 pivots lose digits to
 * cancellation).  Loads and stores stay float32 in both modes.
 * FP32_DELTA (r = 1 only, sgwls_filter / sgwls_interpolate only): float32
 * throughout, each strip's tridiagonal system solved serially by the banded
 * LDL^T of Sec. 2.2 with every pivot carried as its excess over the coupling
 * still to be eliminated, delta_{p+1} = 1 + lambda w_p delta_p / alpha_p,
 * alpha_p = delta_p + lambda w_p, which adds positive terms only (no
 * cancellation).  One thread per strip: a precision reference, about 20x
 * the time of FP64_PIVOT on a 1080p image.  Any other entry point, r != 1,
 * and a non-NULL `saved` return SGWLS_E_UNSUPPORTED.
 * AUTO: each call picks FP32 or FP64_PIVOT on the host (sgwls_resolve_precision):
 *   - from the bound kappa = 1 + 2 lambda sum_{d=1..r} S(d) R_max on the
 *     largest diagonal entry of A_s (Eq. 4 with the weights of Eq. 2; S(d) the
 *     spatial factor, R_max the largest range factor: 1 for omega^exp, 1/eps
 *     for omega^frac, reached where neighbouring guidance values are equal),
 *     FP32 when kappa <= SGWLS_AUTO_KAPPA_MAX and FP64_PIVOT above it (float32
 *     pivots lose about kappa float32 ulps of the solution);
 *   - FP64_PIVOT for every backward call that asks for the lambda gradient,
 *     and for every sgwls_filter call that saves its pass inputs (they feed a
 *     backward that may ask for it): that gradient is a sum over all edges
 *     of terms of both signs, whose cancellation no host bound can predict,
 *     and it inherits the error of the saved inputs.  A caller that needs
 *     no lambda gradient can resolve the precision itself
 *     (sgwls_resolve_precision(p, 0)) and pass it explicitly to both calls.
 *   With lambda_dev, the decision uses p->lambda, which should then bound the
 *   device value.  The workspace queries size an AUTO request for the
 *   precision the call resolves to (backward: for both). */
typedef enum {
  SGWLS_P_FP32 = 0,
  SGWLS_P_FP64_PIVOT = 1,
  SGWLS_P_FP32_DELTA = 2,
  SGWLS_P_AUTO = 3
} sgwls_precision;

/* The kappa threshold of SGWLS_P_AUTO. */
#define SGWLS_AUTO_KAPPA_MAX 64.0

/* Filter parameters.  lambda: Eq. (1).  r: the neighbourhood is
 * (2r+1)x(2r+1) (Eq. 1), 1 <= r <= 4 in this build.  iters: T >= 1 column+row
 * iterations (Sec. 2.3).  stride: the sliding step tau between strip centres
 * (Sec. 2.3), 1 <= stride <= 2r+1.  sigma_s, sigma_r > 0 for SGWLS_W_EXP;
 * alpha_s, alpha_r >= 0 and eps > 0 for SGWLS_W_FRAC (the paper uses
 * eps = 1e-4, Sec. 1). */
typedef struct {
  float lambda;
  int r;
  int iters;
  int stride;
  sgwls_weight kind;
  float sigma_s, sigma_r;
  float alpha_s, alpha_r;
  float eps;
  sgwls_precision prec;
} sgwls_params;

/* Human-readable name of a status code (static storage; never NULL). */
const char* sgwls_status_str(sgwls_status s);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int sgwls_version(void);

/* Host-only validation of a (C, M, N, params) request, exactly as the
 * filter entry points perform it.  Makes no HIP call, so it can be used
 * without a GPU. */
sgwls_status sgwls_validate(int C, int M, int N, const sgwls_params* p);

/* Device workspace bytes needed by sgwls_filter / sgwls_pass /
 * sgwls_pass_stages for one C x M x N image with parameters p; 0 if the
 * request is invalid.  save_for_backward (0 or 1) says whether the filter
 * call will pass `saved`: it decides the precision an SGWLS_P_AUTO call
 * resolves to (the saved pass inputs themselves live in the caller's
 * `saved` buffer).  The filter's workspace starts with a synchronisation
 * area (the fused passes' error word and counters, see SGWLS_ONE_LAUNCH
 * below), then one intermediate image, the transposed guidance and the
 * interface buffers.  For SGWLS_P_FP32_DELTA it is sgwls_filter's workspace
 * in that mode (the synchronisation area, one image plus the eliminated
 * strips of four channels).  Makes no HIP call. */
size_t sgwls_workspace_bytes(int C, int M, int N, const sgwls_params* p, int save_for_backward);

/* The precision a call with parameters p runs in: p->prec itself unless it
 * is SGWLS_P_AUTO, which resolves as described at sgwls_precision
 * (want_lambda_grad = 1 for a backward call that writes the lambda
 * gradient and for a filter call that saves its pass inputs).  -1 (cast)
 * for a NULL p.  Host only. */
sgwls_precision sgwls_resolve_precision(const sgwls_params* p, int want_lambda_grad);

/* One pass of Sec. 2.3 (steps 1-4) on a C x M x N image: direction 0 is
 * the column direction (strips of 2r+1 columns, Sec. 2.1), 1 the row
 * direction (the column pass of the transposed image).  x: input, y: output
 * (must not alias x or g).  lambda_dev: optional device float that, when
 * non-NULL, overrides p->lambda (read by the kernels, no host sync). */
sgwls_status sgwls_pass(int direction, const float* x, const float* g, float* y,
                        int C, int M, int N, const sgwls_params* p,
                        const float* lambda_dev, void* ws, size_t ws_bytes,
                        void* stream);

/* The kernels of one pass, for timing them one at a time.  A pass runs
 * three stages in order: 1 = reduce (every chunk of every subsystem is
 * eliminated and contributes to the Schur complement on the chunk
 * separators), 2 = interface (the separator system of every subsystem is
 * solved), 4 = expand (every chunk is solved with its separators known, and
 * the pixels covered by several subsystems are averaged into y).  `stages`
 * is a bit mask (1..7); stage 2 reads what stage 1 left in ws and stage 4
 * what stage 2 left there, so calling masks 1, 2 and 4 in order on the same
 * ws and stream computes exactly sgwls_pass.  Adding 8 to the mask (direction 0,
 * stride 1, only when the tuned column-pass variants read chunks directly)
 * stores the output transposed: y becomes C planes of N x M, pixel (i, j) of
 * the pass output at y[c*M*N + j*M + i].  sgwls_filter uses this form for
 * every stride-1 pass: each pass is then a column pass, of the image or of
 * its transpose.  Calling masks 1, 2, 4 one at a time computes sgwls_pass
 * for a channel count of one channel block (C = 1 or 3): with more, each
 * stage runs over every block and the interface buffers hold the last one.
 * Other arguments as sgwls_pass. */
sgwls_status sgwls_pass_stages(int stages, int direction, const float* x, const float* g,
                               float* y, int C, int M, int N, const sgwls_params* p,
                               const float* lambda_dev, void* ws, size_t ws_bytes,
                               void* stream);

/* The SG-WLS filter of Sec. 2.3: T iterations of (column pass, row pass).
 * f: input C x M x N; g: guidance M x N; u: output C x M x N, may alias f
 * (must not alias g).  lambda_dev: optional device override of p->lambda.
 * saved: NULL, or a device buffer of 2T*C*M*N floats that receives the
 * input of every pass in order (pass 2t = column pass of iteration t, 2t+1
 * its row pass) for sgwls_backward.  For stride 1 the passes run as column
 * passes of the image and of its transpose, and the inputs of the row
 * passes (odd entries) are then stored transposed: C planes of N x M,
 * pixel (i, j) at [c*M*N + j*M + i].  ws: workspace of
 * sgwls_workspace_bytes(C, M, N, p) bytes. */
sgwls_status sgwls_filter(const float* f, const float* g, float* u,
                          int C, int M, int N, const sgwls_params* p,
                          const float* lambda_dev, float* saved,
                          void* ws, size_t ws_bytes, void* stream);

/* ---- Fused passes (opt-in) ----
 * The environment variable SGWLS_ONE_LAUNCH, read at every sgwls_filter /
 * sgwls_filter_nchw call, replaces the three kernels of each stride-1 pass
 * (Sec. 2.3: chunk elimination, separator systems, re-solve and averaging)
 * by fused launches: 1 = one launch per pass, 2 = chunk elimination and
 * separator systems in one launch, the re-solve in a second; unset or 0 =
 * three launches (the default, and the fastest on MI355X at 1080p).  Fused
 * launches hand data between workgroups through per-strip-group counters in
 * the workspace, with bounded waits: a wait that gives up (after about two
 * seconds, or SGWLS_FUSED_SPIN_LIMIT polls) leaves the results undefined and
 * sets an error word at the start of ws.  sgwls_filter_status synchronises
 * `stream`, returns SGWLS_E_HIP (and clears the word) if it is set, else
 * SGWLS_OK; ws is the workspace of the filter calls to check.  Every call
 * with fused passes clears the word when it starts.  sgwls_filter_noalloc
 * always runs three launches per pass (its workspace is the library's). */
sgwls_status sgwls_filter_status(void* ws, void* stream);

/* ---- sgwls_filter without a caller workspace ----
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): sgwls_filter with
 * its workspace in a static device array of SGWLS_NOALLOC_MAX_BYTES bytes
 * that the library holds on every device it runs on until the process ends.
 * The call allocates nothing.  Arguments as sgwls_filter; SGWLS_E_WORKSPACE
 * (nothing enqueued) when sgwls_workspace_bytes(C, M, N, p, saved != NULL)
 * exceeds the array (1080 x 1920 RGB fits with either precision).  Every call
 * on one device uses the same array: calls that overlap on one device (other
 * streams, other host threads) race and must be serialised by the caller. */
#define SGWLS_NOALLOC_MAX_BYTES ((size_t)96 << 20)
sgwls_status sgwls_filter_noalloc(const float* f, const float* g, float* u,
                                  int C, int M, int N, const sgwls_params* p,
                                  const float* lambda_dev, float* saved, void* stream);

/* ---- NCHW batches of equal-shape images ----
 * sgwls_filter and sgwls_backward over B images of one shape in each launch
 * (the images stacked, blockIdx.z = image), with their own guidance images:
 * f, u, grad_u, grad_f are B x C x M x N; g, grad_g are B x M x N; saved is
 * B x 2T x C x M x N (image b's pass inputs at [b*2T*C*M*N ...], in the
 * layout sgwls_filter documents).  grad_lambda receives the sum over the B
 * images of their lambda gradients (one lambda shared by the batch, as for a
 * learnable lambda), reduced in a fixed order.  Workspaces from the _nchw
 * queries (0 if invalid).  B = 1 is exactly sgwls_filter / sgwls_backward.
 * SGWLS_P_FP32_DELTA is single-image only (SGWLS_E_UNSUPPORTED for B > 1). */
size_t sgwls_workspace_bytes_nchw(int B, int C, int M, int N, const sgwls_params* p,
                                  int save_for_backward);
sgwls_status sgwls_filter_nchw(const float* f, const float* g, float* u, int B, int C, int M,
                               int N, const sgwls_params* p, const float* lambda_dev,
                               float* saved, void* ws, size_t ws_bytes, void* stream);
size_t sgwls_backward_workspace_bytes_nchw(int B, int C, int M, int N, const sgwls_params* p);
sgwls_status sgwls_backward_nchw(const float* g, const float* saved, const float* grad_u,
                                 float* grad_f, float* grad_g, double* grad_lambda, int B, int C,
                                 int M, int N, const sgwls_params* p, const float* lambda_dev,
                                 void* ws, size_t ws_bytes, void* stream);

/* ---- Saved separators (not in the paper) ----
 * A backward pass recomputes its pass solution (Sec. 2.3) alongside the
 * adjoint solve.  sgwls_filter_nchw_seps is sgwls_filter_nchw with `saved`
 * required (entries 1 .. 2T-1 are written; entry 0, pass 0's input, is f
 * itself and is left unwritten, so u must not alias f) that also keeps, in
 * the device buffer seps, the solution of every pass at the chunk
 * separators of the backward's cut (the interface values of Sec. 2.3,
 * steps 2-3, for the backward's chunks; where the forward keeps its own
 * chunks its re-solve stores them).
 * sgwls_backward_nchw_seps is sgwls_backward_nchw that takes them from seps
 * and pass 0's input from f (the forward's f, unchanged; grad_f and grad_g
 * must not alias it), so each of its passes eliminates and solves the
 * separator systems of the adjoint alone (one right-hand side per channel
 * instead of two) before re-solving both.
 * Results agree with the plain pair to rounding.  Both calls run in the
 * precision sgwls_resolve_precision(p, 1) gives (AUTO: as for the lambda
 * gradient, whether or not grad_lambda is wanted), so the backward must get
 * the forward's p, B, C, M, N and its seps unchanged.
 * sgwls_separator_bytes_nchw: bytes of seps for B images, 0 when the case
 * has no such path (then both calls return SGWLS_E_UNSUPPORTED and enqueue
 * nothing): stride 1 with the column-pass kernels reading their chunks
 * directly, and the partitioned precisions.  Layout: the B guidance planes
 * transposed (N x M each, written by the forward, read by the backward
 * instead of transposing g again, so g must be the forward's, unchanged),
 * rounded up to 256 bytes; then per image (image b at b times the per-image
 * bytes): pass 0 .. 2T-1, within a pass its channel blocks (three channels,
 * then single channels), each block its separator solutions (r x cb values
 * per separator, strip after strip) rounded up to 256 bytes.  SGWLS_E_WORKSPACE when seps_bytes is too small;
 * the workspaces are those of the plain calls.  The fused passes
 * (SGWLS_ONE_LAUNCH) do not apply to sgwls_filter_nchw_seps. */
size_t sgwls_separator_bytes_nchw(int B, int C, int M, int N, const sgwls_params* p);
sgwls_status sgwls_filter_nchw_seps(const float* f, const float* g, float* u, int B, int C,
                                    int M, int N, const sgwls_params* p,
                                    const float* lambda_dev, float* saved, void* seps,
                                    size_t seps_bytes, void* ws, size_t ws_bytes, void* stream);
sgwls_status sgwls_backward_nchw_seps(const float* g, const float* f, const float* saved,
                                      const void* seps, size_t seps_bytes,
                                      const float* grad_u, float* grad_f,
                                      float* grad_g, double* grad_lambda, int B, int C, int M,
                                      int N, const sgwls_params* p, const float* lambda_dev,
                                      void* ws, size_t ws_bytes, void* stream);

/* ---- Guided sparse interpolation (Eq. 21) ----
 * u = S(f) / S(h) channel by channel, where S is the SG-WLS filter with
 * guidance g and parameters p (Sec. 2.3) standing in for the inverse of the
 * WLS matrix: f holds the C sparse input planes (0 where no value is known)
 * and h the index map (one M x N plane, 1 where f is known, 0 elsewhere).
 * All pointers are device pointers; u (C planes) must not alias g or h and
 * may alias f.  The quotient is a plain IEEE division: where S(h) is 0 (no
 * known value reaches the pixel, e.g. weights underflowing to 0) u is inf
 * or NaN.  ws: workspace of sgwls_interpolate_workspace_bytes(C, M, N, p)
 * bytes (the C+1 stacked planes plus the filter's workspace).  Errors as for
 * sgwls_filter. */
size_t sgwls_interpolate_workspace_bytes(int C, int M, int N, const sgwls_params* p);
sgwls_status sgwls_interpolate(const float* f, const float* h, const float* g, float* u,
                               int C, int M, int N, const sgwls_params* p,
                               const float* lambda_dev, void* ws, size_t ws_bytes,
                               void* stream);

/* ---- The 2D WLS model (Eqs. 1-4), reference solver ----
 * u = (I + lambda L)^-1 f per channel, where L couples every pixel with the
 * (2r+1) x (2r+1) patch around it (Eq. 1) with the weights of Eq. 2 and
 * |i - j| the Euclidean distance of the two pixels: the global model that
 * SG-WLS approximates, for measuring the approximation.  Solved by
 * Jacobi-preconditioned conjugate gradients from u = 0, one per channel,
 * until max over channels of ||f - A u|| / ||f|| <= tol or max_iters
 * iterations.  p supplies lambda, r (1..4), kind and the weight parameters;
 * iters, stride and prec are ignored.  1 <= C <= 4; u must not alias g (it
 * may alias f).  Checks convergence every 8 iterations, each check a stream
 * synchronisation, so the call cannot be captured into a graph.
 * iters_done and rel_residual (nullable) receive the iterations run and
 * the last checked relative residual.  ws: workspace of
 * sgwls_wls2d_workspace_bytes(C, M, N, p) bytes. */
size_t sgwls_wls2d_workspace_bytes(int C, int M, int N, const sgwls_params* p);
sgwls_status sgwls_wls2d(const float* f, const float* g, float* u, int C, int M, int N,
                         const sgwls_params* p, int max_iters, double tol, int* iters_done,
                         double* rel_residual, void* ws, size_t ws_bytes, void* stream);

/* ---- Kernel variants and autotuning (not in the paper) ----
 * Stride-1 passes can run several compiled kernel variants that differ in
 * how a subsystem is cut into chunks (rows per chunk) and how many chunks
 * one workgroup processes; all variants compute the same result up to
 * float rounding.  A process-wide tuning table maps (radius, channel block,
 * precision, weight kind, direction, size bucket) to a variant; absent
 * entries use variant 0.  The size bucket is round(2 log2(L*W)) of the
 * pass (L = rows along the pass, W = extent across).  The table is guarded
 * by a mutex; concurrent filter calls read it. */

/* Number of compiled variants for radius r, channel block 1 or 3 and
 * precision prec (0 if the triple is invalid). */
int sgwls_variant_count(int r, int channel_block, int prec);

/* Set the variant used for stride-1 passes of this direction, channel block
 * width (1 or 3), image size and parameters.  SGWLS_E_ARG for an unknown
 * variant. */
sgwls_status sgwls_tune_pin(int direction, int channel_block, int M, int N,
                            const sgwls_params* p, int variant);

/* The variant such a pass uses now (-1 for invalid arguments). */
int sgwls_tune_query(int direction, int channel_block, int M, int N, const sgwls_params* p);

/* Forget every tuning entry / number of entries. */
void sgwls_tune_clear(void);
int sgwls_tune_size(void);

/* Time every variant of both pass directions on the given image (each
 * channel block width present in C), `reps` launches each with HIP events
 * on `stream`, and store the fastest in the tuning table.  Synchronises the
 * stream.  x, g, y as for sgwls_pass (y is overwritten); ws of
 * sgwls_workspace_bytes(C, M, N, p) bytes.  chosen (nullable, 4 ints)
 * receives the variant per (direction 0/1) x (channel block 3/1), -1 where
 * nothing was tuned.  Strided passes have nothing to tune (SGWLS_OK). */
sgwls_status sgwls_autotune(const float* x, const float* g, float* y, int C, int M, int N,
                            const sgwls_params* p, void* ws, size_t ws_bytes, void* stream,
                            int reps, int* chosen);

/* Persist / restore the tuning table (single-image and batched entries) as text, tagged with the library
 * version and the caller's device architecture name (e.g. "gfx950").  Load
 * rejects (SGWLS_E_ARG, table unchanged) a file with another version or
 * architecture or any malformed line.  With the environment variable
 * SGWLS_TUNE_CACHE naming a file, the library loads it at the first tuning
 * lookup of the process (for the current device's architecture; a missing,
 * stale or corrupt file is ignored) and saves the table to it after every
 * sgwls_autotune / sgwls_autotune_batched call. */
sgwls_status sgwls_tune_save(const char* path, const char* arch);
sgwls_status sgwls_tune_load(const char* path, const char* arch);

/* ---- Gradients (not in the paper) ----
 * A pass maps x to y = (1/cnt) sum_k scatter_k(A_k^-1 gather_k(x)) (Sec.
 * 2.3, Eq. 5).  For a scalar loss with output gradient ybar, its adjoint is,
 * per strip k: v = gather_k(ybar / cnt); ubar = A_k^-1 v (A_k is symmetric,
 * so the adjoint solve is the same solve); xbar += scatter_k(ubar).  With
 * dA_k/dw_pq = lambda (e_p - e_q)(e_p - e_q)^T and u = A_k^-1 gather_k(x)
 * (recomputed, not stored), every edge (p, q) of Eq. (2) contributes
 * t_pq = -sum_c (ubar_p - ubar_q)(u_p - u_q): lambda t_pq dw_pq/dG to the
 * guidance gradient at both pixels of the edge and w_pq t_pq to the lambda
 * gradient.  Weights are recomputed from g.  omega^frac is not differentiable
 * in G where G_p = G_q and alpha_r <= 1; its derivative is taken as 0 there.
 * The lambda gradient is summed in float64 in a fixed order (deterministic). */

/* Device workspace bytes of sgwls_backward and sgwls_pass_backward for one
 * C x M x N image (0 if the request is invalid).  Makes no HIP call. */
size_t sgwls_backward_workspace_bytes(int C, int M, int N, const sgwls_params* p);

/* Adjoint of one sgwls_pass.  x: the pass input; ybar: gradient of the pass
 * output (C x M x N); xbar (written): gradient of the pass input, must not
 * alias x, ybar or g.  gbar (nullable, M x N, written): guidance gradient.
 * grad_lambda (nullable, one device double, written): lambda gradient.  ws:
 * sgwls_backward_workspace_bytes(C, M, N, p) bytes. */
sgwls_status sgwls_pass_backward(int direction, const float* x, const float* g,
                                 const float* ybar, float* xbar, float* gbar,
                                 double* grad_lambda, int C, int M, int N,
                                 const sgwls_params* p, const float* lambda_dev, void* ws,
                                 size_t ws_bytes, void* stream);

/* Adjoint of sgwls_filter.  saved: the 2T pass inputs that sgwls_filter wrote
 * with the same g, parameters and lambda; grad_u: gradient of the filter
 * output (C x M x N).  Writes grad_f (C x M x N; may alias grad_u, must not
 * alias g or saved) and, when non-NULL, grad_g (M x N) and grad_lambda (one
 * device double), each overwritten.  The passes are traversed in reverse
 * order.  ws: sgwls_backward_workspace_bytes(C, M, N, p) bytes. */
sgwls_status sgwls_backward(const float* g, const float* saved, const float* grad_u,
                            float* grad_f, float* grad_g, double* grad_lambda,
                            int C, int M, int N, const sgwls_params* p,
                            const float* lambda_dev, void* ws, size_t ws_bytes,
                            void* stream);

/* ---- Batches of uneven images (not in the paper) ----
 * B images of independent sizes, each with its own parameters p[b] (host
 * arrays of B entries), are filtered together: every kernel stage of a pass
 * is one persistent launch per (precision, radius) group over all images of
 * that group, whose workgroups stride over the work units (image, channel,
 * block of strips and chunks), largest image first.  With SGWLS_P_AUTO each
 * image resolves its own precision (float32 images keep float32 even when
 * others of the batch need FP64 pivots).  The persistent launches take the
 * images with stride 1, r <= 2 and sides of at most 4104 pixels (r = 1) or
 * 2052 (r = 2); every other image of the batch (r = 3 or 4, stride > 1,
 * longer sides) runs through sgwls_filter in the same call, after them, on
 * the same stream.  Requirements (else SGWLS_E_ARG, or SGWLS_E_UNSUPPORTED
 * for SGWLS_P_FP32_DELTA): every p[b].iters, kind and prec equal, and each
 * image valid for sgwls_filter.  The persistent launches filter images whose
 * channel count is a multiple of 3 three channels at a time (the guidance
 * weights shared by the block) and the others channel by channel.  On a non-default stream that is not being captured, the whole
 * call (2T passes) is captured once into a hipGraph and replayed by later
 * calls with identical arguments (same stream, workspace, pointers, shapes
 * and parameters); otherwise it is enqueued directly (the single-image-path
 * images are always enqueued directly).  u may alias f. */

/* One image of a batch: device pointers and its shape. */
typedef struct {
  const float* f;
  const float* g;
  float* u;
  int C, M, N;
} sgwls_image;

/* Workspace bytes for sgwls_filter_batched over B images (0 if invalid);
 * enough for every batched variant.  Pointers in imgs may be NULL here. */
size_t sgwls_batched_workspace_bytes(const sgwls_image* imgs, const sgwls_params* p, int B);

/* Filter B images.  Uses the variant the tuning table holds for this
 * precision, weight kind and total pixel count (variant 0 if none).  The
 * variant applies to the float32 groups; float64 groups have one. */
sgwls_status sgwls_filter_batched(const sgwls_image* imgs, const sgwls_params* p, int B,
                                  void* ws, size_t ws_bytes, void* stream);

/* Number of compiled batched variants for precision prec (rows per chunk
 * for r = 1 and r = 2, chunks per workgroup); 0 for an invalid prec. */
int sgwls_batched_variant_count(int prec);

/* sgwls_filter_batched with an explicit variant (variant < 0: tuned). */
sgwls_status sgwls_filter_batched_variant(const sgwls_image* imgs, const sgwls_params* p, int B,
                                          int variant, void* ws, size_t ws_bytes, void* stream);

/* Time every batched variant on this batch (`reps` calls each, eagerly, with
 * HIP events on `stream`; synchronises it) and store the fastest in the
 * tuning table; *chosen (nullable) receives it.  Outputs are overwritten. */
sgwls_status sgwls_autotune_batched(const sgwls_image* imgs, const sgwls_params* p, int B,
                                    void* ws, size_t ws_bytes, void* stream, int reps,
                                    int* chosen);

/* Number of cached batched graphs / destroy them all (the cache keeps the 8
 * most recently used). */
int sgwls_batched_graph_count(void);
void sgwls_batched_graph_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* SGWLS_H */
