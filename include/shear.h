/*
 * shear.h -- C ABI of the MI355X (gfx950) digital shearlet filter-bank library.
 *
 * The transform follows "tfShearlab: The TensorFlow Digital Shearlet Transform
 * for Deep Learning" (Andrade-Loarca, Kutyniok):
 *   - system construction: Section 3.4.1 (getshearletsystem2D), built from the
 *     digital construction of Section 2.1 (eqs. (2.1)-(2.6));
 *   - forward transform (decomposition): Algorithm 1 and its listing
 *     (tfsheardec2D), Section 3.4.2;
 *   - inverse transform (reconstruction): Algorithm 2 and its listing
 *     (tfshearrec2D), Section 3.4.2, with the dual-frame weight
 *     W = sum_k |Psi_k|^2;
 *   - adjoint: Algorithm 2 without the division by W.
 *
 * Conventions shared by every entry point
 *   Images are float32, row-major (C order): x[b][r][c], r < rows, c < cols.
 *   Coefficients are float32, planar, row-major: coeffs[b][k][r][c], k < K.
 *   The 2-D DFT is unnormalised and its inverse carries 1/(rows*cols), so
 *     coeffs[b][k] = Re ifft2( fft2(x[b]) * conj(Psi_k) ),
 *     x_rec[b]     = Re ifft2( sum_k fft2(coeffs[b][k]) * Psi_k / W ),
 *     adjoint[b]   = Re ifft2( sum_k fft2(coeffs[b][k]) * Psi_k ).
 *   Spectra at this interface use the paper's centred layout (index
 *   (rows/2, cols/2) is zero frequency, i.e. fftshift of the DFT order) and
 *   are FP64 (re, im) pairs: spectra[k][r][c][2].
 *   Filter order: for scale j = 1..J: cone 1 shears -2^s..2^s, then cone 2
 *   shears -(2^s-1)..(2^s-1), s = shear level of scale j; low-pass last.
 *   Index triples are (cone, scale, shear); the low-pass is (0, 0, 0).
 *
 * Sizes: the GPU path takes rows, cols powers of two in [16, 2048].
 *
 * Ownership and ordering
 *   The caller owns x / coeffs (device memory, e.g. torch tensors) and keeps
 *   them alive until work queued on the stream has finished. A system owns its
 *   device filter sets, twiddle tables and workspace. Transform calls are
 *   asynchronous on the given HIP stream (NULL = default stream) and never
 *   synchronise the host, except when the workspace must grow (first call with
 *   a larger batch; see shear_reserve). Only one call per system may be in
 *   flight at a time: calls on different streams sharing a system race on its
 *   workspace.
 *
 * Empty batches: shear_forward, shear_inverse, shear_adjoint, shear_denoise,
 *   shear_inpaint and shear_shrink_apply with batch == 0 return SHEAR_OK at
 *   once for a non-NULL system: nothing is launched and no other argument is
 *   read (pointers may be NULL). A negative batch is SHEAR_E_INVALID; so is
 *   batch == 0 for shear_reserve, shear_workspace_bytes, shear_autotune and
 *   shear_shrink_train_step.
 *
 * Errors: every int-returning call returns SHEAR_OK or a negative code; no
 * C++ exception crosses this boundary. shear_last_error() gives a message for
 * the most recent failure on the calling thread. Asynchronous kernel faults
 * surface at the caller's next synchronisation. NaN/Inf inputs propagate.
 */
#ifndef SHEAR_H
#define SHEAR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHEAR_OK 0
#define SHEAR_E_INVALID (-1) /* null pointer, negative batch, non-positive count, bad parameter */
#define SHEAR_E_SIZE (-2)    /* size not supported, or a constructed kernel does not fit */
#define SHEAR_E_FRAME (-3)   /* min W <= 1e-10 max W, or non-Hermitian spectra */
#define SHEAR_E_NOMEM (-4)   /* device or host allocation failed / workspace cap too small */
#define SHEAR_E_HIP (-5)     /* a HIP API call or kernel launch failed */
#define SHEAR_E_DEVICE (-6)  /* current device is not the device the system was built on */

typedef struct shear_system shear_system; /* opaque */

typedef struct {
    int rows;                   /* image rows N */
    int cols;                   /* image columns M */
    int n_scales;               /* J >= 1 */
    const int* shear_levels;    /* J entries (each 0..4), or NULL for ceil(j/2), j = 1..J */
    const double* scaling_taps; /* odd-length real 1-D low-pass h, centred; NULL = default
                                   9-tap maxflat design of Section 3.4.1 */
    int n_scaling;              /* length of scaling_taps */
    const double* fan_taps;     /* real 2-D fan filter P, row-major fan_rows x fan_cols, odd
                                   sizes, centred; NULL = default maxflat fan of Section 3.4.1 */
    int fan_rows, fan_cols;
    size_t max_workspace_bytes; /* cap on the device workspace; 0 = 4 GiB */
} shear_build_params;

/* Host only, no device needed (Section 3.4.1 construction, FP64).
 * Computes the filter bank described by p. *K receives the number of filters.
 * spectra_centred (K*rows*cols*2 doubles) and idx (K*3 ints) may be NULL to
 * query K only. Returns SHEAR_E_SIZE when a kernel does not fit in rows x cols
 * or the sizes are outside [4, 4096]. */
int shear_design_spectra(const shear_build_params* p, int* K, double* spectra_centred, int* idx);

/* getshearletsystem2D (Section 3.4.1): builds the system on the current device.
 * Synchronous. *out receives a new system; free it with shear_destroy_system. */
int shear_build_system(const shear_build_params* p, shear_system** out);

/* getshearletsystem2D (Section 3.4.1) for a caller-supplied filter bank: a
 * system from spectra in the paper's centred layout (K*rows*cols*2 doubles,
 * host memory, copied); W = sum_k |Psi_k|^2 and RMS_k are formed as for a
 * built system. The spectra must be Hermitian (DFTs of real kernels):
 * |Psi(-xi) - conj Psi(xi)| <= 1e-9 max|Psi|, else SHEAR_E_FRAME; the frame
 * must satisfy min W > 1e-10 max W, else SHEAR_E_FRAME. idx may be NULL
 * (triples then read (0, 0, k)). Synchronous. */
int shear_system_from_spectra(int rows, int cols, int K, const double* spectra_centred, const int* idx,
                              size_t max_workspace_bytes, shear_system** out);

/* The fields getshearletsystem2D returns besides the filters (Section 3.4.1):
 * sizes, RMS_k = ||Psi_k||_F / sqrt(rows*cols) (K doubles, the weights of the
 * denoising listing of Section 4.2) and the index triples (K*3 ints) of a
 * system. Any output pointer may be NULL. Host only. */
int shear_system_info(const shear_system* s, int* K, int* rows, int* cols, double* rms, int* idx);

/* The filters of getshearletsystem2D (Section 3.4.1) and the dual-frame weight
 * that Algorithm 2 divides by (Section 3.4.2), W = sum_k |Psi_k|^2: copies the
 * FP64 spectra (centred, K*rows*cols*2 doubles) and W (centred, rows*cols
 * doubles) to host memory; either pointer may be NULL. */
int shear_export_spectra(const shear_system* s, double* spectra_centred, double* W_centred);

/* Allocates the device workspace for batches up to `batch`, so that later
 * transform calls with batch <= `batch` never allocate. Synchronous. */
int shear_reserve(shear_system* s, int batch);

/* Device bytes the workspace needs for one call with `batch` images. */
int shear_workspace_bytes(const shear_system* s, int batch, size_t* bytes);

/* tfsheardec2D / Algorithm 1 (Section 3.4.2): x (batch*rows*cols float32,
 * device) -> coeffs (batch*K*rows*cols float32, device). Asynchronous on
 * hip_stream (a hipStream_t, NULL = default). x and coeffs must not overlap. */
int shear_forward(shear_system* s, const float* x, float* coeffs, int batch, void* hip_stream);

/* shear_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same transform, bitwise equal to shear_forward under a panel schedule (it
 * always takes the panel form; the whole-plane forward that shear_set_schedule
 * can select for shear_forward agrees with it to rounding), computed through a fixed
 * 64 MiB device scratch array that the library holds on each GPU it runs on
 * until the process ends, instead of the system's workspace. It calls no
 * hipMalloc, hipFree or other allocating routine and never synchronises.
 * Images are processed in chunks of as many as fit: one image needs (K + 1)
 * planes of rows x cols/2 complex values (K + 1 = 50 planes, 50 MiB, at
 * 512 x 512 with 49 filters); SHEAR_E_SIZE when one image needs more than the
 * scratch holds (e.g. 1024 x 1024 with 49 filters). Every call on a GPU shares
 * that GPU's scratch: calls that overlap on one GPU (other streams, other
 * systems, other threads) race and must be ordered by the caller.
 * Asynchronous on hip_stream. */
int shear_forward_noalloc(shear_system* s, const float* x, float* coeffs, int batch, void* hip_stream);

/* tfshearrec2D / Algorithm 2 (Section 3.4.2): coeffs -> x, dividing the
 * filtered sum by the dual-frame weight W. Asynchronous. */
int shear_inverse(shear_system* s, const float* coeffs, float* x, int batch, void* hip_stream);

/* Adjoint SH* of shear_forward (Algorithm 2 without the division by W):
 * <shear_forward(x), c> = <x, shear_adjoint(c)>. Asynchronous. */
int shear_adjoint(shear_system* s, const float* coeffs, float* x, int batch, void* hip_stream);

/* Shearlet denoising by hard thresholding (Section 4.2): for each image,
 *   y = SH^-1 T SH x,   (T c)(n) = c(n) if |c(n)| >= thresholds[b*K + k], else 0,
 * with SH = shear_forward and SH^-1 = shear_inverse; the paper's rule for the
 * thresholds is delta = K_j * sigma * RMS_k for a filter k of scale j.
 * x, y: batch*rows*cols float32 (device; they may be the same buffer).
 * thresholds: batch*K float32 (device), one per image and filter; a
 * threshold <= 0 keeps every coefficient of its plane, +inf drops them all.
 * kept: batch*K uint32 (device) or NULL; if given, it is cleared and receives
 * the number of coefficients kept per plane. The thresholded coefficients are
 * never written to memory: the threshold sits between the forward row stage
 * and the inverse row stage of one kernel. Asynchronous. */
int shear_denoise(shear_system* s, const float* x, float* y, int batch, const float* thresholds, unsigned* kept,
                  void* hip_stream);

/* Thresholds of the denoising rule of Section 4.2 for shear_denoise:
 *   out[b*K + k] = K_j * sigma[b] * RMS_k  for filter k of scale j,
 * the text's delta_j = K_j sigma per scale, weighted per filter by RMS_k as
 * the listing does. The listing thresholds every plane, the low-pass
 * included; the low-pass belongs to no scale j and takes K_1 (the coarsest
 * scale's factor). sigma: batch noise levels (host); factors: the J values
 * K_1..K_J, coarse to fine (n_factors == J), or NULL for the paper's choice
 * (2.5 on every scale but the finest, 3.8 there); out: batch*K float32
 * (host). Host only: nothing is launched. SHEAR_E_INVALID for NULL pointers,
 * a negative batch or a factor count other than J. */
int shear_denoise_thresholds(const shear_system* s, const double* sigma, int batch, const double* factors,
                             int n_factors, float* out);

/* Decay of Algorithm 3's threshold (Section 4.3): out[i] = delta_i, i < iterations.
 *   SHEAR_DECAY_GEOMETRIC: delta_i = delta_init * lambda^i with
 *     lambda = (delta_min / delta_init)^(1/(iterations-1)), so delta goes from
 *     delta_init to delta_min (the printed lambda = delta_min^(1/(iterations-1))
 *     reaches delta_min only for delta_init = 1; delta_min is read relative to it).
 *   SHEAR_DECAY_LINEAR: delta_i = delta_init * (1 - i/(iterations-1)), down to 0
 *     (delta_min unused).
 * Host only; no system needed. SHEAR_E_INVALID for an unknown kind, a
 * non-positive iteration count or, in the geometric decay, delta_init or
 * delta_min <= 0. */
#define SHEAR_DECAY_GEOMETRIC 0
#define SHEAR_DECAY_LINEAR 1
int shear_delta_schedule(int kind, double delta_init, double delta_min, int iterations, double* out);

/* Per-filter thresholds of Algorithm 3 for shear_inpaint: the scalar delta of
 * iteration i and image b is weighted by each filter's RMS_k, as in the
 * denoising listing of Section 4.2 (every plane, the low-pass included):
 *   out[(i*batch + b)*K + k] = deltas[i*batch + b] * RMS_k.
 * deltas: iterations*batch (host); out: iterations*batch*K float32 (host).
 * Host only. SHEAR_E_INVALID for NULL pointers, iterations < 1 or batch < 0. */
int shear_inpaint_thresholds(const shear_system* s, const double* deltas, int iterations, int batch, float* out);

/* Shearlet inpainting by iterative hard thresholding (Section 4.3, Algorithm 3):
 *   f = 0; for i < iterations:
 *     f = SH^-1 T_i SH ( mask (f_masked - f) + f ),
 * where T_i keeps |c| >= thresholds[i][b][k] (as shear_denoise). The caller
 * chooses the schedule (Algorithm 3 decays a scalar delta geometrically and
 * weights it per filter: thresholds[i][b][k] = delta_i * RMS_k).
 * f_masked, mask, f: batch*rows*cols float32 (device); f receives the result
 * and must not overlap f_masked or mask. thresholds: iterations*batch*K
 * float32 (device). The iteration sequence is captured once into a HIP graph
 * (kept by the system, re-captured when the pointers, batch, iterations or
 * workspace change) and replayed on hip_stream; with per-launch timing on
 * (shear_profile_enable) the launches are issued directly instead. The
 * combination mask (f_masked - f) + f is formed inside the row-FFT kernel.
 * Asynchronous. */
int shear_inpaint(shear_system* s, const float* f_masked, const float* mask, float* f, int batch,
                  const float* thresholds, int iterations, void* hip_stream);

/* Batched inpainting of images of several sizes (Section 4.3, Algorithm 3) in
 * one graph launch: group g < n_groups runs shear_inpaint's iteration sequence
 * with systems[g] (one system per image size) on its batch[g] images. The
 * sequences of all groups are captured once per call shape as parallel
 * branches of one HIP graph, held by systems[0] and re-captured when a
 * system, its schedule or workspace, a pointer, a batch or the iteration count
 * changes; each call replays it with one hipGraphLaunch on hip_stream. Arrays
 * of n_groups entries: systems (distinct, built on the current device),
 * f_masked, mask, f, batch (> 0) and thresholds (iterations*batch[g]*K_g
 * float32 each, device), with the per-group meaning of shear_inpaint. With
 * per-launch timing on in any system, the groups' launches are issued
 * directly, one group after the other. SHEAR_E_INVALID for NULL arrays or
 * entries, a system in two groups, batch[g] <= 0 or iterations < 1.
 * Asynchronous. */
int shear_inpaint_groups(shear_system* const* systems, int n_groups, const float* const* f_masked,
                         const float* const* mask, float* const* f, const int* batch, const float* const* thresholds,
                         int iterations, void* hip_stream);

/* Learned shrinkage (not in the paper: a small network predicts the
 * thresholds of Section 4.2's hard thresholding per coefficient). With
 * z_k = c_k / (sigma_b RMS_k):
 *   h1 = relu(conv3x3(z; W1) + b1), h2 = relu(conv3x3(h1; W2) + b2),
 *   tau_k = softplus(conv3x3(h2; W3) + b3_k)  (0 on the low-pass plane, the last),
 *   shrunk_k = c_k where |z_k| >= tau_k, else 0,
 * conv3x3 a cross-correlation with circular boundary over 3x3 taps, W1 32xKx3x3,
 * W2 32x32x3x3, W3 Kx32x3x3 (FP32, natural order [out][in][dy][dx]), biases FP32.
 * The matrix-core kernels compute with bfloat16 operands (z, weights and the
 * hidden activations rounded to bfloat16) and FP32 accumulation. K <= 64,
 * rows % 8 == 0, cols % 128 == 0 (else SHEAR_E_SIZE). */

/* Bytes of the packed (device) parameter block of a K-filter network. */
int shear_shrink_params_bytes(int K, size_t* bytes);

/* Packs FP32 device parameters into the device block `packed` (bfloat16
 * weights in the kernels' order, padded); asynchronous on hip_stream. */
int shear_shrink_pack(shear_system* s, const float* W1, const float* b1, const float* W2, const float* b2,
                      const float* W3, const float* b3, void* packed, void* hip_stream);

/* coeffs (batch*K*rows*cols float32, device, as shear_forward writes them) ->
 * shrunk (same shape; must not overlap coeffs) and, if tau is non-NULL, the
 * thresholds tau (same shape, noise units). sigma: batch float32 (device),
 * the noise level of each image. The system keeps a workspace of about
 * 128*batch*rows*cols bytes for the two hidden activations (32 bfloat16
 * channels each). Asynchronous. */
int shear_shrink_apply(shear_system* s, const float* coeffs, float* shrunk, float* tau, int batch, const float* sigma,
                       const void* packed, void* hip_stream);

/* Number of FP32 parameters of a K-filter network (577 K + 9280), or
 * SHEAR_E_INVALID. Flat order: W1 [32][K][3][3], b1 [32], W2 [32][32][3][3],
 * b2 [32], W3 [K][32][3][3], b3 [K]. */
int shear_shrink_param_count(int K);

/* One training step of the shrinkage network on a batch of coefficient
 * pairs (c_noisy of images with noise sigma[b], c_clean of the same images
 * without noise; both batch*K*rows*cols float32, device, as shear_forward
 * writes them). The loss replaces the hard threshold by a smooth gate
 * g = sigmoid((|z| - tau) / temperature) and is the mean over images, band
 * planes and pixels of (z g - z_clean)^2, z the noise-normalised coefficients.
 * Forward and backward run on the matrix cores (bfloat16 operands, FP32
 * accumulation; the gradient planes are stored as bfloat16); the weight
 * gradients are summed in a fixed order. Then one Adam step (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected for `step` >= 1, rate lr) updates
 * `params` (flat FP32, device), `grads` receives the gradients (same layout),
 * `adam_state` holds the two moment vectors (2 x param count, zero before
 * step 1) and `packed` is re-packed from the updated parameters. `loss`
 * (one float, device) receives the loss of the step's forward pass.
 * Asynchronous; uses the system's shrinkage workspace. */
int shear_shrink_train_step(shear_system* s, const float* c_noisy, const float* c_clean, int batch, const float* sigma,
                            float* params, float* grads, float* adam_state, void* packed, int step, float lr,
                            float temperature, float* loss, void* hip_stream);

/* Launch kinds reported by shear_profile_read (one kernel symbol each). */
#define SHEAR_KERNEL_ROWS_R2C_IMAGES 0 /* forward: row FFT of the images              */
#define SHEAR_KERNEL_COLS_FWD 1        /* forward: column FFT, x conj filter, IFFT (K-expanding) */
#define SHEAR_KERNEL_ROWS_C2R_COEFFS 2 /* forward: row inverse FFT -> coefficient planes */
#define SHEAR_KERNEL_ROWS_R2C_COEFFS 3 /* inverse/adjoint: row FFT of the coefficient planes */
#define SHEAR_KERNEL_COLS_INV 4        /* inverse/adjoint: column FFT, x filter, sum over k, IFFT */
#define SHEAR_KERNEL_ROWS_C2R_IMAGES 5 /* inverse/adjoint: row inverse FFT -> images   */
#define SHEAR_KERNEL_ROWS_THRESH 6     /* denoising: row inverse FFT, hard threshold, row FFT (in place) */
#define SHEAR_KERNEL_PLANE_FWD 7       /* forward, whole-plane form: filter, column IFFT and row
                                          inverse FFT of one plane per workgroup (its column
                                          spectra pass counts as SHEAR_KERNEL_COLS_FWD) */
#define SHEAR_KERNEL_KINDS 8

/* Per-launch timing (tracing). While enabled, every kernel launch of the
 * system is bracketed by two hipEvents recorded on the caller's stream. */
int shear_profile_enable(shear_system* s, int on);

/* Waits for the recorded events, then writes per kind the number of launches
 * and their summed duration in ms (arrays of SHEAR_KERNEL_KINDS) since the
 * previous read, and clears the record. */
int shear_profile_read(shear_system* s, int* launches, double* total_ms);

/* Column-pass schedule of the separate-launch kernels:
 *   pw_fwd / pw_inv: columns per block (16 or 8; 16 needs cols >= 32);
 *     pw_fwd = cols / 2 (the whole packed plane per workgroup) selects, for
 *     shear_forward, the whole-plane forward where it is compiled (256 x 256
 *     systems with real filter sets): one workgroup filters a plane,
 *     transforms its columns and rows on chip and writes only the
 *     coefficients, so no exchange planes pass through memory; the panel
 *     schedule is kept for the other column passes (denoising, inpainting,
 *     shear_forward_noalloc), and pw_fwd = 8 or 16 returns shear_forward to
 *     it. The column IFFT then runs as 16 x 16 (four steps), so results agree
 *     with the panel form to rounding; kg_fwd and pc_fwd do not apply to it;
 *   kg_fwd / kg_inv: filter groups (1..K: the K filters of a column panel are
 *     split over that many blocks, so that small batches fill the device; the
 *     inverse then adds the groups' partial sums in group order);
 *   pc_fwd / pc_inv: points per thread of the rows-point column FFTs, i.e.
 *     their radix sequence: the default (8 up to 512 points, 16 at 1024 and
 *     2048) or, at 256 and 512 points, 16 (two radix-16 passes), at 1024
 *     points, 8 (a 128-thread FFT group over two wavefronts; with 16-column
 *     blocks, which would need 2048 threads, the default runs instead);
 *     SHEAR_E_INVALID for any other value at that size;
 * in the forward and in the inverse/adjoint column passes; 0 keeps the
 * current value. The forward's results do not depend on the panel width or
 * the filter split (every column and filter goes through the same
 * operations); the points per thread and, in the inverse, the summation order
 * over the filters change the rounding, so results agree to rounding.
 * Drops any captured inpainting graph. */
int shear_set_schedule(shear_system* s, int pw_fwd, int pw_inv, int kg_fwd, int kg_inv, int pc_fwd, int pc_inv);

/* Autotuner: chooses the column-pass schedule of each direction among every
 * compiled panel width, filter split in {1, 2, 4, 8} (at most K; the forward
 * also tries 16 and 32 when batch * cols/16 is below the device's compute
 * units) and points per thread (default and alternative, where there is one),
 * and for the forward also the whole-plane form where it is compiled.
 * Each candidate is timed inside whole shear_forward + shear_inverse steps at
 * this batch size (the forward's candidates with the current inverse schedule,
 * then the inverse's with the chosen forward), on temporary images and
 * coefficients it allocates for the call (batch * (2 + K) * rows * cols
 * floats) and frees before it returns; five interleaved rounds, each
 * candidate keeps the median of its step times. Keeps, for each direction,
 * the candidate with the fewest filter groups among those within 1 % of the
 * fastest median (shear_set_schedule) and reports it through the out-pointers (any
 * may be NULL); the whole-plane forward is taken where its median is below the
 * chosen panel schedule's (pw_fwd then reports cols / 2, and the panel
 * schedule stays set for the other column passes). Synchronous: waits for the device, allocates the workspace for
 * batch if needed, uses the null stream; per-launch timing is paused during the
 * call. SHEAR_E_NOMEM if the temporary buffers cannot be allocated. Drops any
 * captured inpainting graph. */
int shear_autotune(shear_system* s, int batch, int* pw_fwd, int* pw_inv, int* kg_fwd, int* kg_inv, int* pc_fwd,
                   int* pc_inv);

/* Frees a system. The caller must have synchronised every stream that used it. */
void shear_destroy_system(shear_system* s);

/* Static description of an error code. */
const char* shear_strerror(int code);

/* Detail message of the most recent failure on the calling thread ("" if none). */
const char* shear_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SHEAR_H */
