/*
 * s2let_mi355x -- exact spherical harmonic transform on McEwen-Wiaux (MW) sampling and the
 * axisymmetric scale-discretised wavelet transform on the sphere, on one AMD Instinct MI355X
 * (gfx950).  Method: Leistedt, McEwen, Vandergheynst & Wiaux, "S2LET: A code to perform fast
 * wavelet analysis on the sphere" (A&A 2013), Sects. 2-3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Status: 0 = S2LET_OK, negative = error.  Arguments are validated before anything is
 *    launched; an invalid call returns S2LET_EINVAL and has no side effect.  No exception and
 *    no abort crosses this interface.
 *  - Sampling (Sect. 2.1): band-limit k gives k rings theta_t = pi(2t+1)/(2k-1), t < k (ring
 *    k-1 is the south pole, stored 2k-1 times) and 2k-1 samples phi_p = 2 pi p/(2k-1) per ring.
 *    A map is [k][2k-1] row-major, ring by ring: doubles for real signals, interleaved
 *    (re, im) double pairs for complex ones.
 *  - Harmonic coefficients f_lm (l < L, |m| <= l) are [L*L] complex (interleaved doubles) with
 *    f_lm at index l*l + l + m, orthonormal Y_lm with the Condon-Shortley phase.  Real signals
 *    exchange the full Hermitian array (f_{l,-m} = (-1)^m conj f_lm).
 *  - Batches: nmaps >= 1 maps are processed by one call; map i starts at i * (size of one map).
 *  - Pointers named "device" are device (HBM) addresses owned by the caller and must be
 *    16-byte aligned; the library never frees or keeps caller memory.  The library owns only
 *    its plan cache (host-computed tables copied to device memory once per device and size),
 *    released by s2let_finalize().
 *  - ws / ws_bytes: caller-owned device scratch of at least s2let_workspace_size(...) bytes.
 *  - stream: a hipStream_t passed as void*; NULL means the default stream.  Every device call
 *    is asynchronous on that stream; concurrent calls on different streams need separate
 *    workspaces.
 *  - Asynchronous device faults surface as S2LET_EHIP from a later call or s2let_sync().
 *  - Limits: 1 <= L <= S2LET_MAX_L for the harmonic transforms, 3 <= L <= S2LET_MAX_L for the
 *    wavelet transforms; larger L returns S2LET_EUNSUPPORTED.
 */
#ifndef S2LET_MI355X_H
#define S2LET_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  S2LET_OK = 0,
  S2LET_EINVAL = -1,        /* invalid argument (nothing launched) */
  S2LET_ENOMEM = -2,        /* workspace too small, or the plan cache could not allocate */
  S2LET_EHIP = -3,          /* a HIP runtime call failed */
  S2LET_EUNSUPPORTED = -4,  /* valid by the paper, outside this library's limits */
  S2LET_ENOTREADY = -5,     /* s2let_axisym_analysis_noalloc: plan tables not built on this device */
  S2LET_ESCRATCH = -6       /* s2let_axisym_analysis_noalloc: needs more than its static scratch */
};

enum { S2LET_REAL = 0, S2LET_COMPLEX = 1 };                       /* reality */
/* Precision of the Legendre contraction (the recursion, the phi/theta stages and the tiling are FP64
 * in every mode).  S2LET_MIXED_FP32: FP32 matrix-core products with FP32 partial sums carried into
 * FP64; where that is not faster than FP64 (the symmetric-grid synthesis of 32-column batches,
 * whose FP64 running sums leave it one wave per SIMD), the FP64 contraction runs instead.
 * S2LET_MIXED_BF16X3: both operands split into two bfloat16 parts, three products; at L = 2048
 * the inverse transforms' resampling and inverse phi stages, and the phi and theta stages of the
 * wavelet synthesis's per-scale forward transforms, also run in FP32 (rounding near 1e-7 of the
 * maps they transform).  The stated bounds (relative to the largest output) are 2e-6 and 1e-4. */
enum { S2LET_FP64 = 0, S2LET_MIXED_FP32 = 1, S2LET_MIXED_BF16X3 = 2 };
#define S2LET_MAX_L 2048

/* Generating functions of the axisymmetric wavelets (Sect. 2.2).  S2LET_KERNEL_SD: the
 * scale-discretised functions of Eqs. (10)-(16) (the default of every call without a kernel
 * argument).  S2LET_KERNEL_BSPLINE: the B-spline construction of the footnote to Sect. 2.2,
 * k(t) = (3/2) B_3(2 t B^(J-1) / L), kappa_j^2 = k(l/B^(j+1)) - k(l/B^j) for j < J, with the top
 * scale kappa_J^2 = 1 - k(l/B^J) so that the tiling sums to one below L; multiresolution
 * band-limits k_j = min(ceil(L / B^(J-j-2)), L) (Sect. 3.1) and k_Phi = min(ceil(L / B^(J-J_min-1)), L).
 * S2LET_KERNEL_NEEDLET is reserved (the paper does not define it): S2LET_EUNSUPPORTED. */
enum { S2LET_KERNEL_SD = 0, S2LET_KERNEL_BSPLINE = 1, S2LET_KERNEL_NEEDLET = 2 };

/* Scale range (Sect. 2.2, after Eq. (16)): J = ceil(log_B(L-1)), computed exactly in integers
 * as the smallest J with B^J >= L-1.  Returns J, or S2LET_EINVAL unless L >= 3 and B >= 2. */
int s2let_j_max(int L, int B);

/* Band-limit of wavelet scale j (Sect. 3.1): min(B^(j+1), L) with multiresolution, else L.
 * Returns S2LET_EINVAL for j < 0, L < 1 or B < 2. */
int s2let_bandlimit_wav(int j, int L, int B, int multires);

/* Band-limit of the scaling map: min(B^J_min, L) with multiresolution (the support of the
 * scaling kernel of Eq. (16) is l < B^J_min), else L.  S2LET_EINVAL on bad arguments. */
int s2let_bandlimit_scal(int J_min, int L, int B, int multires);

/* Number of samples stored for one map at band-limit k: k*(2k-1) (the (k-1)(2k-1)+1 distinct
 * points of Sect. 2.1 plus the 2k-2 repeats of the south pole).  -1 if k < 1. */
int64_t s2let_mw_size(int k);

/* Samples per map of the concatenated wavelet maps, scales J_min..J in order:
 * sum_j s2let_mw_size(k_j).  -1 on bad arguments. */
int64_t s2let_wav_size(int L, int B, int J_min, int multires);

/* Harmonic kernels of Eqs. (15)-(16) without the sqrt((2l+1)/4pi) factor, which cancels in
 * Eqs. (4), (6) and (8):  kappa[(j-J_min)*L + l] = kappa_B(l/B^j) (Eq. (13)) for j = J_min..J,
 * eta[l] = eta_B(l/B^J_min) (Eq. (14)), l < L.  Host memory, owned by the caller:
 * kappa has (J-J_min+1)*L doubles, eta has L.  k_B of Eq. (12) is evaluated by composite
 * Gauss-Legendre quadrature.  Host-only (no device needed).  S2LET_EINVAL unless
 * L >= 3, B >= 2, 0 <= J_min < J. */
int s2let_tiling_axisym(double* kappa, double* eta, int L, int B, int J_min);

/* Bytes of device workspace needed by mw_forward / mw_inverse (wavelet = 0) or by the
 * wavelet calls (wavelet = 1) for these arguments; 0 on invalid arguments. */
size_t s2let_workspace_size(int L, int B, int J_min, int multires, int reality, int precision,
                            int nmaps, int wavelet);

/* Forward MW spherical harmonic transform, Eq. (2) evaluated exactly by the MW quadrature:
 *   flm (device, out) [nmaps][L*L] complex;  f (device, in) [nmaps][L][2L-1] real or complex.
 * Only band-limited maps are transformed exactly (their south-pole ring is constant). */
int mw_forward(void* flm, const void* f, int L, int reality, int precision, int nmaps,
               void* ws, size_t ws_bytes, void* stream);

/* Inverse MW spherical harmonic transform, Eq. (1) truncated at l < L:
 *   f (device, out) [nmaps][L][2L-1];  flm (device, in) [nmaps][L*L] complex.
 * For reality = S2LET_REAL only f_lm with m >= 0 are read (the rest follow by symmetry). */
int mw_inverse(void* f, const void* flm, int L, int reality, int precision, int nmaps,
               void* ws, size_t ws_bytes, void* stream);

/* Axisymmetric wavelet analysis (Eqs. (4) and (6), computed in harmonic space, then one
 * inverse SHT per scale at its band-limit, Sects. 2.2 and 3.1-3.2):
 *   f_wav  (device, out) [nmaps][s2let_wav_size(L,B,J_min,multires)]: wavelet maps of scales
 *          J_min..J concatenated, scale j an MW map at band-limit k_j;
 *   f_scal (device, out) [nmaps][s2let_mw_size(k_Phi)]: scaling map at k_Phi;
 *   f      (device, in)  [nmaps][L][2L-1].
 * Real input gives real output maps; complex gives complex (interleaved). */
int s2let_axisym_analysis(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min,
                          int multires, int reality, int precision, int nmaps, void* ws,
                          size_t ws_bytes, void* stream);

/* Allocation-free variant of s2let_axisym_analysis, for callers that cannot allocate device
 * memory while they run (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, layouts and result as s2let_axisym_analysis with the
 * S2LET_KERNEL_SD kernels, without ws / ws_bytes: the workspace is a static device array of
 * S2LET_NOALLOC_SCRATCH_BYTES inside the library, one per device, held until the process ends.
 * The call allocates nothing: no hipMalloc, hipFree or allocating library routine, and no
 * profiling events.
 *  - S2LET_ESCRATCH if the call needs more workspace than that array holds, i.e. if
 *    s2let_workspace_size(L, B, J_min, multires, reality, precision, nmaps, 1) exceeds
 *    S2LET_NOALLOC_SCRATCH_BYTES (e.g. 16 real maps at L = 256 fit, at L = 512 they do not).
 *  - S2LET_ENOTREADY if the plan tables for these sizes (recursion coefficients, DFT tables,
 *    wavelet kernels of (L, B, J_min)) have not been built on the current device by an earlier
 *    allocating call: run s2let_axisym_analysis once with the same L, B, J_min and multires first.
 *  - Every call on a device uses that device's one array and leaves its contents behind (no part
 *    of it needs to start at zero): calls that overlap on one device, on different streams or
 *    threads, race and give wrong results.  Serialise them. */
#define S2LET_NOALLOC_SCRATCH_BYTES (64u << 20)
int s2let_axisym_analysis_noalloc(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min,
                                  int multires, int reality, int precision, int nmaps, void* stream);

/* Axisymmetric wavelet synthesis, Eq. (8): a forward SHT of every scale at its band-limit,
 * the harmonic tiling sum, and one inverse SHT at L.  Same layouts as the analysis, with
 * f the output. */
int s2let_axisym_synthesis(void* f, const void* f_wav, const void* f_scal, int L, int B,
                           int J_min, int multires, int reality, int precision, int nmaps,
                           void* ws, size_t ws_bytes, void* stream);

/* Adjoints, for gradients of losses through the transforms.  Each is the adjoint of the linear
 * map computed by the corresponding call above, with respect to the real inner products
 * <f, g> = sum over every stored sample of f g (real maps; Re sum conj(f) g for complex maps,
 * the 2k-1 stored copies of the south pole counted separately) and <a, b> = Re sum_{l,m}
 * conj(a_lm) b_lm over the full [L*L] coefficient array.  Same layouts, workspace and errors
 * as the transforms; output first.
 *
 * mw_inverse_adjoint: flm = S^H f with S the inverse transform of Eq. (1):
 *   flm_lm = sum_{t,p} conj(Y_lm(theta_t, phi_p)) f(theta_t, phi_p).
 * mw_forward_adjoint: f = A^H flm with A the MW quadrature (mw_forward).  For real maps the
 *   result is the real part of A^H flm, i.e. A^H applied to the Hermitian part
 *   (flm_lm + (-1)^m conj flm_{l,-m}) / 2; all L*L coefficients are read. */
int mw_inverse_adjoint(void* flm, const void* f, int L, int reality, int precision, int nmaps,
                       void* ws, size_t ws_bytes, void* stream);
int mw_forward_adjoint(void* f, const void* flm, int L, int reality, int precision, int nmaps,
                       void* ws, size_t ws_bytes, void* stream);

/* Adjoint of s2let_axisym_analysis: f = W^H (f_wav, f_scal), with W the map of Eqs. (4), (6).
 * Layouts as in s2let_axisym_synthesis (f is the output). */
int s2let_axisym_analysis_adjoint(void* f, const void* f_wav, const void* f_scal, int L, int B,
                                  int J_min, int multires, int reality, int precision, int nmaps,
                                  void* ws, size_t ws_bytes, void* stream);

/* Adjoint of s2let_axisym_synthesis (Eq. (8)): (f_wav, f_scal) = Y^H f.  Layouts as in
 * s2let_axisym_analysis (f_wav and f_scal are the outputs). */
int s2let_axisym_synthesis_adjoint(void* f_wav, void* f_scal, const void* f, int L, int B,
                                   int J_min, int multires, int reality, int precision, int nmaps,
                                   void* ws, size_t ws_bytes, void* stream);

/* The band-limit, size, tiling, analysis and synthesis calls above with a choice of generating
 * function (S2LET_KERNEL_*); identical to them for S2LET_KERNEL_SD. */
int s2let_bandlimit_wav_kernel(int j, int L, int B, int multires, int kernel);
int s2let_bandlimit_scal_kernel(int J_min, int L, int B, int multires, int kernel);
int64_t s2let_wav_size_kernel(int L, int B, int J_min, int multires, int kernel);
int s2let_tiling_axisym_kernel(double* kappa, double* eta, int L, int B, int J_min, int kernel);
int s2let_axisym_analysis_kernel(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min,
                                 int multires, int kernel, int reality, int precision, int nmaps, void* ws,
                                 size_t ws_bytes, void* stream);
int s2let_axisym_synthesis_kernel(void* f, const void* f_wav, const void* f_scal, int L, int B, int J_min,
                                  int multires, int kernel, int reality, int precision, int nmaps, void* ws,
                                  size_t ws_bytes, void* stream);

/* Wavelet denoising by hard thresholding (Sect. 4.3).  For white noise with E|n_lm|^2 = sigma^2
 * (Eq. (19)) the wavelet maps of scale j carry noise of standard deviation
 *   sigma_j = sigma * sqrt( sum_l (2l+1)/(4 pi) kappa_j(l)^2 )
 * (the noise-model relation stated, unnumbered, right after Eq. (22), with Psi^j_l0 from Eq. (15)),
 * written to sigma_wav[j - J_min] (host, J - J_min + 1 doubles).  s2let_hard_threshold sets to zero
 * every sample of the wavelet maps (device, layout of s2let_axisym_analysis) of scale j whose
 * magnitude is below thresholds[j - J_min] (host array; Eq. (23) with T_j = 3 sigma_j, read with
 * the magnitude |Y^j|); the scaling maps are not thresholded.  Asynchronous on `stream`. */
int s2let_noise_std_axisym(double* sigma_wav, int L, int B, int J_min, int kernel, double sigma);
int s2let_hard_threshold(void* f_wav, const double* thresholds, int L, int B, int J_min, int multires,
                         int kernel, int reality, int nmaps, void* stream);

/* Batches of maps with uneven band-limits and wavelet parameters: axisymmetric wavelet
 * analysis (Eqs. (4), (6)) and synthesis (Eq. (8)) of map i at band-limit L[i] with parameter
 * B[i], common J_min, multiresolution flag, reality and precision.  Maps with equal (L, B) are
 * processed together in the library's batched kernels; groups run concurrently on worker streams
 * owned by the plan (default priority), forked from and joined back to the caller's stream.
 *
 * Layouts (device memory, caller-owned): maps concatenated in the given order (map i at sample
 * offset map_off[i], [L[i]][2L[i]-1] doubles, or interleaved complex pairs); wavelet maps of map i
 * concatenated as in s2let_axisym_analysis at wav_off[i]; scaling map at scal_off[i].
 * s2let_batch_layout returns the totals {maps, wavelet maps, scaling maps} and the offsets (in
 * doubles; any of the output pointers may be NULL).
 *
 * s2let_batch_create: host-side plan plus device resources owned by the plan (copy descriptors,
 *   streams, events), released by s2let_batch_destroy.  EINVAL unless every L[i] >= 3,
 *   B[i] >= 2 and 0 <= J_min < J(L[i], B[i]); EUNSUPPORTED for L[i] > S2LET_MAX_L.
 * s2let_batch_workspace_size: bytes of caller-owned device workspace for every call below.
 * s2let_batch_analysis: f -> (f_wav, f_scal).
 * s2let_batch_run: analysis, then synthesis of its output: f -> (f_wav, f_scal) and rec.
 * s2let_batch_autotune: times s2let_batch_run over the worker-stream counts {1, 2, 4, 8} and the
 *   maps per batch {4, 8, 16} (real; {2, 4, 8} complex) on the given buffers (synchronising
 *   the stream), keeps the fastest and returns it (pointers may be NULL).  Outputs hold a
 *   complete run afterwards.
 * s2let_batch_graph_capture: runs once eagerly, then captures s2let_batch_run on these buffers
 *   into a HIP graph (stream must not be NULL); s2let_batch_graph_launch replays it on `stream`.
 *   The graph stays bound to the buffers given at capture; changing the configuration
 *   (autotune) discards it. */
typedef struct s2let_batch s2let_batch;
/* Execution modes of a batch plan.  S2LET_BATCH_STREAMS: every (L, B) group runs the batched drivers
 * on a worker stream.  S2LET_BATCH_PERSISTENT (FP64 only): the job runs level by level over every map
 * and scale; the Legendre steps of a level (analysis at L, the inverse transforms of all scales, the
 * forward transforms of all scales, synthesis at L) are work items (batch of up to 32 columns,
 * scale, m pair, node group) sorted by decreasing cost and taken by one persistent launch per tile
 * shape.  Tile shape: waves (64 northern nodes each) per block, 1, 2 or 4, chosen per band-limit
 * bucket k = 64, 128, ..., 2048 (index log2(k) - 6) separately for the analysis and the synthesis
 * kernels; a shape must not exceed the bucket's nodes (64 w <= k/2 rounded up to 64) nor give more
 * than 4 node groups (k/2 <= 256 w).  Band-limits outside the buckets (the scales below 64 and
 * those that are not powers of two) run per transform on the worker streams. */
enum { S2LET_BATCH_STREAMS = 0, S2LET_BATCH_PERSISTENT = 1 };
int s2let_batch_create(s2let_batch** plan, int nmaps, const int* L, const int* B, int J_min, int multires,
                       int reality, int precision);
int s2let_batch_destroy(s2let_batch* plan);
int s2let_batch_layout(const s2let_batch* plan, int64_t* totals, int64_t* map_off, int64_t* wav_off,
                       int64_t* scal_off);
size_t s2let_batch_workspace_size(const s2let_batch* plan);
int s2let_batch_analysis(s2let_batch* plan, void* f_wav, void* f_scal, const void* f, void* ws,
                         size_t ws_bytes, void* stream);
int s2let_batch_run(s2let_batch* plan, void* f_wav, void* f_scal, void* rec, const void* f, void* ws,
                    size_t ws_bytes, void* stream);
int s2let_batch_autotune(s2let_batch* plan, void* f_wav, void* f_scal, void* rec, const void* f, void* ws,
                         size_t ws_bytes, void* stream, int* best_streams, int* best_maps_per_batch,
                         float* best_ms);
int s2let_batch_graph_capture(s2let_batch* plan, void* f_wav, void* f_scal, void* rec, const void* f,
                              void* ws, size_t ws_bytes, void* stream);
int s2let_batch_graph_launch(s2let_batch* plan, void* stream);
/* s2let_batch_set_execution: selects the mode; nw_analysis / nw_synthesis (6 entries each, or NULL
 *   to keep the current ones) are the persistent mode's tile shapes.  EUNSUPPORTED for the persistent
 *   mode with a mixed precision, EINVAL for a shape outside the rules above.  Discards a captured graph.
 * s2let_batch_get_execution: the current mode, worker streams, maps per batch and tile shapes (any
 *   pointer may be NULL; the shape arrays take 6 entries).  s2let_batch_autotune also tries the
 *   persistent mode (FP64), choosing each used bucket's shapes by timing, and keeps whichever mode
 *   is faster. */
int s2let_batch_set_execution(s2let_batch* plan, int mode, const int* nw_analysis, const int* nw_synthesis);
int s2let_batch_get_execution(const s2let_batch* plan, int* mode, int* nstreams, int* maps_per_batch,
                              int* nw_analysis, int* nw_synthesis);

/* Measurement support.  s2let_profile_enable(1) clears previous records and, until
 * s2let_profile_enable(0), brackets every kernel launch of the calls above with a pair of HIP
 * events recorded on the launch stream; the Legendre kernels also count the (l, theta) pairs they
 * actually contract (pairs whose lambda_lm is below 2^-1100 for a whole wavefront are skipped).
 * s2let_profile_query() waits for the recorded events and returns, for one stage, the summed
 * kernel time (ms), the number of launches, the algorithmic flops of those launches (every
 * (l, m, theta) triple: 3 recursion flops plus 2 flops per data column), the flops of the work
 * actually done (retained pairs), and the algorithmic HBM bytes (inputs read once, outputs
 * written once).  Stages: 0 phi forward, 1 theta quadrature, 2 Legendre analysis,
 * 3 Legendre synthesis, 4 phi inverse, 5 harmonic tiling, 6 resampling from the symmetric grid
 * to the MW nodes (the inverse transforms that run their Legendre step on that grid).
 * s2let_profile_query_k() counts only the launches at band-limit k (every launch for k <= 0;
 * the tiling is counted at its destination band-limit).  Host-side, not thread-safe with
 * concurrent transform calls on other threads.  S2LET_EINVAL for a bad stage or null pointer. */
enum { S2LET_STAGE_PHI_FWD = 0, S2LET_STAGE_THETA = 1, S2LET_STAGE_LEG_FWD = 2,
       S2LET_STAGE_LEG_INV = 3, S2LET_STAGE_PHI_INV = 4, S2LET_STAGE_TILE = 5, S2LET_STAGE_RESAMPLE = 6 };
int s2let_profile_enable(int on);
int s2let_profile_query(int stage, double* ms, int64_t* launches, double* flops_full,
                        double* flops_retained, double* bytes);
int s2let_profile_query_k(int stage, int k, double* ms, int64_t* launches, double* flops_full,
                          double* flops_retained, double* bytes);

/* Waits for the stream and reports a pending asynchronous device error as S2LET_EHIP. */
int s2let_sync(void* stream);

/* Releases the plan cache of every device (host and device tables). */
void s2let_finalize(void);

/* Static description of a status code. */
const char* s2let_strerror(int status);

/* The HIP error code (hipError_t) behind the last S2LET_EHIP returned on the calling thread,
 * and its name (static string); hipSuccess / "hipSuccess" if none. */
int s2let_last_hip_error(void);
const char* s2let_last_hip_error_name(void);

/* Library version string. */
const char* s2let_version(void);

#ifdef __cplusplus
}
#endif
#endif /* S2LET_MI355X_H */
