/*
 * ftk.h -- C-ABI of the MI355X (gfx950) FTK rigid-alignment library.
 *
 * FTK ("factorization of the translation kernel", Rangan, Spivak, Anden,
 * Barnett, arXiv 1905.12317) computes, for many n x n images A and
 * templates B, the band-limited inner products
 *
 *     X(delta, gamma) = < R_gamma T_delta A , B >          (Section 2, eq. Xdg)
 *
 * over N user-given shifts delta and all Qa in-plane rotations
 * gamma_r = 2 pi r / Qa.  Images are taken to Fourier-Bessel coefficients
 * a(k_m; q) on M radial quadrature rings (Section 3, eq. aqkcalc); the
 * Bessel translation kernel is replaced by its rank-H operator SVD
 * (Section 4.5, eq. Jsvd / svdtrunc); the result is two dense complex
 * contractions and an angular FFT (the three steps of eq. fbk3).
 *
 * Conventions (all calls):
 *   - pixel images are float32, row-major [n][n]; the first index runs
 *     along x; pixel (i, j) sits at (i dx - 1, j dx - 1), dx = 2/n; the
 *     rotation centre is pixel (n/2, n/2) (Section 2.1);
 *   - shifts are given in pixels (dx, dy); delta = -s undoes an image that
 *     was made as A = T_s R_theta B, and gamma = -theta undoes its rotation;
 *   - the maximum shift radius is given in pixels (it is 2W in the paper's
 *     wavelength units W, Section 2);
 *   - Fourier-Bessel coefficients are complex float32 (re, im) pairs,
 *     layout [count][Qa][M]: q in storage order 0..Qa/2-1, -Qa/2..-1;
 *   - device pointers are plain HIP device allocations; the caller owns
 *     every buffer it passes; streams are hipStream_t passed as void*
 *     (NULL = the null stream); every call that takes a stream is
 *     asynchronous with respect to the host unless stated otherwise;
 *   - return values are FTK_OK (0) or a negative ftk_status; nothing
 *     throws across this boundary; ftk_strerror() names the code and
 *     ftk_last_error_message() gives the detail of the last failure on the
 *     calling thread.
 *   - a plan is not thread safe: calls on one plan must be serialised;
 *     different plans are independent.
 */
#ifndef FTK_H
#define FTK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ftk_plan ftk_plan;

typedef enum ftk_status {
  FTK_OK = 0,
  FTK_EINVAL = -1,       /* an argument is out of its documented range */
  FTK_ENOMEM = -2,       /* host or device allocation failed */
  FTK_EDEVICE = -3,      /* a HIP runtime call failed */
  FTK_ERANGE = -4,       /* a shift lies outside the planned disk */
  FTK_ESTATE = -5,       /* call order violated (e.g. align before set_shifts) */
  FTK_EUNSUPPORTED = -6  /* size not supported by the device kernels */
} ftk_status;

typedef enum ftk_precision {
  FTK_FP32 = 0,   /* both contractions on FP32 MFMA */
  FTK_BF16X3 = 1, /* split bf16 (hi + lo) with three products, FP32 accumulate */
  FTK_FP16 = 2    /* one fp16 product per term, FP32 accumulate; operands scaled by
                     powers of two per call (max |a|, max |b|) and per SVD term
                     (the 2 pi w G rows and the shift panel), Section 4.5 factors
                     kept in FP64 on the host.  About 11 significant bits per
                     operand: errors of a few 1e-4 of the pair scale, for
                     eps >= 1e-3 */,
  FTK_FP16X3 = 3  /* split fp16 (hi + lo) with three products, FP32 accumulate,
                     on the power-of-two scaled operands of FTK_FP16: about 22
                     significant bits per product (errors of order 1e-6 of the
                     pair scale), for eps down to 1e-5 */
} ftk_precision;

/* Best pose of one image-template pair: the largest Re X over the shift
 * list and the Qa rotations.  shift indexes the ftk_set_shifts array,
 * rot is r in gamma_r = 2 pi r / Qa.  Ties go to the lowest shift index,
 * then the lowest r. */
typedef struct ftk_pose {
  float value;
  int32_t shift;
  int32_t rot;
} ftk_pose;

typedef struct ftk_plan_info_t {
  int n;              /* pixels per side */
  int M;              /* radial quadrature nodes */
  int Qa;             /* angular samples = Fourier-Bessel modes = rotations */
  int H;              /* retained SVD terms (both signs of l) */
  int L;              /* largest |l| retained */
  int N;              /* shifts currently set (0 before ftk_set_shifts) */
  int precision;      /* ftk_precision */
  int nufft_width;    /* spreading kernel width of the transform */
  int nufft_grid;     /* oversampled grid size of the transform */
  double shift_radius_px;
  double eps;
  double sigma_next;  /* largest discarded singular value (<= eps) */
  double kmax;        /* pi n / 2 */
  size_t coeff_bytes_per_image; /* 8 * M * Qa */
  size_t device_bytes;          /* device memory held by the plan now */
  int weighted;                 /* 1: operator SVD with a k-side weight */
  int rotations;                /* rotations per pose search: U Qa (ftk_plan_set_rotations) */
  int ctf;                      /* 1: joint translation-CTF factorisation (ftk_plan_create_ctf) */
} ftk_plan_info_t;

/* Contrast transfer function of ftk_plan_create_ctf: the isotropic
 * weak-phase model C(s; tau) = -(sqrt(1 - A^2) sin chi + A cos chi),
 * chi = pi lambda tau s^2 - (pi/2) Cs lambda^3 s^4, s the spatial frequency
 * in 1/Angstrom (s = 1 / (2 pixel) at k = Kmax), tau the defocus (Angstrom,
 * underfocus positive).  No envelope, no astigmatism. */
typedef struct ftk_ctf_t {
  double wavelength_A;        /* electron wavelength, [0, 1] (0.019687 at 300 kV) */
  double cs_mm;               /* spherical aberration, [0, 100] */
  double amplitude_contrast;  /* A, [0, 1] */
  double pixel_A;             /* pixel size, (0, 100] */
  double defocus_min_A;       /* planned defocus range tmin < tmax, |tau| <= 1e6 */
  double defocus_max_A;
} ftk_ctf_t;

/* Build a plan (host FP64 planning, then upload of the device tables on the
 * current HIP device).
 *   n       : image side, 4 <= n <= 1024, even
 *   K       : radial quadrature nodes M, 1 <= K <= 512 (Gauss-Jacobi(0,1)
 *             rule for k dk on [0, pi n/2], Section 3.1); the reduced
 *             precision forms (every form but FTK_FP32) need K to be a
 *             multiple of 8 (FTK_EUNSUPPORTED otherwise)
 *   Q       : angular samples Qa = number of modes = number of rotations
 *             (eq. aqkcalc with Qa = 2Q of the paper).  The device kernels
 *             take Q in {64, 128, 192, 256, 384} (a multiple of 64 of the
 *             form 2^a 3^b, at most 384); any other Q is FTK_EUNSUPPORTED,
 *             an odd Q or Q outside [8, 4096] FTK_EINVAL
 *   W       : maximum shift radius in pixels, 0 < W <= n/4
 *   (n)     : besides, the transform's oversampled grid (the smallest
 *             2^a 3^b >= 2n) must not exceed 4096 (FTK_EUNSUPPORTED)
 *   eps     : truncation level, every operator singular value > eps is
 *             kept (Section 4.5 and Theorem t:rank), 0 < eps < 1
 *   precision : ftk_precision
 * On success *out owns the plan; release it with ftk_plan_destroy.
 * Errors: FTK_EINVAL, FTK_EUNSUPPORTED, FTK_ENOMEM, FTK_EDEVICE. */
int ftk_plan_create(ftk_plan** out, int n, int K, int Q, double W, double eps, int precision);

/* ftk_plan_create with a k-side weight in the operator SVD (Section 4.5,
 * the remark on alternative weight functions): the SVD of each J_l(delta k)
 * is taken with the measure p(k) k dk on [0, Kmax] in place of k dk,
 *   p(k) = c sum_{j < nterms} alpha[j] exp(-beta[j] (k / Kmax)^2),
 * alpha[j] >= 0 (not all 0), beta[j] >= 0, finite, host arrays copied by
 * the call, c set so that p has mean 1 over the disk of radius Kmax.  Every
 * Sigma > eps is kept as before, now in the p-weighted norm: with p shaped
 * like the power spectrum of the templates, fewer terms reach a given
 * accuracy of the inner products (the remark's purpose).  nterms = 0 is
 * ftk_plan_create.  Errors: as ftk_plan_create; FTK_EINVAL for bad terms. */
int ftk_plan_create_weighted(ftk_plan** out, int n, int K, int Q, double W, double eps, int precision,
                             const double* alpha, const double* beta, int nterms);

/* Release the plan and all device memory it holds.  NULL is allowed.  The
 * caller must make sure no work that uses the plan is still in flight. */
void ftk_plan_destroy(ftk_plan* plan);

/* Fill *out with the plan's sizes.  Errors: FTK_EINVAL (NULL pointers). */
int ftk_plan_info(const ftk_plan* plan, ftk_plan_info_t* out);

/* Set the N shifts (host array [N][2] of (dx, dy) in pixels) that the
 * alignment evaluates; builds the shift-side table
 * Y[delta][zeta] = u_zeta(Kmax |delta|) exp(-i l_zeta (omega + pi/2))
 * (Section 4.5) in FP64 and uploads it.  Synchronous.  The plan copies the
 * shifts.  1 <= N <= 65536.  Any |delta| > W (beyond a 1e-9 relative
 * margin) returns FTK_ERANGE: the factorisation only holds inside the
 * planned disk (eq. Jsvd).  Errors: FTK_EINVAL, FTK_ERANGE, FTK_ENOMEM,
 * FTK_EDEVICE. */
int ftk_set_shifts(ftk_plan* plan, const double* shifts_px, int N);

/* Pixel images -> Fourier-Bessel coefficients (Section 3.2: type-2 NUFFT
 * onto the polar grid, then a length-Qa DFT per ring, eq. aqkcalc).
 *   imgs   : device float32 [cnt][n][n]
 *   coeffs : device complex float32 [cnt][Qa][M] (caller allocated,
 *            cnt * coeff_bytes_per_image bytes)
 * cnt >= 0 (0 is a no-op).  Uses plan-owned scratch (grown on demand with
 * hipMalloc, so the first call with a larger cnt may allocate).
 * Errors: FTK_EINVAL, FTK_ENOMEM, FTK_EDEVICE. */
int ftk_transform(ftk_plan* plan, const float* imgs, int cnt, void* coeffs, void* stream);

/* Alignment from Fourier-Bessel coefficients (the three steps of eq. fbk3,
 * with the shift contraction applied before the rotation FFT).
 *   img_coeffs  : device [nA][Qa][M] complex float32 (images A)
 *   tmpl_coeffs : device [nB][Qa][M] complex float32 (templates B)
 *   X           : device float32 [nA][nB][N][Qa] or NULL.  If given, every
 *                 inner product X(delta_s, gamma_r) is written.
 *   best        : device ftk_pose [nA][nB] or NULL.
 * At least one of X, best must be non-NULL unless nA or nB is 0 (then the
 * call is a no-op).  nA, nB >= 0.  Requires
 * ftk_set_shifts first (else FTK_ESTATE).  Plan-owned workspace is grown
 * on demand.  Errors: FTK_EINVAL, FTK_ESTATE, FTK_ENOMEM, FTK_EDEVICE. */
int ftk_align_coeffs(ftk_plan* plan, const void* img_coeffs, int nA, const void* tmpl_coeffs,
                     int nB, float* X, ftk_pose* best, void* stream);

/* Size of the fixed device scratch of ftk_align_coeffs_noalloc (256 MiB).
 * The library holds it on every GPU it runs on until the process ends. */
#define FTK_NOALLOC_SCRATCH_BYTES (256u * 1024u * 1024u)

/* ftk_align_coeffs for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with every buffer the call
 * needs (pose keys, 8 nA nB bytes; the Step 1 template operand; the data
 * scales of the fp16 forms; and the Zhat staging of at least one image
 * against all nB templates) carved from one fixed device array of
 * FTK_NOALLOC_SCRATCH_BYTES per GPU.  It calls no hipMalloc, hipFree or
 * allocating library routine and records no stage timing.  Arguments,
 * layouts and ownership as ftk_align_coeffs.
 * The scratch keeps the last call's contents; every call initialises what
 * it reads.  Calls that overlap on one GPU (different streams or host
 * threads) share the array and race: the caller serialises them.
 * Errors: FTK_EUNSUPPORTED when the call needs more than the scratch (the
 * message states the sizes), otherwise as ftk_align_coeffs (never
 * FTK_ENOMEM). */
int ftk_align_coeffs_noalloc(ftk_plan* plan, const void* img_coeffs, int nA, const void* tmpl_coeffs,
                             int nB, float* X, ftk_pose* best, void* stream);

/* Alignment from pixels: ftk_transform of images and templates into
 * plan-owned coefficient buffers, then ftk_align_coeffs.
 *   images    : device float32 [nA][n][n]
 *   templates : device float32 [nB][n][n]
 * Other arguments and errors as ftk_align_coeffs. */
int ftk_align(ftk_plan* plan, const float* images, int nA, const float* templates, int nB,
              float* X, ftk_pose* best, void* stream);

/* Two-pass alignment from coefficients: `coarse` (for example an FTK_FP16
 * plan) aligns every pair into best; then, per image, the k templates with
 * the largest coarse best values (ties: lower template number) are aligned
 * again by `fine` (for example an FTK_BF16X3 plan), and those k poses
 * replace the coarse ones in best.  Each pose is the argmax over shifts and
 * rotations of the inner products of eq. fbk3, as in ftk_align_coeffs.  The
 * plans must share n, K, Q and W (FTK_EINVAL otherwise); their precision,
 * eps and k-side weight (hence H) may differ, so the coarse pass may use a
 * cheaper factorisation than the fine one.  The caller sets the same shifts
 * on both (only their count N is checked); ftk_transform gives the same
 * coefficients under either plan.
 *   best      : device ftk_pose [nA][nB], every pair
 *   best_t    : device int32 [nA]: per image, the template with the largest
 *               refined value (ties: lower template number), or NULL
 *   best_pose : device ftk_pose [nA], its pose, or NULL (with best_t)
 * 1 <= k <= min(nB, 64).  Workspace of the fine plan grows on demand.
 * Errors: FTK_EINVAL, FTK_ESTATE, FTK_ENOMEM, FTK_EDEVICE. */
int ftk_align_refined(ftk_plan* coarse, ftk_plan* fine, const void* img_coeffs, int nA, const void* tmpl_coeffs,
                      int nB, int k, ftk_pose* best, int32_t* best_t, ftk_pose* best_pose, void* stream);

/* Joint translation and CTF factorisation (Section 7.1, other 2D kernels):
 * a plan whose SVD terms factorise F(delta, k) C(|k|; tau) into
 * Y_zeta(delta, tau) G_zeta(k), so that one alignment searches shifts,
 * defocus values and rotations: X(delta, tau, gamma) = <R_gamma T_delta C_tau
 * A, B> (equal to aligning A with the CTF-filtered template C_tau B).  Per
 * angular mode l the SVD is that of J_l(x y) C(y; tau) from L2(y dy) on
 * [0, 1] to L2(x dx dtau) on [0, pi W] x [tmin, tmax] (defocus measure of
 * mass 1), kept above eps as in ftk_plan_create.  The kernels are those of
 * every plan; only the tables (and H, which grows with the defocus range)
 * differ.  Poses are set with ftk_set_poses (one defocus per shift);
 * ftk_set_shifts and ftk_bft_align refuse such plans.  Other arguments and
 * errors as ftk_plan_create (FTK_EINVAL for CTF parameters out of range). */
int ftk_plan_create_ctf(ftk_plan** out, int n, int K, int Q, double W, double eps, int precision,
                        const ftk_ctf_t* ctf);

/* Poses (shift_i, defocus_i), i < N, of a plan with a CTF: shifts_px as in
 * ftk_set_shifts, defocus_A [N] within the planned range (FTK_ERANGE
 * otherwise).  The pose index plays the part of the shift index in X and in
 * ftk_pose.shift.  On a plan without a CTF, defocus_A must be NULL and the
 * call is ftk_set_shifts.  Errors as ftk_set_shifts. */
int ftk_set_poses(ftk_plan* plan, const double* shifts_px, const double* defocus_A, int N);

/* Shift windows for the learned proposal's restricted search: window b
 * holds the plan's shifts whose radius |delta| lies within half_width_px of
 * centers_px[b] (an annulus: rotation-invariant features fix the size of a
 * shift, not its direction).  For each window the library keeps the
 * shift-side panels of that subset.  ftk_align_proposed (ftk_mlp.h) with a
 * network of n_shift = nw bins then aligns each confidently proposed image
 * only over the window of its predicted bin; the poses still index the
 * plan's full shift list.  nw = 0 removes the windows; ftk_set_shifts
 * removes them too.  Errors: FTK_EINVAL (a window without shifts, bad
 * arguments), FTK_ESTATE (no shifts), FTK_EUNSUPPORTED (plan with a CTF),
 * FTK_ENOMEM. */
int ftk_plan_set_shift_windows(ftk_plan* plan, const double* centers_px, int nw, double half_width_px);

/* Rotation upsampling (the remark after eq. 1dfft: zero-padding the angular
 * sum samples more rotations at little cost).  With upsample = U > 1 the
 * alignments of this plan evaluate X on U Q rotations gamma_r = 2 pi r / (U Q),
 * r = 0 .. U Q - 1: X = Re sum_q e^{-i q gamma} Xhat(delta, q) over the Q
 * modes (the Nyquist mode as its cosine), which at every U-th rotation equals
 * the Q-rotation result.  X then has rows of U Q values ([nA][nB][N][U Q])
 * and ftk_pose.rot runs over [0, U Q).  Implemented as U passes of the
 * Q-point rotation FFT on Xhat(q) e^{-i q 2 pi u / (U Q)}, u = 0 .. U - 1,
 * Step 3 handing Xhat over through device memory (Q/2 x 2 N' floats per pair,
 * N' = N rounded up to 16, counted against the staging size).  Applies to
 * ftk_align, ftk_align_coeffs, ftk_align_lists, ftk_bft_align, batches and
 * ftk_align_refined (both plans with the same U); not to the FP16 form
 * (FTK_EUNSUPPORTED at alignment) nor to ftk_align_coeffs_noalloc.
 * upsample = 1 (the default) restores Q rotations.
 * Errors: FTK_EINVAL (upsample outside [1, 16]). */
int ftk_plan_set_rotations(ftk_plan* plan, int upsample);

/* Brute-force translations (BFT, Section 6.2 of the paper), the method the
 * paper compares FTK with, on the plan's grids and shifts: for every image
 * and shift, the translated Fourier-Bessel coefficients T_delta a(k_m; q)
 * (the ring samples times the translation phase exp(-i k . delta) of eq. Fdk,
 * then the ring DFT of eq. aqkcalc); for every pair and shift, eq. fbk2
 * with l_max = 0, Xhat(delta, q) = 2 pi sum_m w_m T_delta a conj b; then
 * the rotation FFT of eq. 1dfft and the argmax.  Its X equals the direct
 * inner product on the polar quadrature (no SVD, no truncation) up to FP32
 * rounding.  FP32 throughout, whatever the plan's precision form; the SVD
 * tables are not used.  Arguments, layouts, ownership and results as
 * ftk_align (pixels in, X [nA][nB][N][Q] optional, best [nA][nB]).  The
 * plan's workspace grows by the translated coefficients of one chunk of
 * images ((Q/2 + 1) N' K complex, N' = N rounded up to 32 or 64, per image)
 * and an Xhat staging of Q/2 x 2 N' floats per pair; images are chunked to
 * the staging size of ftk_plan_set_tuning.  Stage timing: the translation
 * is stage 5, the contraction stage 1, the rotation FFT stage 2.
 * Errors: FTK_EINVAL, FTK_ESTATE (no shifts), FTK_ENOMEM, FTK_EUNSUPPORTED,
 * FTK_EDEVICE. */
int ftk_bft_align(ftk_plan* plan, const float* images, int nA, const float* templates, int nB, float* X,
                  ftk_pose* best, void* stream);

/* Brute-force rotations (Section 6.1, eq. 2dconv), the paper's other
 * comparison method: for every rotation gamma_r = 2 pi r / R (R = Q times
 * the plan's rotation upsampling factor, 1 unless ftk_plan_set_rotations)
 * the correlation of the image with the rotated template through the 2D
 * convolution theorem on the Cartesian Fourier grid of the pixel DFT,
 *   X(delta, r) = pi^2 sum_k exp(-i k . delta) Ahat(k) conj(Bhat(R_gamma k)),
 * k = pi (u, v) over the integer points of the disk u^2 + v^2 <= (n/2)^2,
 * Ahat and Bhat the type-2 NUFFT of the pixels at those points (rotated for
 * the template).  It approximates the same inner product as ftk_align on a
 * Cartesian instead of a polar quadrature (the two agree to rounding for
 * images whose spectra vanish at Kmax; they differ by the quadratures'
 * error otherwise).  The shifts are those of ftk_set_shifts, evaluated on
 * the product grid of their distinct x and y offsets (any list is allowed;
 * lattices cost least).  FP32 whatever the plan's precision form; the SVD
 * tables are not used.  Arguments, ownership and results as ftk_bft_align:
 * pixels in, X [nA][nB][N][R] optional, best [nA][nB] (rotation index in
 * [0, R)); asynchronous on the stream after a short host wait for the
 * call's tables (so not for use under stream capture).  The plan's workspace grows by the image spectra
 * ((n/2 + 1) x (n + 4) complex per image) and the spectra of one chunk of
 * templates at all R rotations (R times that per template), templates
 * chunked to the staging size of ftk_plan_set_tuning.  Stage timing: the
 * fine grids stage 0, the spectra stage 6, the correlation stage 7.
 * Errors: FTK_EINVAL, FTK_ESTATE (no shifts), FTK_ENOMEM, FTK_EUNSUPPORTED
 * (a plan with a CTF, R not a multiple of 64), FTK_EDEVICE. */
int ftk_bfr_align(ftk_plan* plan, const float* images, int nA, const float* templates, int nB, float* X,
                  ftk_pose* best, void* stream);

/* FP64 planning tables, host only (no device work, usable without a GPU):
 * the same truncation and factor tables a plan with these arguments uses.
 * Pass NULL for any output not wanted; sizes come from *H_out (call once
 * with all outputs NULL to get H).
 *   ell   : int32 [H]        l_zeta
 *   sigma : double [H]       Sigma_zeta
 *   G     : double [H][K]    Sigma_zeta v_zeta(k_m / Kmax)
 *   k, w  : double [K]       radial nodes and weights
 *   Y     : double [N][H][2] u_zeta(Kmax|delta|) e^{-i l (omega + pi/2)}
 *           (needs shifts_px [N][2], else pass N = 0)
 *   sigma_next : largest discarded singular value
 * Errors: FTK_EINVAL, FTK_ERANGE. */
int ftk_plan_tables(int n, int K, double W, double eps, const double* shifts_px, int N,
                    int* H_out, int32_t* ell, double* sigma, double* G, double* k, double* w,
                    double* Y, double* sigma_next);
/* ftk_plan_tables with the k-side weight of ftk_plan_create_weighted
 * (alpha, beta, nterms as there; nterms = 0: ftk_plan_tables). */
int ftk_plan_tables_weighted(int n, int K, double W, double eps, const double* alpha, const double* beta,
                             int nterms, const double* shifts_px, int N, int* H_out, int32_t* ell, double* sigma,
                             double* G, double* k, double* w, double* Y, double* sigma_next);

/* ftk_plan_tables for a plan with a CTF: Y [N][H][2] for the poses
 * (shifts_px [N][2], defocus_A [N]); other outputs as ftk_plan_tables. */
int ftk_plan_tables_ctf(int n, int K, double W, double eps, const ftk_ctf_t* ctf, const double* shifts_px,
                        const double* defocus_A, int N, int* H_out, int32_t* ell, double* sigma, double* G,
                        double* k, double* w, double* Y, double* sigma_next);

/* Stage timing.  While enabled, the plan records a pair of HIP events on the
 * caller's stream around every kernel launch it makes, tagged with a stage:
 *   0 transform (pixels -> coefficients)
 *   1 Step 1: image x template contraction per mode (eq. fbk3)
 *   2 Step 3 + rotation FFT + argmax (eq. fbk3, eq. 1dfft)
 *   3 bookkeeping (pose key init / conversion)
 *   4 operand preparation (templates embedded, and split for bf16x3,
 *     into Step 1's lane order, once per call)
 *   5 translated coefficients of ftk_bft_align
 *   6 Cartesian spectra of ftk_bfr_align (fine grid interpolated)
 *   7 correlation of ftk_bfr_align
 * ftk_plan_profile(plan, 1) enables (and clears), 0 disables.
 * ftk_plan_stage_times waits for the recorded events, writes per-stage sums
 * of elapsed milliseconds and launch counts into ms[nstages] and
 * launches[nstages] (either may be NULL), and clears the record.
 * Errors: FTK_EINVAL, FTK_EDEVICE. */
int ftk_plan_profile(ftk_plan* plan, int enable);
int ftk_plan_stage_times(ftk_plan* plan, double* ms, int64_t* launches, int nstages);

/* Launch shapes of a plan's alignment kernels.  They change speed only:
 * every choice gives the same results (each pair's sums are taken in the
 * same order whatever the shape).  A field left 0 takes the built-in
 * default (an FTK_STEP3_WAVES, FTK_STEP1_ZBLK or FTK_STAGE_MB environment
 * variable, read at plan creation, overrides that default).
 *   step3_waves : most waves per Step 3 workgroup, each wave owning 16
 *                 shifts; 1..16, lowered to what LDS allows (default 16)
 *   step1_zblk  : SVD terms per Step 1 workgroup, 64 or 128, lowered to 64
 *                 when H (padded to 64) is not a multiple of 128 or the
 *                 tile does not fit LDS (default 128; FTK_FP16: 64;
 *                 list alignments of up to 16 templates per image: 64)
 *   step1_wgs   : Step 1 splits its template sweep until the grid holds
 *                 about this many workgroups; 64..65536 (default 4096)
 *   stage_mib   : the Step 1 -> Step 3 staging buffer, MiB; images are
 *                 processed in chunks that fit; 16..65536 (default 8192) */
typedef struct ftk_tuning_t {
  int step3_waves;
  int step1_zblk;
  int step1_wgs;
  int stage_mib;
} ftk_tuning_t;

/* Set (NULL fields checked, 0 = default) or read the plan's tuning.
 * ftk_plan_get_tuning reports the values in force, defaults resolved.
 * Errors: FTK_EINVAL (NULL pointer, value out of range). */
int ftk_plan_set_tuning(ftk_plan* plan, const ftk_tuning_t* tuning);
int ftk_plan_get_tuning(const ftk_plan* plan, ftk_tuning_t* out);

/* ---- Ragged batches ---------------------------------------------------
 * A batch runs many independent alignment problems ("stacks") whose plans
 * differ in n, K, Q, W (hence H) and N, as one unit of work on one stream.
 * The paper treats each problem on its own (the method of Section 4 per
 * image-template set); the batch only schedules them:
 *   - one device workspace per lane, sized at creation for the largest
 *     stack, is lent to every plan while its stack runs, so running the
 *     batch allocates nothing;
 *   - stacks are ordered by a cost model (Step 1 + Step 3 flop of the
 *     stack) and dealt to `lanes` streams forked from the caller's stream,
 *     largest first onto the least loaded lane, so one lane's kernel tails
 *     overlap the other's work;
 *   - with FTK_BATCH_GRAPH, the first ftk_batch_run captures every launch
 *     of every stack (fork and join included) into one hipGraph and each
 *     run replays it with one hipGraphLaunch;
 *   - with FTK_BATCH_AUTOTUNE, ftk_batch_create times candidate launch
 *     shapes (ftk_tuning_t) of each stack's plan on a slice of that stack
 *     and keeps the fastest; results are cached per shape in the process
 *     and, if FTK_TUNE_CACHE names a file, across processes (one text line
 *     per shape).  Tuning changes speed only, never results.
 * Each stack's outputs equal those of ftk_align on the same plan and
 * inputs.  The batch keeps the launch shapes of each stack (the plan's
 * tuning at creation, or the autotuner's choice) and lends them to the
 * plan while the stack runs; the plans' own tuning is left unchanged. */
typedef struct ftk_batch ftk_batch;

typedef struct ftk_stack {
  ftk_plan* plan;          /* plan of this stack, shifts already set */
  const float* images;     /* device float32 [nA][n][n] */
  int nA;
  const float* templates;  /* device float32 [nB][n][n] */
  int nB;
  float* X;                /* device float32 [nA][nB][N][Qa] or NULL */
  ftk_pose* best;          /* device ftk_pose [nA][nB] or NULL */
} ftk_stack;

enum {
  FTK_BATCH_GRAPH = 1,     /* capture once, replay as one hipGraph */
  FTK_BATCH_AUTOTUNE = 2   /* time launch shapes per stack at creation */
};

typedef struct ftk_batch_info_t {
  int count;               /* stacks */
  int lanes;               /* streams the stacks are dealt to */
  int graph_nodes;         /* nodes of the captured graph (0 before capture) */
  size_t workspace_bytes;  /* device bytes of all lane workspaces */
  double cost_gflop;       /* cost model total */
  double tune_ms;          /* host time spent autotuning at creation */
} ftk_batch_info_t;

/* Create a batch over `count` stacks (the array is copied; the buffers and
 * plans it names must outlive the batch and keep their addresses).  Every
 * stack needs its plan's shifts set, nA, nB >= 0 and, if nA nB > 0, both
 * pixel pointers and at least one of X, best.  Several stacks may share a
 * plan.  lanes is 1 to 4 (one hardware queue each).  All device memory the batch needs is allocated
 * here.  With FTK_BATCH_AUTOTUNE the call runs kernels on `stream` over
 * the first images and templates of each stack (into batch-owned buffers;
 * the stacks' outputs are not written) and waits for them.
 * Errors: FTK_EINVAL, FTK_ESTATE (shifts not set), FTK_ENOMEM,
 * FTK_EDEVICE and those of ftk_align. */
int ftk_batch_create(ftk_batch** out, const ftk_stack* stacks, int count, int lanes, int flags, void* stream);

/* Run every stack once, asynchronously on `stream`.  Allocates nothing
 * (workspaces were sized at creation).  With FTK_BATCH_GRAPH the first run
 * captures the graph on `stream` (which must not be the null stream:
 * FTK_EINVAL) and launches it; later runs only launch it.  Inputs may change between runs;
 * shapes, plans and buffer addresses may not.  A batch is not thread safe
 * and its runs on different streams must not overlap.  While a batch
 * runs, its plans must not be used by other calls.  Errors: FTK_EINVAL,
 * FTK_EDEVICE and those of ftk_align. */
int ftk_batch_run(ftk_batch* batch, void* stream);

int ftk_batch_info(const ftk_batch* batch, ftk_batch_info_t* out);

/* Release the batch (graph, streams, workspaces).  NULL is allowed.  Work
 * in flight must be finished first. */
void ftk_batch_destroy(ftk_batch* batch);

/* Static name of a status code. */
const char* ftk_strerror(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char* ftk_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* FTK_H */
