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
  FTK_BF16X3 = 1  /* split bf16 (hi + lo) with three products, FP32 accumulate */
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
} ftk_plan_info_t;

/* Build a plan (host FP64 planning, then upload of the device tables on the
 * current HIP device).
 *   n       : image side, 4 <= n <= 1024, even
 *   K       : radial quadrature nodes M, 1 <= K <= 512 (Gauss-Jacobi(0,1)
 *             rule for k dk on [0, pi n/2], Section 3.1)
 *   Q       : angular samples Qa = number of modes = number of rotations;
 *             even, of the form 2^a 3^b, 8 <= Q <= 4096 (eq. aqkcalc with
 *             Qa = 2Q of the paper)
 *   W       : maximum shift radius in pixels, 0 < W <= n/4
 *   eps     : truncation level, every operator singular value > eps is
 *             kept (Section 4.5 and Theorem t:rank), 0 < eps < 1
 *   precision : ftk_precision
 * On success *out owns the plan; release it with ftk_plan_destroy.
 * Errors: FTK_EINVAL, FTK_EUNSUPPORTED, FTK_ENOMEM, FTK_EDEVICE. */
int ftk_plan_create(ftk_plan** out, int n, int K, int Q, double W, double eps, int precision);

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

/* Alignment from pixels: ftk_transform of images and templates into
 * plan-owned coefficient buffers, then ftk_align_coeffs.
 *   images    : device float32 [nA][n][n]
 *   templates : device float32 [nB][n][n]
 * Other arguments and errors as ftk_align_coeffs. */
int ftk_align(ftk_plan* plan, const float* images, int nA, const float* templates, int nB,
              float* X, ftk_pose* best, void* stream);

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

/* Stage timing.  While enabled, the plan records a pair of HIP events on the
 * caller's stream around every kernel launch it makes, tagged with a stage:
 *   0 transform (pixels -> coefficients)
 *   1 Step 1: image x template contraction per mode (eq. fbk3)
 *   2 Step 3 + rotation FFT + argmax (eq. fbk3, eq. 1dfft)
 *   3 bookkeeping (pose key init / conversion)
 * ftk_plan_profile(plan, 1) enables (and clears), 0 disables.
 * ftk_plan_stage_times waits for the recorded events, writes per-stage sums
 * of elapsed milliseconds and launch counts into ms[nstages] and
 * launches[nstages] (either may be NULL), and clears the record.
 * Errors: FTK_EINVAL, FTK_EDEVICE. */
int ftk_plan_profile(ftk_plan* plan, int enable);
int ftk_plan_stage_times(ftk_plan* plan, double* ms, int64_t* launches, int nstages);

/* Static name of a status code. */
const char* ftk_strerror(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char* ftk_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* FTK_H */
