// Internal interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct TransformArgs {
  const float* imgs;     // [cnt][n][n]
  float2* coeffs;        // [cnt][Qa][M], or null: stop after the fine grid (scratchG)
  float2* polar;         // [cnt][M][Qa] ring samples Ahat(k_m, psi_p) / Qa, or null
  float2* scratchH;      // [cnt][n][nf]
  float2* scratchG;      // [cnt][nf][nf] (transposed: [l2][l1])
  const float* deapod;   // [n] per-dimension deconvolution and scale
  const float2* tw_nf;   // [nf] exp(-2 pi i k / nf)
  const float2* tw_qa;   // [Qa] exp(-2 pi i k / Qa)
  const int* pt_base;    // [M * Qa/2][2] first fine-grid index (mod nf) per dimension
  const float* pt_ker;   // [M * Qa/2][2][w] spreading-kernel weights per dimension
  int n, nf, M, Qa, w;
};

size_t transform_lds_bytes(int nf, int Qa, int nwaves);
// waves per transform workgroup: FTK_TRANSFORM_WAVES (default 16), lowered until LDS fits
int transform_waves(int nf, int Qa);
hipError_t launch_transform(const TransformArgs& args, int cnt, hipStream_t stream);

// Step 1 (eq. fbk3): Zhat of every pair of the call, into the staging below.
struct Step1Args {
  const float2* a;       // image coefficients [nA][Qa][M] (chunk base)
  const float2* b;       // template coefficients [nB][Qa][M]
  const float* cz;       // [H_pad][M]: 2 pi w_m Sigma v(k_m), 0 on padding
  const int* ell;        // [H_pad]: l_zeta, 0 on padding
  const float2* ta;      // brute-force translations only: translated coefficients (launch_step1_bft)
  void* zs;              // Zhat staging, layout by form (below)
  const float* r32;      // embedded template operand, FP32 lane order (tmpl_prep)
  const void* r16;       // embedded template operand, bf16 hi/lo or fp16 lane order (tmpl_prep)
  const float* dscale;   // FP16 form: device [1/s_a, 1/s_b] (power-of-two data scales); else null
  int nA, nB, M, Qa, H_pad, L;
  int zblk;              // zeta per workgroup (64 or 128)
  int tparts;            // template row tiles split over this many workgroups
  // template operand addressing: row tile t of image A at mode q is tile
  // q tiles_per_q + A img_tiles + t.  Plain: tiles_per_q = ceil(nB/16),
  // img_tiles = 0; per-image lists: nB = K, img_tiles = ceil(K/16),
  // tiles_per_q = nA img_tiles
  int tiles_per_q;
  int img_tiles;
};

// Zhat staging written by Step 1 and read by Step 3: Qa/2 rows of q per pair,
// row 0 holding Zhat(0) + i Zhat(Qa/2) (the Nyquist mode folded in), and
// K index k' = c H_pad + zeta (c = 0 real, 1 imaginary part).  4 Qa H_pad
// bytes per pair in the FP32 and split forms, half that in the FP16 form:
//   FP32:       [pair][q][k'] float
//   split:      [pair][k' / 32][q][32 hi of k' % 32][32 lo], bf16 (split
//               bf16) or fp16 (split fp16, scaled by 1 / (s_a s_b sg_zeta))
//               (one 128-byte row per q and chunk of 32 k': Step 3 copies
//               whole chunks into LDS without converting them)
//   FP16:       [pair][k' / 64][q][64 fp16 of k' % 64] (the same 128-byte
//               rows, 64 k' each), scaled by 1 / (s_a s_b sg_zeta)
// Step 3 + rotation FFT + argmax.
struct Step3Args {
  const void* zs;        // Zhat staging (above)
  const float* yt;       // [2 H_pad][2 N_pad] real embedding of Y, transposed
  const uint16_t* yt_hi; // reduced-precision copies (bf16 or fp16 in MFMA lane order)
  const uint16_t* yt_lo;
  float* X;              // [pairs][N][Qa] or nullptr
  const float* xscale;   // device scalar multiplying the X outputs (FP16 and split-fp16 forms), or null
  unsigned long long* keys;  // [pairs]
  const float2* tw_qa;   // [Qa]
  const void* rot16;     // FP16 form with Qa <= 256: the rotation transform tables (rot16_table_bytes), or null
  float* xhat;           // or: Xhat out [pairs][Qa/2][2][N_pad] instead of the rotation sum (upsampling)
  int up;                // rotation upsampling factor of launch_xhat_rotate (1: none)
  int pairs, Qa, H_pad, N, N_pad;
  int nwaves;            // waves per workgroup; each wave owns 16 shifts
  int nblk;              // workgroups per pair (shift blocks); 1-D grid of pairs * nblk
};

size_t step3_lds_bytes(int Qa, int nwaves);
hipError_t launch_step3(const Step3Args& args, int precision, hipStream_t stream);
// Step 1 with the template operand embedded once per call (kern_step1.hip):
// Zhat staging as described above Step3Args; the template operand still
// covers q = 0 .. Qa/2 (Qa/2 + 1 slices).
size_t tmpl_prep_bytes(int nB, int M, int Qa, int precision);
size_t tmpl_prep_tile_bytes(size_t tiles, int M, int Qa, int precision);
// precision: 0 FP32, 1 split-bf16, 2 FP16, 3 split-fp16 (2 and 3: dscale[1]
// scales b)
hipError_t launch_tmpl_prep(const float2* b, void* out, int nB, int M, int Qa, int precision, const float* dscale,
                            hipStream_t stream);
// per-image template lists [.][K] for images a0 .. a0 + na - 1 of the call
hipError_t launch_tmpl_prep_lists(const float2* b, void* out, int nB, int M, int Qa, int precision,
                                  const float* dscale, const int* lists, int K, int na, int a0, hipStream_t stream);
size_t step1_v2_lds_bytes(int M, int zb, int precision);
hipError_t launch_step1_v2(const Step1Args& args, int precision, hipStream_t stream);

// Step 3 of the split forms (kern_align_bf16.hip): split bf16, or split fp16
// (fp16 = true; then args.xscale must be set)
size_t step3_bf16_lds_bytes(int Qa, int nwaves);
hipError_t launch_step3_bf16(const Step3Args& args, bool fp16, hipStream_t stream);

// FP16 form (kern_align_fp16.hip): Step 3 with one FP16 product per term
// (same LDS footprint as the split form), and the per-call data scales of the
// FP16 and split-fp16 forms: scales[0..1] = max |a|, max |b| (as float bits,
// reduced here), then scales[2] = 2^e_data / s_a, scales[3] = 2^e_data / s_b,
// scales[4] = s_a s_b s_y 2^e_x, scales[5] = 2^e_z, with s the power of two
// at or above each maximum (1 for an all-zero input).  The FP16 form uses
// e_data = e_x = e_z = 0; the split-fp16 form lifts its operands to the top
// of the fp16 range (kernels of kern_step1.hip multiply Step 1's FP32 result
// by 2^e_z before splitting it, and X is multiplied back by scales[4]).
// With Step3Args::rot16 set (Qa <= 256), Step 3 runs the two-tile kernel:
// the shift contraction transposed (Zhat as the A operand; the fp16 shift
// panel then has, per tile of 16 shifts, column 16 c + dl in place of row
// 2 dl + c) and the rotation transform on MFMA from the fp16 tables T_E, T_O
// of the even and odd modes, rows r < Qa/2:
//   T[r][q, c]: q = 0: 1 (c = 0), (-1)^r (c = 1);
//               q > 0: 2 cos(2 pi q r / Qa) (c = 0), 2 sin(...) (c = 1)
// stored as 1 KB fragments (parity p, row tile t, K step s) of the
// 16x16x32 MFMA's A operand: lane l, element e holds r = 16 t + l % 16,
// c = (l / 16) % 2, q = 32 s + 8 (e / 2) + 4 (l / 32) + 2 (e % 2) + p, at
// half index (((p Qa/32 + t) Qa/64 + s) 64 + l) 8 + e.
size_t step3_fp16_lds_bytes(int Qa, int nwaves);
size_t rot16_table_bytes(int Qa);  // 0 where the MFMA transform does not apply
size_t step3_fp16_rot_lds_bytes(int Qa, int nwaves);
hipError_t launch_step3_fp16(const Step3Args& args, hipStream_t stream);
hipError_t launch_fp16_scales(const float* a, size_t a_count, const float* b, size_t b_count, float s_y,
                              float* scales, int e_data, int e_x, int e_z, hipStream_t stream);

hipError_t launch_keys_init(unsigned long long* keys, size_t count, hipStream_t stream);
// vscale: device scalar multiplying the pose values (FP16 and split-fp16 forms), or null
hipError_t launch_keys_to_poses(const unsigned long long* keys, void* poses, size_t count, int Qa,
                                const float* vscale, hipStream_t stream);

// Brute-force translations (Section 6.2 of the paper), kern_bft.hip and
// launch_step1_bft.  Per image A and shift delta the translated coefficients
//   Ta[A][q][delta][m] = sum_p Ahat(k_m, psi_p) / Qa e^{-i k_m (dx cos psi_p + dy sin psi_p)} e^{-2 pi i q p / Qa}
// for q = 0 .. Qa/2 (Hermitian symmetry of a real image), zero for the
// padded shifts delta >= N; then Step 1 with zeta = delta, no mode offset
// and P_delta(m; q) = 2 pi w_m Ta gives Xhat(delta, q) directly in the
// FTK staging layout (H_pad = the padded shift count), and the rotation
// epilogue of Step 3 runs on it without a shift contraction.
struct BftTranslateArgs {
  const float2* polar;   // [nA][M][Qa] (TransformArgs::polar)
  float2* ta;            // [nA][Qa/2 + 1][N_pad][M]
  const float2* kd;      // [N][M]: (k_m dx, k_m dy) of shift delta, image units
  const float2* tw_qa;   // [Qa] exp(-2 pi i k / Qa)
  int nA, M, Qa, N, N_pad;
};
size_t bft_translate_lds_bytes(int Qa);
hipError_t launch_bft_translate(const BftTranslateArgs& args, hipStream_t stream);
// Step 1 on the translated coefficients (Step1Args::ta set, H_pad = N_pad,
// cz = [M] 2 pi w_m, zblk = 32, 64 or 128)
hipError_t launch_step1_bft(const Step1Args& args, hipStream_t stream);
// rotation FFT + argmax of Xhat read from HBM (Step3Args: zs = Xhat rows
// [pair][Qa/2][2][H_pad], X, xscale, keys, tw_qa, pairs, Qa, H_pad, N, up);
// one wave per 16 shifts of a pair, nwaves (<= 4) waves per workgroup.
// up = U > 1: U Qa rotations (X rows of U Qa values, pose index delta U Qa +
// rotation), as U passes of the Qa-point transform on phase-shifted Xhat.
size_t xhat_rotate_lds_bytes(int Qa, int nwaves, int up);
hipError_t launch_xhat_rotate(const Step3Args& args, hipStream_t stream);

// Brute-force rotations (Section 6.1, eq. 2dconv).  Spectra on the
// Cartesian disk grid k = pi (u, v), u^2 + v^2 <= V^2 (V = n / 2), stored as
// half-disk rows v = 0..V of Up complex values at j = u + V (zero outside
// the disk and for j > 2V), per image and rotation: out[img][R][V + 1][Up].
struct BfrSpectraArgs {
  const float2* grid;   // [cnt][nf][nf] fine grids of the transform's first stage ([l2][l1])
  float2* out;          // [cnt][R or 1][V + 1][Up]
  const double* cs;     // [R / 4] (cos, sin) of gamma_r = 2 pi r / R (quarter form only)
  int cnt, nf, w, V, Up, R;
  int quarter;          // 1: rotations r < R / 4 over the full disk, scattered to all R by quarter turns
  double s_per_u;       // fine-grid units per unit of u: pi dx / h
  float beta;           // spreading kernel shape
  float scale;          // the grid holds Ahat / Qa
  int patch;            // side of the LDS patch of fine grid per tile, >= bfr_spectra_patch(s_per_u)
};
int bfr_spectra_patch(double s_per_u);
hipError_t launch_bfr_spectra(const BfrSpectraArgs& args, hipStream_t stream);

// The correlation over the product grid of the requested shifts' x and y
// offsets: rows are images (64 per workgroup), columns (template, rotation,
// x offset) (32 per workgroup); per Fourier row v an MFMA sum over u, then
// the y offsets of the pass accumulated in registers; argmax keys and X.
constexpr int kBfrDy = 17;  // y offsets per pass
struct BfrCorrArgs {
  const float2* sa;     // image spectra [nA][V + 1][Up]
  const float2* sb;     // template spectra of the chunk [nBc][R][V + 1][Up]
  const float2* ex;     // [Dx][Up] exp(-2 pi i (j - V) x_ix / n)
  const float2* ey;     // [Dy_pad][V + 1] pi^2 c_v exp(-2 pi i v y_iy / n), c_0 = 1, c_v = 2
  const int4* chunks;   // [nch] (v, first j, K-steps of 4, last chunk of its row)
  const int* head;      // [Dx * Dy] lowest shift index at (x_ix, y_iy), -1 for none
  const int* nxt;       // [N] next shift index at the same point, -1 for none
  unsigned long long* keys;  // [nA][nB] pose keys (index shift * R + rotation)
  float* X;             // [nA][nB][N][R] or null
  int nA, nB, B0, nBc, R, Dx, Dy, iy0, N, V, Up, nch;
};
size_t bfr_corr_lds_bytes(int V);
hipError_t launch_bfr_corr(const BfrCorrArgs& args, hipStream_t stream);
