// Internal interface of the template-proposal kernels (kern_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// C[i][j] = sum_k A(i, k) B(k, j) with A(i, k) = A[i sai + k sak] and
// B(k, j) = B[k sbk + j sbj] (one of sai/sak and one of sbk/sbj must be 1),
// FP32 accumulation; epilogue z = acc + bias[j], z *= (mask[i][j] > 0) if
// mask, C = z (FP32) if C, Cb = relu(z) or z (operand type) if Cb.
struct GemmArgs {
  const void* A;
  const void* B;
  int M, N, K;
  long long sai, sak, sbk, sbj;
  float* C;
  long long ldc;
  void* Cb;
  long long ldcb;
  const float* bias;
  const float* mask;
  long long ldm;
  int relu;
  float* part;         // bf16 GEMMs split over K: FP32 partial sums (gemm_part_floats), or null
  size_t part_floats;
};

// Launch shape of a bf16 GEMM: 128 x 128 tiles when there are at least 256
// of them, else 64 x 64; K split into kparts when the grid is small.
struct GemmPlan {
  bool big = false;
  int kparts = 1;
};
GemmPlan gemm_plan(int M, int N, int K);
// FP32 workspace a bf16 GEMM of this shape needs for its K parts (0: none)
size_t gemm_part_floats(int M, int N, int K);

// bf16 = 1: operands are bf16 (v_mfma_f32_32x32x16_bf16); 0: FP32 operands
// (v_mfma_f32_32x32x2_f32).
hipError_t launch_gemm(const GemmArgs& g, int bf16, hipStream_t s);

// X[b][f] = (x[row][f] - mu[f]) * inv_sigma[f], row = idx ? idx[b] : b,
// written in the operand type.
hipError_t launch_standardise(const float* x, const int32_t* idx, int B, int D, const float* mu,
                              const float* inv_sigma, void* X, int bf16, hipStream_t s);

// Two-head softmax cross-entropy, one row per workgroup: labels of row b are
// lab_t[r], lab_s[r] with r = idx ? idx[b] : b.  dZ = (softmax - onehot) / B
// (FP32 and operand-type copies), row_loss[b] = CE_t + CE_s.
hipError_t launch_softmax_ce(const float* logits, int B, int D, int ldz, int n_t, int n_s, const int32_t* lab_t,
                             const int32_t* lab_s, const int32_t* idx, float* dZ, void* dZb, int bf16,
                             float* row_loss, hipStream_t s);
// loss = sum(row_loss[0..B)) / B, one workgroup, fixed order.
hipError_t launch_mean(const float* row_loss, int B, float* loss, hipStream_t s);
// db[j] = sum_b dZ[b][j]
hipError_t launch_colsum(const float* dZ, int B, int N, int ld, float* db, hipStream_t s);
// AdamW on n parameters; refreshes the operand-type copy wc if non-null.
hipError_t launch_adamw(float* w, const float* g, float* m, float* v, size_t n, float lr, float beta1, float beta2,
                        float eps, float wd, float bc1, float bc2, void* wc, int bf16, hipStream_t s);
// Copy FP32 -> operand type.
hipError_t launch_convert(const float* w, size_t n, void* wc, int bf16, hipStream_t s);
// kind 0: F[a][m n_q + q] = |coeffs[a][q][m]|^2; kind 1: signed square roots
// of the cross-ring products a(k1; q) conj a(k2; q) (n_q blocks of n_r^2)
hipError_t launch_features(const float2* coeffs, int nA, int Qa, int M, int kind, int n_r, int n_q, float* F,
                           hipStream_t s);
// per row: top-k template logits (ties to the lower index), their softmax
// mass over the template head, and the argmax of the shift head
hipError_t launch_topk(const float* logits, int rows, int D, int n_t, int n_s, int k, int32_t* top, float* mass,
                       int32_t* sbin, hipStream_t s);
// best template per row from per-pair poses (value, shift, rot)
hipError_t launch_best_template(const void* poses, const int32_t* lists, int nA, int K, int32_t* best_t,
                                void* best_pose, hipStream_t s);
// rows with mass < tau, in increasing order: list[0..count), count[0]
hipError_t launch_select_below(const float* mass, int nA, float tau, int32_t* list, int32_t* count, int32_t* flag,
                               hipStream_t s);
// dst[i] = src[list[i]] for rows of `row_bytes` bytes (multiple of 8)
hipError_t launch_gather_rows(const void* src, const int32_t* list, int count, size_t row_bytes, void* dst,
                              hipStream_t s);
// dst[i] = src[list[i]] for rows of row_words 4-byte words
hipError_t launch_gather_words(const void* src, const int32_t* list, int count, size_t row_words, void* dst,
                               hipStream_t s);
// dst[list[i]][j] = src[i][j] for pose rows of K poses, shift indices mapped
// through map (or kept when map is null)
hipError_t launch_scatter_poses(const void* src, const int32_t* list, int count, int K, const int32_t* map, void* dst,
                                hipStream_t s);
// dst[list[i]] = src[i] for int32 and 12-byte pose rows
hipError_t launch_scatter_results(const int32_t* bt, const void* bp, const int32_t* list, int count, int32_t* dst_t,
                                  void* dst_p, hipStream_t s);
