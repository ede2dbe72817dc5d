// Two-pass alignment: a coarse plan (for example the FP16 form) over every
// pair, then, per image, the k templates with the largest coarse best values
// aligned again by a fine plan (for example the split-bf16 form).  The pair's
// best pose is the argmax of eq. fbk3's X over shifts and rotations in both
// passes; the fine pass only replaces the coarse poses of the listed pairs.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ftk_mlp.h"
#include "mlp_kernels.h"
#include "plan_internal.h"

using namespace ftkint;

namespace {

constexpr int kThreads = 256;

struct PoseR {
  float value;
  int32_t shift;
  int32_t rot;
};

// larger value first, then the lower template number; NaN ranks last
__device__ __forceinline__ bool before(float v, int i, float w, int j) { return v > w || (v == w && i < j); }
__device__ __forceinline__ float clean(float x) { return (x == x) ? x : -__builtin_inff(); }

// per image (one workgroup): the k templates with the largest pose values,
// in rank order, by k block-wide selections of the best remaining entry
__global__ void __launch_bounds__(kThreads) pose_topk_kernel(const PoseR* __restrict__ best, int nB, int k,
                                                             int32_t* __restrict__ lists) {
  __shared__ float rv[kThreads / 64];
  __shared__ int ri[kThreads / 64];
  const PoseR* row = best + static_cast<size_t>(blockIdx.x) * nB;
  float pv = __builtin_inff();
  int pi = -1;
  for (int r = 0; r < k; ++r) {
    float bv = -__builtin_inff();
    int bi = 0x7fffffff;
    for (int j = threadIdx.x; j < nB; j += kThreads) {
      const float v = clean(row[j].value);
      if (before(pv, pi, v, j) && before(v, j, bv, bi)) {
        bv = v;
        bi = j;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float ov = __shfl_xor(bv, o);
      const int oi = __shfl_xor(bi, o);
      if (before(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
      }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      rv[threadIdx.x >> 6] = bv;
      ri[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    bv = rv[0];
    bi = ri[0];
    for (int w = 1; w < kThreads / 64; ++w)
      if (before(rv[w], ri[w], bv, bi)) {
        bv = rv[w];
        bi = ri[w];
      }
    if (threadIdx.x == 0) lists[static_cast<size_t>(blockIdx.x) * k + r] = bi;
    pv = bv;
    pi = bi;
  }
}

// best[i][lists[i][j]] = refined[i][j]
__global__ void scatter_poses_kernel(const PoseR* __restrict__ refined, const int32_t* __restrict__ lists, int nA,
                                     int k, int nB, PoseR* __restrict__ best) {
  const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<size_t>(nA) * k) return;
  const size_t i = t / k;
  const int j = lists[t];
  if (j >= 0 && j < nB) best[i * nB + j] = refined[t];
}

// The two passes read the same coefficients and shifts; their factorisations
// (eps, k-side weight, hence H) may differ: the coarse pass may use a cheaper
// one, the fine pass gives the refined values.
bool same_shape(const ftk_plan* a, const ftk_plan* b) {
  return a->n == b->n && a->M == b->M && a->Qa == b->Qa && a->up == b->up && a->W == b->W && a->N == b->N;
}

}  // namespace

extern "C" {

int ftk_align_refined(ftk_plan* coarse, ftk_plan* fine, const void* img_coeffs, int nA, const void* tmpl_coeffs,
                      int nB, int k, ftk_pose* best, int32_t* best_t, ftk_pose* best_pose, void* stream) {
  if (!coarse || !fine) return fail(FTK_EINVAL, "ftk_align_refined: NULL plan");
  if (nA < 0 || nB < 0) return fail(FTK_EINVAL, "ftk_align_refined: negative count");
  if (coarse->N <= 0 || fine->N <= 0) return fail(FTK_ESTATE, "ftk_align_refined: call ftk_set_shifts first");
  if (!same_shape(coarse, fine)) return fail(FTK_EINVAL, "ftk_align_refined: the plans differ in n, K, Q, rotations, W or N");
  if (nA == 0 || nB == 0) return FTK_OK;
  if (k < 1 || k > 64 || k > nB) return fail(FTK_EINVAL, "ftk_align_refined: k must be in [1, min(nB, 64)]");
  if (!img_coeffs || !tmpl_coeffs || !best) return fail(FTK_EINVAL, "ftk_align_refined: NULL buffer");
  if ((best_t == nullptr) != (best_pose == nullptr))
    return fail(FTK_EINVAL, "ftk_align_refined: best_t and best_pose go together");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = ftk_align_coeffs(coarse, img_coeffs, nA, tmpl_coeffs, nB, nullptr, best, stream);
  if (rc != FTK_OK) return rc;
  // lists [nA][k] int32, then the refined poses [nA][k]
  const size_t n = static_cast<size_t>(nA) * k;
  const size_t lbytes = (n * sizeof(int32_t) + 255) / 256 * 256;
  Workspace& ws = *fine->ws;
  if (ws.refine.ensure(lbytes + n * sizeof(ftk_pose)) != hipSuccess)
    return fail(FTK_ENOMEM, "ftk_align_refined: list buffer");
  int32_t* lists = ws.refine.as<int32_t>();
  ftk_pose* refined = reinterpret_cast<ftk_pose*>(static_cast<char*>(ws.refine.ptr) + lbytes);
  hipLaunchKernelGGL(pose_topk_kernel, dim3(nA), dim3(kThreads), 0, s, reinterpret_cast<const PoseR*>(best), nB, k,
                     lists);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "ftk_align_refined: top-k");
  rc = ftk_align_lists(fine, img_coeffs, nA, tmpl_coeffs, nB, lists, k, refined, stream);
  if (rc != FTK_OK) return rc;
  hipLaunchKernelGGL(scatter_poses_kernel, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     reinterpret_cast<const PoseR*>(refined), lists, nA, k, nB, reinterpret_cast<PoseR*>(best));
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "ftk_align_refined: scatter");
  if (best_t && (e = launch_best_template(refined, lists, nA, k, best_t, best_pose, s)) != hipSuccess)
    return hip_fail(e, "ftk_align_refined: best template");
  return FTK_OK;
}

}  // extern "C"
