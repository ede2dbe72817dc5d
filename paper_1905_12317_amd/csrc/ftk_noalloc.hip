// ftk_align_coeffs_noalloc: Steps 1-3 and the argmax with every buffer the
// call needs (Zhat staging, pose keys, the Step 1 template operand, the data
// scales of the fp16 forms) carved from one fixed device array, so that the
// call allocates no device memory.  The kernels and their order are those of
// ftk_align_coeffs; only the staging may hold fewer images per chunk, which
// does not change any result (each pair's sums run in the same order).
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan_internal.h"

using namespace ftkint;

namespace {

// The fixed scratch.  Host code never passes this name to a kernel or a
// copy: on the host it is only a stand-in for the symbol; its device address
// (one copy per GPU) comes from hipGetSymbolAddress below.
__device__ __align__(256) unsigned char scratch[FTK_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the scratch on the current device, looked up once per
// device with that device current.
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "ftk_align_coeffs_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(FTK_EDEVICE, "ftk_align_coeffs_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "ftk_align_coeffs_noalloc: hipGetSymbolAddress");
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return FTK_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" {

int ftk_align_coeffs_noalloc(ftk_plan* p, const void* img_coeffs, int nA, const void* tmpl_coeffs, int nB, float* X,
                             ftk_pose* best, void* stream) {
  if (!p) return fail(FTK_EINVAL, "ftk_align_coeffs_noalloc: NULL plan");
  if (nA < 0 || nB < 0) return fail(FTK_EINVAL, "ftk_align_coeffs_noalloc: negative count");
  if (p->N <= 0) return fail(FTK_ESTATE, "ftk_align_coeffs_noalloc: call ftk_set_shifts first");
  if (nA == 0 || nB == 0) return FTK_OK;
  if (!X && !best) return fail(FTK_EINVAL, "ftk_align_coeffs_noalloc: X and best are both NULL");
  if (!img_coeffs || !tmpl_coeffs) return fail(FTK_EINVAL, "ftk_align_coeffs_noalloc: NULL coefficients");
  if (p->up > 1) return fail(FTK_EUNSUPPORTED, "ftk_align_coeffs_noalloc: rotation upsampling is not available");
  // layout of the scratch: pose keys, template operand, data scales, staging
  const int prec = prec_code(p);
  const size_t keys = align256(static_cast<size_t>(nA) * nB * sizeof(unsigned long long));
  const size_t tmpl = align256(tmpl_prep_bytes(nB, p->M, p->Qa, prec));
  const size_t scl = (prec == 2 || prec == 3) ? 256 : 0;
  const size_t per_image = stage_bytes_per_pair(p) * static_cast<size_t>(nB);
  const size_t fixed = keys + tmpl + scl;
  if (fixed > FTK_NOALLOC_SCRATCH_BYTES || FTK_NOALLOC_SCRATCH_BYTES - fixed < per_image)
    return fail(FTK_EUNSUPPORTED, "ftk_align_coeffs_noalloc: the call needs more than the fixed scratch of " +
                                      std::to_string(FTK_NOALLOC_SCRATCH_BYTES) + " bytes (pose keys " +
                                      std::to_string(keys) + ", template operand " + std::to_string(tmpl) +
                                      ", staging of one image " + std::to_string(per_image) + ")");
  void* base = nullptr;
  const int rc = scratch_address(&base);
  if (rc != FTK_OK) return rc;
  unsigned char* b = static_cast<unsigned char*>(base);
  const size_t room = FTK_NOALLOC_SCRATCH_BYTES - fixed;
  const AlignBufs buf{b + fixed, reinterpret_cast<unsigned long long*>(b), b + keys,
                      scl ? reinterpret_cast<float*>(b + keys + tmpl) : nullptr,
                      static_cast<int>(std::min<size_t>(static_cast<size_t>(nA), room / per_image)), nullptr};
  return align_run(p, img_coeffs, nA, tmpl_coeffs, nB, nullptr, 0, X, best, buf, nullptr, stream);
}

}  // extern "C"
