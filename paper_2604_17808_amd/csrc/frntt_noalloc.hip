// The allocation-free transform entry point: for callers that cannot
// allocate (code under hipGraph stream capture, tight serving loops, harnesses
// that forbid hipMalloc). Its passes ping-pong through a file-scope device
// array instead of context scratch, and its pass twiddles come from the split
// tables built at context creation, so nothing is allocated or built on any
// call.
#include <hip/hip_runtime.h>

#include "frntt_internal.hpp"

namespace frntt {

// 2^20 elements (32 MiB): one transform of up to 2^20 elements, or a batch of
// smaller ones. Every GPU the library runs on holds its own copy until the
// process ends.
constexpr size_t kNoallocMaxElems = size_t(1) << kNoallocMaxLog;
static __device__ __align__(256) u32x4 scratch[2 * kNoallocMaxElems];

// Device address of this GPU's copy of `scratch` (the array's name is a host
// stand-in, not a device address). Called once per context, with the
// context's device current.
int noalloc_scratch_address(void** out) {
  *out = nullptr;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  *out = p;
  return 0;
}

int transform_noalloc(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, hipStream_t stream) {
  if (!ctx || (!data && batch > 0)) return FRNTT_EINVAL;
  if (batch < 0 || kind < FRNTT_FWD || kind > FRNTT_COSET_INV) return FRNTT_EINVAL;
  if (log_n < 0 || log_n > ctx->max_log_n || log_n > kMasterLog) return FRNTT_ERANGE;
  if (((uintptr_t)data & 31) != 0) return FRNTT_EALIGN;
  if (batch == 0) return FRNTT_OK;
  if ((((int64_t)batch) << log_n) > (int64_t)kNoallocMaxElems) return FRNTT_ERANGE;
  if (!ctx->noalloc_scratch) return FRNTT_ESTATE;
  if (ctx->flags & FRNTT_VALIDATE) {
    const uint64_t count = (uint64_t)batch << log_n;
    hipLaunchKernelGGL(validate_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       (const u32x4*)data, count, ctx->valid_flag);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(ctx, e);
  }
  if (log_n == 0) return FRNTT_OK;  // identity
  int algo = 0;
  Plan plan;
  resolve_plan(ctx, FRNTT_ALGO_AUTO, log_n, &algo, &plan);
  PassParams passes[4];
  int n = 0;
  const int rc = build_passes_into(ctx, plan, log_n, batch, kind, data, ctx->noalloc_scratch, passes, &n, algo,
                                   /*capturing=*/true, /*no_tables=*/true);
  if (rc) return rc;
  return launch_passes(ctx, passes, n, algo, stream);
}

}  // namespace frntt

extern "C" int ntt_transform_noalloc(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, void* stream) {
  return frntt::transform_noalloc(ctx, data, log_n, batch, kind, (hipStream_t)stream);
}
