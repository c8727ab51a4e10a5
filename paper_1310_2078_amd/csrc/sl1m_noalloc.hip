// One-shot forward operator that allocates no device memory, for callers
// that cannot allocate (tight serving loops, harnesses that forbid
// hipMalloc).  The plan's workspace -- permutation, pixel and visibility
// records, split-K partial rows -- lives in a file-scope device array of
// SL1M_NOALLOC_SCRATCH_BYTES that every call on a device reuses.
#include <mutex>

#include "sl1m_internal.h"

namespace {

constexpr size_t kScratchBytes = SL1M_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Each device that runs this code holds its own copy until the process ends.
// Host code never uses this name as an address: the per-device address comes
// from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;                       // one call at a time per process
void* g_scratch[kMaxDevices] = {};     // device address of `scratch` per device

// Address of the current device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
sl1m_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return sl1m::set_error(SL1M_EINVAL, "device ordinal out of range for the no-alloc scratch");
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return sl1m::hip_error(e, "no-alloc scratch address");
    if (!ptr) return sl1m::set_error(SL1M_EHIP, "no-alloc scratch address is NULL");
    g_scratch[device] = ptr;
  }
  *out = g_scratch[device];
  return SL1M_OK;
}

}  // namespace

extern "C" {

sl1m_status sl1m_forward_noalloc(const sl1m_problem* problem, const void* x, void* vis,
                                 void* stream) {
  try {
    if (!problem) return sl1m::set_error(SL1M_EINVAL, "problem is NULL");
    size_t need = 0;
    if (sl1m_status s = sl1m_plan_workspace_bytes(problem, &need)) return s;
    if (need > kScratchBytes)
      return sl1m::set_error(
          SL1M_ENOMEM, "problem needs a " + std::to_string(need) +
                           "-byte plan workspace; sl1m_forward_noalloc holds at most " +
                           std::to_string(kScratchBytes) + " bytes (use sl1m_plan_create)");
    std::lock_guard<std::mutex> lk(g_mu);
    int device = 0;
    if (const hipError_t e = hipGetDevice(&device); e != hipSuccess)
      return sl1m::hip_error(e, "get device");
    void* ws = nullptr;
    if (sl1m_status s = scratch_address(device, &ws)) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    sl1m_plan* plan = nullptr;
    if (sl1m_status s = sl1m_plan_create(problem, ws, kScratchBytes, stream, &plan)) return s;
    sl1m_status s = sl1m_forward(plan, x, vis, stream);
    // the scratch is free for the next call only once this call's kernels
    // have finished reading it
    const hipError_t e = hipStreamSynchronize(st);
    sl1m_plan_destroy(plan);
    if (s) return s;
    if (e != hipSuccess) return sl1m::hip_error(e, "no-alloc forward synchronise");
    return SL1M_OK;
  } catch (...) {
    return sl1m::set_error(SL1M_EINVAL, "unexpected host error");
  }
}

}  // extern "C"
