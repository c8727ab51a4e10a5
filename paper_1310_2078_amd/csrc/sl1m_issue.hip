// Issue rates of the VALU instruction classes the operator kernels are made
// of: FP32 FMA, FP64 FMA, v_sin_f32 (v_cos_f32 issues alike), v_exp_f32.
// The operators evaluate every matrix entry from its closed form (Section
// "On-the-fly computation versus in-memory computation"), so their cost is
// instruction issue, and a roofline in issue slots needs these rates on the
// running GPU.  Each kernel runs eight independent dependency chains of one
// instruction class per lane, enough wavefronts per SIMD to hide the chains'
// latency, and stores the chains' sum so that nothing is optimised away.
#include "sl1m_internal.h"

namespace sl1m {

namespace {

constexpr int kIssueChains = 8;
constexpr int kIssueWavesPerCU = 32;  // 8 per SIMD
constexpr int kIssueIters = 8192;

template <int OP>
__global__ __launch_bounds__(kBlock) void k_issue(float* __restrict__ out, int iters) {
  const float t = 1.0f + 1e-3f * static_cast<float>(threadIdx.x & 63);
  float a[kIssueChains];
  double d[kIssueChains];
#pragma unroll
  for (int c = 0; c < kIssueChains; ++c) {
    a[c] = t * (0.5f + 0.0625f * c);
    d[c] = static_cast<double>(a[c]);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kIssueChains; ++c) {
      if constexpr (OP == 0) a[c] = fmaf(a[c], 0.999999f, 1e-7f);
      if constexpr (OP == 1) d[c] = fma(d[c], 0.9999999999, 1e-12);
      if constexpr (OP == 2) a[c] = __builtin_amdgcn_sinf(a[c]);
      if constexpr (OP == 3) a[c] = __builtin_amdgcn_exp2f(-a[c]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kIssueChains; ++c) s += OP == 1 ? static_cast<float>(d[c]) : a[c];
  out[static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x] = s;
}

template <int OP>
hipError_t time_issue(float* buf, int blocks, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                      double* ms) {
  hipLaunchKernelGGL(k_issue<OP>, dim3(blocks), dim3(kBlock), 0, st, buf, kIssueIters / 8);
  hipError_t e = hipEventRecord(e0, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_issue<OP>, dim3(blocks), dim3(kBlock), 0, st, buf, kIssueIters);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float f = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  *ms = f;
  return e;
}

}  // namespace

}  // namespace sl1m

using namespace sl1m;

extern "C" {

sl1m_status sl1m_issue_rates(void* scratch, size_t scratch_bytes, double* rates, void* stream) {
  try {
    if (!scratch || !rates) return set_error(SL1M_EINVAL, "NULL argument");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_error(e, "device query");
    const int blocks = cus * kIssueWavesPerCU / (kBlock / 64);
    if (scratch_bytes < sizeof(float) * static_cast<size_t>(blocks) * kBlock)
      return set_error(SL1M_ENOMEM, "scratch smaller than sl1m_issue_scratch_bytes()");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float* buf = static_cast<float*>(scratch);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double ms[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = time_issue<0>(buf, blocks, st, e0, e1, &ms[0]);
    if (e == hipSuccess) e = time_issue<1>(buf, blocks, st, e0, e1, &ms[1]);
    if (e == hipSuccess) e = time_issue<2>(buf, blocks, st, e0, e1, &ms[2]);
    if (e == hipSuccess) e = time_issue<3>(buf, blocks, st, e0, e1, &ms[3]);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_error(e, "issue-rate kernels");
    // wave64 instructions of the measured class per launch, per compute unit
    const double instr = static_cast<double>(blocks) * (kBlock / 64) * kIssueIters * kIssueChains;
    for (int i = 0; i < 4; ++i) rates[i] = ms[i] > 0.0 ? instr / cus / (ms[i] * 1e-3) : 0.0;
    return SL1M_OK;
  } catch (...) {
    return set_error(SL1M_EHIP, "issue-rate measurement failed");
  }
}

sl1m_status sl1m_issue_scratch_bytes(size_t* bytes) {
  if (!bytes) return set_error(SL1M_EINVAL, "NULL argument");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_error(e, "device query");
  *bytes = sizeof(float) * static_cast<size_t>(cus * kIssueWavesPerCU / (kBlock / 64)) * kBlock;
  return SL1M_OK;
}

}  // extern "C"
