// Measured ceilings of the device: the empirical counterpart of the
// roofline (section "Roofline Model", which measures its CPU's peaks with
// a microbenchmark instead of taking the data sheet's).  Each probe runs
// one small kernel long enough to fill every compute unit and times it with
// HIP events:
//   FMA:  eight independent chains of FMAs with a constant multiplier and
//         addend, which the compiler encodes in the two-operand (VOP2)
//         form v_fmamk_f32;
//   FMA_VOP3: the same chains with both operands in registers, encoded as
//         the three-operand (VOP3) v_fma_f32, which issues at half the
//         rate of the VOP2 form on gfx950;
//   EXP:  eight independent chains x <- 2^-x (v_exp_f32 with a negated
//         source, which costs nothing);
//   RCP:  eight independent chains x <- 1/x (v_rcp_f32);
//   LOG:  eight chains x <- -log2(2^-x) alternating v_exp_f32 and
//         v_log_f32, both counted (with the EXP rate the caller separates
//         the two);
//   COPY: a device-to-device copy of `bytes` with 16-byte vector loads and
//         stores, counted as bytes read plus bytes written;
//   MFMA: four independent accumulators of v_mfma_f32_16x16x32_bf16 per
//         wave, 16 x 16 x 32 x 2 FLOP each.
// Results are written out under a condition the device cannot know to be
// false, so the chains are not optimized away.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fib.h"

namespace fib {
int set_error(int code, const char* msg);

namespace {

constexpr int kChains = 8;
constexpr int kBlocks = 256 * 64;  // 64 workgroups of 256 threads per compute unit
constexpr int kThreads = 256;

template <int KIND>
__global__ __launch_bounds__(kThreads) void k_probe_valu(int iters, float seed, float* sink) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * (float)c + 1e-7f * (float)threadIdx.x;
  const float b = 0.999f, d = 1e-3f;
  // the same constants in registers the compiler cannot see through
  float rb = b, rd = d;
  asm volatile("" : "+v"(rb), "+v"(rd));
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        if constexpr (KIND == FIB_PROBE_FMA) x[c] = fmaf(x[c], b, d);
        if constexpr (KIND == FIB_PROBE_FMA_VOP3) x[c] = fmaf(x[c], rb, rd);
        if constexpr (KIND == FIB_PROBE_EXP) x[c] = __builtin_amdgcn_exp2f(-x[c]);
        if constexpr (KIND == FIB_PROBE_RCP) x[c] = __builtin_amdgcn_rcpf(x[c]);
        if constexpr (KIND == FIB_PROBE_LOG)
          x[c] = -__builtin_amdgcn_logf(__builtin_amdgcn_exp2f(-x[c]));
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  if (s == 12345.678f) sink[blockIdx.x * kThreads + threadIdx.x] = s;
}

// Four 16-byte loads in flight per thread before their stores; n is a
// multiple of 4 * blockDim.x * gridDim.x is not required (the tail is
// guarded).
__global__ __launch_bounds__(256) void k_probe_copy(const uint4* __restrict__ src,
                                                    uint4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float seed, float* sink) {
  v8bf a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(seed + 0.001f * (float)(threadIdx.x + e));
    b[e] = (__bf16)(seed - 0.002f * (float)e);
  }
  v4f acc[4] = {};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  if (s == 12345.678f) sink[blockIdx.x * 256 + threadIdx.x] = s;
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  bool ok() const { return a && b; }
  Timer() {
    if (hipEventCreate(&a) != hipSuccess) a = nullptr;
    if (hipEventCreate(&b) != hipSuccess) b = nullptr;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace
}  // namespace fib

extern "C" int fib_probe(int32_t kind, int64_t bytes, double* rate) {
  using namespace fib;
  if (!rate) return set_error(FIB_EINVAL, "null output");
  *rate = 0.0;
  if (kind < FIB_PROBE_FMA || kind > FIB_PROBE_FMA_VOP3)
    return set_error(FIB_EINVAL, "unknown probe");
  if (kind == FIB_PROBE_COPY && (bytes < (1 << 20) || bytes > ((int64_t)64 << 30)))
    return set_error(FIB_EINVAL, "copy probe size must lie in [1 MiB, 64 GiB]");
  Timer t;
  if (!t.ok()) return set_error(FIB_EHIP, "hipEventCreate failed");
  float* sink = nullptr;
  void *src = nullptr, *dst = nullptr;
  const int iters = kind == FIB_PROBE_MFMA_BF16 ? 32 : 1024;
  double ops = 0.0, ms = 0.0;
  hipError_t e = hipSuccess;
  auto run = [&](auto launch) -> hipError_t {
    launch();  // warm-up: code object load, clocks
    hipError_t r = hipDeviceSynchronize();
    if (r != hipSuccess) return r;
    if ((r = hipEventRecord(t.a, nullptr)) != hipSuccess) return r;
    launch();
    if ((r = hipEventRecord(t.b, nullptr)) != hipSuccess) return r;
    if ((r = hipEventSynchronize(t.b)) != hipSuccess) return r;
    float f = 0.0f;
    r = hipEventElapsedTime(&f, t.a, t.b);
    ms = f;
    return r;
  };
  if (kind == FIB_PROBE_COPY) {
    const int64_t n = bytes / 16;
    if (hipMalloc(&src, (size_t)n * 16) != hipSuccess || hipMalloc(&dst, (size_t)n * 16) != hipSuccess) {
      (void)hipFree(src);
      return set_error(FIB_ENOMEM, "probe buffers");
    }
    e = hipMemset(src, 0, (size_t)n * 16);
    if (e == hipSuccess)
      e = run([&] {
        hipLaunchKernelGGL(k_probe_copy, dim3(256 * 32), dim3(256), 0, nullptr,
                           (const uint4*)src, (uint4*)dst, n);
      });
    ops = 2.0 * 16.0 * (double)n;
  } else {
    if (hipMalloc(&sink, sizeof(float) * kBlocks * kThreads) != hipSuccess)
      return set_error(FIB_ENOMEM, "probe buffer");
    const double lanes = (double)kBlocks * kThreads;
    if (kind == FIB_PROBE_MFMA_BF16) {
      e = run([&] { hipLaunchKernelGGL(k_probe_mfma, dim3(kBlocks), dim3(256), 0, nullptr, iters, 0.5f, sink); });
      ops = (double)kBlocks * 4.0 /* waves */ * iters * 8.0 * 4.0 * 16.0 * 16.0 * 32.0 * 2.0;
    } else {
      const double per_lane = (double)iters * 8.0 * kChains;
      if (kind == FIB_PROBE_FMA)
        e = run([&] { hipLaunchKernelGGL(k_probe_valu<FIB_PROBE_FMA>, dim3(kBlocks), dim3(kThreads), 0, nullptr, iters, 0.5f, sink); });
      if (kind == FIB_PROBE_FMA_VOP3)
        e = run([&] { hipLaunchKernelGGL(k_probe_valu<FIB_PROBE_FMA_VOP3>, dim3(kBlocks), dim3(kThreads), 0, nullptr, iters, 0.5f, sink); });
      if (kind == FIB_PROBE_EXP)
        e = run([&] { hipLaunchKernelGGL(k_probe_valu<FIB_PROBE_EXP>, dim3(kBlocks), dim3(kThreads), 0, nullptr, iters, 0.5f, sink); });
      if (kind == FIB_PROBE_RCP)
        e = run([&] { hipLaunchKernelGGL(k_probe_valu<FIB_PROBE_RCP>, dim3(kBlocks), dim3(kThreads), 0, nullptr, iters, 0.5f, sink); });
      if (kind == FIB_PROBE_LOG)
        e = run([&] { hipLaunchKernelGGL(k_probe_valu<FIB_PROBE_LOG>, dim3(kBlocks), dim3(kThreads), 0, nullptr, iters, 0.5f, sink); });
      ops = lanes * per_lane * (kind == FIB_PROBE_LOG ? 2.0 : 1.0);
    }
  }
  if (e == hipSuccess) e = hipGetLastError();
  (void)hipFree(sink);
  (void)hipFree(src);
  (void)hipFree(dst);
  if (e != hipSuccess) return set_error(FIB_EHIP, hipGetErrorString(e));
  if (!(ms > 0.0)) return set_error(FIB_EHIP, "probe took no measurable time");
  *rate = ops / (ms * 1e-3);
  return FIB_OK;
}
