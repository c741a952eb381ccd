// Calibration kernels: attainable matrix-core rate and HBM bandwidth of the
// device, measured with the instruction shapes the solver uses
// (helm_device_peaks).
#include <algorithm>
#include <cstring>

#include "api_common.h"

namespace helm {
namespace kern {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int PROBE_CHAINS = 8;   // independent accumulators per wave

// back-to-back 16x16x4 MFMAs on PROBE_CHAINS independent accumulators
__global__ void __launch_bounds__(256) k_probe_mfma_f32(float* out, int iters) {
  v4f acc[PROBE_CHAINS];
  for (int j = 0; j < PROBE_CHAINS; ++j) acc[j] = v4f{0, 0, 0, 0};
  const float a = threadIdx.x * 1e-3f, b = 1.0001f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < PROBE_CHAINS; ++j)
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
  }
  float s = 0;
  for (int j = 0; j < PROBE_CHAINS; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void __launch_bounds__(256) k_probe_mfma_f64(double* out, int iters) {
  v4d acc[PROBE_CHAINS];
  for (int j = 0; j < PROBE_CHAINS; ++j) acc[j] = v4d{0, 0, 0, 0};
  const double a = threadIdx.x * 1e-3, b = 1.0001;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < PROBE_CHAINS; ++j)
      acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  }
  double s = 0;
  for (int j = 0; j < PROBE_CHAINS; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
// streaming read (sum per thread) and copy, 16-byte accesses, grid-stride
__global__ void __launch_bounds__(256) k_probe_read(const float4* __restrict__ x, float* out,
                                                    long long n) {
  const long long st = (long long)gridDim.x * 256;
  float s = 0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += st) {
    const float4 v = x[i];
    s += v.x + v.y + v.z + v.w;
  }
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ void __launch_bounds__(256) k_probe_copy(const float4* __restrict__ x,
                                                    float4* __restrict__ y, long long n) {
  constexpr int U = 4;
  const long long st = (long long)gridDim.x * 256 * U;
  for (long long i = blockIdx.x * 256LL * U + threadIdx.x; i < n; i += st) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = (i + u * 256 < n) ? x[i + u * 256] : float4{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * 256 < n) y[i + u * 256] = v[u];
  }
}

}  // namespace
}  // namespace kern
}  // namespace helm

using namespace helm;

extern "C" int helm_device_peaks(int device, double* mfma_f32_tflops, double* mfma_f64_tflops,
                                 double* hbm_read_gbps, double* hbm_copy_gbps) {
  return guard([&] {
    HELM_HIP(hipSetDevice(device));
    struct OwnedStream {
      hipStream_t s = nullptr;
      ~OwnedStream() {
        if (s) {
          (void)hipStreamSynchronize(s);
          (void)hipStreamDestroy(s);
        }
      }
    } os;
    HELM_HIP(hipStreamCreate(&os.s));
    hipStream_t st = os.s;
    EventPair ev;
    int cus = 0;
    HELM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    const int blocks = std::max(1, cus) * 8, threads = 256;
    const long long bytes = 2LL << 30;   // 2 GiB per buffer
    const long long n4 = bytes / 16;
    DevMem out, x, y;
    out.alloc((size_t)blocks * 64 * threads * sizeof(double));
    x.alloc((size_t)bytes);
    y.alloc((size_t)bytes);
    HELM_HIP(hipMemsetAsync(x.p, 0, (size_t)bytes, st));
    auto best_ms = [&](auto&& launch) {
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HELM_HIP(hipEventRecord(ev.a, st));
        launch();
        HELM_HIP(hipEventRecord(ev.b, st));
        best = std::min(best, (float)ev.elapsed_ms(st));
      }
      return (double)best;
    };
    const int iters = 4000;
    const double mfma_flops = (double)blocks * 4 * iters * kern::PROBE_CHAINS * 2048.0;
    double ms = best_ms([&] {
      hipLaunchKernelGGL(kern::k_probe_mfma_f32, dim3(blocks), dim3(threads), 0, st,
                         out.as<float>(), iters);
    });
    if (mfma_f32_tflops) *mfma_f32_tflops = mfma_flops / ms / 1e9;
    ms = best_ms([&] {
      hipLaunchKernelGGL(kern::k_probe_mfma_f64, dim3(blocks), dim3(threads), 0, st,
                         out.as<double>(), iters);
    });
    if (mfma_f64_tflops) *mfma_f64_tflops = mfma_flops / ms / 1e9;
    const int sgrid = std::max(1, cus) * 4;
    ms = best_ms([&] {
      hipLaunchKernelGGL(kern::k_probe_read, dim3(sgrid), dim3(256), 0, st,
                         x.as<const float4>(), out.as<float>(), n4);
    });
    if (hbm_read_gbps) *hbm_read_gbps = (double)bytes / ms / 1e6;
    ms = best_ms([&] {
      hipLaunchKernelGGL(kern::k_probe_copy, dim3(std::max(1, cus) * 64), dim3(256), 0, st,
                         x.as<const float4>(), y.as<float4>(), n4);
    });
    if (hbm_copy_gbps) *hbm_copy_gbps = 2.0 * (double)bytes / ms / 1e6;
    HELM_HIP(hipGetLastError());
    HELM_HIP(hipStreamSynchronize(st));
    return HELM_OK;
  });
}
