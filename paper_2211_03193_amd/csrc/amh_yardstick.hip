// amh_yardstick.hip -- achievable-bandwidth yardsticks for the roofline of the sweep
// kernel (declared in include/amh_yardstick.h).  They are not part of the sampler:
// they measure, on the GPU at hand, what the memory system delivers to the access
// patterns the sweep kernel uses (Sec. 2.4 maps the pair sums of the energy onto the
// GPU; here those pair sums gather 16-byte spline stencils from the distogram table).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "amh.h"
#include "amh_yardstick.h"

namespace {

// Streaming read of n float4 (grid-stride, coalesced); one float per thread is
// written so that the loads stay live.
__global__ void stream_kernel(const float4* __restrict__ src, int64_t n, float* __restrict__ sink) {
  float acc = 0.0f;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = src[e];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// 32-bit mixing step (xorshift-multiply), used only to spread the gathers.
__device__ __forceinline__ uint32_t mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Independent 16-byte gathers: gather m of thread t reads the 4 floats at
// table + row * stride + bin, row and bin drawn from a hash of (t, m); every lane of a
// wavefront reads its own row, as the near-pair evaluation of a global sweep does.
__global__ void gather_kernel(const float* __restrict__ table, int64_t rows, int stride, int max_bin,
                              int per_thread, float* __restrict__ sink) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  float acc = 0.0f;
  uint32_t h = mix(t * 0x9E3779B9u + 1u);
#pragma unroll 4
  for (int m = 0; m < per_thread; ++m) {
    h = mix(h + (uint32_t)m);
    const int64_t row = (int64_t)((uint64_t)h * (uint64_t)rows >> 32);
    const int bin = (int)((h >> 3) % (uint32_t)(max_bin + 1));
    const float* q = table + row * stride + bin;
    acc += (q[0] + q[1]) + (q[2] + q[3]);
  }
  sink[t] = acc;
}

// LDS reads: each thread reads float4 values at a lane-dependent stride from a
// 64-KiB block of LDS, as the tile tests of a global sweep read the C-beta array.
__global__ void __launch_bounds__(512) lds_kernel(int per_thread, float* __restrict__ sink) {
  __shared__ float4 buf[4096];
  for (int e = threadIdx.x; e < 4096; e += blockDim.x)
    buf[e] = make_float4((float)e, 1.0f, 2.0f, 3.0f);
  __syncthreads();
  float acc = 0.0f;
  int idx = (threadIdx.x * 7) & 4095;
#pragma unroll 8
  for (int m = 0; m < per_thread; ++m) {
    const float4 v = buf[idx];
    acc += (v.x + v.y) + (v.z + v.w);
    idx = (idx + 64 + (m & 7)) & 4095;
  }
  sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

extern "C" {

amh_status amh_yard_stream(const float* src_dev, int64_t n_float4, int32_t blocks, float* sink_dev,
                           void* stream) {
  if (!src_dev || !sink_dev || n_float4 < 1 || blocks < 1) return AMH_E_INVAL;
  hipLaunchKernelGGL(stream_kernel, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<const float4*>(src_dev), n_float4, sink_dev);
  return hipGetLastError() == hipSuccess ? AMH_OK : AMH_E_DEVICE;
}

amh_status amh_yard_gather(const float* table_dev, int64_t rows, int32_t stride, int32_t max_bin,
                           int32_t per_thread, int32_t blocks, float* sink_dev, void* stream) {
  if (!table_dev || !sink_dev || rows < 1 || stride < 4 || max_bin < 0 || max_bin + 4 > stride ||
      per_thread < 1 || blocks < 1)
    return AMH_E_INVAL;
  hipLaunchKernelGGL(gather_kernel, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     table_dev, rows, stride, max_bin, per_thread, sink_dev);
  return hipGetLastError() == hipSuccess ? AMH_OK : AMH_E_DEVICE;
}

amh_status amh_yard_lds(int32_t per_thread, int32_t blocks, float* sink_dev, void* stream) {
  if (!sink_dev || per_thread < 1 || blocks < 1) return AMH_E_INVAL;
  hipLaunchKernelGGL(lds_kernel, dim3(blocks), dim3(512), 0, reinterpret_cast<hipStream_t>(stream),
                     per_thread, sink_dev);
  return hipGetLastError() == hipSuccess ? AMH_OK : AMH_E_DEVICE;
}

}  // extern "C"
