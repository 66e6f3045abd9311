// Device self-calibration for roofline reporting: the sustained rate of the
// FP32 and BF16 matrix cores on back-to-back independent MFMAs, and the
// device-memory bandwidth of a plain vector copy.  Not an operation of the
// method; it tells what this chip sustains beside its datasheet peaks.
#include "kxg_device.h"

namespace kxg {
namespace {

typedef __bf16 bf16x8p __attribute__((ext_vector_type(8)));

// Every wave keeps four independent accumulators busy for `iters` rounds of
// four MFMAs (no dependency between consecutive instructions).  The sum of
// the accumulators is stored only when it equals a value it cannot take for
// these inputs, so the work is kept without a store per thread.
__global__ __launch_bounds__(256) void k_peak_f32(int iters, float *__restrict__ sink)
{
    floatx16 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[j][e] = 0.0f;
    const float a = 1e-3f * (float)(threadIdx.x & 63), b = 1.0f + 1e-6f * (float)(blockIdx.x & 255);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) s += acc[j][e];
    if (s == -1.0f) sink[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_bf16(int iters, float *__restrict__ sink)
{
    floatx16 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[j][e] = 0.0f;
    bf16x8p a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(1e-3f * (float)((threadIdx.x + e) & 63));
        b[e] = (__bf16)(1.0f + 1e-2f * (float)e);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) s += acc[j][e];
    if (s == -1.0f) sink[blockIdx.x * 256 + threadIdx.x] = s;
}

// Grid-stride copy of n 16-byte vectors.
__global__ __launch_bounds__(256) void k_copy16(const float4 *__restrict__ src, float4 *__restrict__ dst, long n)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) dst[q] = src[q];
}

// Read of n 16-byte vectors, non-temporal like the stream kernels' loads:
// each workgroup takes a contiguous chunk, eight vectors in flight per
// thread; kept alive like the MFMA loops.  sink holds gridDim.x * 256 floats.
typedef float f4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_read16(const f4v *__restrict__ src, long n, float *__restrict__ sink)
{
    const long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long beg = (long)blockIdx.x * chunk;
    const long end = beg + chunk < n ? beg + chunk : n;
    f4v a = {0.0f, 0.0f, 0.0f, 0.0f};
    for (long q = beg + threadIdx.x; q < end; q += 8 * 256) {
        f4v x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long r = q + 256 * u;
            x[u] = r < end ? __builtin_nontemporal_load(src + r) : f4v{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) a += x[u];
    }
    const float s = (a.x + a.y) + (a.z + a.w);
    if (s == -1.0f) sink[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

// Flop of one launch of each MFMA probe: waves x iters x 4 MFMAs x flop per MFMA.
hipError_t launch_peak_mfma(int bf16, int nwg, int iters, float *sink, hipStream_t s)
{
    if (bf16) hipLaunchKernelGGL(k_peak_bf16, dim3(nwg), dim3(256), 0, s, iters, sink);
    else hipLaunchKernelGGL(k_peak_f32, dim3(nwg), dim3(256), 0, s, iters, sink);
    return hipGetLastError();
}

hipError_t launch_copy16(const void *src, void *dst, long nvec, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy16, dim3(8192), dim3(256), 0, s, static_cast<const float4 *>(src),
                       static_cast<float4 *>(dst), nvec);
    return hipGetLastError();
}

hipError_t launch_read16(const void *src, long nvec, float *sink, int nwg, hipStream_t s)
{
    hipLaunchKernelGGL(k_read16, dim3(nwg), dim3(256), 0, s, static_cast<const f4v *>(src), nvec, sink);
    return hipGetLastError();
}

}  // namespace kxg
