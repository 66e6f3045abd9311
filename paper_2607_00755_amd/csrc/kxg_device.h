// Device helpers shared by the GEMM translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "kxg_geom.h"

namespace kxg {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap so that consecutive logical indices share an XCD: workgroups
// that read the same slice of A (same i-block and K split, different batch
// tiles) then hit the same L2.
__device__ inline int xcd_logical(int bid, int nwg)
{
    if (nwg % 8 != 0) return bid;
    return (bid % 8) * (nwg / 8) + bid / 8;
}

// Reduce the 4 waves' accumulators of a workgroup (fixed order 0+1+2+3) and
// store the FP32 partial of this K split.  32x32 MFMA result layout: register
// e of lane l holds row 8*(e/4) + 4*(l/32) + e%4, column l%32.  Every wave
// parks its accumulators in LDS as [wave][bb][e/4][lane][4]; wave q then sums
// registers 4q..4q+3 of all four and stores those rows.  `lds` holds
// 4*BBW*16*64 floats.
template <int BBW>
__device__ inline void store_tile(floatx16 (&acc)[BBW], float *lds, float *__restrict__ part, int sp,
                           int bpad, int ipad, int brow0, int icol0)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float4 *l4 = reinterpret_cast<float4 *>(lds);
#pragma unroll
    for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
        for (int g = 0; g < 4; ++g)
            l4[((wave * BBW + bb) * 4 + g) * 64 + lane] =
                make_float4(acc[bb][4 * g], acc[bb][4 * g + 1], acc[bb][4 * g + 2], acc[bb][4 * g + 3]);
    __syncthreads();
    float *dst = part + (long)sp * bpad * ipad;
#pragma unroll
    for (int bb = 0; bb < BBW; ++bb) {
        float4 v = l4[((0 * BBW + bb) * 4 + wave) * 64 + lane];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
            const float4 x = l4[((w * BBW + bb) * 4 + wave) * 64 + lane];
            v.x += x.x;
            v.y += x.y;
            v.z += x.z;
            v.w += x.w;
        }
        const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int row = brow0 + bb * 32 + 8 * wave + 4 * (lane >> 5) + c;
            dst[(long)row * ipad + icol0 + (lane & 31)] = vv[c];
        }
    }
}

}  // namespace kxg
