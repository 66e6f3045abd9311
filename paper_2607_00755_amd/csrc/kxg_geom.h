// Geometry of the block-packed GEMM operands, shared by the host tables and
// the GEMM kernels.
#pragma once

namespace kxg {

constexpr int kBlk = 16;             // (k,m) block edge of the packed GEMM layout
constexpr int kIBlk = 32;            // output rows (i) per MFMA tile
constexpr int kBRows = 32;           // distributions per MFMA tile
constexpr int kWaves = 4;            // waves per GEMM workgroup (split K)
#ifndef KXG_F32_SS
#define KXG_F32_SS 4   // dk steps per super-step of the FP32 GEMM (work units)
#endif
constexpr int kF32SS = KXG_F32_SS;

}  // namespace kxg
