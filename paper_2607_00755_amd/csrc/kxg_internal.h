// Internal declarations shared by the libkxg translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/kxg.h"
#include "kxg_geom.h"

namespace kxg {

void set_error(const char *fmt, ...);

#define KXG_TRY_HIP(expr)                                                   \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) {                                             \
            ::kxg::set_error("%s failed: %s", #expr, hipGetErrorString(e_)); \
            return KXG_EHIP;                                                \
        }                                                                   \
    } while (0)

constexpr int kMaxN = 1024;          // largest grid
constexpr int kMaxDevices = 64;      // devices the allocation-free evaluation keeps a scratch address for
#ifndef KXG_PSTREAM_UNROLL
#define KXG_PSTREAM_UNROLL 8   // 16-byte loads in flight per thread in the packed FP64 stream
#endif
constexpr int kPStreamPairs = 128;   // kept pairs one packed-stream workgroup stages (its chunk spans at most this)
// largest chunk of the packed stream of element size `bytes`: one round of
// 16-byte loads per thread (256 threads)
constexpr int pstream_chunk(int bytes) { return KXG_PSTREAM_UNROLL * 256 * (16 / bytes); }
static_assert(pstream_chunk(4) / 256 <= kPStreamPairs, "a chunk spans at most kPStreamPairs pairs");

// Tuning of the GEMM launches (overridable at build time).
#ifndef KXG_GEMM_WG_TARGET
#define KXG_GEMM_WG_TARGET 512   // workgroups of one FP32 GEMM launch at the handle's largest batch
#endif
#ifndef KXG_LDS_WG_TARGET
#define KXG_LDS_WG_TARGET 512   // workgroups of one 16-bit GEMM launch at the handle's largest batch
#endif
#ifndef KXG_LDS_SS
#define KXG_LDS_SS 2   // dk steps per LDS stage of the 16-bit GEMM
#endif
#ifndef KXG_LDS_STEP_COST
#define KXG_LDS_STEP_COST 2.0   // cost of a 16-bit super-step besides its MFMAs, in blocks multiplied
#endif
#ifndef KXG_PSTREAM_ROWS_TARGET
#define KXG_PSTREAM_ROWS_TARGET 2048   // non-empty workgroups of a packed FP64 stream launch aimed at
#endif
#ifndef KXG_LDS_BBW
#define KXG_LDS_BBW 2   // 32-row batch blocks per wave of the 16-bit GEMM
#endif
#ifndef KXG_LDS_IBW
#define KXG_LDS_IBW 4   // i-blocks per workgroup of the 16-bit GEMM
#endif

// Geometry of the block-packed GEMM operand: the (k,m) plane is cut into
// 16x16 blocks; only blocks with kb <= mb are stored (off-diagonal blocks hold
// A[i,k,m] + A[i,m,k], diagonal blocks hold A as is), which is exact for the
// gain sum_{k,m} A f_k f_m.  A unit of K progress ("dk step") is one row k of
// one block: 16 values of K.
struct Geometry {
    int nb = 0;        // ceil(n/16)
    int npairs = 0;    // nb (nb+1)/2 stored blocks
    int nib = 0;       // ceil(n/32) output row tiles
    int ipad = 0;      // nib * 32
    long dksteps = 0;  // npairs * 16
};

// K-slot (split partial) counts of the i-blocks, 16 bits each for up to 32
// i-blocks (n <= 1024), handed to the epilogue by value so that no load
// of a table delays the loads of the partials.
struct SlotCounts {
    uint64_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int per_block = 0;          // 0: every row has the call's nsplit slots
};

// Per-handle (or per-stepper) evaluation workspace.
struct Workspace {
    void *part = nullptr;       // split partial gains
    size_t part_bytes = 0;
    float *fop = nullptr;       // FP32 operand, natural order  [nb][bpad][16]
    float *fpar = nullptr;      // FP32 operand, parity order  [nb][bpad][2][8]
    float *fscale = nullptr;    // per-distribution power-of-two scale [bpad]
    int bpad_cap = 0;
    int b_cap = 0;              // largest batch; the loss-rate buffer [b_cap][n] ends part
};

}  // namespace kxg

struct kxg_kernel {
    int n = 0;
    double mass = 1, gdof = 1, m2 = 1;
    int nmu = 18, quad = 0;
    int b_cap = 1;
    uint32_t prec_mask = 0;
    std::vector<double> p, dp, E, K, h;
    double *d_p = nullptr, *d_dp = nullptr, *d_E = nullptr, *d_K = nullptr, *d_h = nullptr;
    double *d_A64 = nullptr;     // [n][n][n] FP64 master, m fastest
    double *d_RT = nullptr;      // [n][n] R transposed: RT[j][i] = R[i][j]
    double *d_R = nullptr;       // [n][n] R in row order
    float *d_G32 = nullptr;      // packed GEMM operand, FP32
    uint16_t *d_Gbf = nullptr;   // packed GEMM operand, BF16 hi/lo
    uint16_t *d_Gh = nullptr;    // packed GEMM operand, FP16 hi/lo (row-scaled)
    float *d_hrow = nullptr;     // [ipad] FP16 row scales (powers of two)
    int *d_pairs = nullptr;      // [npairs][2] (kb, mb)
    // FP32 GEMM over the non-zero (i-block, pair) blocks only: the pairs of
    // each i-block whose 32 x 16 x 16 block of A (both orderings) has a
    // non-zero, i-block by i-block; G32 holds these blocks in that order.
    int *d_pairs_c = nullptr;    // [ncomp][2] (kb, mb)
    int *d_cib = nullptr;        // [ncomp] i-block of each compacted pair
    int *d_units = nullptr;      // [nunits][4] (i-block, slot, first, end super-step)
    kxg::SlotCounts nslot;       // K slots (partials) of each i-block
    long ncomp = 0;              // non-zero (i-block, pair) blocks
    long nnz_packed = 0;         // entries of the k <= m packing of A' = A - delta_ik R_im that carry a weight
    int nunits = 0, maxslots = 0;
    // the same for the 16-bit operands, per group of KXG_LDS_IBW i-blocks
    // (union of their non-zero pairs); Gbf/Gh hold [block][i-block of the
    // group][dk][hi|lo][lane][8]
    int *d_pairs16 = nullptr, *d_cit16 = nullptr, *d_units16 = nullptr;
    int *d_act16 = nullptr;      // [ncomp16] i-blocks [0, act) of the group hold the pair's non-zero blocks
    long mult16 = 0;             // (i-block, pair) blocks multiplied: the sum of d_act16
    kxg::SlotCounts nslot16;
    long ncomp16 = 0;
    int nunits16 = 0, maxslots16 = 0;
    // Operands of the plain (stream) evaluations: the same non-zero
    // (i-block, pair) blocks as the FP32 GEMM, row by row: row i holds the
    // 16 x 16 blocks of its i-block's kept pairs, [pair][dk][dm]; FP64 for
    // FP64 evaluations, FP32 for the single-distribution FP32 handles
    double *d_P64 = nullptr;
    float *d_P32 = nullptr;
    int *d_pairs64 = nullptr;    // [ncomp64][2] (kb, mb), i-block by i-block, then [ncomp64] their i-blocks
    int *d_ib64 = nullptr;       // [nib][2] first kept pair and count of each i-block
    long ncomp64 = 0;
    int chunk64 = 0, nsplit64 = 0;   // FP64: values per stream workgroup, K splits (partials) per row
    int chunk32 = 0, nsplit32 = 0;   // FP32: the same
    // Operands of the exact forms (handles built with brackets): A[i,k,m]
    // itself (not symmetrised, no loss) and the interpolation bracket j_L
    // (0xFFFF: cut) on the (i-block, kb, mb) blocks, in both orders, of the
    // pairs with a structural weight, row by row like P64 ([block][dk][dm]);
    // A in FP64 and/or FP32
    double *d_AX64 = nullptr;
    float *d_AX32 = nullptr;
    uint16_t *d_JX = nullptr;
    int *d_xpairs = nullptr;     // [nx][2] (kb, mb) of the ordered blocks, i-block by i-block, then [nx] their i-blocks
    int *d_xib = nullptr;        // [nib][2] first block and count of each i-block
    long nx = 0;
    int chunkx64 = 0, nsplitx64 = 0, chunkx32 = 0, nsplitx32 = 0;
    double *d_invdK = nullptr;   // [n] 1 / (K_{j+1} - K_j) (0 for the last point)
    kxg::Geometry geo;
    size_t bytes[5] = {0, 0, 0, 0, 0};
    size_t held = 0;             // device bytes held by the handle
    kxg::Workspace ws;
};

namespace kxg {

// Launchers (device code in the .hip files).
hipError_t launch_build_A(const kxg_kernel &k, const double *d_xmu, const double *d_wmu,
                          hipStream_t s);
hipError_t launch_build_R(const kxg_kernel &k, hipStream_t s);
hipError_t launch_derive(kxg_kernel &k, hipStream_t s);
hipError_t launch_block_nz(const kxg_kernel &k, unsigned char *flags, unsigned int *nnz,
                           hipStream_t s);
hipError_t launch_pack_f32(const kxg_kernel &k, hipStream_t s);
hipError_t launch_pack_rows(const kxg_kernel &k, hipStream_t s);
hipError_t launch_pack_16(const kxg_kernel &k, int ibw, hipStream_t s);
hipError_t launch_pack_exact(const kxg_kernel &k, hipStream_t s);
// device self-calibration (kxg_probe.hip)
hipError_t launch_peak_mfma(int bf16, int nwg, int iters, float *sink, hipStream_t s);
hipError_t launch_copy16(const void *src, void *dst, long nvec, hipStream_t s);
hipError_t launch_read16(const void *src, long nvec, float *sink, int nwg, hipStream_t s);
// FP32 GEMM over the kept blocks: nwg = batch tiles x work units, bbw
// 32-row b-blocks per wave (1, 2 or 4)
hipError_t launch_gemm_f32(int bbw, int nwg, const float *G, const float *fop, const float *fpar,
                           const int *pairs, const int *units, int bpad, int ipad, int nbt, float *part,
                           hipStream_t s);
// 16-bit GEMM (kxg_gemm16.hip): split = 3, 2 or 1 products of the hi+lo
// split; nwg = batch tiles x work units
hipError_t launch_gemm16(bool f16, int split, int nwg, const uint16_t *G, const float *fop, const int *pairs,
                         const int *act, const int *units, int nib, int bpad, int ipad, int nbt, float *part,
                         hipStream_t s);

struct StepArgs;
// Evaluate C[f] for B rows; with `step` the epilogue applies that stepper
// update instead of writing C (C and diag may then be null).
kxg_status eval_impl(const kxg_kernel &k, const Workspace &ws, int prec, const double *f,
                     int B, double *C, uint32_t flags, double *diag, hipStream_t s,
                     const StepArgs *step = nullptr);
// kxg_eval with the call's workspace in the library's static device array
// (no allocation); KXG_EINVAL if the call needs more than that array holds.
kxg_status eval_noalloc_impl(const kxg_kernel &k, int prec, const double *f, int B, double *C,
                             uint32_t flags, double *diag, hipStream_t s);
kxg_status prep_operands(const kxg_kernel &k, const Workspace &ws, int prec, const double *f,
                         int B, hipStream_t s);
kxg_status alloc_workspace(const kxg_kernel &k, int b_cap, Workspace &ws);
void free_workspace(Workspace &ws);
hipError_t launch_moments(const kxg_kernel &k, const double *f, int B, double *out,
                          hipStream_t s);


// Gain-kernel profiling (events around each launch while a profile is open).
void profile_mark_begin(hipStream_t s);
void profile_mark_end(hipStream_t s);

}  // namespace kxg
