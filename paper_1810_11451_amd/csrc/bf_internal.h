// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bf.h"

// One product of a batch, as the kernels read it (32 bytes).
struct BfItem {
    const float2 *S;   // f x 60 complex64, row-major
    float2 *R;         // 64 x 60 complex64, row-major
    int32_t w_id;
    int32_t f;
    int32_t pad0;
    int32_t pad1;
};

// Header of a device descriptor block.  Layout of a block:
//   [BfHeader, 64 B][sink, kSinkBytes][BfItem x n_items]
// `next` is the claim counter of the persistent schedule and `done` counts
// finished workgroups; the last workgroup to finish puts both back to zero,
// so a block can be replayed (graphs) without clearing it in between.
// The sink is scratch that lets every memory access of the kernels be
// unconditional: loads for f = 0 products read it and the stores of the
// four padding columns (60..63) of each row land in it.
struct BfHeader {
    uint32_t next;
    uint32_t done;
    uint32_t n_items;
    uint32_t pad[13];
};
constexpr size_t kSinkBytes = 8192;
inline size_t block_bytes(int n_items) { return 64 + kSinkBytes + (size_t)n_items * 32; }
static_assert(sizeof(BfItem) == 32, "BfItem layout");
static_assert(sizeof(BfHeader) == 64, "BfHeader layout");

namespace bfk {

constexpr int kM = BF_M;
constexpr int kB = BF_B;
constexpr int kFMax = BF_FMAX;
constexpr int kPairsMax = (kFMax + 1) / 2;   // K pairs of S rows
constexpr int kWaves = 4;                    // one wave per 16 antennas
constexpr int kThreads = 64 * kWaves;

// Operand layout of one W for the FP32 matrix-core form: float2 entries
// [kWaves][pairs][64 lanes]; see bf_kernels.hip.
inline size_t fp32_w_stride(int pairs) { return (size_t)kWaves * pairs * 64; }

// Split-form operand layouts (16-bit types): per W, per form; see
// bf_kernels.hip.  Sizes are in bytes.
size_t lp_w_bytes(int f_max);

hipError_t launch_w_transform_fp32(const float2 *w_dev, int n_w, int f_max, float2 *a_out,
                                   int pairs, hipStream_t st);
hipError_t launch_w_transform_lp(const float2 *w_dev, int n_w, int f_max, int prec,
                                 void *a_out, float *w_scale_out, hipStream_t st);

struct LaunchCfg {
    int prec;        // bf_prec
    int schedule;    // 0 one product per workgroup, 1 persistent with atomic claim
    int grid;        // workgroups
    bool vec16;      // all S 16-byte aligned
};

hipError_t launch_apply(const LaunchCfg &cfg, BfHeader *blk, int n_items, const void *a_pool,
                        size_t a_w_stride, int pairs, const float *w_scale, hipStream_t st);

// Workgroups of the apply kernel that fit on one CU at once.
int apply_occupancy(int prec, int schedule, bool vec16);

}  // namespace bfk
