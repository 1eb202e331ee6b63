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

// One request of a serving launch, as uploaded (32 bytes): n_s S blocks of
// one W and f, block k reading S + k f 60 and writing R + k 64 60 complex
// elements, which become items item0 .. item0 + n_s - 1 of the launch's
// descriptor block.  The device expands them (launch_expand), so the host
// packs one record per request instead of one item per block.
struct BfReqRec {
    const float2 *S;   // first S block (null when f = 0)
    float2 *R;         // first R block
    int32_t w_id;
    int32_t f;
    int32_t n_s;
    int32_t item0;
};
static_assert(sizeof(BfReqRec) == 32, "BfReqRec layout");
static_assert(sizeof(BfHeader) == 64, "BfHeader layout");

// Position in the item list of the i-th of n items when the items are dealt
// to the G workgroups of a wave-specialised launch in contiguous blocks.
// That schedule splits the list into min(G, 8) contiguous parts, one per
// XCD (workgroup b runs on XCD b % 8), and workgroup j of part x, one of nb
// in that part, takes positions lo + j, lo + j + nb, lo + j + 2 nb, ...
// (bfk::ws_share).  Dealing the part's items in order to its workgroups,
// the first ones to workgroup 0, the next to workgroup 1 and so on, puts
// items that are consecutive in the list, for instance of one W, in
// consecutive products of one workgroup.  A bijection of 0 .. n - 1.
__host__ __device__ inline int ws_deal(int i, int n, int G)
{
    const int X = G < 8 ? G : 8;
    if (X <= 0)
        return i;
    const int q = n / X, r = n % X;
    // part x holds positions lo .. lo + cnt - 1
    const int x = i < (q + 1) * r ? i / (q + 1) : r + (q > 0 ? (i - (q + 1) * r) / q : 0);
    const int lo = x * q + (x < r ? x : r);
    const int cnt = q + (x < r ? 1 : 0);
    const int nb = G / X + (x < G % X ? 1 : 0);
    const int s = i - lo;
    const int a = cnt / nb, b = cnt % nb;   // workgroups j < b take a + 1 items, the others a
    int j, k;
    if (s < b * (a + 1)) {
        j = s / (a + 1);
        k = s % (a + 1);
    } else {
        const int s2 = s - b * (a + 1);
        j = b + s2 / a;
        k = s2 % a;
    }
    return lo + j + k * nb;
}

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
// Three-product FP32 form, two layouts of each W one after the other (the
// kernels form Wr + Wi with one FP32 add):
//   32 x 32 tiles: floats [2 antenna halves][pairs][2][64 lanes], the 2
//     being Wr and Wi of the lane's (antenna, flow);
//   16 x 16 tiles, at fp32_3m16_offset: floats [4 antenna blocks][steps]
//     [2][64 lanes], steps = ceil(pairs / 2) blocks of 4 flows.
constexpr size_t fp32_3m16_offset(int pairs) { return (size_t)2 * pairs * 2 * 64; }
constexpr int fp32_3m16_steps(int pairs) { return (pairs + 1) / 2; }
constexpr size_t fp32_3m_w_stride(int pairs)
{
    return fp32_3m16_offset(pairs) + (size_t)4 * fp32_3m16_steps(pairs) * 2 * 64;
}

// Device-side view of a plan, as the apply kernels need it.
struct PlanDev {
    const float2 *a_fp32;     // FP32 form: kWaves x pairs x 64 float2 per W
    int a_fp32_stride;        // float2 per W
    int pairs;                // ceil(f_max / 2)
    const float *a_3m;        // three-product form: both layouts, a_3m_stride floats per W
    int a_3m_stride;          // floats per W
    const void *lp_hi;        // plain 16-bit forms: kWaves x chunks x 64 x 16 bytes per W
    const int *lp_exp;        // per-W power-of-two exponent of the 16-bit operands
    int lp_stride;            // 16-byte units per W
    int lp_chunks;            // ceil(f_max / 8)
    const uint32_t *lp_wc;    // 16-bit forms, compact: parts x 64 antennas x 40 flows dwords per W
    int lp_wc_stride;         // dwords per W
};

constexpr int kLpFlows = 8;   // flows per 16-bit matrix-core step (K = 16 real)
inline int lp_chunks(int f_max) { return (f_max + kLpFlows - 1) / kLpFlows; }
inline size_t lp_w_units(int f_max) { return (size_t)kWaves * lp_chunks(f_max) * 64; }
// Compact 16-bit W (wave-specialised schedule): per part (hi, then lo for
// the split forms) one dword per (antenna, flow < 40), (re, im) codes of the
// scaled entry, flows past f_max zero.
constexpr int kLpWcFlows = 40;
constexpr size_t kLpWcPart = (size_t)BF_M * kLpWcFlows;
inline size_t lp_wc_stride(bool split) { return (split ? 2 : 1) * kLpWcPart; }

hipError_t launch_w_transform_fp32(const float2 *w_dev, int n_w, int f_max, float2 *a_out,
                                   int pairs, hipStream_t st);
hipError_t launch_w_transform_3m(const float2 *w_dev, int n_w, int f_max, float *a_out,
                                 int pairs, hipStream_t st);
// bf16 selects BF16 (else FP16); hi (null when the plan has no plain form)
// receives the plain forms' operand layout, wc the compact layout
// (lp_wc_stride(split) dwords per W: the lo part only when split).
hipError_t launch_w_transform_lp(const float2 *w_dev, int n_w, int f_max, bool bf16, void *hi,
                                 bool split, int *w_exp, uint32_t *wc, hipStream_t st);

struct LaunchCfg {
    int prec;        // bf_prec
    int schedule;    // 0 one product per workgroup, 1 persistent with atomic claim,
                     // 2 persistent static share with prefetch, 3 wave-specialised
    int grid;        // workgroups
    bool vec16;      // all S 16-byte aligned
    bool stage;      // R rows staged in LDS and written as contiguous 16-byte stores
    int producers;   // schedule 3: producer waves per workgroup (4, 8 or 12)
    int depth;       // schedule 3: products of S prefetched in producer registers (1..3)
    bool tile16;     // schedule 3, three-product form: 8 matrix-core waves on 16 x 16 tiles
    bool w_dma;      // tile16: the matrix-core waves copy W into LDS (global-to-LDS loads)
    bool s_dma;      // w_dma, and the producers copy S into three LDS buffers the same way
    hipEvent_t ev_start = nullptr;   // if set, recorded at the kernel's own start and end
    hipEvent_t ev_stop = nullptr;    // (hipExtLaunchKernel), for timing the kernel alone
};

hipError_t launch_apply(const LaunchCfg &cfg, BfHeader *blk, int n_items, const PlanDev &pd,
                        hipStream_t st);

// Writes the header and the n_items items of descriptor block blk from
// n_recs request records (their item ranges tile 0 .. n_items - 1).  With
// deal_grid > 0, item i goes to position ws_deal(i, n_items, deal_grid).
hipError_t launch_expand(const BfReqRec *recs, int n_recs, BfHeader *blk, int n_items, int deal_grid,
                         hipStream_t st);

// Workgroups of the apply kernel that fit on one CU at once.
int apply_occupancy(int prec, int schedule, bool vec16, bool stage);

}  // namespace bfk
