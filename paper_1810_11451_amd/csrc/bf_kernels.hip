// gfx950 kernels for the batched beamforming product R = W x S.
//
// The product (Section III of the paper, beamforming paragraph and its
// equation) is a complex 64 x f by f x 60 matrix product per item.  It is
// computed as a real GEMM on the matrix cores:
//
//   rows    m = 2 i + c     (antenna i, c = 0 real part, c = 1 imaginary part)
//   columns n = j           (resource element j, padded 60 -> 64)
//   K index (k, q)          (flow k, q = 0 real part of S, q = 1 imaginary part)
//
//   A[(i,c)][(k,q)] = [[ Wr, -Wi ], [ Wi, Wr ]] (row c, column q) of W[i][k]
//   B[(k,q)][j]     = Re S[k][j] (q = 0) or Im S[k][j] (q = 1)
//
// so that C[(i,0)][j] = sum Wr Sr - Wi Si = Re R[i][j] and
//         C[(i,1)][j] = sum Wi Sr + Wr Si = Im R[i][j].
// The 2 x 2 real block form of each W entry is built once at plan time
// (W is constant); S is read in its own interleaved layout, and the
// accumulator pairs (c = 0, 1) land in adjacent registers, so R is written
// in its own interleaved layout as 8-byte complex values.
//
// Workgroup: 4 waves; wave w owns antennas 16w .. 16w+15 (32 real rows,
// one 32 x 32 matrix-core tile in M) and both 32-column tiles in N.  S is
// staged once per item in LDS and read by all four waves.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bf_internal.h"

namespace bfk {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f3v __attribute__((ext_vector_type(3)));
// Global-memory (address space 1) views, so that accesses through pointers
// read from descriptors compile to global_* rather than flat_* instructions.
typedef __attribute__((address_space(1))) f2v g_f2v;
typedef __attribute__((address_space(1))) const f2v g_cf2v;
typedef __attribute__((address_space(1))) const f4v g_cf4v;
typedef __attribute__((address_space(1))) f4v g_f4v;
// Descriptors are never written by a kernel; reading them through the
// constant address space lets the compiler use scalar loads, which wait on
// their own counter instead of behind the vector memory queue.
typedef __attribute__((address_space(4))) const BfItem c_item;

// Item k of a share that starts at p and takes every stride-th item.
__device__ __forceinline__ BfItem item_at(c_item *p, int k, int stride)
{
    const int i = k * stride;
    BfItem d;
    d.S = p[i].S;
    d.R = p[i].R;
    d.w_id = p[i].w_id;
    d.f = p[i].f;
    d.pad0 = d.pad1 = 0;
    return d;
}

constexpr int kLdsCols = 64;   // LDS row pitch of a staged S, in complex elements

// ---------------------------------------------------------------------------
// Plan-time operand layout, FP32 form.
//
// For v_mfma_f32_32x32x2_f32, lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32].  One instruction covers two K indices; here they are
// (k = 2p + l/32, q) for a fixed q, so pair p of S rows feeds two
// instructions: q = 0 takes the real parts, q = 1 the imaginary parts.
// Lane l of wave w holds, for pair p, the float2 (A for q = 0, A for q = 1)
// of real row m = l % 32, i.e. antenna i = 16 w + (l % 32) / 2, c = l % 2,
// flow k = 2 p + l / 32:
//   c = 0:  ( Wr, -Wi )       c = 1:  ( Wi, Wr )
// Flows k >= f_max hold zeros.
__global__ void w_transform_fp32_kernel(const float2 *__restrict__ w, int n_w, int f_max,
                                        float2 *__restrict__ a, int pairs)
{
    const size_t total = (size_t)n_w * kWaves * pairs * 64;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int lane = (int)(idx % 64);
        const int p = (int)((idx / 64) % pairs);
        const int wave = (int)((idx / (64 * (size_t)pairs)) % kWaves);
        const size_t wi = idx / (64 * (size_t)pairs * kWaves);
        const int i = 16 * wave + (lane & 31) / 2;
        const int c = lane & 1;
        const int k = 2 * p + (lane >> 5);
        float2 out = make_float2(0.f, 0.f);
        if (k < f_max) {
            const float2 v = w[(wi * kM + i) * (size_t)f_max + k];
            out = c == 0 ? make_float2(v.x, -v.y) : make_float2(v.y, v.x);
        }
        a[idx] = out;
    }
}

hipError_t launch_w_transform_fp32(const float2 *w_dev, int n_w, int f_max, float2 *a_out,
                                   int pairs, hipStream_t st)
{
    const size_t total = (size_t)n_w * kWaves * pairs * 64;
    if (total == 0)
        return hipSuccess;
    const int block = 256;
    const size_t want = (total + block - 1) / block;
    const int grid = (int)(want < 65535 ? want : 65535);
    hipLaunchKernelGGL(w_transform_fp32_kernel, dim3(grid), dim3(block), 0, st, w_dev, n_w,
                       f_max, a_out, pairs);
    return hipGetLastError();
}

// Plan-time operand layouts, three-product FP32 form, both per W (Wr and Wi
// planes; flows k >= f_max hold zeros; the kernels form Wr + Wi):
//   32 x 32 tiles (v_mfma_f32_32x32x2_f32, real rows = antennas): lane l of
//     antenna half mt holds, for pair p, antenna 32 mt + l % 32 and flow
//     2p + l / 32;
//   16 x 16 tiles (v_mfma_f32_16x16x4_f32), after the first: lane l of
//     antenna block rb holds, for step s, antenna 16 rb + l % 16 and flow
//     4s + l / 16 (the instruction's A operand: row l % 16, K index l / 16).
__global__ void w_transform_3m_kernel(const float2 *__restrict__ w, int n_w, int f_max,
                                      float *__restrict__ a, int pairs)
{
    const size_t per_w = fp32_3m_w_stride(pairs);
    const size_t off16 = fp32_3m16_offset(pairs);
    const int steps = fp32_3m16_steps(pairs);
    const size_t total = (size_t)n_w * per_w;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t wi = idx / per_w;
        const size_t e = idx - wi * per_w;
        const int lane = (int)(e % 64);
        const int c = (int)((e / 64) % 2);
        int i, k;
        if (e < off16) {
            // (half mt, pair p, component c, lane)
            const int p = (int)((e / (64 * 2)) % pairs);
            const int mt = (int)(e / (64 * 2 * (size_t)pairs));
            i = 32 * mt + (lane & 31);
            k = 2 * p + (lane >> 5);
        } else {
            // (block rb, step s, component c, lane)
            const size_t e16 = e - off16;
            const int s = (int)((e16 / (64 * 2)) % steps);
            const int rb = (int)(e16 / (64 * 2 * (size_t)steps));
            i = 16 * rb + (lane & 15);
            k = 4 * s + (lane >> 4);
        }
        float out = 0.f;
        if (k < f_max) {
            const float2 v = w[(wi * kM + i) * (size_t)f_max + k];
            out = c == 0 ? v.x : v.y;
        }
        a[idx] = out;
    }
}

hipError_t launch_w_transform_3m(const float2 *w_dev, int n_w, int f_max, float *a_out,
                                 int pairs, hipStream_t st)
{
    const size_t total = (size_t)n_w * fp32_3m_w_stride(pairs);
    if (total == 0)
        return hipSuccess;
    const int block = 256;
    const size_t want = (total + block - 1) / block;
    const int grid = (int)(want < 65535 ? want : 65535);
    hipLaunchKernelGGL(w_transform_3m_kernel, dim3(grid), dim3(block), 0, st, w_dev, n_w, f_max,
                       a_out, pairs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Memory access discipline.  Every global load and store inside the
// per-product loop is unconditional: indices are clamped into range (the
// duplicate loads are harmless) and the stores of the four padding columns
// go to a sink area of the descriptor block.  With no branches around
// memory instructions the compiler can count outstanding operations and
// wait for exactly the ones a value depends on, so the next product's S
// loads stay in flight while the matrix cores work on the current one.

constexpr int kChunks16 = (kFMax * kB / 2 + kThreads - 1) / kThreads;   // 5
constexpr int kChunks8 = (kFMax * kB + kThreads - 1) / kThreads;        // 9

// Waits until every vector memory operation of this wave has completed
// (gfx9 s_waitcnt encoding: vmcnt = 0, expcnt and lgkmcnt not waited on).
__device__ __forceinline__ void wait_vmem_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <bool kVec16>
struct SRegs {
    f4v v[kChunks16];
};
template <>
struct SRegs<false> {
    f2v v[kChunks8];
};

// Issues the loads of one S (f x 60 complex) into registers: thread t takes
// 16-byte chunks t, t + 256, ... (8-byte elements when S is only 8-byte
// aligned).  For f = 0, S must point at the sink and one chunk is read.
// S is loaded through the caches (here and in the producers' p_load_s):
// streaming hints cost about 8% on batches of mixed f and gained nothing
// measurable at full width.
template <bool kVec16>
__device__ __forceinline__ void load_s(SRegs<kVec16> &r, const float2 *__restrict__ S, int f,
                                       int tid = threadIdx.x)
{
    if constexpr (kVec16) {
        g_cf4v *src = (g_cf4v *)S;
        const int last = (f > 0 ? f * (kB / 2) : 1) - 1;
#pragma unroll
        for (int u = 0; u < kChunks16; ++u) {
            const int c = min(tid + u * kThreads, last);
            r.v[u] = src[c];
        }
    } else {
        g_cf2v *src = (g_cf2v *)S;
        const int last = (f > 0 ? f * kB : 1) - 1;
#pragma unroll
        for (int u = 0; u < kChunks8; ++u) {
            const int c = min(tid + u * kThreads, last);
            r.v[u] = src[c];
        }
    }
}

// Writes the registers of load_s to LDS: row k of S (480 bytes) to LDS row
// k (pitch 64 complex).  For odd f, row f is cleared so the second half of
// the last K pair multiplies zeros.
template <bool kVec16>
__device__ __forceinline__ void put_s(f2v *__restrict__ lds, const SRegs<kVec16> &r, int f,
                                      int tid = threadIdx.x)
{
    if constexpr (kVec16) {
        const int chunks = f * (kB / 2);
#pragma unroll
        for (int u = 0; u < kChunks16; ++u) {
            const int c = tid + u * kThreads;
            if (c < chunks) {
                const int row = c / (kB / 2);
                const int col2 = c - row * (kB / 2);
                *reinterpret_cast<f4v *>(lds + row * kLdsCols + 2 * col2) = r.v[u];
            }
        }
    } else {
        const int elems = f * kB;
#pragma unroll
        for (int u = 0; u < kChunks8; ++u) {
            const int c = tid + u * kThreads;
            if (c < elems) {
                const int row = c / kB;
                const int col = c - row * kB;
                lds[row * kLdsCols + col] = r.v[u];
            }
        }
    }
    if (f & 1) {
        if (tid < kLdsCols)
            lds[f * kLdsCols + tid] = f2v{0.f, 0.f};
    }
}

// Writes the two 32 x 32 accumulator tiles of one wave to R.  Register r of
// lane l holds real row 8 (r / 4) + 4 (l / 32) + r % 4 and column l % 32,
// so registers (r, r + 1), r even, are (Re, Im) of antenna
// 4 (r / 4) + 2 (l / 32) + (r % 4) / 2 within the wave's 16.  Columns
// 60..63 of the second tile are padding; those lanes write to the sink.
__device__ __forceinline__ void store_r(float2 *__restrict__ Rp, float2 *__restrict__ sink,
                                        int wave, int lane, const floatx16 &acc0,
                                        const floatx16 &acc1)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    g_f2v *base = (g_f2v *)Rp + (size_t)(16 * wave) * kB;
    g_f2v *pad = (g_f2v *)sink + lane;
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
        const int il = 4 * (r >> 2) + 2 * h + ((r & 3) >> 1);
        g_f2v *row = base + il * kB;
        g_f2v *dst1 = n < kB - 32 ? row + 32 + n : pad;
        __builtin_nontemporal_store(f2v{acc0[r], acc0[r + 1]}, row + n);
        __builtin_nontemporal_store(f2v{acc1[r], acc1[r + 1]}, dst1);
    }
}

// Issues kN stores into the sink: as many as one product's R write issues
// (16 for store_r, 8 for write_r_staged).  Placed after the first S loads
// of a persistent loop, it makes the loop-entry path carry the same
// outstanding-operation pattern as the back edge (S loads followed by the
// R stores), so the compiler's wait before the first LDS write counts only
// the S loads on both paths instead of falling back to the stricter count.
template <int kN>
__device__ __forceinline__ void prime_store_count(float2 *__restrict__ sink, int lane)
{
    g_f2v *pad = (g_f2v *)sink + lane;
#pragma unroll
    for (int k = 0; k < kN; ++k)
        __builtin_nontemporal_store(f2v{0.f, 0.f}, pad + 64 * k);
}

// R of one wave: rows 16 wave .. 16 wave + 15, i.e. 960 complex values
// (7680 bytes) contiguous in memory.
constexpr int kWaveOut = 16 * kB;

// Writes the wave's two accumulator tiles to R through the wave's own LDS
// area: first to LDS in R's row-major layout, then read back and written
// as 7 contiguous 16-byte stores plus one 8-byte store per lane (whole
// 128-byte lines, no padding lanes).  Only this wave touches its area, and
// a wave's LDS operations complete in order, so no barrier is needed.
__device__ __forceinline__ void stage_acc(f2v *__restrict__ stage, int lane, const floatx16 &acc0,
                                          const floatx16 &acc1)
{
    const int h = lane >> 5;
    const int n = lane & 31;
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
        const int il = 4 * (r >> 2) + 2 * h + ((r & 3) >> 1);
        stage[il * kB + n] = f2v{acc0[r], acc0[r + 1]};
        if (n < kB - 32)
            stage[il * kB + 32 + n] = f2v{acc1[r], acc1[r + 1]};
    }
}

__device__ __forceinline__ void store_staged(float2 *__restrict__ Rp, const f2v *__restrict__ stage,
                                             int wave, int lane)
{
    g_f2v *dst = (g_f2v *)Rp + (size_t)(16 * wave) * kB;
    const f4v *src4 = reinterpret_cast<const f4v *>(stage);
#pragma unroll
    for (int u = 0; u < 7; ++u) {
        const int c = u * 64 + lane;
        __builtin_nontemporal_store(src4[c], (g_f4v *)dst + c);
    }
    __builtin_nontemporal_store(stage[896 + lane], dst + 896 + lane);
}

__device__ __forceinline__ void write_r_staged(float2 *__restrict__ Rp, f2v *__restrict__ stage,
                                               int wave, int lane, const floatx16 &acc0,
                                               const floatx16 &acc1)
{
    stage_acc(stage, lane, acc0, acc1);
    store_staged(Rp, stage, wave, lane);
}

template <bool kStage>
__device__ __forceinline__ void write_r(float2 *__restrict__ Rp, float2 *__restrict__ sink,
                                        f2v *__restrict__ stage, int wave, int lane,
                                        const floatx16 &acc0, const floatx16 &acc1)
{
    if constexpr (kStage)
        write_r_staged(Rp, stage, wave, lane, acc0, acc1);
    else
        store_r(Rp, sink, wave, lane, acc0, acc1);
}
template <bool kStage>
constexpr int kStoresPerProduct = kStage ? 8 : 16;

// ---------------------------------------------------------------------------
// FP32 apply kernels.

// Loads wave `wave`'s A operands of pool entry w into registers (pairs >= 1;
// entries past `pairs` repeat the last one and are never used).
__device__ __forceinline__ void load_a_fp32(f2v (&a)[kPairsMax], const float2 *__restrict__ apool,
                                            int w, int a_w_stride, int pairs, int wave, int lane)
{
    const g_cf2v *ap = (const g_cf2v *)(apool + (size_t)w * a_w_stride + (size_t)wave * pairs * 64 + lane);
#pragma unroll
    for (int p = 0; p < kPairsMax; ++p)
        a[p] = ap[min(p, pairs - 1) * 64];
}

// One product from a staged S: 2 * np matrix-core steps per 32 x 32 tile.
__device__ __forceinline__ void contract_fp32(const f2v *__restrict__ lds, const f2v (&a)[kPairsMax],
                                              int f, int lane, floatx16 &acc0, floatx16 &acc1)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    const int np = (f + 1) >> 1;
    acc0 = floatx16{};
    acc1 = floatx16{};
    if (np == kPairsMax) {
        // Full width: straight-line code, so the LDS reads of later pairs can
        // be issued while earlier pairs are on the matrix cores.
#pragma unroll
        for (int p = 0; p < kPairsMax; ++p) {
            const f2v b0 = lds[(2 * p + h) * kLdsCols + n];
            const f2v b1 = lds[(2 * p + h) * kLdsCols + 32 + n];
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b0.x, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b1.x, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b0.y, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b1.y, acc1, 0, 0, 0);
        }
        return;
    }
#pragma unroll
    for (int p = 0; p < kPairsMax; ++p) {
        if (p < np) {
            const f2v b0 = lds[(2 * p + h) * kLdsCols + n];
            const f2v b1 = lds[(2 * p + h) * kLdsCols + 32 + n];
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b0.x, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b1.x, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b0.y, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b1.y, acc1, 0, 0, 0);
        }
    }
}

// contract_fp32 for the wave-specialised schedule: once a pair's matrix-core
// steps are issued its operand registers are free, and they are reloaded
// there with the same pair of pool entry w_next (the next product's W), so
// the next W arrives during this product's chain at no register cost.
__device__ __forceinline__ void contract_fp32_reload(const f2v *__restrict__ lds, f2v (&a)[kPairsMax],
                                                     int f, int lane, floatx16 &acc0, floatx16 &acc1,
                                                     const float2 *__restrict__ apool, int w_next,
                                                     int a_w_stride, int pairs, int wave)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    const int np = (f + 1) >> 1;
    const g_cf2v *nx = (const g_cf2v *)(apool + (size_t)w_next * a_w_stride + (size_t)wave * pairs * 64 + lane);
    acc0 = floatx16{};
    acc1 = floatx16{};
    // The staged rows are read ahead of their products (rows past f hold
    // older data and feed no product) in batches of 6 pairs: batch k is
    // issued once pair 6k - 4 is, so at most 10 pairs occupy registers.
    constexpr int kBatch = 6, kLead = 4;
    f2v b0[kPairsMax], b1[kPairsMax];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
        b0[q] = lds[(2 * q + h) * kLdsCols + n];
        b1[q] = lds[(2 * q + h) * kLdsCols + 32 + n];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < kPairsMax; ++p) {
        if (p + kLead < kPairsMax && (p + kLead) % kBatch == 0) {
#pragma unroll
            for (int q = p + kLead; q < p + kLead + kBatch; ++q) {
                b0[q] = lds[(2 * q + h) * kLdsCols + n];
                b1[q] = lds[(2 * q + h) * kLdsCols + 32 + n];
            }
        }
        if (p < np) {
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b0[p].x, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b1[p].x, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b0[p].y, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b1[p].y, acc1, 0, 0, 0);
        }
        a[p] = nx[min(p, pairs - 1) * 64];
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ---------------------------------------------------------------------------
// Three-product FP32 form.  Wave w of a workgroup owns the 32 x 32 quadrant
// (antennas 32 mt .. 32 mt + 31, columns 32 nt .. 32 nt + 31), mt = w / 2,
// nt = w % 2, and accumulates T1 = Wr Sr, T2 = Wi Si, T3 = (Wr + Wi)(Sr + Si)
// over the flows; then Re R = T1 - T2 and Im R = (T3 - T1) - T2.

// Operands of pool entry w for antenna half mt: Wr and Wi, 2 registers per
// pair, read from the plan's component planes (pairs >= 1); the third
// operand Wr + Wi is formed at each matrix-core step.  The product uses `need`
// (>= 1) pairs; the loads of later pairs repeat the last used one, so they
// hit in cache instead of fetching W columns the product does not use, and
// those registers feed no matrix-core step.
__device__ __forceinline__ void load_a_3m(f2v (&a)[kPairsMax], const float *__restrict__ apool,
                                          int w, int a_w_stride, int pairs, int mt, int lane,
                                          int need)
{
    typedef __attribute__((address_space(1))) const float g_cf;
    const g_cf *ap = (const g_cf *)(apool + (size_t)w * a_w_stride + (size_t)mt * pairs * 128 + lane);
    const int last = min(pairs, need) - 1;
#pragma unroll
    for (int p = 0; p < kPairsMax; ++p) {
        const int q = min(p, last);
        a[p] = f2v{ap[(2 * q) * 64], ap[(2 * q + 1) * 64]};
    }
}

__device__ __forceinline__ void mfma3(const f3v &a, const f2v &b, floatx16 &t1, floatx16 &t2,
                                      floatx16 &t3)
{
    t1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, t1, 0, 0, 0);
    t2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, t2, 0, 0, 0);
    t3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.x + b.y, t3, 0, 0, 0);
}

// Contracts the staged S (LDS, pitch kLdsCols) and writes the wave's
// quadrant of R, row-major 64 x 60, into `tile` (LDS).
__device__ __forceinline__ void contract_stage_3m(const f2v *__restrict__ lds,
                                                  const f2v (&a)[kPairsMax], int f, int wave,
                                                  int lane, f2v *__restrict__ tile)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    const int mt = wave >> 1;
    const int nt = wave & 1;
    const int np = (f + 1) >> 1;
    floatx16 t1 = {}, t2 = {}, t3 = {};
    const f2v *col = lds + h * kLdsCols + 32 * nt + n;
    if (np == kPairsMax) {
        // All B operands are read before the first product: each wait then
        // covers only the oldest outstanding read, and the matrix core never
        // idles on LDS latency inside the chain.
        f2v b[kPairsMax];
#pragma unroll
        for (int p = 0; p < kPairsMax; ++p)
            b[p] = col[2 * p * kLdsCols];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int p = 0; p < kPairsMax; ++p)
            mfma3(f3v{a[p].x, a[p].y, a[p].x + a[p].y}, b[p], t1, t2, t3);
    } else {
#pragma unroll
        for (int p = 0; p < kPairsMax; ++p)
            if (p < np)
                mfma3(f3v{a[p].x, a[p].y, a[p].x + a[p].y}, col[2 * p * kLdsCols], t1, t2, t3);
    }
    const int j = 32 * nt + n;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 32 * mt + 8 * (r >> 2) + 4 * h + (r & 3);
        if (j < kB)
            tile[i * kB + j] = f2v{t1[r] - t2[r], (t3[r] - t1[r]) - t2[r]};
    }
}

// Row r of a wave's 32 x 32 quadrant of R (staged in LDS, 64 x 60
// row-major) from the three products: Re = T1 - T2, Im = (T3 - T1) - T2.
__device__ __forceinline__ void stage_row_3m(const floatx16 &t1, const floatx16 &t2, const floatx16 &t3,
                                             int r, int wave, int lane, f2v *__restrict__ tile)
{
    const int h = lane >> 5;
    const int i = 32 * (wave >> 1) + 8 * (r >> 2) + 4 * h + (r & 3);
    const int j = 32 * (wave & 1) + (lane & 31);
    if (j < kB)
        tile[i * kB + j] = f2v{t1[r] - t2[r], (t3[r] - t1[r]) - t2[r]};
}

// The three-product chain of one product for the wave-specialised schedule,
// with the operands of W staged in LDS by the producer waves as two
// component planes, [2 halves][pairs][2][64 lanes] floats (Wr, Wi; the
// third operand Wr + Wi is formed right before its matrix-core step, as the
// plan rounds it).  The A and B values of each pair are read ahead of its
// products in batches of 6 pairs: batch k is issued once pair 6k - 4 is, so at most 10 pairs occupy
// registers and each wait covers only the oldest reads.  kFull (f > 34):
// every batch is read, in straight-line code; otherwise only the batches
// holding pairs below ceil(f / 2).  Rows past f and pairs past the plan's
// hold older data and feed no product.
// With kEpi, the previous product's accumulators (p1, p2, p3) are staged to
// `prev_tile` one row per pair during the chain, so the epilogue runs while
// the matrix cores are busy instead of after they drain.
template <bool kEpi, bool kFull>
__device__ __forceinline__ void chain_3m_body(const f2v *__restrict__ lds, const float *__restrict__ lds_a,
                                              int pairs, int np, int wave, int lane, floatx16 &t1,
                                              floatx16 &t2, floatx16 &t3, const floatx16 &p1,
                                              const floatx16 &p2, const floatx16 &p3,
                                              f2v *__restrict__ prev_tile)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    const int mt = wave >> 1;
    const int nt = wave & 1;
    constexpr int kBatch = 6, kLead = 4;
    const f2v *col = lds + h * kLdsCols + 32 * nt + n;
    const float *ab = lds_a + mt * pairs * 128 + lane;
    t1 = floatx16{};
    t2 = floatx16{};
    t3 = floatx16{};
    f2v a[kPairsMax];
    f2v b[kPairsMax];
    if (kFull || np > 0) {
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            b[q] = col[2 * q * kLdsCols];
            a[q] = f2v{ab[(2 * q) * 64], ab[(2 * q + 1) * 64]};
        }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < kPairsMax; ++p) {
        if (p + kLead < kPairsMax && (p + kLead) % kBatch == 0 && (kFull || p + kLead < np)) {
#pragma unroll
            for (int q = p + kLead; q < p + kLead + kBatch; ++q) {
                b[q] = col[2 * q * kLdsCols];
                a[q] = f2v{ab[(2 * q) * 64], ab[(2 * q + 1) * 64]};
            }
        }
        if (kFull || p < np)
            mfma3(f3v{a[p].x, a[p].y, a[p].x + a[p].y}, b[p], t1, t2, t3);
        if constexpr (kEpi) {
            if (p < 16)
                stage_row_3m(p1, p2, p3, p, wave, lane, prev_tile);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <bool kEpi>
__device__ __forceinline__ void chain_3m_lds(const f2v *__restrict__ lds, const float *__restrict__ lds_a,
                                             int pairs, int f, int wave, int lane, floatx16 &t1,
                                             floatx16 &t2, floatx16 &t3, const floatx16 &p1,
                                             const floatx16 &p2, const floatx16 &p3,
                                             f2v *__restrict__ prev_tile)
{
    const int np = (f + 1) >> 1;
    if (np == kPairsMax)
        chain_3m_body<kEpi, true>(lds, lds_a, pairs, np, wave, lane, t1, t2, t3, p1, p2, p3, prev_tile);
    else
        chain_3m_body<kEpi, false>(lds, lds_a, pairs, np, wave, lane, t1, t2, t3, p1, p2, p3, prev_tile);
}

__device__ __forceinline__ void stage_3m(const floatx16 &t1, const floatx16 &t2, const floatx16 &t3,
                                         int wave, int lane, f2v *__restrict__ tile)
{
#pragma unroll
    for (int r = 0; r < 16; ++r)
        stage_row_3m(t1, t2, t3, r, wave, lane, tile);
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on
// XCD b % 8).  This maps the blocks of each XCD onto one contiguous eighth
// of the (W-id ordered) item list, so each XCD's L2 holds only the W
// operands of its own eighth.  A bijection of [0, n) for any n.
__device__ __forceinline__ int xcd_contiguous(int b, int n)
{
    const int x = b & 7;
    const int j = b >> 3;
    const int q = n >> 3;
    const int r = n & 7;
    return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ float2 *sink_of(BfHeader *blk)
{
    return reinterpret_cast<float2 *>(reinterpret_cast<char *>(blk) + sizeof(BfHeader));
}

// kSched 0 for the three-product form: one product per workgroup.
template <bool kVec16>
__global__ __launch_bounds__(kThreads) void apply_fp32_3m_single(BfHeader *__restrict__ blk,
                                                                 const BfItem *__restrict__ items,
                                                                 int n_items,
                                                                 const float *__restrict__ apool,
                                                                 int a_w_stride, int pairs)
{
    __shared__ f2v lds_s[kFMax * kLdsCols];
    __shared__ f2v tile[kWaves * kWaveOut];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float2 *sink = sink_of(blk);
    const int it = xcd_contiguous(blockIdx.x, n_items);
    const BfItem d = items[it];
    f2v a[kPairsMax];
    SRegs<kVec16> sr;
    load_s<kVec16>(sr, d.f > 0 ? d.S : sink, d.f);
    if (pairs > 0)
        load_a_3m(a, apool, d.w_id, a_w_stride, pairs, wave >> 1, lane, max((d.f + 1) >> 1, 1));
    put_s<kVec16>(lds_s, sr, d.f);
    __syncthreads();
    contract_stage_3m(lds_s, a, d.f, wave, lane, tile);
    __syncthreads();
    store_staged(d.R, tile + wave * kWaveOut, wave, lane);
}

// kSched 0: one product per workgroup.
template <bool kVec16, bool kStage>
__global__ __launch_bounds__(kThreads) void apply_fp32_single(BfHeader *__restrict__ blk,
                                                              const BfItem *__restrict__ items,
                                                              int n_items,
                                                              const float2 *__restrict__ apool,
                                                              int a_w_stride, int pairs)
{
    __shared__ f2v lds_s[kFMax * kLdsCols];
    __shared__ f2v stage[kStage ? kWaves : 1][kStage ? kWaveOut : 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float2 *sink = sink_of(blk);
    const int it = xcd_contiguous(blockIdx.x, n_items);
    const BfItem d = items[it];
    f2v a[kPairsMax];
    SRegs<kVec16> sr;
    load_s<kVec16>(sr, d.f > 0 ? d.S : sink, d.f);
    if (pairs > 0)
        load_a_fp32(a, apool, d.w_id, a_w_stride, pairs, wave, lane);
    put_s<kVec16>(lds_s, sr, d.f);
    __syncthreads();
    floatx16 acc0, acc1;
    contract_fp32(lds_s, a, d.f, lane, acc0, acc1);
    write_r<kStage>(d.R, sink, stage[kStage ? wave : 0], wave, lane, acc0, acc1);
}

// kSched 1: persistent; workgroups claim items from blk->next.  The last
// workgroup to finish re-arms the counters, so graphs can replay it.
template <bool kVec16>
__global__ __launch_bounds__(kThreads) void apply_fp32_claim(BfHeader *__restrict__ blk,
                                                             const BfItem *__restrict__ items,
                                                             int n_items,
                                                             const float2 *__restrict__ apool,
                                                             int a_w_stride, int pairs)
{
    __shared__ f2v lds_s[kFMax * kLdsCols];
    __shared__ int claim;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float2 *sink = sink_of(blk);
    f2v a[kPairsMax];
    int cur_w = -1;

    if (threadIdx.x == 0)
        claim = (int)atomicAdd(&blk->next, 1u);
    __syncthreads();
    int it = __builtin_amdgcn_readfirstlane(claim);
    while (it < n_items) {
        const BfItem d = items[it];
        SRegs<kVec16> sr;
        load_s<kVec16>(sr, d.f > 0 ? d.S : sink, d.f);
        if (d.w_id != cur_w && pairs > 0) {
            cur_w = d.w_id;
            load_a_fp32(a, apool, cur_w, a_w_stride, pairs, wave, lane);
        }
        put_s<kVec16>(lds_s, sr, d.f);
        __syncthreads();
        if (threadIdx.x == 0)
            claim = (int)atomicAdd(&blk->next, 1u);
        floatx16 acc0, acc1;
        contract_fp32(lds_s, a, d.f, lane, acc0, acc1);
        store_r(d.R, sink, wave, lane, acc0, acc1);
        __syncthreads();   // LDS is reused by the next item; `claim` is ready
        it = __builtin_amdgcn_readfirstlane(claim);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&blk->done, 1u);
        if (prev == gridDim.x - 1) {
            atomicExch(&blk->next, 0u);
            atomicExch(&blk->done, 0u);
        }
    }
}

// Uniform fields of a descriptor read with a vector load (all lanes read
// the same 32 bytes), so that waiting for it does not wait for later loads.
struct DescV {
    const float2 *S;
    float2 *R;
    int w_id;
    int f;
};
__device__ __forceinline__ DescV load_desc_v(const BfItem *items, int it)
{
    typedef int i4v __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) const i4v g_ci4v;
    const g_ci4v *p = (const g_ci4v *)(items + it);
    const i4v lo = p[0];
    const i4v hi = p[1];
    DescV d;
    d.S = (const float2 *)(((uint64_t)(uint32_t)lo.y << 32) | (uint32_t)lo.x);
    d.R = (float2 *)(((uint64_t)(uint32_t)lo.w << 32) | (uint32_t)lo.z);
    d.w_id = hi.x;
    d.f = hi.y;
    return d;
}
__device__ __forceinline__ DescV uniform(const DescV &d)
{
    DescV u;
    const uint64_t s = (uint64_t)d.S;
    const uint64_t r = (uint64_t)d.R;
    u.S = (const float2 *)(((uint64_t)__builtin_amdgcn_readfirstlane((int)(s >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)s));
    u.R = (float2 *)(((uint64_t)__builtin_amdgcn_readfirstlane((int)(r >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)r));
    u.w_id = __builtin_amdgcn_readfirstlane(d.w_id);
    u.f = __builtin_amdgcn_readfirstlane(d.f);
    return u;
}

// kSched 2: persistent with a static assignment and software pipelining.
// Group x (= XCD x for grids of 8 or more blocks) owns one contiguous
// range of the item list and its blocks take turns through it; every item
// is covered, since a non-empty range always has at least one block (the
// grid is at most n_items).  Per iteration, in issue order:
//   S(i) registers -> LDS buffer; [A reload if the W id changes];
//   descriptor of item i+2 requested; barrier;
//   S(i+1) loads issued; matrix-core steps on item i; R(i) stored.
// The waits before the next iteration's LDS write cover S(i+1) only, so
// S(i+1) and R(i) traffic overlaps the compute.  Two LDS buffers alternate
// (the one written in iteration i+1 was last read in iteration i-1, before
// iteration i's barrier).
template <bool kVec16, bool kStage>
__global__ __launch_bounds__(kThreads) void apply_fp32_stream(BfHeader *__restrict__ blk,
                                                              const BfItem *__restrict__ items,
                                                              int n_items,
                                                              const float2 *__restrict__ apool,
                                                              int a_w_stride, int pairs)
{
    __shared__ f2v lds_s[2][kFMax * kLdsCols];
    __shared__ f2v stage[kStage ? kWaves : 1][kStage ? kWaveOut : 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float2 *sink = sink_of(blk);

    const int G = gridDim.x;
    const int X = G < 8 ? G : 8;
    const int x = blockIdx.x % X;
    const int j = blockIdx.x / X;
    const int nb = G / X + (x < G % X ? 1 : 0);
    const int q = n_items / X, r = n_items % X;
    const int lo = x * q + (x < r ? x : r);
    const int hi = lo + q + (x < r ? 1 : 0);

    int it = lo + j;
    if (it >= hi)
        return;
    const int last = hi - 1;
    DescV d = uniform(load_desc_v(items, it));
    int nxt = it + nb;
    DescV dn = load_desc_v(items, min(nxt, last));
    SRegs<kVec16> sr;
    load_s<kVec16>(sr, d.f > 0 ? d.S : sink, d.f);
    prime_store_count<kStoresPerProduct<kStage>>(sink, lane);
    f2v a[kPairsMax];
    int cur_w = -1;
    int buf = 0;
    while (true) {
        put_s<kVec16>(lds_s[buf], sr, d.f);
        if (d.w_id != cur_w && pairs > 0) {
            cur_w = d.w_id;
            load_a_fp32(a, apool, cur_w, a_w_stride, pairs, wave, lane);
            wait_vmem_all();
        }
        const int nn = nxt + nb;
        const DescV dnn = load_desc_v(items, min(nn, last));
        __syncthreads();
        const bool more = nxt < hi;
        const DescV du = uniform(dn);
        load_s<kVec16>(sr, du.f > 0 ? du.S : sink, du.f);
        floatx16 acc0, acc1;
        contract_fp32(lds_s[buf], a, d.f, lane, acc0, acc1);
        write_r<kStage>(d.R, sink, stage[kStage ? wave : 0], wave, lane, acc0, acc1);
        if (!more)
            break;
        d = du;
        dn = dnn;
        nxt = nn;
        buf ^= 1;
    }
}

// kSched 3: wave-specialised persistent kernel (FP32 forms).  4 + kProd
// waves per workgroup: waves 0-3 (one per SIMD) only run matrix-core steps
// from LDS; the kProd producer waves only move data.  Per product t of the
// workgroup's share (every nb-th item of its XCD's range):
//   consumers: contract S(t) from s_buf[t % 2] (three-product form: with the
//              W operands from a_buf[t % 2]), results -> r_buf[t % 2] (the
//              three-product form stages them during product t + 1);
//   producers: write R(t-1) (three-product form: R(t-2)) from LDS with
//              contiguous 16-byte stores; move S(t+1) (and W(t+1)) from
//              registers to LDS; issue
//              the loads for product t+1+kDepth into the register set that
//              product t+1 has just left;
//   one barrier.
// A buffer written in iteration t was last read in iteration t-1, before
// that iteration's barrier; one written in t is read in t+1.  The two roles
// run separate loops with the same number of barriers, so neither role's
// memory waits hold up the other's instructions.  kDepth register sets give
// each load kDepth products' time to arrive.  The four-product form keeps W
// in consumer registers and reloads them during each chain; the
// three-product form's operands (3 per pair) would not fit beside its three
// accumulators, so they come through LDS, copied once per workgroup instead
// of once per wave.

// Exponent e with 2^e <= m < 2^(e+1) for the bit pattern m of a positive
// float (0 for m == 0), clamped so that 2^-e is a normal float.
__device__ __forceinline__ int exp_of_bits(uint32_t m)
{
    if (m == 0)
        return 0;
    const int e = (int)(m >> 23) - 127;
    return e < -126 ? -126 : (e > 126 ? 126 : e);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

// Producer-side staging over kProd waves, in 16-byte chunks with clamped
// indices: S of one product and, for the three-product form, the operands
// of its W in one of the plan's two layouts (kW = 1: 32 x 32 tiles, kW = 2:
// 16 x 16 tiles; kW = 0: no W).  The 32 x 32 layout is 2 halves x pairs x 2
// planes x 64 floats (Wr, Wi; 32 chunks per pair); the producers load it in
// units of one 4-lane chunk of each plane (2 halves x pairs x 16 units).
// The 16 x 16 layout is 4 blocks x steps x 2 planes x 64 floats, loaded in
// plain 16-byte chunks.  Both are staged in LDS in the plan's layout; the
// consumers form Wr + Wi with one FP32 add.
constexpr int kWUnitsMax = kPairsMax * 32;
constexpr int kWFloatsMax = kPairsMax * 256;   // staged in LDS (either layout fits)
constexpr int kSteps16Max = (kPairsMax + 1) / 2;          // blocks of 4 flows
constexpr int kW16ChunksMax = 4 * kSteps16Max * 2 * 16;   // 16-byte chunks of a 16 x 16 layout W
static_assert(4 * kSteps16Max * 2 * 64 <= kWFloatsMax, "16 x 16 layout fits the W buffer");

template <int kProd, int kW = 0>
struct PRegs {
    static constexpr int kN = (kFMax * kB / 2 + 64 * kProd - 1) / (64 * kProd);
    static constexpr int kWRounds = kW == 2 ? (kW16ChunksMax + 64 * kProd - 1) / (64 * kProd)
                                            : (kWUnitsMax + 64 * kProd - 1) / (64 * kProd);
    static constexpr int kNW = kW == 1 ? 2 * kWRounds : (kW == 2 ? kWRounds : 1);
    f4v v[kN];
    f4v w[kNW];
};

template <int kProd, int kW>
__device__ __forceinline__ void p_load_s(PRegs<kProd, kW> &r, const float2 *__restrict__ S, int f, int ptid)
{
    g_cf4v *src = (g_cf4v *)S;
    const int last = (f > 0 ? f * (kB / 2) : 1) - 1;
#pragma unroll
    for (int u = 0; u < PRegs<kProd, kW>::kN; ++u)
        r.v[u] = src[min(ptid + u * 64 * kProd, last)];
}

// Chunk index (in the plan's and the staged layout) of the Wr chunk of unit
// u: half h, pair q, 4-lane group j; the Wi chunk follows 16 chunks later.
__device__ __forceinline__ int w_unit_chunk(int u, int pairs)
{
    const int per_half = pairs * 16;
    const int h = u >= per_half ? 1 : 0;
    const int rem = u - h * per_half;
    return h * pairs * 32 + (rem >> 4) * 32 + (rem & 15);
}

// W operands (L2-resident pool: plain loads, no streaming hint).  Only the
// first `need` (>= 1) pairs of each half are used by
// the product; units of later pairs load the last used pair's unit again
// (a cache hit; nothing of them reaches LDS).  Units past the end repeat
// the last unit.
template <int kProd>
__device__ __forceinline__ void p_load_w(PRegs<kProd, 1> &r, const float *__restrict__ wsrc, int pairs,
                                         int need, int ptid)
{
    g_cf4v *src = (g_cf4v *)wsrc;
    const int units = pairs * 32;
    const int last_q = min(pairs, need) - 1;
#pragma unroll
    for (int k = 0; k < PRegs<kProd, 1>::kWRounds; ++k) {
        int u = min(ptid + k * 64 * kProd, units - 1);
        const int per_half = pairs * 16;
        const int h = u >= per_half ? 1 : 0;
        const int rem = u - h * per_half;
        u = h * per_half + min(rem >> 4, last_q) * 16 + (rem & 15);
        const int c = w_unit_chunk(u, pairs);
        r.w[2 * k] = src[c];
        r.w[2 * k + 1] = src[c + 16];
    }
}

// Puts the Wr and Wi planes of the first `need` pairs of each antenna half
// (the only ones the product's chain reads) into the staged layout,
// [2 halves][pairs][2][64] floats, the plan's own.
template <int kProd>
__device__ __forceinline__ void p_put_w(float *__restrict__ lds_a, const PRegs<kProd, 1> &r, int pairs,
                                        int need, int ptid)
{
    const int per_half = pairs * 16;
    const int used = min(pairs, need) * 16;
#pragma unroll
    for (int k = 0; k < PRegs<kProd, 1>::kWRounds; ++k) {
        const int u = ptid + k * 64 * kProd;
        if (u < 2 * per_half && (u < per_half ? u : u - per_half) < used) {
            f4v *dst = reinterpret_cast<f4v *>(lds_a) + w_unit_chunk(u, pairs);
            dst[0] = r.w[2 * k];
            dst[16] = r.w[2 * k + 1];
        }
    }
}

// The 16 x 16 layout of one W (`steps` blocks of 4 flows per antenna block
// and plane): chunk u holds floats 4 (u % 16) .. of the 64 lanes of block
// u / 32 / steps, step (u / 32) % steps, plane (u / 16) % 2.  Only steps
// below `need` (>= 1) are used by the product; chunks of later steps load
// the last used step's chunk again (a cache hit) and are not staged.
__device__ __forceinline__ int w16_chunk(int u, int steps, int need)
{
    const int s = (u >> 5) % steps;
    return s < need ? u : u - ((s - need + 1) << 5);
}

template <int kProd>
__device__ __forceinline__ void p_load_w16(PRegs<kProd, 2> &r, const float *__restrict__ wsrc, int steps,
                                           int need, int ptid)
{
    g_cf4v *src = (g_cf4v *)wsrc;
    const int units = steps * 128;
#pragma unroll
    for (int k = 0; k < PRegs<kProd, 2>::kWRounds; ++k)
        r.w[k] = src[w16_chunk(min(ptid + k * 64 * kProd, units - 1), steps, need)];
}

template <int kProd>
__device__ __forceinline__ void p_put_w16(float *__restrict__ lds_a, const PRegs<kProd, 2> &r, int steps,
                                          int need, int ptid)
{
    const int units = steps * 128;
#pragma unroll
    for (int k = 0; k < PRegs<kProd, 2>::kWRounds; ++k) {
        const int u = ptid + k * 64 * kProd;
        if (u < units && ((u >> 5) % steps) < need)
            reinterpret_cast<f4v *>(lds_a)[u] = r.w[k];
    }
}

// Puts S into LDS row by row (pitch kLdsCols).  The rows between f and the
// next multiple of the contraction's flow granularity (2 flows for the
// 32 x 32 tiles, 4 for the 16 x 16 tiles) are cleared, so that the unused
// part of the last step multiplies zeros.
template <int kProd, int kW>
__device__ __forceinline__ void p_put_s(f2v *__restrict__ lds, const PRegs<kProd, kW> &r, int f, int ptid)
{
    const int chunks = f * (kB / 2);
#pragma unroll
    for (int u = 0; u < PRegs<kProd, kW>::kN; ++u) {
        const int c = ptid + u * 64 * kProd;
        if (c < chunks) {
            const int row = c / (kB / 2);
            const int col2 = c - row * (kB / 2);
            *reinterpret_cast<f4v *>(lds + row * kLdsCols + 2 * col2) = r.v[u];
        }
    }
    if constexpr (kW >= 2) {
        const int gap = ((f + 3) & ~3) - f;
        if (ptid < gap * kLdsCols)
            lds[f * kLdsCols + ptid] = f2v{0.f, 0.f};
    } else if (f & 1) {
        if (ptid < kLdsCols)
            lds[f * kLdsCols + ptid] = f2v{0.f, 0.f};
    }
}

// Writes the whole staged R tile (64 x 60 complex, 1920 16-byte chunks) with
// kProd waves.  Chunk indices past the end are clamped: those threads write
// the last chunk again with the same data, so every store is unconditional.
template <int kProd>
constexpr int kPStoreRounds = (kM * kB / 2 + 64 * kProd - 1) / (64 * kProd);

template <int kProd>
__device__ __forceinline__ void p_store_r(float2 *__restrict__ Rp, const f2v *__restrict__ tile, int ptid)
{
    constexpr int kChunks = kM * kB / 2;
    constexpr int kRounds = kPStoreRounds<kProd>;
    g_f4v *dst = (g_f4v *)Rp;
    const f4v *src = reinterpret_cast<const f4v *>(tile);
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
        const int c = min(ptid + u * 64 * kProd, kChunks - 1);
        __builtin_nontemporal_store(src[c], dst + c);
    }
}

// Everything the producers move for one product: its S and, for the
// three-product form, its W operands.
template <int kProd, int kW>
__device__ __forceinline__ void p_load_item(PRegs<kProd, kW> &r, const BfItem &d, bool real, float2 *sink,
                                            const void *apool, int a_w_stride, int pairs, int ptid)
{
    p_load_s<kProd, kW>(r, real && d.f > 0 ? d.S : sink, real ? d.f : 0, ptid);
    if constexpr (kW == 1)
        p_load_w<kProd>(r, static_cast<const float *>(apool) + (size_t)d.w_id * a_w_stride, pairs,
                        max((d.f + 1) >> 1, 1), ptid);
    if constexpr (kW == 2)
        p_load_w16<kProd>(r, static_cast<const float *>(apool) + (size_t)d.w_id * a_w_stride +
                                 fp32_3m16_offset(pairs),
                          fp32_3m16_steps(pairs), max((d.f + 3) >> 2, 1), ptid);
}

// Largest |Re|, |Im| (as float bits) over the valid chunks of a staged S.
template <int kProd, int kW>
__device__ __forceinline__ uint32_t p_absmax(const PRegs<kProd, kW> &r, int f, int ptid)
{
    const int chunks = f * (kB / 2);
    uint32_t m = 0;
#pragma unroll
    for (int u = 0; u < PRegs<kProd, kW>::kN; ++u) {
        if (ptid + u * 64 * kProd < chunks) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                m = max(m, __float_as_uint(r.v[u][e]) & 0x7fffffffu);
        }
    }
    return m;
}

// Puts one product's data into LDS.  kMax (16-bit forms): each producer wave
// also leaves the largest |Re|, |Im| of its part of S in smax[wave], from
// which the consumers take the product's power-of-two scale.
template <int kProd, int kW, bool kMax>
__device__ __forceinline__ void p_put_item(f2v *__restrict__ s_lds, float *__restrict__ a_lds,
                                           uint32_t *__restrict__ smax, const PRegs<kProd, kW> &r,
                                           int f, int pairs, int ptid)
{
    p_put_s<kProd, kW>(s_lds, r, f, ptid);
    if constexpr (kW == 1)
        p_put_w<kProd>(a_lds, r, pairs, max((f + 1) >> 1, 1), ptid);
    if constexpr (kW == 2)
        p_put_w16<kProd>(a_lds, r, fp32_3m16_steps(pairs), max((f + 3) >> 2, 1), ptid);
    if constexpr (kMax) {
        const uint32_t m = wave_max_u32(p_absmax<kProd, kW>(r, f, ptid));
        if ((ptid & 63) == 0)
            smax[ptid >> 6] = m;
    }
}

// Staged W operands of the workgroup (three-product form only).
template <bool k3M>
struct WBuf {
    float v[2][kWFloatsMax];
};
template <>
struct WBuf<false> {
    float v[2][1];
};

// LDS shared by the two roles of the wave-specialised kernels: S of two
// products, R of two products, the three-product form's W operands and the
// 16-bit forms' per-wave S maxima (kProd entries per product).  The member
// order sets which buffers the 16-bit offset field of LDS instructions can
// reach from one base register; the orders below are the ones that keep
// each form's kernel free of register spills.
template <bool k3M, int kProd>
struct WsLds {
    alignas(16) f2v s_buf[2][kFMax * kLdsCols];
    alignas(16) f2v r_buf[2][kM * kB];
    alignas(16) WBuf<k3M> a_buf;
    alignas(16) uint32_t smax[2][kProd];
};
template <int kProd>
struct WsLds<true, kProd> {
    alignas(16) f2v r_buf[2][kM * kB];
    alignas(16) f2v s_buf[2][kFMax * kLdsCols];
    alignas(16) WBuf<true> a_buf;
    alignas(16) uint32_t smax[2][kProd];
};

// One producer iteration t >= kLag: R(t - kLag) out (the consumers staged it
// by the end of iteration t - 1), the data of product t+1 into LDS from
// register set kPut, the loads for product t+1+kDepth into that set.  Past
// the end of the share the descriptor index is clamped and the S loads read
// the sink, so every memory instruction is unconditional; a put past the
// end fills LDS buffers nobody reads any more.
template <int kProd, int kDepth, int kPut, int kW, bool kMax, int kLag>
__device__ __forceinline__ void ws_produce_step(PRegs<kProd, kW> (&sr)[kDepth], c_item *my, int stride,
                                                int t, int n_my, float2 *sink, WsLds<kW != 0, kProd> &L,
                                                const void *apool, int a_w_stride, int pairs, int ptid)
{
    p_store_r<kProd>(item_at(my, t - kLag, stride).R, L.r_buf[(t - kLag) & 1], ptid);
    const BfItem d1 = item_at(my, min(t + 1, n_my - 1), stride);
    p_put_item<kProd, kW, kMax>(L.s_buf[(t + 1) & 1], L.a_buf.v[(t + 1) & 1], L.smax[(t + 1) & 1],
                                sr[kPut], d1.f, pairs, ptid);
    const int tn = t + 1 + kDepth;
    const BfItem dn = item_at(my, min(tn, n_my - 1), stride);
    p_load_item<kProd, kW>(sr[kPut], dn, tn < n_my, sink, apool, a_w_stride, pairs, ptid);
}

// The producer role of the wave-specialised kernels (threads 64 kCons ..,
// after the kCons matrix-core waves): product 0 straight to LDS, products
// u = 1..kDepth into register set u % kDepth, then one iteration per
// barrier of the consumers.  The consumers stage R(t) during iteration t
// (four-product and 16-bit forms) or t + 1 (three-product form, epilogue
// folded into the next chain), so iteration t writes R(t - kLag).  kW selects the W layout the
// producers stage (0: none; 3: none, with S cleared to the 16 x 16 tiles' granularity, for the
// kernel whose matrix-core waves copy W themselves).
template <int kProd, int kDepth, int kW, bool kMax, int kCons = kWaves>
__device__ __forceinline__ void ws_producer(c_item *my, int stride, int n_my, float2 *sink,
                                            WsLds<kW != 0, kProd> &L, const void *apool, int a_w_stride,
                                            int pairs)
{
    constexpr int kLag = kW != 0 ? 2 : 1;
    const int ptid = threadIdx.x - 64 * kCons;
    PRegs<kProd, kW> sr[kDepth];
    {
        const BfItem d0 = item_at(my, 0, stride);
        p_load_item<kProd, kW>(sr[0], d0, true, sink, apool, a_w_stride, pairs, ptid);
        p_put_item<kProd, kW, kMax>(L.s_buf[0], L.a_buf.v[0], L.smax[0], sr[0], d0.f, pairs, ptid);
    }
    // Each load group is preceded by as many sink stores as an iteration
    // issues R stores, and so is product 0, which has no R to write: the
    // outstanding memory operations at the loop's entry then follow the
    // same pattern as at its back edge, and the compiler's wait before
    // each put counts only the loads that put needs.
    const int plane = ptid & 63;
#pragma unroll
    for (int u = 1; u <= kDepth; ++u) {
        prime_store_count<kPStoreRounds<kProd>>(sink, plane);
        const BfItem d = item_at(my, min(u, n_my - 1), stride);
        p_load_item<kProd, kW>(sr[u % kDepth], d, u < n_my, sink, apool, a_w_stride, pairs, ptid);
    }
    __syncthreads();
    // The first kLag iterations have no R to write and issue sink stores
    // instead.
#pragma unroll
    for (int t0 = 0; t0 < kLag; ++t0) {
        prime_store_count<kPStoreRounds<kProd>>(sink, plane);
        const BfItem d1 = item_at(my, min(t0 + 1, n_my - 1), stride);
        p_put_item<kProd, kW, kMax>(L.s_buf[(t0 + 1) & 1], L.a_buf.v[(t0 + 1) & 1], L.smax[(t0 + 1) & 1],
                                     sr[(t0 + 1) % kDepth], d1.f, pairs, ptid);
        const int tn = t0 + 1 + kDepth;
        const BfItem dn = item_at(my, min(tn, n_my - 1), stride);
        p_load_item<kProd, kW>(sr[(t0 + 1) % kDepth], dn, tn < n_my, sink, apool, a_w_stride, pairs,
                                ptid);
        __syncthreads();
    }
    // Iterations kLag .. n_my + kLag - 2 in groups of kDepth, so that every
    // register set index is a constant: iteration t puts product t+1 from
    // set (t+1) % kDepth.  The loop has a single exit at its end (a break
    // in the middle becomes a flow block inside the loop, whose pessimistic
    // memory-count state would then reach the loop's first put); the
    // remaining iterations follow it.
    static_assert(kDepth >= 1 && kDepth <= 3, "prefetch depth");
    const int groups = (n_my - 1) / kDepth;
    const int rest = (n_my - 1) - groups * kDepth;
    constexpr int kP0 = (kLag + 1) % kDepth, kP1 = (kLag + 2) % kDepth, kP2 = (kLag + 3) % kDepth;
    int t = kLag;
    for (int g = 0; g < groups; ++g) {
        ws_produce_step<kProd, kDepth, kP0, kW, kMax, kLag>(sr, my, stride, t, n_my, sink, L, apool,
                                                             a_w_stride, pairs, ptid);
        __syncthreads();
        if constexpr (kDepth >= 2) {
            ws_produce_step<kProd, kDepth, kP1, kW, kMax, kLag>(sr, my, stride, t + 1, n_my, sink, L,
                                                                 apool, a_w_stride, pairs, ptid);
            __syncthreads();
        }
        if constexpr (kDepth >= 3) {
            ws_produce_step<kProd, kDepth, kP2, kW, kMax, kLag>(sr, my, stride, t + 2, n_my, sink, L,
                                                                 apool, a_w_stride, pairs, ptid);
            __syncthreads();
        }
        t += kDepth;
    }
    if constexpr (kDepth >= 2) {
        if (rest >= 1) {
            ws_produce_step<kProd, kDepth, kP0, kW, kMax, kLag>(sr, my, stride, t, n_my, sink, L, apool,
                                                                 a_w_stride, pairs, ptid);
            __syncthreads();
        }
    }
    if constexpr (kDepth >= 3) {
        if (rest >= 2) {
            ws_produce_step<kProd, kDepth, kP1, kW, kMax, kLag>(sr, my, stride, t + 1, n_my, sink, L,
                                                                 apool, a_w_stride, pairs, ptid);
            __syncthreads();
        }
    }
    p_store_r<kProd>(item_at(my, n_my - 1, stride).R, L.r_buf[(n_my - 1) & 1], ptid);
}

// The share of a workgroup of the wave-specialised kernels: the nb
// workgroups of an XCD take its items round-robin (item lo + j + k nb is
// product k of workgroup j), so at any moment they work on one contiguous
// window of the item list: R is written as one advancing front per XCD,
// which keeps HBM pages open far better than nb separate fronts would.
// Returns the number of products; *start and *stride locate them.
__device__ __forceinline__ int ws_share(int n_items, int *start, int *stride)
{
    const int G = gridDim.x;
    const int X = G < 8 ? G : 8;
    const int x = blockIdx.x % X;
    const int j = blockIdx.x / X;
    const int nb = G / X + (x < G % X ? 1 : 0);
    const int q = n_items / X, r = n_items % X;
    const int lo = x * q + (x < r ? x : r);
    const int cnt = q + (x < r ? 1 : 0);
    *start = lo + j;
    *stride = nb;
    return j < cnt ? (cnt - j + nb - 1) / nb : 0;
}

// The consumer role of apply_fp32_ws (threads 0 .. 64 kWaves - 1).
template <bool k3M, int kProd>
__device__ __forceinline__ void ws_fp32_consumer(c_item *my, int stride, int n_my, WsLds<k3M, kProd> &L,
                                                 const void *apool, int a_w_stride, int pairs, int wave,
                                                 int lane)
{
    int f = item_at(my, 0, stride).f;
    if constexpr (k3M) {
        // Product k's chain runs with product k - 1's epilogue folded in
        // (two accumulator sets, A for even k, B for odd k); the last
        // product's epilogue gets an iteration of its own, so the R of
        // product k is staged during iteration k + 1 and drained by the
        // producers in iteration k + 2.
        floatx16 a1, a2, a3, b1, b2, b3;
        __syncthreads();
        chain_3m_lds<false>(L.s_buf[0], L.a_buf.v[0], pairs, f, wave, lane, a1, a2, a3, a1, a2, a3,
                            nullptr);
        __builtin_amdgcn_sched_barrier(0);
        f = item_at(my, min(1, n_my - 1), stride).f;
        __syncthreads();
        int k = 1;
        while (true) {
            if (k >= n_my) {
                stage_3m(a1, a2, a3, wave, lane, L.r_buf[(k - 1) & 1]);
                __syncthreads();
                break;
            }
            chain_3m_lds<true>(L.s_buf[k & 1], L.a_buf.v[k & 1], pairs, f, wave, lane, b1, b2, b3, a1,
                               a2, a3, L.r_buf[(k - 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            f = item_at(my, min(k + 1, n_my - 1), stride).f;
            __syncthreads();
            ++k;
            if (k >= n_my) {
                stage_3m(b1, b2, b3, wave, lane, L.r_buf[(k - 1) & 1]);
                __syncthreads();
                break;
            }
            chain_3m_lds<true>(L.s_buf[k & 1], L.a_buf.v[k & 1], pairs, f, wave, lane, a1, a2, a3, b1,
                               b2, b3, L.r_buf[(k - 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            f = item_at(my, min(k + 1, n_my - 1), stride).f;
            __syncthreads();
            ++k;
        }
    } else {
        // W of product t is in registers when t starts; the chain of t
        // reloads them with W of t + 1 (the last product reloads its own).
        f2v a[kPairsMax];
        load_a_fp32(a, static_cast<const float2 *>(apool), item_at(my, 0, stride).w_id, a_w_stride,
                    pairs, wave, lane);
        int w_next = item_at(my, min(1, n_my - 1), stride).w_id;
        __syncthreads();
        for (int t = 0; t < n_my; ++t) {
            floatx16 acc0, acc1;
            contract_fp32_reload(L.s_buf[t & 1], a, f, lane, acc0, acc1,
                                 static_cast<const float2 *>(apool), w_next, a_w_stride, pairs, wave);
            stage_acc(L.r_buf[t & 1] + wave * kWaveOut, lane, acc0, acc1);
            __builtin_amdgcn_sched_barrier(0);
            f = item_at(my, min(t + 1, n_my - 1), stride).f;
            w_next = item_at(my, min(t + 2, n_my - 1), stride).w_id;
            __syncthreads();
        }
    }
}

// kSched 3: wave-specialised persistent kernel (FP32 forms).  S must be
// 16-byte aligned (the host routes other batches elsewhere).
template <bool k3M, int kProd, int kDepth>
__global__ __launch_bounds__(64 * (kWaves + kProd)) void apply_fp32_ws(
    BfHeader *__restrict__ blk, const BfItem *__restrict__ items, int n_items,
    const void *__restrict__ apool, int a_w_stride, int pairs)
{
    __shared__ WsLds<k3M, kProd> L;
    const int wave8 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    float2 *sink = sink_of(blk);
    int start, stride;
    const int n_my = ws_share(n_items, &start, &stride);
    if (n_my <= 0)
        return;

    c_item *my = (c_item *)items + start;
    if (wave8 < kWaves) {
        // consumer.  f of product t is read at the end of product t - 1,
        // where the barrier waits for it: a wait for a scalar read also waits
        // for every LDS read, so it must not fall among the chain's.
        ws_fp32_consumer<k3M, kProd>(my, stride, n_my, L, apool, a_w_stride, pairs, wave8, lane);
    } else {
        ws_producer<kProd, kDepth, k3M, false>(my, stride, n_my, sink, L, apool, a_w_stride, pairs);
    }
}

// ---------------------------------------------------------------------------
// FP32 forms on 16 x 16 tiles (v_mfma_f32_16x16x4_f32, the same
// matrix-core rate as the 32 x 32 x 2 form), with eight matrix-core waves,
// two per SIMD: a single wave per SIMD loses about a quarter of the matrix
// core to its own LDS reads and epilogue, which a second wave on the SIMD
// overlaps.  Matrix-core wave cw owns antennas 16 rb .. 16 rb + 15
// (rb = cw / 2) and columns 32 cb .. 32 cb + 31 (cb = cw % 2) as two 16 x 16
// tiles that share their A operands.  For v_mfma_f32_16x16x4_f32 lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] (K = 4 flows per step)
// and receives column l % 16, rows 4 (l / 16) + v of the tile in register v.
// Both forms read the same operands, Wr and Wi from the 16 x 16 W layout
// and S as staged; the three-product form keeps three accumulators per
// tile (Wr Sr, Wi Si, (Wr + Wi)(Sr + Si)), the four-product form (k4) two
// (Re R, Im R).
constexpr int kCons16 = 8;
template <bool k4>
constexpr int kAcc16 = k4 ? 2 : 3;

__device__ __forceinline__ void mfma3_16(float ar, float ai, float as, f2v b, floatx4 &t1, floatx4 &t2,
                                         floatx4 &t3)
{
    t1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b.x, t1, 0, 0, 0);
    t2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, b.y, t2, 0, 0, 0);
    t3 = __builtin_amdgcn_mfma_f32_16x16x4f32(as, b.x + b.y, t3, 0, 0, 0);
}

// One step of the four-product form on both tiles: Re R += Wr Sr - Wi Si,
// Im R += Wr Si + Wi Sr (the complex product of Section III written as four
// real ones).  Each accumulator's second update comes four instructions
// after its first, so no instruction waits for the one before it.
__device__ __forceinline__ void mfma4_16(float ar, float ai, f2v b0, f2v b1, floatx4 (&acc)[2][2])
{
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b0.x, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b0.y, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b1.x, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b1.y, acc[1][1], 0, 0, 0);
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, b0.y, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, b0.x, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, b1.y, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, b1.x, acc[1][1], 0, 0, 0);
}

// Row (t, v) of the epilogue of wave cw's two tiles, e = 4 t + v (0..7):
// Re R = T1 - T2, Im R = (T3 - T1) - T2 (three-product form) or the two
// accumulators as they are (k4) into the staged R tile (64 x 60
// row-major) at antenna 16 rb + 4 (lane / 16) + v, column 32 cb + 16 t +
// lane % 16; columns 60..63 are not written.
template <bool k4>
__device__ __forceinline__ void stage_row_16(const floatx4 (&acc)[2][kAcc16<k4>], int e, int cw, int lane,
                                             f2v *__restrict__ tile)
{
    const int t = e >> 2;
    const int v = e & 3;
    const int j = 32 * (cw & 1) + 16 * t + (lane & 15);
    const int i = 16 * (cw >> 1) + 4 * (lane >> 4) + v;
    if (j < kB) {
        if constexpr (k4) {
            tile[i * kB + j] = f2v{acc[t][0][v], acc[t][1][v]};
        } else {
            const floatx4 &t1 = acc[t][0], &t2 = acc[t][1], &t3 = acc[t][2];
            tile[i * kB + j] = f2v{t1[v] - t2[v], (t3[v] - t1[v]) - t2[v]};
        }
    }
}

// One product's chain for wave cw: `steps` blocks of 4 flows (kFull: all
// kSteps16Max), operands read from the staged S (row pitch kLdsCols) and
// the staged W (16 x 16 layout, `plan_steps` steps per block), each step's
// reads issued three steps ahead of its matrix-core work.  acc[t][m] is the
// m-th accumulator of tile t.  With kEpi, the
// previous product's accumulators `prev` are staged to `prev_tile` one row
// per step during the chain, so that this wave's epilogue falls between its
// own matrix-core steps (where the other wave of the SIMD fills the matrix
// core) instead of after the chain, where both waves of a SIMD would reach
// it together.
template <bool k4, bool kFull, bool kEpi>
__device__ __forceinline__ void chain_16(const f2v *__restrict__ s_lds, const float *__restrict__ w_lds,
                                         int plan_steps, int steps, int cw, int lane,
                                         floatx4 (&acc)[2][kAcc16<k4>], const floatx4 (&prev)[2][kAcc16<k4>],
                                         f2v *__restrict__ prev_tile)
{
    constexpr int kAhead = 3;
    const int rb = cw >> 1;
    const int cb = cw & 1;
    const f2v *col = s_lds + (lane >> 4) * kLdsCols + 32 * cb + (lane & 15);
    const float *wa = w_lds + rb * plan_steps * 128 + lane;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int m = 0; m < kAcc16<k4>; ++m)
            acc[t][m] = floatx4{};
    float ar[kSteps16Max], ai[kSteps16Max];
    f2v b0[kSteps16Max], b1[kSteps16Max];
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
        if (kFull || q < steps) {
            ar[q] = wa[q * 128];
            ai[q] = wa[q * 128 + 64];
            b0[q] = col[4 * q * kLdsCols];
            b1[q] = col[4 * q * kLdsCols + 16];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < kSteps16Max; ++q) {
        const int qn = q + kAhead;
        if (qn < kSteps16Max && (kFull || qn < steps)) {
            ar[qn] = wa[qn * 128];
            ai[qn] = wa[qn * 128 + 64];
            b0[qn] = col[4 * qn * kLdsCols];
            b1[qn] = col[4 * qn * kLdsCols + 16];
        }
        if (kFull || q < steps) {
            if constexpr (k4) {
                mfma4_16(ar[q], ai[q], b0[q], b1[q], acc);
            } else {
                const float as = ar[q] + ai[q];
                mfma3_16(ar[q], ai[q], as, b0[q], acc[0][0], acc[0][1], acc[0][2]);
                mfma3_16(ar[q], ai[q], as, b1[q], acc[1][0], acc[1][1], acc[1][2]);
            }
        }
        if constexpr (kEpi) {
            if (q < 8)
                stage_row_16<k4>(prev, q, cw, lane, prev_tile);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <bool k4, bool kEpi>
__device__ __forceinline__ void chain_16_any(const f2v *__restrict__ s_lds, const float *__restrict__ w_lds,
                                             int plan_steps, int f, int cw, int lane,
                                             floatx4 (&acc)[2][kAcc16<k4>], const floatx4 (&prev)[2][kAcc16<k4>],
                                             f2v *__restrict__ prev_tile)
{
    const int steps = (f + 3) >> 2;
    if (steps == kSteps16Max)
        chain_16<k4, true, kEpi>(s_lds, w_lds, plan_steps, steps, cw, lane, acc, prev, prev_tile);
    else
        chain_16<k4, false, kEpi>(s_lds, w_lds, plan_steps, steps, cw, lane, acc, prev, prev_tile);
}

// The matrix-core role of the 16 x 16 kernels.  Product k's chain runs with
// product k - 1's epilogue folded in (two accumulator sets, A for even k, B
// for odd k); the last product's epilogue gets an iteration of its own, so
// the R of product k is staged during iteration k + 1 and written out by the
// producers in iteration k + 2.  f of product k + 1 is read at the end of
// product k, where the barrier waits for it anyway.
// Direct global-to-LDS copy (global_load_lds_dwordx4) of the 16 x 16 layout
// W of one pool entry, the steps a product of f flows reads, into the LDS
// buffer dst, by matrix-core wave cw: instruction k of the wave copies the
// 16-byte units 512 k + 64 cw + lane.  Such a load writes LDS at its
// wave-uniform base (M0) plus 16 bytes per lane, so each instruction covers
// 64 consecutive units; the units of unused steps are left out lane by lane.
// No registers hold the data and no LDS write instruction is issued: the
// copy costs the matrix-core waves three load instructions per product.
constexpr int kW16DmaRounds = (kW16ChunksMax + 64 * kCons16 - 1) / (64 * kCons16);

__device__ __forceinline__ void dma_w16(float *__restrict__ dst, const float *__restrict__ wsrc,
                                        int plan_steps, int f, int cw, int lane)
{
    typedef __attribute__((address_space(1))) const void g_cv;
    typedef __attribute__((address_space(3))) void l_v;
    const int units = plan_steps * 128;
    const int need = max((f + 3) >> 2, 1);
#pragma unroll
    for (int k = 0; k < kW16DmaRounds; ++k) {
        const int base = 512 * k + 64 * cw;   // wave-uniform
        if (base < units) {
            const int u = base + lane;
            if (((u >> 5) % plan_steps) < need)
                __builtin_amdgcn_global_load_lds((g_cv *)(wsrc + 4 * u), (l_v *)(dst + 4 * base), 16, 0, 0);
        }
    }
}

// The pool entry and the number of 4-flow steps of W that each of the two
// LDS W buffers holds, for matrix-core waves that copy W themselves.
struct W16Held {
    int id0 = -1, id1 = -1;
    int st0 = 0, st1 = 0;
};

// The W buffer that the product with descriptor dn reads, given that the
// product before it reads buffer cur: cur again when that buffer holds the
// same pool entry with at least the steps dn needs (consecutive products
// of one W, as a W-sorted order gives them, copy it once); otherwise the
// other buffer, into which dn's W copy is issued here.  Every matrix-core
// wave takes the same decision (the descriptors are wave-uniform scalar
// loads) and copies its own part of the buffer.
__device__ __forceinline__ int w16_take(int cur, const BfItem &dn, W16Held &h, float *b0, float *b1,
                                        const float *__restrict__ w16, int a_w_stride, int plan_steps, int cw,
                                        int lane)
{
    const int need = max((dn.f + 3) >> 2, 1);
    if (dn.w_id == (cur ? h.id1 : h.id0) && need <= (cur ? h.st1 : h.st0))
        return cur;
    const int o = cur ^ 1;
    dma_w16(o ? b1 : b0, w16 + (size_t)dn.w_id * a_w_stride, plan_steps, dn.f, cw, lane);
    if (o) {
        h.id1 = dn.w_id;
        h.st1 = need;
    } else {
        h.id0 = dn.w_id;
        h.st0 = need;
    }
    return o;
}

// Waits for this wave's outstanding vector-memory loads (here only the W
// copies) and nothing else: s_waitcnt vmcnt(0) with expcnt and lgkmcnt at
// their maximum.
__device__ __forceinline__ void dma_wait()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

template <bool k4, int kProd, bool kDma, int kSBufs, class Lds>
__device__ __forceinline__ void ws16_consumer(c_item *my, int stride, int n_my, Lds &L,
                                              const float *__restrict__ apool, int a_w_stride, int pairs, int cw,
                                              int lane)
{
    const int plan_steps = fp32_3m16_steps(pairs);
    const float *w16 = apool + fp32_3m16_offset(pairs);
    floatx4 accA[2][kAcc16<k4>], accB[2][kAcc16<k4>];
    // With kDma the matrix-core waves copy each product's W themselves: W of
    // product k + 1, unless the buffer of product k already holds it, into
    // the other buffer while chain k runs (that buffer was last read by an
    // earlier chain, which every matrix-core wave finished before the
    // barrier that opened iteration k), complete before the barrier that
    // closes iteration k.  Without kDma the producers stage W of product k
    // in buffer k & 1.
    BfItem d = item_at(my, 0, stride);
    int f = d.f;
    W16Held held;
    int wb = 0;      // W buffer of the chain that runs next (kDma)
    int wn = 0;      // W buffer of the product after it (kDma)
    if constexpr (kDma) {
        dma_w16(L.a_buf.v[0], w16 + (size_t)d.w_id * a_w_stride, plan_steps, d.f, cw, lane);
        held.id0 = d.w_id;
        held.st0 = max((d.f + 3) >> 2, 1);
        dma_wait();
    }
    __syncthreads();
    if constexpr (kDma) {
        d = item_at(my, min(1, n_my - 1), stride);
        wn = w16_take(wb, d, held, L.a_buf.v[0], L.a_buf.v[1], w16, a_w_stride, plan_steps, cw, lane);
    }
    chain_16_any<k4, false>(L.s_buf[0], L.a_buf.v[0], plan_steps, f, cw, lane, accA, accA, nullptr);
    int sb = 0;   // S buffer of product k: k % kSBufs
    __builtin_amdgcn_sched_barrier(0);
    f = item_at(my, min(1, n_my - 1), stride).f;
    if constexpr (kDma)
        dma_wait();
    __syncthreads();
    wb = wn;
    int k = 1;
    while (true) {
        if (k >= n_my) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                stage_row_16<k4>(accA, e, cw, lane, L.r_buf[(k - 1) & 1]);
            __syncthreads();
            break;
        }
        if constexpr (kDma) {
            d = item_at(my, min(k + 1, n_my - 1), stride);
            wn = w16_take(wb, d, held, L.a_buf.v[0], L.a_buf.v[1], w16, a_w_stride, plan_steps, cw, lane);
        }
        sb = sb + 1 == kSBufs ? 0 : sb + 1;
        chain_16_any<k4, true>(L.s_buf[sb], L.a_buf.v[kDma ? wb : (k & 1)], plan_steps, f, cw, lane, accB,
                               accA, L.r_buf[(k - 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        f = item_at(my, min(k + 1, n_my - 1), stride).f;
        if constexpr (kDma)
            dma_wait();
        __syncthreads();
        wb = wn;
        ++k;
        if (k >= n_my) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                stage_row_16<k4>(accB, e, cw, lane, L.r_buf[(k - 1) & 1]);
            __syncthreads();
            break;
        }
        if constexpr (kDma) {
            d = item_at(my, min(k + 1, n_my - 1), stride);
            wn = w16_take(wb, d, held, L.a_buf.v[0], L.a_buf.v[1], w16, a_w_stride, plan_steps, cw, lane);
        }
        sb = sb + 1 == kSBufs ? 0 : sb + 1;
        chain_16_any<k4, true>(L.s_buf[sb], L.a_buf.v[kDma ? wb : (k & 1)], plan_steps, f, cw, lane, accA,
                               accB, L.r_buf[(k - 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        f = item_at(my, min(k + 1, n_my - 1), stride).f;
        if constexpr (kDma)
            dma_wait();
        __syncthreads();
        wb = wn;
        ++k;
    }
}

// LDS of the 16 x 16 three-product kernel whose producers copy S with
// direct global-to-LDS loads: three S buffers (S of product t + 2 is copied
// while the matrix-core waves work on t and t + 1 waits), W and R double
// buffered.
template <int kProd>
struct WsLds3 {
    alignas(16) f2v r_buf[2][kM * kB];
    alignas(16) f2v s_buf[3][kFMax * kLdsCols];
    alignas(16) WBuf<true> a_buf;
    alignas(16) uint32_t smax[2][kProd];
};

// Direct global-to-LDS copy of one product's S (f rows of 60 complex,
// contiguous, 16-byte aligned) into an S buffer (rows of kLdsCols complex) by
// producer wave pw: 16-byte unit v of the buffer (row v / 32, complex columns
// 2 (v % 32) and 2 (v % 32) + 1) comes from S + 60 row + 2 (v % 32).
// Instruction k of the wave covers units 512 k + 64 pw .. + 63 (the load
// writes LDS at its wave-uniform base plus 16 bytes per lane); the padding
// columns 60..63 and rows from f on are left out lane by lane.
constexpr int kSDmaRounds = (kFMax * 32 + 64 * 8 - 1) / (64 * 8);

__device__ __forceinline__ void dma_s(f2v *__restrict__ dst, const float2 *__restrict__ S, int f, int pw,
                                      int lane)
{
    typedef __attribute__((address_space(1))) const void g_cv;
    typedef __attribute__((address_space(3))) void l_v;
    const int units = f * 32;
#pragma unroll
    for (int k = 0; k < kSDmaRounds; ++k) {
        const int base = 512 * k + 64 * pw;   // wave-uniform
        if (base < units) {
            const int v = base + lane;
            const int row = v >> 5;
            const int c2 = v & 31;
            if (v < units && c2 < kB / 2)
                __builtin_amdgcn_global_load_lds((g_cv *)(S + kB * row + 2 * c2), (l_v *)(dst + 2 * base), 16,
                                                 0, 0);
        }
    }
}

// Clears S rows f .. 4 ceil(f / 4) - 1 of an S buffer (the last step's
// flows past f), with plain LDS writes, before that buffer's copy is issued.
__device__ __forceinline__ void clear_s_tail(f2v *__restrict__ dst, int f, int ptid)
{
    const int gap = ((f + 3) & ~3) - f;
    if (ptid < gap * kLdsCols)
        dst[f * kLdsCols + ptid] = f2v{0.f, 0.f};
}

// Barrier of the S-copying producers.  __syncthreads releases at workgroup
// scope, and with a global-to-LDS load in flight that release waits for
// every outstanding vector-memory operation: the copy of S(t + 2) just
// issued, and the R stores.  Here the LDS writes are completed explicitly
// (lgkmcnt(0)) and the copy the next chain needs was waited for before the
// next one was issued, so the barrier itself waits for nothing more; the
// compiler fences keep LDS accesses on their side of it (LDS has no cache
// to invalidate).
__device__ __forceinline__ void producer_barrier()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt and expcnt at their maximum
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// The producer role of the 16 x 16 kernel with S copied by direct loads
// (kProd = 8 waves).  Iteration t (between the barriers that open and close
// product t's chain) writes R(t - 2), waits for its vector-memory operations
// older than those stores (the copy of S(t + 1), issued at the end of
// iteration t - 1), then clears the tail rows of S(t + 2)'s buffer and
// issues its copy: the copy has the whole next iteration to land.  The
// barrier count matches the matrix-core waves' (n_my + 2).
template <int kProd>
__device__ __forceinline__ void ws_producer_sdma(c_item *my, int stride, int n_my, float2 *sink,
                                                 WsLds3<kProd> &L)
{
    static_assert(kProd == 8, "the S copy covers a product with 8 waves");
    const int ptid = threadIdx.x - 64 * kCons16;
    const int pw = __builtin_amdgcn_readfirstlane(ptid >> 6);
    const int lane = ptid & 63;
    {
        const BfItem d0 = item_at(my, 0, stride);
        clear_s_tail(L.s_buf[0], d0.f, ptid);
        if (d0.f > 0)
            dma_s(L.s_buf[0], d0.S, d0.f, pw, lane);
        if (n_my > 1) {
            const BfItem d1 = item_at(my, 1, stride);
            clear_s_tail(L.s_buf[1], d1.f, ptid);
            if (d1.f > 0)
                dma_s(L.s_buf[1], d1.S, d1.f, pw, lane);
        }
        dma_wait();
    }
    producer_barrier();
    int sb = 2;   // S buffer of product t + 2
    for (int t = 0; t < n_my; ++t) {
        if (t >= 2)
            p_store_r<kProd>(item_at(my, t - 2, stride).R, L.r_buf[t & 1], ptid);
        else
            prime_store_count<kPStoreRounds<kProd>>(sink, lane);
        // (every lane issued exactly kPStoreRounds stores since the copy of
        // S(t + 1): waiting until at most that many remain completes it)
        __builtin_amdgcn_s_waitcnt(0x0F70 | kPStoreRounds<kProd>);
        if (t + 2 < n_my) {
            const BfItem d = item_at(my, t + 2, stride);
            clear_s_tail(L.s_buf[sb], d.f, ptid);
            if (d.f > 0)
                dma_s(L.s_buf[sb], d.S, d.f, pw, lane);
        }
        sb = sb + 1 == 3 ? 0 : sb + 1;
        producer_barrier();
    }
    if (n_my >= 2)
        p_store_r<kProd>(item_at(my, n_my - 2, stride).R, L.r_buf[n_my & 1], ptid);
    producer_barrier();
    p_store_r<kProd>(item_at(my, n_my - 1, stride).R, L.r_buf[(n_my - 1) & 1], ptid);
}

// The 16 x 16 kernels with both operands copied by direct global-to-LDS
// loads: the matrix-core waves copy W (as in the kDma kernels below), the 8
// producer waves copy S and write R.
template <bool k4>
__device__ __forceinline__ void ws16_sdma_body(WsLds3<8> &L, BfHeader *__restrict__ blk,
                                               const BfItem *__restrict__ items, int n_items,
                                               const void *__restrict__ apool, int a_w_stride, int pairs)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    float2 *sink = sink_of(blk);
    int start, stride;
    const int n_my = ws_share(n_items, &start, &stride);
    if (n_my <= 0)
        return;

    c_item *my = (c_item *)items + start;
    if (wave < kCons16)
        ws16_consumer<k4, 8, true, 3>(my, stride, n_my, L, static_cast<const float *>(apool), a_w_stride, pairs,
                                      wave, lane);
    else
        ws_producer_sdma<8>(my, stride, n_my, sink, L);
}

// kSched 3 on 16 x 16 tiles: 8 matrix-core waves and kProd producer waves
// (with kDma the matrix-core waves copy W themselves).  S must be 16-byte
// aligned and the plan's f_max at least 1 (the host routes other batches
// elsewhere).
template <bool k4, int kProd, int kDepth, bool kDma>
__device__ __forceinline__ void ws16_body(WsLds<true, kProd> &L, BfHeader *__restrict__ blk,
                                          const BfItem *__restrict__ items, int n_items,
                                          const void *__restrict__ apool, int a_w_stride, int pairs)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    float2 *sink = sink_of(blk);
    int start, stride;
    const int n_my = ws_share(n_items, &start, &stride);
    if (n_my <= 0)
        return;

    c_item *my = (c_item *)items + start;
    if (wave < kCons16)
        ws16_consumer<k4, kProd, kDma, 2>(my, stride, n_my, L, static_cast<const float *>(apool), a_w_stride,
                                          pairs, wave, lane);
    else
        ws_producer<kProd, kDepth, kDma ? 3 : 2, false, kCons16>(my, stride, n_my, sink, L, apool,
                                                                 a_w_stride, pairs);
}

// The three-product form (Section III's complex product with three real
// ones) on 16 x 16 tiles.
__global__ __launch_bounds__(64 * (kCons16 + 8)) void apply_fp32_3m16_ws_sdma(
    BfHeader *__restrict__ blk, const BfItem *__restrict__ items, int n_items,
    const void *__restrict__ apool, int a_w_stride, int pairs)
{
    __shared__ WsLds3<8> L;
    ws16_sdma_body<false>(L, blk, items, n_items, apool, a_w_stride, pairs);
}

template <int kProd, int kDepth, bool kDma>
__global__ __launch_bounds__(64 * (kCons16 + kProd)) void apply_fp32_3m16_ws(
    BfHeader *__restrict__ blk, const BfItem *__restrict__ items, int n_items,
    const void *__restrict__ apool, int a_w_stride, int pairs)
{
    __shared__ WsLds<true, kProd> L;
    ws16_body<false, kProd, kDepth, kDma>(L, blk, items, n_items, apool, a_w_stride, pairs);
}

// The four-product FP32 form on 16 x 16 tiles, reading the W layout of the
// three-product form (Wr and Wi per lane).
__global__ __launch_bounds__(64 * (kCons16 + 8)) void apply_fp32_4m16_ws_sdma(
    BfHeader *__restrict__ blk, const BfItem *__restrict__ items, int n_items,
    const void *__restrict__ apool, int a_w_stride, int pairs)
{
    __shared__ WsLds3<8> L;
    ws16_sdma_body<true>(L, blk, items, n_items, apool, a_w_stride, pairs);
}

template <int kProd, int kDepth, bool kDma>
__global__ __launch_bounds__(64 * (kCons16 + kProd)) void apply_fp32_4m16_ws(
    BfHeader *__restrict__ blk, const BfItem *__restrict__ items, int n_items,
    const void *__restrict__ apool, int a_w_stride, int pairs)
{
    __shared__ WsLds<true, kProd> L;
    ws16_body<true, kProd, kDepth, kDma>(L, blk, items, n_items, apool, a_w_stride, pairs);
}

// ---------------------------------------------------------------------------
// 16-bit forms: FP16 / BF16, plain and 2-term split.
//
// The same real GEMM as the FP32 form, on v_mfma_f32_32x32x16_{f16,bf16}:
// one instruction covers K = 16 real indices, i.e. 8 flows x (re, im).  In
// step t, operand slot s of lane l (row or column l % 32, half h = l / 32)
// holds K index (flow 8t + 4h + s / 2, part s % 2).  A and B use the same
// assignment, so the instruction sums over exactly these K indices.
//
// Scaling (exact, powers of two): W is stored times 2^-eW (plan time, eW
// from the largest |Re|, |Im| of that W) and each S times 2^-eS (eS from
// the largest |Re|, |Im| of that S, found in the kernel), so operands are
// near 1 and far from FP16's range limits.  Split forms store
//   hi = RN(x),  lo = RN((x - hi) * 2^sh),  sh = 11 (FP16) or 8 (BF16),
// which keeps lo out of FP16's subnormal range; hi*hi and the cross terms
// hi*lo + lo*hi use separate FP32 accumulators, lo*lo is dropped, and
//   R = 2^(eW + eS) * (C_hh + 2^-sh * C_cross).

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u4v g_cu4v;

constexpr int kLpFlowsMax = ((kFMax + kLpFlows - 1) / kLpFlows) * kLpFlows;   // 40
constexpr int kLpChunksMax = kLpFlowsMax / kLpFlows;                            // 5
constexpr int kLpPitch = kLpFlowsMax + 4;   // dwords per LDS column: 8 lanes cover all banks

template <bool kBf16>
struct Lp;
template <>
struct Lp<false> {
    typedef _Float16 T;
    typedef _Float16 T2 __attribute__((ext_vector_type(2)));
    static constexpr int kShift = 11;
    __device__ static floatx16 mfma(u4v a, u4v b, floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8v, a),
                                                      __builtin_bit_cast(h8v, b), c, 0, 0, 0);
    }
};
template <>
struct Lp<true> {
    typedef __bf16 T;
    typedef __bf16 T2 __attribute__((ext_vector_type(2)));
    static constexpr int kShift = 8;
    __device__ static floatx16 mfma(u4v a, u4v b, floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8v, a),
                                                       __builtin_bit_cast(b8v, b), c, 0, 0, 0);
    }
};

template <bool kBf16>
__device__ __forceinline__ unsigned short to16(float x)
{
    return __builtin_bit_cast(unsigned short, (typename Lp<kBf16>::T)x);
}
template <bool kBf16>
__device__ __forceinline__ float from16(unsigned short b)
{
    return (float)__builtin_bit_cast(typename Lp<kBf16>::T, b);
}
// hi and lo (scaled by 2^kShift) 16-bit codes of x.
template <bool kBf16>
__device__ __forceinline__ void split16(float x, unsigned short &hi, unsigned short &lo)
{
    hi = to16<kBf16>(x);
    lo = to16<kBf16>((x - from16<kBf16>(hi)) * (float)(1 << Lp<kBf16>::kShift));
}

// Plan time: one block per W.  Operand layout (hi part; the plain forms'
// per-lane operands): [kWaves][chunks][64 lanes][8 x 16-bit], slot s of
// lane l in step t being real row m = l % 32 of the wave (antenna
// 16 wave + m / 2, c = m % 2) and K index (flow 8t + 4(l / 32) + s / 2,
// part q = s % 2):
//   (c, q) = (0, 0): Wr   (0, 1): -Wi   (1, 0): Wi   (1, 1): Wr.
//
// Compact layout (wc): per part (hi, then lo when `split`) dword 40 i + k
// holds the (re, im) codes of entry (antenna i, flow k < 40) of the scaled
// W, zero past f_max; the same codes as the operand layout, whose -Wi
// entries are the negated (sign-flipped) codes.  The split forms read only
// this layout.
template <bool kBf16>
__global__ __launch_bounds__(256) void w_transform_lp_kernel(const float2 *__restrict__ w, int f_max,
                                                             int chunks,
                                                             unsigned short *__restrict__ hi,
                                                             bool split,
                                                             int *__restrict__ w_exp,
                                                             uint32_t *__restrict__ wc)
{
    __shared__ uint32_t wmax[kThreads / 64];
    const size_t wi = blockIdx.x;
    const float2 *W = w + wi * kM * (size_t)f_max;
    uint32_t m = 0;
    for (int e = threadIdx.x; e < kM * f_max; e += blockDim.x) {
        const float2 v = W[e];
        m = max(m, max(__float_as_uint(v.x) & 0x7fffffffu, __float_as_uint(v.y) & 0x7fffffffu));
    }
    m = wave_max_u32(m);
    if ((threadIdx.x & 63) == 0)
        wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    m = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    const int ew = exp_of_bits(m);
    const float scale = __builtin_amdgcn_ldexpf(1.0f, -ew);
    if (threadIdx.x == 0)
        w_exp[wi] = ew;
    const size_t per_w = (size_t)kWaves * chunks * 64 * 8;
    for (size_t idx = threadIdx.x; hi && idx < per_w; idx += blockDim.x) {
        const int s = (int)(idx % 8);
        const int lane = (int)((idx / 8) % 64);
        const int t = (int)((idx / 512) % chunks);
        const int wave = (int)(idx / (512 * (size_t)chunks));
        const int mrow = lane & 31;
        const int i = 16 * wave + mrow / 2;
        const int c = mrow & 1;
        const int q = s & 1;
        const int k = kLpFlows * t + 4 * (lane >> 5) + (s >> 1);
        float x = 0.f;
        if (k < f_max) {
            const float2 v = W[(size_t)i * f_max + k];
            x = c == 0 ? (q == 0 ? v.x : -v.y) : (q == 0 ? v.y : v.x);
        }
        if (hi)
            hi[wi * per_w + idx] = to16<kBf16>(x * scale);
    }
    const size_t part = (size_t)kM * kLpWcFlows;
    uint32_t *dst = wc + wi * part * (split ? 2 : 1);
    for (int idx = threadIdx.x; idx < (int)part; idx += blockDim.x) {
        const int i = idx / kLpWcFlows;
        const int k = idx - i * kLpWcFlows;
        const float2 v = k < f_max ? W[(size_t)i * f_max + k] : make_float2(0.f, 0.f);
        unsigned short rh, rl, ih, il;
        split16<kBf16>(v.x * scale, rh, rl);
        split16<kBf16>(v.y * scale, ih, il);
        dst[idx] = (uint32_t)rh | ((uint32_t)ih << 16);
        if (split)
            dst[part + idx] = (uint32_t)rl | ((uint32_t)il << 16);
    }
}

hipError_t launch_w_transform_lp(const float2 *w_dev, int n_w, int f_max, bool bf16, void *hi,
                                 bool split, int *w_exp, uint32_t *wc, hipStream_t st)
{
    const int chunks = lp_chunks(f_max);
    if (n_w <= 0 || chunks == 0)
        return hipSuccess;
    if (bf16)
        hipLaunchKernelGGL(w_transform_lp_kernel<true>, dim3(n_w), dim3(256), 0, st, w_dev, f_max,
                           chunks, static_cast<unsigned short *>(hi), split, w_exp, wc);
    else
        hipLaunchKernelGGL(w_transform_lp_kernel<false>, dim3(n_w), dim3(256), 0, st, w_dev, f_max,
                           chunks, static_cast<unsigned short *>(hi), split, w_exp, wc);
    return hipGetLastError();
}

// Largest |Re|, |Im| (as float bits) over the valid part of staged S registers.
template <bool kVec16>
__device__ __forceinline__ uint32_t absmax_bits(const SRegs<kVec16> &r, int f)
{
    const int tid = threadIdx.x;
    uint32_t m = 0;
    if constexpr (kVec16) {
        const int chunks = f * (kB / 2);
#pragma unroll
        for (int u = 0; u < kChunks16; ++u) {
            if (tid + u * kThreads < chunks) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    m = max(m, __float_as_uint(r.v[u][e]) & 0x7fffffffu);
            }
        }
    } else {
        const int elems = f * kB;
#pragma unroll
        for (int u = 0; u < kChunks8; ++u) {
            if (tid + u * kThreads < elems) {
                m = max(m, __float_as_uint(r.v[u][0]) & 0x7fffffffu);
                m = max(m, __float_as_uint(r.v[u][1]) & 0x7fffffffu);
            }
        }
    }
    return m;
}

// Writes one complex value (scaled) as packed 16-bit (re, im) codes.
template <bool kBf16, bool kSplit>
__device__ __forceinline__ void put_c16(uint32_t *__restrict__ bhi, uint32_t *__restrict__ blo,
                                        int col, int k, float re, float im)
{
    unsigned short rh, rl, ih, il;
    split16<kBf16>(re, rh, rl);
    split16<kBf16>(im, ih, il);
    bhi[col * kLpPitch + k] = (uint32_t)rh | ((uint32_t)ih << 16);
    if (kSplit)
        blo[col * kLpPitch + k] = (uint32_t)rl | ((uint32_t)il << 16);
}

// Stages S (already in registers) into the transposed 16-bit LDS tile:
// column j holds flows 0..39 of column j as packed (re, im).  Flows
// [f, 8 ceil(f / 8)) are cleared.
template <bool kBf16, bool kSplit, bool kVec16>
__device__ __forceinline__ void put_s_lp(uint32_t *__restrict__ bhi, uint32_t *__restrict__ blo,
                                         const SRegs<kVec16> &r, int f, float scale)
{
    const int tid = threadIdx.x;
    if constexpr (kVec16) {
        const int chunks = f * (kB / 2);
#pragma unroll
        for (int u = 0; u < kChunks16; ++u) {
            const int c = tid + u * kThreads;
            if (c < chunks) {
                const int row = c / (kB / 2);
                const int col = 2 * (c - row * (kB / 2));
                put_c16<kBf16, kSplit>(bhi, blo, col, row, r.v[u][0] * scale, r.v[u][1] * scale);
                put_c16<kBf16, kSplit>(bhi, blo, col + 1, row, r.v[u][2] * scale, r.v[u][3] * scale);
            }
        }
    } else {
        const int elems = f * kB;
#pragma unroll
        for (int u = 0; u < kChunks8; ++u) {
            const int c = tid + u * kThreads;
            if (c < elems) {
                const int row = c / kB;
                const int col = c - row * kB;
                put_c16<kBf16, kSplit>(bhi, blo, col, row, r.v[u][0] * scale, r.v[u][1] * scale);
            }
        }
    }
    const int fpad = (f + kLpFlows - 1) & ~(kLpFlows - 1);
    const int gap = fpad - f;
    if (gap > 0) {
        for (int e = tid; e < kB * gap; e += kThreads) {
            const int col = e / gap;
            const int k = f + (e - col * gap);
            bhi[col * kLpPitch + k] = 0u;
            if (kSplit)
                blo[col * kLpPitch + k] = 0u;
        }
    }
}

template <bool kSplit>
struct LpA {
    u4v hi[kLpChunksMax];
    u4v lo[kSplit ? kLpChunksMax : 1];
};

// A operands of the plain forms from the plan's per-lane operand layout.
__device__ __forceinline__ void load_a_lp(LpA<false> &a, const PlanDev &pd, int w, int wave, int lane)
{
    const size_t base = (size_t)w * pd.lp_stride + (size_t)wave * pd.lp_chunks * 64 + lane;
    const g_cu4v *h = (const g_cu4v *)pd.lp_hi + base;
#pragma unroll
    for (int t = 0; t < kLpChunksMax; ++t)
        a.hi[t] = h[min(t, pd.lp_chunks - 1) * 64];
}

// Matrix-core steps of one product from the staged 16-bit tile, then the
// rescaled result to R.
template <bool kBf16, bool kSplit>
__device__ __forceinline__ void contract_lp(const uint32_t *__restrict__ bhi,
                                            const uint32_t *__restrict__ blo, const LpA<kSplit> &a,
                                            int f, int eo, int lane, floatx16 &o0, floatx16 &o1)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    const int tc = (f + kLpFlows - 1) / kLpFlows;
    floatx16 hh0 = {}, hh1 = {}, cr0 = {}, cr1 = {};
#pragma unroll
    for (int t = 0; t < kLpChunksMax; ++t) {
        if (t < tc) {
            const int k0 = kLpFlows * t + 4 * h;
            const u4v b0 = *reinterpret_cast<const u4v *>(bhi + n * kLpPitch + k0);
            const u4v b1 = *reinterpret_cast<const u4v *>(bhi + (32 + n) * kLpPitch + k0);
            hh0 = Lp<kBf16>::mfma(a.hi[t], b0, hh0);
            hh1 = Lp<kBf16>::mfma(a.hi[t], b1, hh1);
            if constexpr (kSplit) {
                const u4v l0 = *reinterpret_cast<const u4v *>(blo + n * kLpPitch + k0);
                const u4v l1 = *reinterpret_cast<const u4v *>(blo + (32 + n) * kLpPitch + k0);
                cr0 = Lp<kBf16>::mfma(a.hi[t], l0, cr0);
                cr1 = Lp<kBf16>::mfma(a.hi[t], l1, cr1);
                cr0 = Lp<kBf16>::mfma(a.lo[t], b0, cr0);
                cr1 = Lp<kBf16>::mfma(a.lo[t], b1, cr1);
            }
        }
    }
    const float back = __builtin_amdgcn_ldexpf(1.0f, -Lp<kBf16>::kShift);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        float v0 = hh0[r], v1 = hh1[r];
        if constexpr (kSplit) {
            v0 = __builtin_fmaf(cr0[r], back, v0);
            v1 = __builtin_fmaf(cr1[r], back, v1);
        }
        o0[r] = __builtin_amdgcn_ldexpf(v0, eo);
        o1[r] = __builtin_amdgcn_ldexpf(v1, eo);
    }
}

// kSched 3 for the 16-bit forms: wave-specialised, with the producers
// splitting S into 16-bit operands as they put it into LDS, so each value
// is converted once and the consumers only read operands and issue
// matrix-core steps.  The producers also stage each product's W, in the
// plan's compact layout (one dword of (re, im) codes per entry and part),
// from which the consumers form their operands; the consumers then issue
// no memory loads at all.  A product's power-of-two scale must be known
// before its conversion: the producers publish the largest |Re|, |Im| of
// their part of product t + 2 in iteration t (smax, per wave) and convert
// product t + 1 with the scale published for it in iteration t - 1.  This
// needs S in producer registers two products ahead of its put (depth >= 2);
// the loads of a product have kDepth - 1 iterations to arrive.
//
// LDS operand layout of S (per part, hi and lo): dword ((k / 4) 64 + c) 4 +
// k % 4 holds (re, im) of flow k, column c as two 16-bit codes, so the
// operand of lane (column n, half h) in chunk t is the 16 bytes at group
// 2t + h.
constexpr int kLpB = (kLpFlowsMax / 4) * 64 * 4;   // dwords per part: 40 flows x 64 columns
constexpr int kLpWcP = kM * kLpWcFlows;            // dwords per part of a compact W
static_assert(kLpWcFlows == kLpFlowsMax, "compact W covers the padded flows");

// Every member starts on a 16-byte boundary (its 16-byte accesses would
// otherwise be split).
template <int kProd, bool kSplit>
struct WsLdsLp {
    alignas(16) uint32_t b_hi[2][kLpB];
    alignas(16) uint32_t b_lo[2][kSplit ? kLpB : 4];
    alignas(16) uint32_t w[2][(kSplit ? 2 : 1) * kLpWcP];
    alignas(16) f2v r_buf[2][kM * kB];
    alignas(16) uint32_t smax[2][kProd];
    int es[2];
};

// One product's S and (unless the consumers stage W, kWC) its compact W in
// producer registers.
template <int kProd, bool kSplit, bool kWC = false>
struct PRegsLp {
    static constexpr int kWChunks = (kSplit ? 2 : 1) * kLpWcP / 4;
    static constexpr int kNW = kWC ? 1 : (kWChunks + 64 * kProd - 1) / (64 * kProd);
    PRegs<kProd, false> s;
    f4v w[kNW];
};

// hi and lo (scaled by 2^kShift) 16-bit codes of a complex value, packed as
// (re, im) pairs; the same rounding as split16, two values per instruction.
template <bool kBf16, bool kSplit>
__device__ __forceinline__ void split_pair(f2v v, uint32_t &hi, uint32_t &lo)
{
    typedef typename Lp<kBf16>::T2 T2;
    const T2 h = __builtin_convertvector(v, T2);
    hi = __builtin_bit_cast(uint32_t, h);
    if constexpr (kSplit) {
        const f2v r = (v - __builtin_convertvector(h, f2v)) * (float)(1 << Lp<kBf16>::kShift);
        lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, T2));
    }
}

// Every producer wave leaves the largest |Re|, |Im| of its part of a staged S.
template <int kProd>
__device__ __forceinline__ void p_publish_max(uint32_t *__restrict__ smax, const PRegs<kProd, false> &r,
                                              int f, int ptid)
{
    const uint32_t m = wave_max_u32(p_absmax<kProd, false>(r, f, ptid));
    if ((ptid & 63) == 0)
        smax[ptid >> 6] = m;
}

// Converts a staged S (scale 2^-es, es from the published maxima) into the
// 16-bit operand layout, flows f .. 8 ceil(f / 8) - 1 cleared, and copies
// the staged W (kWC: the consumers stage W).  One lane leaves es for the
// consumers.
template <bool kBf16, bool kSplit, int kProd, bool kWC>
__device__ __forceinline__ void p_put_lp(uint32_t *__restrict__ bhi, uint32_t *__restrict__ blo,
                                         uint32_t *__restrict__ wl, const uint32_t *__restrict__ smax,
                                         int *__restrict__ es_out, const PRegsLp<kProd, kSplit, kWC> &r, int f,
                                         int ptid)
{
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kProd; ++i)
        m = max(m, smax[i]);
    const int es = exp_of_bits(m);
    const float sc = __builtin_amdgcn_ldexpf(1.0f, -es);
    if (ptid == 0)
        *es_out = es;
    const int chunks = f * (kB / 2);
#pragma unroll
    for (int u = 0; u < PRegs<kProd, false>::kN; ++u) {
        const int c = ptid + u * 64 * kProd;
        if (c < chunks) {
            const int row = c / (kB / 2);
            const int col = 2 * (c - row * (kB / 2));
            const int d = ((row >> 2) * 64 + col) * 4 + (row & 3);
            uint32_t h0, l0 = 0, h1, l1 = 0;
            split_pair<kBf16, kSplit>(f2v{r.s.v[u][0], r.s.v[u][1]} * sc, h0, l0);
            split_pair<kBf16, kSplit>(f2v{r.s.v[u][2], r.s.v[u][3]} * sc, h1, l1);
            bhi[d] = h0;
            bhi[d + 4] = h1;
            if constexpr (kSplit) {
                blo[d] = l0;
                blo[d + 4] = l1;
            }
        }
    }
    const int fpad = (f + kLpFlows - 1) & ~(kLpFlows - 1);
    const int gap = fpad - f;
    for (int e = ptid; e < 64 * gap; e += 64 * kProd) {
        const int col = e / gap;
        const int k = f + (e - col * gap);
        const int d = ((k >> 2) * 64 + col) * 4 + (k & 3);
        bhi[d] = 0u;
        if constexpr (kSplit)
            blo[d] = 0u;
    }
    if constexpr (!kWC) {
#pragma unroll
        for (int u = 0; u < PRegsLp<kProd, kSplit, kWC>::kNW; ++u) {
            const int c = ptid + u * 64 * kProd;
            if (c < PRegsLp<kProd, kSplit, kWC>::kWChunks)
                reinterpret_cast<f4v *>(wl)[c] = r.w[u];
        }
    }
}

// Loads of product u (S and compact W) into a register set; past the end
// the S loads read the sink (f = 0) and W is the last product's.
template <int kProd, bool kSplit, bool kWC>
__device__ __forceinline__ void p_load_lp(PRegsLp<kProd, kSplit, kWC> &r, c_item *my, int stride, int u,
                                          int n_my, float2 *sink, const PlanDev &pd, int ptid)
{
    const BfItem d = item_at(my, min(u, n_my - 1), stride);
    const bool real = u < n_my;
    p_load_s<kProd, false>(r.s, real && d.f > 0 ? d.S : sink, real ? d.f : 0, ptid);
    if constexpr (!kWC) {
        g_cf4v *src = (g_cf4v *)(pd.lp_wc + (size_t)d.w_id * pd.lp_wc_stride);
        constexpr int kLast = PRegsLp<kProd, kSplit, kWC>::kWChunks - 1;
#pragma unroll
        for (int q = 0; q < PRegsLp<kProd, kSplit, kWC>::kNW; ++q)
            r.w[q] = src[min(ptid + q * 64 * kProd, kLast)];
    }
}

// The compact W of pool entry w staged by the kWaves consumer waves
// (thread ctid < 64 kWaves): loads into registers, then a copy into LDS.
template <bool kSplit>
struct CRegsW {
    static constexpr int kChunks = (kSplit ? 2 : 1) * kLpWcP / 4;
    static constexpr int kN = (kChunks + 64 * kWaves - 1) / (64 * kWaves);
    f4v w[kN];
};

template <bool kSplit>
__device__ __forceinline__ void c_load_w(CRegsW<kSplit> &r, const PlanDev &pd, int w, int ctid)
{
    g_cf4v *src = (g_cf4v *)(pd.lp_wc + (size_t)w * pd.lp_wc_stride);
#pragma unroll
    for (int q = 0; q < CRegsW<kSplit>::kN; ++q)
        r.w[q] = src[min(ctid + q * 64 * kWaves, CRegsW<kSplit>::kChunks - 1)];
}

template <bool kSplit>
__device__ __forceinline__ void c_put_w(uint32_t *__restrict__ wl, const CRegsW<kSplit> &r, int ctid)
{
#pragma unroll
    for (int q = 0; q < CRegsW<kSplit>::kN; ++q) {
        const int c = ctid + q * 64 * kWaves;
        if (c < CRegsW<kSplit>::kChunks)
            reinterpret_cast<f4v *>(wl)[c] = r.w[q];
    }
}

// One producer iteration t >= 1: R(t - 1) out, product t + 1 converted from
// set kPut, the maxima of product t + 2 (set kMax) published, the loads of
// product t + 1 + kDepth into set kPut.
template <bool kBf16, bool kSplit, int kProd, int kDepth, int kPut, int kMax, bool kWC>
__device__ __forceinline__ void ws_lp_step(PRegsLp<kProd, kSplit, kWC> (&sr)[kDepth], c_item *my, int stride,
                                           int t, int n_my, float2 *sink, WsLdsLp<kProd, kSplit> &L,
                                           const PlanDev &pd, int ptid)
{
    p_store_r<kProd>(item_at(my, t - 1, stride).R, L.r_buf[(t - 1) & 1], ptid);
    const int f1 = item_at(my, min(t + 1, n_my - 1), stride).f;
    const int f2 = t + 2 < n_my ? item_at(my, t + 2, stride).f : 0;
    p_put_lp<kBf16, kSplit, kProd, kWC>(L.b_hi[(t + 1) & 1], L.b_lo[kSplit ? (t + 1) & 1 : 0], L.w[(t + 1) & 1],
                                   L.smax[(t + 1) & 1], &L.es[(t + 1) & 1], sr[kPut], f1, ptid);
    p_publish_max<kProd>(L.smax[t & 1], sr[kMax].s, f2, ptid);
    p_load_lp<kProd, kSplit, kWC>(sr[kPut], my, stride, t + 1 + kDepth, n_my, sink, pd, ptid);
}

// The producer role (threads 64 kWaves ..).  Barriers: one before product
// 0's conversion, then as the consumers: one before product 0 is used and
// one after each product.
template <bool kBf16, bool kSplit, int kProd, int kDepth, bool kWC>
__device__ __forceinline__ void ws_producer_lp(c_item *my, int stride, int n_my, float2 *sink,
                                               WsLdsLp<kProd, kSplit> &L, const PlanDev &pd)
{
    static_assert(kDepth >= 2 && kDepth <= 3, "prefetch depth");
    const int ptid = threadIdx.x - 64 * kWaves;
    const int plane = ptid & 63;
    PRegsLp<kProd, kSplit, kWC> sr[kDepth];
    // Each load group is preceded by as many sink stores as an iteration
    // issues R stores, so that the outstanding memory operations at the
    // loop's entry follow the pattern of its back edge.
#pragma unroll
    for (int u = 0; u < kDepth; ++u) {
        prime_store_count<kPStoreRounds<kProd>>(sink, plane);
        p_load_lp<kProd, kSplit, kWC>(sr[u], my, stride, u, n_my, sink, pd, ptid);
    }
    p_publish_max<kProd>(L.smax[0], sr[0].s, item_at(my, 0, stride).f, ptid);
    __syncthreads();
    p_put_lp<kBf16, kSplit, kProd, kWC>(L.b_hi[0], L.b_lo[0], L.w[0], L.smax[0], &L.es[0], sr[0],
                                   item_at(my, 0, stride).f, ptid);
    p_publish_max<kProd>(L.smax[1], sr[1].s, 1 < n_my ? item_at(my, 1, stride).f : 0, ptid);
    prime_store_count<kPStoreRounds<kProd>>(sink, plane);
    p_load_lp<kProd, kSplit, kWC>(sr[0], my, stride, kDepth, n_my, sink, pd, ptid);
    __syncthreads();
    // iteration 0: no R to write yet
    {
        prime_store_count<kPStoreRounds<kProd>>(sink, plane);
        const int f1 = item_at(my, min(1, n_my - 1), stride).f;
        const int f2 = 2 < n_my ? item_at(my, 2, stride).f : 0;
        p_put_lp<kBf16, kSplit, kProd, kWC>(L.b_hi[1], L.b_lo[kSplit ? 1 : 0], L.w[1], L.smax[1], &L.es[1], sr[1],
                                       f1, ptid);
        p_publish_max<kProd>(L.smax[0], sr[2 % kDepth].s, f2, ptid);
        p_load_lp<kProd, kSplit, kWC>(sr[1], my, stride, 1 + kDepth, n_my, sink, pd, ptid);
        __syncthreads();
    }
    // Iterations 1 .. n_my - 1 in groups of kDepth (constant register set
    // indices; a single exit at the loop's end), then the remainder.
    const int groups = (n_my - 1) / kDepth;
    const int rest = (n_my - 1) - groups * kDepth;
    constexpr int kA0 = 2 % kDepth, kB0 = 3 % kDepth;
    constexpr int kA1 = 3 % kDepth, kB1 = 4 % kDepth;
    constexpr int kA2 = 4 % kDepth, kB2 = 5 % kDepth;
    int t = 1;
    for (int g = 0; g < groups; ++g) {
        ws_lp_step<kBf16, kSplit, kProd, kDepth, kA0, kB0, kWC>(sr, my, stride, t, n_my, sink, L, pd, ptid);
        __syncthreads();
        ws_lp_step<kBf16, kSplit, kProd, kDepth, kA1, kB1, kWC>(sr, my, stride, t + 1, n_my, sink, L, pd, ptid);
        __syncthreads();
        if constexpr (kDepth >= 3) {
            ws_lp_step<kBf16, kSplit, kProd, kDepth, kA2, kB2, kWC>(sr, my, stride, t + 2, n_my, sink, L, pd,
                                                               ptid);
            __syncthreads();
        }
        t += kDepth;
    }
    if (rest >= 1) {
        ws_lp_step<kBf16, kSplit, kProd, kDepth, kA0, kB0, kWC>(sr, my, stride, t, n_my, sink, L, pd, ptid);
        __syncthreads();
    }
    if constexpr (kDepth >= 3) {
        if (rest >= 2) {
            ws_lp_step<kBf16, kSplit, kProd, kDepth, kA1, kB1, kWC>(sr, my, stride, t + 1, n_my, sink, L, pd,
                                                               ptid);
            __syncthreads();
        }
    }
    p_store_r<kProd>(item_at(my, n_my - 1, stride).R, L.r_buf[(n_my - 1) & 1], ptid);
}

// Matrix-core steps of one chunk for one 32-column tile.
template <bool kBf16, bool kSplit>
__device__ __forceinline__ void lp_mma(const u4v &ahi, const u4v &alo, const u4v &bh, const u4v &bl,
                                       floatx16 &hh, floatx16 &cr)
{
    hh = Lp<kBf16>::mfma(ahi, bh, hh);
    if constexpr (kSplit) {
        cr = Lp<kBf16>::mfma(ahi, bl, cr);
        cr = Lp<kBf16>::mfma(alo, bh, cr);
    }
}

// Operand of a lane from four compact dwords (flows k .. k + 3 of its
// antenna): real rows (c = 0) take (Wr, -Wi), i.e. the sign of the high
// half flipped; imaginary rows (c = 1) take (Wi, Wr), the halves swapped.
__device__ __forceinline__ u4v lp_a_of(u4v x, uint32_t rot, uint32_t flip)
{
    u4v a;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        a[j] = __builtin_amdgcn_alignbit(x[j], x[j], rot) ^ flip;
    return a;
}

// One product from the 16-bit operands in LDS (result scaled by 2^eo),
// staged into `stage`: both 32-column tiles, chunk by chunk, W operands
// formed from the staged compact W.
template <bool kBf16, bool kSplit>
__device__ __forceinline__ void lp_chain_ws(const uint32_t *__restrict__ bhi, const uint32_t *__restrict__ blo,
                                            const uint32_t *__restrict__ wl, int f, int eo, int wave, int lane,
                                            f2v *__restrict__ stage)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    const int tc = (f + kLpFlows - 1) / kLpFlows;
    const u4v *ph = reinterpret_cast<const u4v *>(bhi) + h * 64 + n;
    const u4v *pl = reinterpret_cast<const u4v *>(blo) + h * 64 + n;
    // this lane's real row: antenna 16 wave + n / 2, component n % 2
    const u4v *pw = reinterpret_cast<const u4v *>(wl + (16 * wave + (n >> 1)) * kLpWcFlows + 4 * h);
    const uint32_t rot = (n & 1) ? 16u : 0u;
    const uint32_t flip = (n & 1) ? 0u : 0x80000000u;
    floatx16 hh0 = {}, hh1 = {}, cr0 = {}, cr1 = {};
    const u4v zero = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int t = 0; t < kLpChunksMax; ++t) {
        if (tc == kLpChunksMax || t < tc) {
            const int g = 2 * t * 64;
            const u4v ahi = lp_a_of(pw[2 * t], rot, flip);
            const u4v alo = kSplit ? lp_a_of(pw[kLpWcP / 4 + 2 * t], rot, flip) : zero;
            lp_mma<kBf16, kSplit>(ahi, alo, ph[g], kSplit ? pl[g] : zero, hh0, cr0);
            lp_mma<kBf16, kSplit>(ahi, alo, ph[g + 32], kSplit ? pl[g + 32] : zero, hh1, cr1);
        }
    }
    const float back = __builtin_amdgcn_ldexpf(1.0f, -Lp<kBf16>::kShift);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        float v0 = hh0[r], v1 = hh1[r];
        if constexpr (kSplit) {
            v0 = __builtin_fmaf(cr0[r], back, v0);
            v1 = __builtin_fmaf(cr1[r], back, v1);
        }
        hh0[r] = __builtin_amdgcn_ldexpf(v0, eo);
        hh1[r] = __builtin_amdgcn_ldexpf(v1, eo);
    }
    stage_acc(stage, lane, hh0, hh1);
}

// S must be 16-byte aligned and the plan's f_max at least 1 (the host routes
// other batches elsewhere).
template <bool kBf16, bool kSplit, int kProd, int kDepth, bool kWC>
__global__ __launch_bounds__(64 * (kWaves + kProd)) void apply_lp_ws(BfHeader *__restrict__ blk,
                                                                     const BfItem *__restrict__ items,
                                                                     int n_items, PlanDev pd)
{
    __shared__ WsLdsLp<kProd, kSplit> L;
    const int wave8 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    float2 *sink = sink_of(blk);
    int start, stride;
    const int n_my = ws_share(n_items, &start, &stride);
    if (n_my <= 0)
        return;

    c_item *my = (c_item *)items + start;
    if (wave8 < kWaves) {
        // consumer.  The scalar reads for later products (f of t + 1, the W
        // exponent of t + 1) are issued at the end of product t, where the
        // barrier waits for them anyway.
        // With kWC the consumers also stage W: product t + 1's W is loaded
        // while product t's chain runs and copied into LDS before the
        // barrier (the producers then move S only).
        const int wave = wave8;
        int f = item_at(my, 0, stride).f;
        int ew = pd.lp_exp[item_at(my, 0, stride).w_id];
        CRegsW<kSplit> wr;
        if constexpr (kWC) {
            c_load_w<kSplit>(wr, pd, item_at(my, 0, stride).w_id, threadIdx.x);
            c_put_w<kSplit>(L.w[0], wr, threadIdx.x);
        }
        __syncthreads();
        __syncthreads();
        for (int t = 0; t < n_my; ++t) {
            if constexpr (kWC)
                c_load_w<kSplit>(wr, pd, item_at(my, min(t + 1, n_my - 1), stride).w_id, threadIdx.x);
            lp_chain_ws<kBf16, kSplit>(L.b_hi[t & 1], L.b_lo[kSplit ? t & 1 : 0], L.w[t & 1], f,
                                       ew + L.es[t & 1], wave, lane, L.r_buf[t & 1] + wave * kWaveOut);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (kWC)
                c_put_w<kSplit>(L.w[(t + 1) & 1], wr, threadIdx.x);
            const BfItem dn = item_at(my, min(t + 1, n_my - 1), stride);
            f = dn.f;
            ew = pd.lp_exp[dn.w_id];
            __syncthreads();
        }
    } else {
        ws_producer_lp<kBf16, kSplit, kProd, kDepth, kWC>(my, stride, n_my, sink, L, pd);
    }
}

constexpr int kLpTile = 64 * kLpPitch;   // dwords per staged 16-bit tile

// kSched 0 for the 16-bit forms: one product per workgroup.
// A operands of the split forms (hi and lo parts) for one wave (16
// antennas, both components) and all chunks of a W, formed from the plan's
// compact layout as the wave-specialised consumers form them: lane l's row
// is antenna 16 wave + (l % 32) / 2, component l % 2, and lanes l and l ^ 1
// read the same dwords, so a wave loads half the bytes a per-lane operand
// layout would take.  (For the plain forms the per-lane layout measured
// faster and is kept.)
__device__ __forceinline__ void load_a_lp(LpA<true> &a, const PlanDev &pd, int w, int wave, int lane)
{
    constexpr bool kSplit = true;
    const int h = lane >> 5;
    const int n = lane & 31;
    const g_cu4v *src = (const g_cu4v *)(pd.lp_wc + (size_t)w * pd.lp_wc_stride +
                                         (16 * wave + (n >> 1)) * kLpWcFlows + 4 * h);
    const uint32_t rot = (n & 1) ? 16u : 0u;
    const uint32_t flip = (n & 1) ? 0u : 0x80000000u;
    u4v raw[kSplit ? 2 * kLpChunksMax : kLpChunksMax];
#pragma unroll
    for (int t = 0; t < kLpChunksMax; ++t)
        raw[t] = src[2 * t];
    if constexpr (kSplit) {
#pragma unroll
        for (int t = 0; t < kLpChunksMax; ++t)
            raw[kLpChunksMax + t] = src[kLpWcP / 4 + 2 * t];
    }
#pragma unroll
    for (int t = 0; t < kLpChunksMax; ++t)
        a.hi[t] = lp_a_of(raw[t], rot, flip);
    if constexpr (kSplit) {
#pragma unroll
        for (int t = 0; t < kLpChunksMax; ++t)
            a.lo[t] = lp_a_of(raw[kLpChunksMax + t], rot, flip);
    }
}

template <bool kBf16, bool kSplit, bool kVec16, bool kStage>
__global__ __launch_bounds__(kThreads) void apply_lp_single(BfHeader *__restrict__ blk,
                                                            const BfItem *__restrict__ items,
                                                            int n_items, PlanDev pd)
{
    __shared__ uint32_t lds_hi[kLpTile];
    __shared__ uint32_t lds_lo[kSplit ? kLpTile : 1];
    __shared__ uint32_t smax[kWaves];
    __shared__ f2v stage[kStage ? kWaves : 1][kStage ? kWaveOut : 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float2 *sink = sink_of(blk);
    const int it = xcd_contiguous(blockIdx.x, n_items);
    const BfItem d = items[it];
    SRegs<kVec16> sr;
    load_s<kVec16>(sr, d.f > 0 ? d.S : sink, d.f);
    LpA<kSplit> a;
    int ew = 0;
    if (pd.lp_chunks > 0) {
        load_a_lp(a, pd, d.w_id, wave, lane);
        ew = pd.lp_exp[d.w_id];
    }
    const uint32_t m = wave_max_u32(absmax_bits<kVec16>(sr, d.f));
    if (lane == 0)
        smax[wave] = m;
    __syncthreads();
    const int es = exp_of_bits(max(max(smax[0], smax[1]), max(smax[2], smax[3])));
    put_s_lp<kBf16, kSplit, kVec16>(lds_hi, lds_lo, sr, d.f, __builtin_amdgcn_ldexpf(1.0f, -es));
    __syncthreads();
    floatx16 o0, o1;
    contract_lp<kBf16, kSplit>(lds_hi, lds_lo, a, d.f, ew + es, lane, o0, o1);
    write_r<kStage>(d.R, sink, stage[kStage ? wave : 0], wave, lane, o0, o1);
}

// kSched 2 for the 16-bit forms: persistent, static share, next S
// prefetched during the current product's matrix-core steps (as
// apply_fp32_stream, with an extra barrier for the per-product scale).
template <bool kBf16, bool kSplit, bool kVec16, bool kStage>
__global__ __launch_bounds__(kThreads) void apply_lp_stream(BfHeader *__restrict__ blk,
                                                            const BfItem *__restrict__ items,
                                                            int n_items, PlanDev pd)
{
    __shared__ uint32_t lds_hi[2][kLpTile];
    __shared__ uint32_t lds_lo[2][kSplit ? kLpTile : 1];
    __shared__ uint32_t smax[2][kWaves];
    __shared__ f2v stage[kStage ? kWaves : 1][kStage ? kWaveOut : 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float2 *sink = sink_of(blk);

    const int G = gridDim.x;
    const int X = G < 8 ? G : 8;
    const int x = blockIdx.x % X;
    const int j = blockIdx.x / X;
    const int nb = G / X + (x < G % X ? 1 : 0);
    const int q = n_items / X, r = n_items % X;
    const int lo = x * q + (x < r ? x : r);
    const int hi = lo + q + (x < r ? 1 : 0);

    int it = lo + j;
    if (it >= hi)
        return;
    const int last = hi - 1;
    DescV d = uniform(load_desc_v(items, it));
    int nxt = it + nb;
    DescV dn = load_desc_v(items, min(nxt, last));
    SRegs<kVec16> sr;
    load_s<kVec16>(sr, d.f > 0 ? d.S : sink, d.f);
    prime_store_count<kStoresPerProduct<kStage>>(sink, lane);
    LpA<kSplit> a;
    int cur_w = -1;
    int ew = 0;
    int buf = 0;
    while (true) {
        const uint32_t m = wave_max_u32(absmax_bits<kVec16>(sr, d.f));
        if (lane == 0)
            smax[buf][wave] = m;
        if (d.w_id != cur_w && pd.lp_chunks > 0) {
            cur_w = d.w_id;
            load_a_lp(a, pd, cur_w, wave, lane);
            ew = pd.lp_exp[cur_w];
            wait_vmem_all();
        }
        const int nn = nxt + nb;
        const DescV dnn = load_desc_v(items, min(nn, last));
        __syncthreads();
        const int es = exp_of_bits(max(max(smax[buf][0], smax[buf][1]), max(smax[buf][2], smax[buf][3])));
        put_s_lp<kBf16, kSplit, kVec16>(lds_hi[buf], lds_lo[buf], sr, d.f,
                                        __builtin_amdgcn_ldexpf(1.0f, -es));
        __syncthreads();
        const bool more = nxt < hi;
        const DescV du = uniform(dn);
        load_s<kVec16>(sr, du.f > 0 ? du.S : sink, du.f);
        floatx16 o0, o1;
        contract_lp<kBf16, kSplit>(lds_hi[buf], lds_lo[buf], a, d.f, ew + es, lane, o0, o1);
        write_r<kStage>(d.R, sink, stage[kStage ? wave : 0], wave, lane, o0, o1);
        if (!more)
            break;
        d = du;
        dn = dnn;
        nxt = nn;
        buf ^= 1;
    }
}

static const BfItem *items_of(BfHeader *blk)
{
    return reinterpret_cast<const BfItem *>(reinterpret_cast<const char *>(blk) +
                                            sizeof(BfHeader) + kSinkBytes);
}

// Launches an apply kernel; with the timing events of the configuration
// set, through hipExtLaunchKernel, which records them at the kernel's own
// start and end.
#define BF_LAUNCH(cfg, kernel, grid, block, st, ...)                                          \
    do {                                                                                      \
        if ((cfg).ev_start)                                                                   \
   hipExtLaunchKernelGGL(kernel, grid, block, 0, st, (cfg).ev_start, (cfg).ev_stop, 0, \
                         __VA_ARGS__);                                               \
        else                                                                                  \
   hipLaunchKernelGGL(kernel, grid, block, 0, st, __VA_ARGS__);                      \
    } while (0)

// Schedule 3 on 16 x 16 tiles, both FP32 forms (k4: four products), both
// reading the three-product W layout.
template <bool k4>
static hipError_t launch_ws16(const LaunchCfg &cfg, BfHeader *blk, int n_items, const void *apool,
                              int a_stride, int pairs, hipStream_t st)
{
    const BfItem *items = items_of(blk);
    const dim3 grid(cfg.grid);
    const dim3 block(64 * (kCons16 + 8));
    if (cfg.s_dma) {
        if constexpr (k4)
            BF_LAUNCH(cfg, apply_fp32_4m16_ws_sdma, grid, block, st, blk, items, n_items, apool, a_stride, pairs);
        else
            BF_LAUNCH(cfg, apply_fp32_3m16_ws_sdma, grid, block, st, blk, items, n_items, apool, a_stride, pairs);
    } else if (cfg.w_dma) {
        if constexpr (k4)
            BF_LAUNCH(cfg, (apply_fp32_4m16_ws<8, 2, true>), grid, block, st, blk, items, n_items, apool,
                      a_stride, pairs);
        else
            BF_LAUNCH(cfg, (apply_fp32_3m16_ws<8, 2, true>), grid, block, st, blk, items, n_items, apool,
                      a_stride, pairs);
    } else if (cfg.depth >= 2) {
        if constexpr (k4)
            BF_LAUNCH(cfg, (apply_fp32_4m16_ws<8, 2, false>), grid, block, st, blk, items, n_items, apool,
                      a_stride, pairs);
        else
            BF_LAUNCH(cfg, (apply_fp32_3m16_ws<8, 2, false>), grid, block, st, blk, items, n_items, apool,
                      a_stride, pairs);
    } else {
        if constexpr (k4)
            BF_LAUNCH(cfg, (apply_fp32_4m16_ws<8, 1, false>), grid, block, st, blk, items, n_items, apool,
                      a_stride, pairs);
        else
            BF_LAUNCH(cfg, (apply_fp32_3m16_ws<8, 1, false>), grid, block, st, blk, items, n_items, apool,
                      a_stride, pairs);
    }
    return hipGetLastError();
}

// Schedule 3 launch: producer waves and S prefetch depth from the variant.
template <bool k3M>
static hipError_t launch_ws(const LaunchCfg &cfg, BfHeader *blk, int n_items, const void *apool,
                   int a_stride, int pairs, hipStream_t st)
{
    const BfItem *items = items_of(blk);
    const dim3 grid(cfg.grid);
    if (k3M && cfg.tile16)
        return launch_ws16<false>(cfg, blk, n_items, apool, a_stride, pairs, st);
    if (cfg.producers == 4)
        BF_LAUNCH(cfg, (apply_fp32_ws<k3M, 4, 1>), grid, dim3(64 * 8), st, blk, items,
                  n_items, apool, a_stride, pairs);
    else if (!k3M && cfg.producers == 12 && cfg.depth == 2)
        // (the three-product form's two accumulator sets do not fit 16 waves'
        // register share; the host gives it at most 8 producers)
        BF_LAUNCH(cfg, (apply_fp32_ws<false, 12, 2>), grid, dim3(64 * 16), st, blk, items,
                  n_items, apool, a_stride, pairs);
    else if (!k3M && cfg.producers == 12)
        BF_LAUNCH(cfg, (apply_fp32_ws<false, 12, 1>), grid, dim3(64 * 16), st, blk, items,
                  n_items, apool, a_stride, pairs);
    else if (cfg.depth == 3)
        BF_LAUNCH(cfg, (apply_fp32_ws<k3M, 8, 3>), grid, dim3(64 * 12), st, blk, items,
                  n_items, apool, a_stride, pairs);
    else if (cfg.depth == 2)
        BF_LAUNCH(cfg, (apply_fp32_ws<k3M, 8, 2>), grid, dim3(64 * 12), st, blk, items,
                  n_items, apool, a_stride, pairs);
    else
        BF_LAUNCH(cfg, (apply_fp32_ws<k3M, 8, 1>), grid, dim3(64 * 12), st, blk, items,
                  n_items, apool, a_stride, pairs);
    return hipGetLastError();
}

template <bool kVec16, bool kStage>
static hipError_t launch_fp32_t(const LaunchCfg &cfg, BfHeader *blk, int n_items,
                                const PlanDev &pd, hipStream_t st)
{
    const BfItem *items = items_of(blk);
    switch (cfg.schedule) {
    case 0:
        BF_LAUNCH(cfg, (apply_fp32_single<kVec16, kStage>), dim3(n_items), dim3(kThreads), st,
                  blk, items, n_items, pd.a_fp32, pd.a_fp32_stride, pd.pairs);
        break;
    case 1:
        BF_LAUNCH(cfg, apply_fp32_claim<kVec16>, dim3(cfg.grid), dim3(kThreads), st, blk,
                  items, n_items, pd.a_fp32, pd.a_fp32_stride, pd.pairs);
        break;
    case 3:
        if (cfg.tile16)
            return launch_ws16<true>(cfg, blk, n_items, (const void *)pd.a_3m, pd.a_3m_stride, pd.pairs, st);
        return launch_ws<false>(cfg, blk, n_items, (const void *)pd.a_fp32, pd.a_fp32_stride, pd.pairs, st);
    default:
        BF_LAUNCH(cfg, (apply_fp32_stream<kVec16, kStage>), dim3(cfg.grid), dim3(kThreads), st, blk,
                  items, n_items, pd.a_fp32, pd.a_fp32_stride, pd.pairs);
        break;
    }
    return hipGetLastError();
}

template <bool kVec16>
static hipError_t launch_3m_t(const LaunchCfg &cfg, BfHeader *blk, int n_items, const PlanDev &pd,
                              hipStream_t st)
{
    const BfItem *items = items_of(blk);
    if (cfg.schedule == 0)
        BF_LAUNCH(cfg, apply_fp32_3m_single<kVec16>, dim3(n_items), dim3(kThreads), st, blk,
                  items, n_items, pd.a_3m, pd.a_3m_stride, pd.pairs);
    else
        return launch_ws<true>(cfg, blk, n_items, (const void *)pd.a_3m, pd.a_3m_stride, pd.pairs, st);
    return hipGetLastError();
}

template <bool kBf16, bool kSplit, bool kVec16, bool kStage>
static hipError_t launch_lp_t(const LaunchCfg &cfg, BfHeader *blk, int n_items, const PlanDev &pd,
                              hipStream_t st)
{
    const BfItem *items = items_of(blk);
    if (cfg.schedule == 0)
        BF_LAUNCH(cfg, (apply_lp_single<kBf16, kSplit, kVec16, kStage>), dim3(n_items),
                  dim3(kThreads), st, blk, items, n_items, pd);
    else
        BF_LAUNCH(cfg, (apply_lp_stream<kBf16, kSplit, kVec16, kStage>), dim3(cfg.grid),
                  dim3(kThreads), st, blk, items, n_items, pd);
    return hipGetLastError();
}

// Schedule 3 for the 16-bit forms: producer waves and S prefetch depth from
// the variant.  The consumer waves stage W (kWC): with the producers moving
// S only, the split forms went from 182.4 to 168.2 us and plain FP16 from
// 152.0 to 148.7 us on the gain workload (12 producers, same box).
template <bool kBf16, bool kSplit>
static hipError_t launch_lp_ws(const LaunchCfg &cfg, BfHeader *blk, int n_items, const PlanDev &pd,
                               hipStream_t st)
{
    const BfItem *items = items_of(blk);
    const dim3 grid(cfg.grid);
    if (cfg.producers == 4)
        BF_LAUNCH(cfg, (apply_lp_ws<kBf16, kSplit, 4, 2, true>), grid, dim3(64 * 8), st, blk, items,
                  n_items, pd);
    else if (cfg.producers == 12)
        BF_LAUNCH(cfg, (apply_lp_ws<kBf16, kSplit, 12, 2, true>), grid, dim3(64 * 16), st, blk, items,
                  n_items, pd);
    else if (cfg.depth >= 3)
        BF_LAUNCH(cfg, (apply_lp_ws<kBf16, kSplit, 8, 3, true>), grid, dim3(64 * 12), st, blk, items,
                  n_items, pd);
    else
        BF_LAUNCH(cfg, (apply_lp_ws<kBf16, kSplit, 8, 2, true>), grid, dim3(64 * 12), st, blk, items,
                  n_items, pd);
    return hipGetLastError();
}

template <bool kBf16, bool kSplit>
static hipError_t launch_lp_v(const LaunchCfg &cfg, BfHeader *blk, int n_items, const PlanDev &pd,
                              hipStream_t st)
{
    if (cfg.schedule == 3)
        return launch_lp_ws<kBf16, kSplit>(cfg, blk, n_items, pd, st);
    if (cfg.stage)
        return cfg.vec16 ? launch_lp_t<kBf16, kSplit, true, true>(cfg, blk, n_items, pd, st)
                         : launch_lp_t<kBf16, kSplit, false, true>(cfg, blk, n_items, pd, st);
    return cfg.vec16 ? launch_lp_t<kBf16, kSplit, true, false>(cfg, blk, n_items, pd, st)
                     : launch_lp_t<kBf16, kSplit, false, false>(cfg, blk, n_items, pd, st);
}

hipError_t launch_apply(const LaunchCfg &cfg, BfHeader *blk, int n_items, const PlanDev &pd,
                        hipStream_t st)
{
    if (n_items <= 0 || cfg.grid <= 0)
        return hipSuccess;
    switch (cfg.prec) {
    case BF_FP32:
        if (cfg.stage)
            return cfg.vec16 ? launch_fp32_t<true, true>(cfg, blk, n_items, pd, st)
                             : launch_fp32_t<false, true>(cfg, blk, n_items, pd, st);
        return cfg.vec16 ? launch_fp32_t<true, false>(cfg, blk, n_items, pd, st)
                         : launch_fp32_t<false, false>(cfg, blk, n_items, pd, st);
    case BF_FP32_3M:
        return cfg.vec16 ? launch_3m_t<true>(cfg, blk, n_items, pd, st)
                         : launch_3m_t<false>(cfg, blk, n_items, pd, st);
    case BF_FP16: return launch_lp_v<false, false>(cfg, blk, n_items, pd, st);
    case BF_BF16: return launch_lp_v<true, false>(cfg, blk, n_items, pd, st);
    case BF_FP16X2: return launch_lp_v<false, true>(cfg, blk, n_items, pd, st);
    case BF_BF16X2: return launch_lp_v<true, true>(cfg, blk, n_items, pd, st);
    }
    return hipErrorNotSupported;
}

// Expansion of serving requests into items: wave r writes the items of
// record r, lane k (and k + 64, ...) block k; thread 0 of the grid writes
// the header.  The counters start at zero for the apply kernel that
// follows on the same stream.
__global__ void __launch_bounds__(256) expand_requests_kernel(const BfReqRec *recs, int n_recs, BfHeader *blk,
                                                              BfItem *items, int n_items, int deal_grid)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        blk->next = 0;
        blk->done = 0;
        blk->n_items = (uint32_t)n_items;
    }
    const int r = (int)((blockIdx.x * blockDim.x + threadIdx.x) / 64);
    if (r >= n_recs)
        return;
    const int lane = threadIdx.x & 63;
    const BfReqRec q = recs[r];
    for (int k = lane; k < q.n_s; k += 64) {
        BfItem d;
        d.S = q.f > 0 ? q.S + (size_t)k * q.f * kB : nullptr;
        d.R = q.R + (size_t)k * kM * kB;
        d.w_id = q.w_id;
        d.f = q.f;
        d.pad0 = 0;
        d.pad1 = 0;
        const int i = q.item0 + k;
        items[deal_grid > 0 ? ws_deal(i, n_items, deal_grid) : i] = d;
    }
}

hipError_t launch_expand(const BfReqRec *recs, int n_recs, BfHeader *blk, int n_items, int deal_grid,
                         hipStream_t st)
{
    if (n_recs <= 0)
        return hipSuccess;
    const int grid = (n_recs + 3) / 4;   // four records (waves) per workgroup
    hipLaunchKernelGGL(expand_requests_kernel, dim3(grid), dim3(256), 0, st, recs, n_recs, blk,
                       const_cast<BfItem *>(items_of(blk)), n_items, deal_grid);
    return hipGetLastError();
}

template <typename K>
static int occ_of(K kernel, int threads = kThreads)
{
    int blocks = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, threads, 0);
    return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

template <bool kBf16, bool kSplit, bool kStage>
static int occ_lp(int schedule, bool vec16)
{
    if (schedule == 3)
        return occ_of(apply_lp_ws<kBf16, kSplit, 4, 2, true>, 512);
    if (schedule == 0)
        return vec16 ? occ_of(apply_lp_single<kBf16, kSplit, true, kStage>)
                     : occ_of(apply_lp_single<kBf16, kSplit, false, kStage>);
    return vec16 ? occ_of(apply_lp_stream<kBf16, kSplit, true, kStage>)
                 : occ_of(apply_lp_stream<kBf16, kSplit, false, kStage>);
}

template <bool kStage>
static int occ_fp32(int schedule, bool vec16)
{
    switch (schedule) {
    case 0: return vec16 ? occ_of(apply_fp32_single<true, kStage>) : occ_of(apply_fp32_single<false, kStage>);
    case 1: return vec16 ? occ_of(apply_fp32_claim<true>) : occ_of(apply_fp32_claim<false>);
    case 3: return occ_of(apply_fp32_ws<false, 4, 1>, 512);
    default: return vec16 ? occ_of(apply_fp32_stream<true, kStage>) : occ_of(apply_fp32_stream<false, kStage>);
    }
}

template <bool kStage>
static int occ_any(int prec, int schedule, bool vec16)
{
    switch (prec) {
    case BF_FP32_3M:
        if (schedule == 0)
            return vec16 ? occ_of(apply_fp32_3m_single<true>) : occ_of(apply_fp32_3m_single<false>);
        return occ_of(apply_fp32_ws<true, 4, 1>, 512);
    case BF_FP16: return occ_lp<false, false, kStage>(schedule, vec16);
    case BF_BF16: return occ_lp<true, false, kStage>(schedule, vec16);
    case BF_FP16X2: return occ_lp<false, true, kStage>(schedule, vec16);
    case BF_BF16X2: return occ_lp<true, true, kStage>(schedule, vec16);
    default: return occ_fp32<kStage>(schedule, vec16);
    }
}

int apply_occupancy(int prec, int schedule, bool vec16, bool stage)
{
    return stage ? occ_any<true>(prec, schedule, vec16) : occ_any<false>(prec, schedule, vec16);
}

}  // namespace bfk
