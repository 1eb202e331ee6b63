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
#include <hip/hip_runtime.h>

#include "bf_internal.h"

namespace bfk {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
// Global-memory (address space 1) views, so that accesses through pointers
// read from descriptors compile to global_* rather than flat_* instructions.
typedef __attribute__((address_space(1))) f2v g_f2v;
typedef __attribute__((address_space(1))) const f2v g_cf2v;
typedef __attribute__((address_space(1))) const f4v g_cf4v;

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

// ---------------------------------------------------------------------------
// Staging S into LDS.  Row k of S (60 complex = 480 bytes) goes to LDS row
// k (pitch 64 complex).  With 16-byte aligned S each thread moves 16-byte
// chunks (30 per row); otherwise 8-byte elements.  For odd f, row f is
// cleared so the second half of the last K pair multiplies zeros.
template <bool kVec16>
__device__ __forceinline__ void stage_s(f2v *__restrict__ lds, const float2 *__restrict__ S, int f)
{
    const int tid = threadIdx.x;
    if (kVec16) {
        g_cf4v *src = (g_cf4v *)S;
        const int chunks = f * (kB / 2);
        for (int c = tid; c < chunks; c += kThreads) {
            const int row = c / (kB / 2);
            const int col2 = c - row * (kB / 2);
            const f4v v = __builtin_nontemporal_load(src + c);
            *reinterpret_cast<f4v *>(lds + row * kLdsCols + 2 * col2) = v;
        }
    } else {
        g_cf2v *src = (g_cf2v *)S;
        const int elems = f * kB;
        for (int c = tid; c < elems; c += kThreads) {
            const int row = c / kB;
            const int col = c - row * kB;
            lds[row * kLdsCols + col] = __builtin_nontemporal_load(src + c);
        }
    }
    if (f & 1) {
        for (int c = tid; c < kLdsCols; c += kThreads)
            lds[f * kLdsCols + c] = f2v{0.f, 0.f};
    }
}

// Writes the two 32 x 32 accumulator tiles of one wave to R.  Register r of
// lane l holds real row 8 (r / 4) + 4 (l / 32) + r % 4 and column l % 32,
// so registers (r, r + 1), r even, are (Re, Im) of antenna
// 4 (r / 4) + 2 (l / 32) + (r % 4) / 2 within the wave's 16.
__device__ __forceinline__ void store_r(float2 *__restrict__ Rp, int wave, int lane,
                                        const floatx16 &acc0, const floatx16 &acc1)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    g_f2v *base = (g_f2v *)Rp + (size_t)(16 * wave) * kB;
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
        const int il = 4 * (r >> 2) + 2 * h + ((r & 3) >> 1);
        g_f2v *row = base + il * kB;
        __builtin_nontemporal_store(f2v{acc0[r], acc0[r + 1]}, row + n);
        if (n < kB - 32)
            __builtin_nontemporal_store(f2v{acc1[r], acc1[r + 1]}, row + 32 + n);
    }
}

// ---------------------------------------------------------------------------
// FP32 apply kernel.
//   kSched 0: workgroup b computes item b.
//   kSched 1: persistent; workgroups claim items from blk->next.
template <int kSched, bool kVec16>
__global__ __launch_bounds__(kThreads) void apply_fp32_kernel(BfHeader *__restrict__ blk,
                                                              const BfItem *__restrict__ items,
                                                              int n_items,
                                                              const float2 *__restrict__ apool,
                                                              int a_w_stride, int pairs)
{
    __shared__ f2v lds_s[kFMax * kLdsCols];
    __shared__ int claim;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = lane >> 5;
    const int n = lane & 31;

    f2v a[kPairsMax];
    int cur_w = -1;

    int it;
    if (kSched == 0) {
        it = blockIdx.x;
    } else {
        if (threadIdx.x == 0)
            claim = (int)atomicAdd(&blk->next, 1u);
        __syncthreads();
        it = claim;
    }
    it = __builtin_amdgcn_readfirstlane(it);

    while (it < n_items) {
        const BfItem d = items[it];
        const int f = d.f;
        const int np = (f + 1) >> 1;

        if (d.w_id != cur_w) {
            cur_w = d.w_id;
            const float2 *ap = apool + (size_t)cur_w * a_w_stride + (size_t)wave * pairs * 64 + lane;
#pragma unroll
            for (int p = 0; p < kPairsMax; ++p)
                a[p] = p < pairs ? reinterpret_cast<const f2v &>(ap[p * 64]) : f2v{0.f, 0.f};
        }

        stage_s<kVec16>(lds_s, d.S, f);
        __syncthreads();

        if (kSched == 1 && threadIdx.x == 0)
            claim = (int)atomicAdd(&blk->next, 1u);

        floatx16 acc0 = {};
        floatx16 acc1 = {};
#pragma unroll
        for (int p = 0; p < kPairsMax; ++p) {
            if (p < np) {
                const f2v b0 = lds_s[(2 * p + h) * kLdsCols + n];
                const f2v b1 = lds_s[(2 * p + h) * kLdsCols + 32 + n];
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b0.x, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b1.x, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b0.y, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b1.y, acc1, 0, 0, 0);
            }
        }
        store_r(d.R, wave, lane, acc0, acc1);
        __syncthreads();   // LDS is reused by the next item; `claim` is ready

        if (kSched == 0)
            break;
        it = __builtin_amdgcn_readfirstlane(claim);
    }

    if (kSched == 1 && threadIdx.x == 0) {
        // The last workgroup out re-arms the block for the next replay.
        __threadfence();
        const uint32_t prev = atomicAdd(&blk->done, 1u);
        if (prev == gridDim.x - 1) {
            atomicExch(&blk->next, 0u);
            atomicExch(&blk->done, 0u);
        }
    }
}

size_t lp_w_bytes(int) { return 0; }

hipError_t launch_w_transform_lp(const float2 *, int, int, int, void *, float *, hipStream_t)
{
    return hipErrorNotSupported;
}

template <int kSched, bool kVec16>
static hipError_t launch_fp32_t(const LaunchCfg &cfg, BfHeader *blk, int n_items,
                                const void *a_pool, size_t a_w_stride, int pairs, hipStream_t st)
{
    hipLaunchKernelGGL((apply_fp32_kernel<kSched, kVec16>), dim3(cfg.grid), dim3(kThreads), 0, st,
                       blk, reinterpret_cast<const BfItem *>(blk + 1), n_items,
                       static_cast<const float2 *>(a_pool), (int)a_w_stride, pairs);
    return hipGetLastError();
}

hipError_t launch_apply(const LaunchCfg &cfg, BfHeader *blk, int n_items, const void *a_pool,
                        size_t a_w_stride, int pairs, const float *, hipStream_t st)
{
    if (n_items <= 0 || cfg.grid <= 0)
        return hipSuccess;
    if (cfg.prec != BF_FP32)
        return hipErrorNotSupported;
    if (cfg.schedule == 0)
        return cfg.vec16 ? launch_fp32_t<0, true>(cfg, blk, n_items, a_pool, a_w_stride, pairs, st)
                         : launch_fp32_t<0, false>(cfg, blk, n_items, a_pool, a_w_stride, pairs, st);
    return cfg.vec16 ? launch_fp32_t<1, true>(cfg, blk, n_items, a_pool, a_w_stride, pairs, st)
                     : launch_fp32_t<1, false>(cfg, blk, n_items, a_pool, a_w_stride, pairs, st);
}

int apply_occupancy(int prec, int schedule, bool vec16)
{
    if (prec != BF_FP32)
        return 1;
    int blocks = 0;
    hipError_t e;
    if (schedule == 0)
        e = vec16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, apply_fp32_kernel<0, true>, kThreads, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, apply_fp32_kernel<0, false>, kThreads, 0);
    else
        e = vec16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, apply_fp32_kernel<1, true>, kThreads, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, apply_fp32_kernel<1, false>, kThreads, 0);
    return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

}  // namespace bfk
