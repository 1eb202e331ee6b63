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
template <bool kVec16>
__device__ __forceinline__ void load_s(SRegs<kVec16> &r, const float2 *__restrict__ S, int f)
{
    const int tid = threadIdx.x;
    if constexpr (kVec16) {
        g_cf4v *src = (g_cf4v *)S;
        const int last = (f > 0 ? f * (kB / 2) : 1) - 1;
#pragma unroll
        for (int u = 0; u < kChunks16; ++u) {
            const int c = min(tid + u * kThreads, last);
            r.v[u] = __builtin_nontemporal_load(src + c);
        }
    } else {
        g_cf2v *src = (g_cf2v *)S;
        const int last = (f > 0 ? f * kB : 1) - 1;
#pragma unroll
        for (int u = 0; u < kChunks8; ++u) {
            const int c = min(tid + u * kThreads, last);
            r.v[u] = __builtin_nontemporal_load(src + c);
        }
    }
}

// Writes the registers of load_s to LDS: row k of S (480 bytes) to LDS row
// k (pitch 64 complex).  For odd f, row f is cleared so the second half of
// the last K pair multiplies zeros.
template <bool kVec16>
__device__ __forceinline__ void put_s(f2v *__restrict__ lds, const SRegs<kVec16> &r, int f)
{
    const int tid = threadIdx.x;
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

// Issues as many stores as store_r (16), into the sink.  Placed after the
// first S loads of a persistent loop, it makes the loop-entry path carry the
// same outstanding-operation pattern as the back edge (S loads followed by
// 16 stores), so the compiler's wait before the first LDS write counts only
// the S loads on both paths instead of falling back to the stricter count.
__device__ __forceinline__ void prime_store_count(float2 *__restrict__ sink, int lane)
{
    g_f2v *pad = (g_f2v *)sink + lane;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        __builtin_nontemporal_store(f2v{0.f, 0.f}, pad + 64 * k);
}

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
__device__ __forceinline__ void contract_store_fp32(const f2v *__restrict__ lds,
                                                    const f2v (&a)[kPairsMax], int f,
                                                    float2 *__restrict__ R, float2 *__restrict__ sink,
                                                    int wave, int lane)
{
    const int h = lane >> 5;
    const int n = lane & 31;
    const int np = (f + 1) >> 1;
    floatx16 acc0 = {};
    floatx16 acc1 = {};
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
    store_r(R, sink, wave, lane, acc0, acc1);
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

// kSched 0: one product per workgroup.
template <bool kVec16>
__global__ __launch_bounds__(kThreads) void apply_fp32_single(BfHeader *__restrict__ blk,
                                                              const BfItem *__restrict__ items,
                                                              int n_items,
                                                              const float2 *__restrict__ apool,
                                                              int a_w_stride, int pairs)
{
    __shared__ f2v lds_s[kFMax * kLdsCols];
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
    contract_store_fp32(lds_s, a, d.f, d.R, sink, wave, lane);
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
        contract_store_fp32(lds_s, a, d.f, d.R, sink, wave, lane);
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
template <bool kVec16>
__global__ __launch_bounds__(kThreads) void apply_fp32_stream(BfHeader *__restrict__ blk,
                                                              const BfItem *__restrict__ items,
                                                              int n_items,
                                                              const float2 *__restrict__ apool,
                                                              int a_w_stride, int pairs)
{
    __shared__ f2v lds_s[2][kFMax * kLdsCols];
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
    prime_store_count(sink, lane);
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
        contract_store_fp32(lds_s[buf], a, d.f, d.R, sink, wave, lane);
        if (!more)
            break;
        d = du;
        dn = dnn;
        nxt = nn;
        buf ^= 1;
    }
}

size_t lp_w_bytes(int) { return 0; }

hipError_t launch_w_transform_lp(const float2 *, int, int, int, void *, float *, hipStream_t)
{
    return hipErrorNotSupported;
}

template <bool kVec16>
static hipError_t launch_fp32_t(const LaunchCfg &cfg, BfHeader *blk, int n_items,
                                const float2 *a_pool, int a_w_stride, int pairs, hipStream_t st)
{
    const BfItem *items = reinterpret_cast<const BfItem *>(reinterpret_cast<const char *>(blk) +
                                                           sizeof(BfHeader) + kSinkBytes);
    switch (cfg.schedule) {
    case 0:
        hipLaunchKernelGGL(apply_fp32_single<kVec16>, dim3(n_items), dim3(kThreads), 0, st, blk,
                           items, n_items, a_pool, a_w_stride, pairs);
        break;
    case 1:
        hipLaunchKernelGGL(apply_fp32_claim<kVec16>, dim3(cfg.grid), dim3(kThreads), 0, st, blk,
                           items, n_items, a_pool, a_w_stride, pairs);
        break;
    default:
        hipLaunchKernelGGL(apply_fp32_stream<kVec16>, dim3(cfg.grid), dim3(kThreads), 0, st, blk,
                           items, n_items, a_pool, a_w_stride, pairs);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_apply(const LaunchCfg &cfg, BfHeader *blk, int n_items, const void *a_pool,
                        size_t a_w_stride, int pairs, const float *, hipStream_t st)
{
    if (n_items <= 0 || cfg.grid <= 0)
        return hipSuccess;
    if (cfg.prec != BF_FP32)
        return hipErrorNotSupported;
    const float2 *a = static_cast<const float2 *>(a_pool);
    return cfg.vec16 ? launch_fp32_t<true>(cfg, blk, n_items, a, (int)a_w_stride, pairs, st)
                     : launch_fp32_t<false>(cfg, blk, n_items, a, (int)a_w_stride, pairs, st);
}

template <typename K>
static int occ_of(K kernel)
{
    int blocks = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, kThreads, 0);
    return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

int apply_occupancy(int prec, int schedule, bool vec16)
{
    if (prec != BF_FP32)
        return 1;
    switch (schedule) {
    case 0: return vec16 ? occ_of(apply_fp32_single<true>) : occ_of(apply_fp32_single<false>);
    case 1: return vec16 ? occ_of(apply_fp32_claim<true>) : occ_of(apply_fp32_claim<false>);
    default: return vec16 ? occ_of(apply_fp32_stream<true>) : occ_of(apply_fp32_stream<false>);
    }
}

}  // namespace bfk
