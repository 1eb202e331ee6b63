// Filter stage on gfx950: y = IFFT(FFT(s) * H) for a batch of 2048-sample
// blocks (Section III, the filter paragraph), H the FFT of the zero-padded
// filter sequence, computed once per filter with the same transform.
//
// One workgroup of 256 threads transforms a block with the Stockham passes
// of bf_fft.h, the intermediate results going through two swizzled LDS
// buffers (no bank conflicts).  The inverse transform is the forward one applied to the
// conjugate: IFFT(Z) = conj(FFT(conj(Z))) / 2048.  The forward transform
// leaves thread t with X[t + 256 q], which is exactly the input pattern of
// the next forward transform, so the multiply by H, the conjugation and the
// second transform follow in registers.  Persistent workgroups keep their
// twiddle factors and their entries of H in registers across blocks; HBM
// sees each block read once and written once.
#include <hip/hip_runtime.h>

#include "bf_filter_internal.h"
#include "bf_fft.h"

namespace bff {

typedef float nf2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const nf2 g_cnf2;
typedef __attribute__((address_space(1))) nf2 g_nf2;

// Entry i of a read-only global complex array.
__device__ __forceinline__ float2 ld2(const float2 *__restrict__ p, int i)
{
    const nf2 a = ((g_cnf2 *)p)[i];
    return make_float2(a.x, a.y);
}

struct Twiddles {
    float2 p2[7], p3[7], p4[2][3];
};

__device__ __forceinline__ void load_twiddles(Twiddles &w, const float2 *__restrict__ table, int t)
{
#pragma unroll
    for (int r = 1; r < 8; ++r) {
        w.p2[r - 1] = ld2(table, tw_pass2(t, r));
        w.p3[r - 1] = ld2(table, tw_pass3(t, r));
    }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 1; r < 4; ++r)
            w.p4[b][r - 1] = ld2(table, tw_pass4(t + 256 * b, r));
}

// Forward 2048-point FFT of the block held as v[q] = x[t + 256 q]; on return
// v[q] = X[t + 256 q].  lds_a / lds_b: two buffers of kLdsPad entries.  The
// leading barrier keeps this call's first writes away from the previous
// call's last reads.
__device__ __forceinline__ void fft2048(float2 (&v)[8], float2 *__restrict__ lds_a,
                                        float2 *__restrict__ lds_b, const Twiddles &w, int t)
{
    // pass 1: radix 8, span 1 (no twiddles), registers -> A
    dft8(v);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r)
        lds_a[pad(out_pass1(t, r))] = v[r];
    __syncthreads();
    // pass 2: radix 8, span 8, A -> B
#pragma unroll
    for (int r = 0; r < 8; ++r)
        v[r] = lds_a[pad(t + 256 * r)];
#pragma unroll
    for (int r = 1; r < 8; ++r)
        v[r] = cmul(v[r], w.p2[r - 1]);
    dft8(v);
#pragma unroll
    for (int r = 0; r < 8; ++r)
        lds_b[pad(out_pass2(t, r))] = v[r];
    __syncthreads();
    // pass 3: radix 8, span 64, B -> A
#pragma unroll
    for (int r = 0; r < 8; ++r)
        v[r] = lds_b[pad(t + 256 * r)];
#pragma unroll
    for (int r = 1; r < 8; ++r)
        v[r] = cmul(v[r], w.p3[r - 1]);
    dft8(v);
#pragma unroll
    for (int r = 0; r < 8; ++r)
        lds_a[pad(out_pass3(t, r))] = v[r];
    __syncthreads();
    // pass 4: radix 4, span 512, butterflies t and t + 256, A -> registers:
    // butterfly i writes X[i + 512 r], i.e. v[2 r + b] = X[t + 256 (2 r + b)]
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int i = t + 256 * b;
        float2 u0 = lds_a[pad(i)];
        float2 u1 = cmul(lds_a[pad(i + 512)], w.p4[b][0]);
        float2 u2 = cmul(lds_a[pad(i + 1024)], w.p4[b][1]);
        float2 u3 = cmul(lds_a[pad(i + 1536)], w.p4[b][2]);
        dft4(u0, u1, u2, u3);
        v[b] = u0;
        v[2 + b] = u1;
        v[4 + b] = u2;
        v[6 + b] = u3;
    }
}

// kFilter: y = IFFT(FFT(x) * H) per block; otherwise y = FFT(x) (used once
// per filter to compute H).  Workgroup g handles blocks g, g + G, ...
template <bool kFilter>
__global__ __launch_bounds__(kThreads) void filter_kernel(const float2 *x, float2 *y, int n_blocks,
                                                          const float2 *__restrict__ table,
                                                          const float2 *__restrict__ H)
{
    __shared__ float2 lds_a[kLdsPad];
    __shared__ float2 lds_b[kLdsPad];
    const int t = threadIdx.x;
    Twiddles w;
    load_twiddles(w, table, t);
    float2 h[8];
    if constexpr (kFilter) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            h[q] = ld2(H, t + 256 * q);
    }
    const float scale = 1.0f / kN;   // exact: 2^-11
    for (int blk = blockIdx.x; blk < n_blocks; blk += gridDim.x) {
        // Blocks may be filtered in place (x == y): a block is read whole
        // before any of it is written, and blocks do not overlap.
        g_cnf2 *src = (g_cnf2 *)(x + (size_t)blk * kN) + t;
        g_nf2 *dst = (g_nf2 *)(y + (size_t)blk * kN) + t;
        float2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const nf2 a = __builtin_nontemporal_load(src + 256 * q);
            v[q] = make_float2(a.x, a.y);
        }
        fft2048(v, lds_a, lds_b, w, t);
        if constexpr (kFilter) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                v[q] = cconj(cmul(v[q], h[q]));
            fft2048(v, lds_a, lds_b, w, t);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                v[q] = make_float2(v[q].x * scale, -v[q].y * scale);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            __builtin_nontemporal_store(nf2{v[q].x, v[q].y}, dst + 256 * q);
    }
}

hipError_t launch_filter(const float2 *x, float2 *y, int n_blocks, const float2 *table,
                         const float2 *H, int grid, hipStream_t st)
{
    if (n_blocks <= 0)
        return hipSuccess;
    if (H)
        hipLaunchKernelGGL(filter_kernel<true>, dim3(grid), dim3(kThreads), 0, st, x, y, n_blocks,
                           table, H);
    else
        hipLaunchKernelGGL(filter_kernel<false>, dim3(grid), dim3(kThreads), 0, st, x, y, n_blocks,
                           table, nullptr);
    return hipGetLastError();
}

int filter_occupancy()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, filter_kernel<true>, kThreads, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace bff
