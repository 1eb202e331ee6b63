// HBM reference kernels.  A plain streaming copy of known size measures
// achievable bandwidth next to the spec-sheet peak and scales the
// FETCH_SIZE / WRITE_SIZE counters (bytes a counter reports for a copy
// whose traffic is known); read-only and write-only streams give the
// ceilings of each direction alone.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f4v __attribute__((ext_vector_type(4)));

// Each thread moves kU 16-byte chunks per step (all loads first), blocks
// stride over the buffer; kNt selects non-temporal loads and stores.
template <int kU, bool kNt>
__global__ __launch_bounds__(256) void copy_kernel(const f4v *__restrict__ src,
                                                   f4v *__restrict__ dst, size_t n)
{
    const size_t step = (size_t)gridDim.x * 256 * kU;
    for (size_t base = (size_t)blockIdx.x * 256 * kU + threadIdx.x; base < n; base += step) {
        f4v v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = base + (size_t)u * 256;
            if (i < n)
                v[u] = kNt ? __builtin_nontemporal_load(src + i) : src[i];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = base + (size_t)u * 256;
            if (i < n) {
                if (kNt)
                    __builtin_nontemporal_store(v[u], dst + i);
                else
                    dst[i] = v[u];
            }
        }
    }
}

// Read-only stream: each thread sums what it reads and writes one value
// per thread (negligible traffic), so the loads cannot be dropped.
template <int kU>
__global__ __launch_bounds__(256) void read_kernel(const f4v *__restrict__ src, f4v *__restrict__ dst,
                                                   size_t n)
{
    const size_t step = (size_t)gridDim.x * 256 * kU;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    for (size_t base = (size_t)blockIdx.x * 256 * kU + threadIdx.x; base < n; base += step) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = base + (size_t)u * 256;
            if (i < n)
                acc += __builtin_nontemporal_load(src + i);
        }
    }
    dst[(size_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

// Write-only stream of a constant.
template <int kU>
__global__ __launch_bounds__(256) void write_kernel(f4v *__restrict__ dst, size_t n, float v)
{
    const size_t step = (size_t)gridDim.x * 256 * kU;
    const f4v x = {v, v, v, v};
    for (size_t base = (size_t)blockIdx.x * 256 * kU + threadIdx.x; base < n; base += step) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t i = base + (size_t)u * 256;
            if (i < n)
                __builtin_nontemporal_store(x, dst + i);
        }
    }
}

// variant: bit 0 = non-temporal, bits 1-2 = log2 of the per-thread unroll.
// mode: 0 copy, 1 read only (dst needs grid * 256 * 16 bytes), 2 write only.
extern "C" int bfprobe_stream(const void *src, void *dst, uint64_t bytes, int grid, int variant,
                              int mode, void *stream)
{
    if (!dst || (bytes & 15) || grid <= 0 || variant < 0 || variant > 7 || mode < 0 || mode > 2 ||
        (mode != 2 && !src))
        return -1;
    const size_t n = bytes / 16;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const f4v *s = static_cast<const f4v *>(src);
    f4v *d = static_cast<f4v *>(dst);
    if (mode == 1) {
        hipLaunchKernelGGL((read_kernel<4>), dim3(grid), dim3(256), 0, st, s, d, n);
    } else if (mode == 2) {
        hipLaunchKernelGGL((write_kernel<4>), dim3(grid), dim3(256), 0, st, d, n, 1.0f);
    } else {
        switch (variant) {
        case 0: hipLaunchKernelGGL((copy_kernel<1, false>), dim3(grid), dim3(256), 0, st, s, d, n); break;
        case 1: hipLaunchKernelGGL((copy_kernel<1, true>), dim3(grid), dim3(256), 0, st, s, d, n); break;
        case 2: hipLaunchKernelGGL((copy_kernel<2, false>), dim3(grid), dim3(256), 0, st, s, d, n); break;
        case 3: hipLaunchKernelGGL((copy_kernel<2, true>), dim3(grid), dim3(256), 0, st, s, d, n); break;
        case 4: hipLaunchKernelGGL((copy_kernel<4, false>), dim3(grid), dim3(256), 0, st, s, d, n); break;
        case 5: hipLaunchKernelGGL((copy_kernel<4, true>), dim3(grid), dim3(256), 0, st, s, d, n); break;
        case 6: hipLaunchKernelGGL((copy_kernel<8, false>), dim3(grid), dim3(256), 0, st, s, d, n); break;
        default: hipLaunchKernelGGL((copy_kernel<8, true>), dim3(grid), dim3(256), 0, st, s, d, n); break;
        }
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

extern "C" int bfprobe_copy(const void *src, void *dst, uint64_t bytes, int grid, int variant,
                            void *stream)
{
    return bfprobe_stream(src, dst, bytes, grid, variant, 0, stream);
}

// Matrix-core reference: each wave runs `iters` steps of four independent
// v_mfma_f32_32x32x2_f32 chains from registers (no memory traffic inside
// the loop), so the measured rate is what the FP32 matrix cores sustain at
// the clock the chip runs under that load.  Each thread writes one value
// (out needs grid * 256 floats) so nothing is dropped.
typedef float floatx16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void mfma_kernel(float *__restrict__ out, int iters)
{
    floatx16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    const float a = 1.0f + 1e-7f * (float)threadIdx.x;
    const float b = 1.0f - 1e-7f * (float)blockIdx.x;
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, a, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(b, b, c3, 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r)
        s += c0[r] + c1[r] + c2[r] + c3[r];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// Flops per call: grid * 4 waves * iters * 4 MFMAs * 4096.
extern "C" int bfprobe_mfma(float *out, int grid, int iters, void *stream)
{
    if (!out || grid <= 0 || iters <= 0)
        return -1;
    hipLaunchKernelGGL(mfma_kernel, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), out,
                       iters);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
