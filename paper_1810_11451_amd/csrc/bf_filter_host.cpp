// Filter stage, host side: the filter plan (twiddle table and H = FFT of the
// zero-padded filter sequence, both on the device) and the batched apply.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>

#include "bf.h"
#include "bf_filter_internal.h"
#include "bf_host.h"

struct bf_filter_s {
    int device = 0;
    int grid_cap = 1;          // persistent workgroups that fit on the device
    int n_taps = 0;
    float2 *table = nullptr;   // exp(-2 pi i m / 2048), m < 2048
    float2 *H = nullptr;       // FFT of the zero-padded filter sequence
};

static constexpr int kFilterN = 2048;

extern "C" bf_status bf_filter_destroy(bf_filter flt)
{
    if (!flt)
        return bf_fail(BF_ERR_INVALID, "filter is null");
    (void)hipDeviceSynchronize();
    if (flt->table)
        (void)hipFree(flt->table);
    if (flt->H)
        (void)hipFree(flt->H);
    delete flt;
    return BF_OK;
}

extern "C" bf_status bf_filter_create(bf_filter *out, const void *h, int32_t n_taps, void *hip_stream)
{
    if (!out)
        return bf_fail(BF_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!h)
        return bf_fail(BF_ERR_INVALID, "h is null");
    if (n_taps < 1 || n_taps > kFilterN)
        return bf_fail(BF_ERR_INVALID, "n_taps %d outside [1, %d]", n_taps, kFilterN);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    bf_filter f = new (std::nothrow) bf_filter_s();
    if (!f)
        return bf_fail(BF_ERR_OOM, "filter allocation");
    f->n_taps = n_taps;
    auto fail_dev = [&](const char *what, hipError_t e) {
        bf_filter_destroy(f);
        return bf_fail(e == hipErrorOutOfMemory ? BF_ERR_OOM : BF_ERR_DEVICE, "%s: %s", what,
                       hipGetErrorString(e));
    };
    hipError_t e = hipGetDevice(&f->device);
    int cus = 1;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, f->device);
    if (e != hipSuccess)
        return fail_dev("device query", e);
    f->grid_cap = std::max(1, cus) * bff::filter_occupancy();

    // Twiddle factors in double precision, rounded once to float.
    std::vector<float2> table(kFilterN), taps(kFilterN, make_float2(0.f, 0.f));
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < kFilterN; ++m) {
        const double a = -two_pi * m / kFilterN;
        table[(size_t)m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    const float2 *hin = static_cast<const float2 *>(h);
    std::copy(hin, hin + n_taps, taps.begin());

    float2 *tmp = nullptr;
    e = hipMalloc(&f->table, kFilterN * sizeof(float2));
    if (e == hipSuccess)
        e = hipMalloc(&f->H, kFilterN * sizeof(float2));
    if (e == hipSuccess)
        e = hipMalloc(&tmp, kFilterN * sizeof(float2));
    if (e == hipSuccess)
        e = hipMemcpyAsync(f->table, table.data(), kFilterN * sizeof(float2), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(tmp, taps.data(), kFilterN * sizeof(float2), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)   // H = FFT(h zero-padded), with the same transform
        e = bff::launch_filter(tmp, f->H, 1, f->table, nullptr, 1, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (tmp)
        (void)hipFree(tmp);
    if (e != hipSuccess)
        return fail_dev("filter spectrum", e);
    *out = f;
    return BF_OK;
}

extern "C" bf_status bf_filter_spectrum(bf_filter flt, void *H_out)
{
    if (!flt || !H_out)
        return bf_fail(BF_ERR_INVALID, "null argument");
    hipError_t e = hipMemcpy(H_out, flt->H, kFilterN * sizeof(float2), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "hipMemcpy(H): %s", hipGetErrorString(e));
    return BF_OK;
}

extern "C" bf_status bf_filter_apply(bf_filter flt, int32_t batch, const void *x, void *y,
                                     void *hip_stream)
{
    if (!flt)
        return bf_fail(BF_ERR_INVALID, "filter is null");
    if (batch < 0)
        return bf_fail(BF_ERR_INVALID, "batch %d < 0", batch);
    if (batch == 0)
        return BF_OK;
    if (!x || !y)
        return bf_fail(BF_ERR_INVALID, "x or y is null");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 7u)
        return bf_fail(BF_ERR_INVALID, "x and y must be 8-byte aligned");
    const uintptr_t xs = reinterpret_cast<uintptr_t>(x), ys = reinterpret_cast<uintptr_t>(y);
    const uintptr_t bytes = (uintptr_t)batch * kFilterN * sizeof(float2);
    if (xs != ys && xs < ys + bytes && ys < xs + bytes)
        return bf_fail(BF_ERR_INVALID, "x and y overlap without being the same buffer");
    const int grid = std::min<int>(batch, flt->grid_cap);
    hipError_t e = bff::launch_filter(static_cast<const float2 *>(x), static_cast<float2 *>(y), batch,
                                      flt->table, flt->H, grid, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess)
        return bf_fail(BF_ERR_DEVICE, "filter launch: %s", hipGetErrorString(e));
    return BF_OK;
}
