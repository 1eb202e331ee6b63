// Device entry points of the filter stage (bf_filter.hip) used by the host
// code of the library.
#pragma once

#include <hip/hip_runtime.h>

namespace bff {

// y = IFFT(FFT(x) * H) for n_blocks blocks of 2048 complex samples when H is
// given, else y = FFT(x).  table: exp(-2 pi i m / 2048), m < 2048.  grid:
// persistent workgroups (each takes every grid-th block).
hipError_t launch_filter(const float2 *x, float2 *y, int n_blocks, const float2 *table,
                         const float2 *H, int grid, hipStream_t st);

// Workgroups of the filter kernel that fit on one CU at once.
int filter_occupancy();

}  // namespace bff
