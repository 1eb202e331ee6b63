// Building blocks of the 2048-point FFT used by the filter stage
// (Section III: y = IFFT(MULT(FFT(s))), all FFT sizes 2048).
//
// The transform is a Stockham autosort FFT with radices 8, 8, 8, 4 over a
// workgroup of 256 threads holding 8 points each.  Pass m (radix R, span p =
// product of the earlier radices, T = 2048 / R butterflies) lets butterfly i
// read x[i + r T] (r < R), multiply entry r by exp(-2 pi i r k / (p R)) with
// k = i mod p, take the length-R DFT and write entry r to
// y[(i / p) p R + k + r p]; the output of the last pass is in natural order.
// Pass 1 reads the thread's own registers (the global-load pattern
// t + 256 r is its input pattern) and the last pass leaves thread t with
// X[t + 256 q], q < 8, which is again the first pass's input pattern, so an
// inverse transform can follow without an LDS round trip.
//
// Everything here is plain arithmetic on float2 and integer index maps, so
// it compiles for the host as well as for gfx950.
#pragma once

#include <hip/hip_runtime.h>

namespace bff {

constexpr int kN = 2048;
constexpr int kThreads = 256;
constexpr int kPts = 8;                   // points per thread
constexpr int kLdsPad = kN;               // LDS entries per buffer (swizzled, no padding)

// LDS position of entry j: its row of 16 entries (128 bytes) stays, the
// position inside the row is XORed with h(row) = (row & 7) ^ (bit 2 of row
// << 3).  With 8-byte accesses checked for bank conflicts over groups of 16
// lanes, every access pattern of the passes then touches 16 different
// positions per group: the stride-8 writes of pass 1 (rows differ in their
// low 3 bits), the group-of-8 writes of pass 2 (bit 3 set apart by bit 2
// of the row) and all unit-stride accesses (one row, a bijection within it).
__host__ __device__ inline int pad(int j)
{
    const int row = j >> 4;
    return j ^ ((row & 7) ^ (((row >> 2) & 1) << 3));
}

__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiplication by -i: (x + i y)(-i) = y - i x
__host__ __device__ inline float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }

// In-place length-4 DFT, exponent sign -1.
__host__ __device__ inline void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3)
{
    const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    const float2 t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// In-place length-8 DFT, exponent sign -1: X[k] = E[k] + w^k O[k] and
// X[k + 4] = E[k] - w^k O[k], E / O the length-4 DFTs of the even / odd
// entries and w = exp(-2 pi i / 8) = (1 - i) / sqrt(2).
__host__ __device__ inline void dft8(float2 (&v)[8])
{
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const float r = 0.70710678118654752440f;
    // w^1 o1 = (1 - i) o1 / sqrt(2); w^2 o2 = -i o2; w^3 o3 = -(1 + i) o3 / sqrt(2)
    const float2 p1 = make_float2((o1.x + o1.y) * r, (o1.y - o1.x) * r);
    const float2 p2 = mul_mi(o2);
    const float2 p3 = make_float2((o3.y - o3.x) * r, -(o3.x + o3.y) * r);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, p1);
    v[5] = csub(e1, p1);
    v[2] = cadd(e2, p2);
    v[6] = csub(e2, p2);
    v[3] = cadd(e3, p3);
    v[7] = csub(e3, p3);
}

// Twiddle table index of entry r of butterfly i in each pass (the table
// holds exp(-2 pi i m / 2048), m < 2048); all indices stay below 2048.
__host__ __device__ inline int tw_pass2(int t, int r) { return r * (t & 7) * 32; }     // p = 8, R = 8
__host__ __device__ inline int tw_pass3(int t, int r) { return r * (t & 63) * 4; }     // p = 64, R = 8
__host__ __device__ inline int tw_pass4(int i, int r) { return r * i; }                // p = 512, R = 4

// Output position of entry r of butterfly i in passes 1-3 (radix 8).
__host__ __device__ inline int out_pass1(int t, int r) { return 8 * t + r; }
__host__ __device__ inline int out_pass2(int t, int r) { return (t >> 3) * 64 + (t & 7) + 8 * r; }
__host__ __device__ inline int out_pass3(int t, int r) { return (t >> 6) * 512 + (t & 63) + 64 * r; }

}  // namespace bff
