// Shared device-side definitions of the porestokes library (gfx950).
//
// Every sweep kernel variant calls the same inline routines below for the
// per-face and per-cell arithmetic, with explicit fma() calls and the whole
// library built with -ffp-contract=off, so that the variants (single launch,
// batched launch, two-pass launch) produce bitwise identical iterates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codes.h"

namespace ps {

// Second derivative across the flow from a stencil code:
//   d2 = a (v[-1] + v[+1]) + b v[0] + gp v[+2] + gm v[-2].
// Faces beyond a wall are solid and hold an exact zero, so one formula
// covers every case of App. B:
//   code 0 (no wall, case 6):      a = 1,   b = -2
//   L      (case 4):               a = 2,   b = -5,    gp = -1/5   (v[-1] = 0)
//   R      (case 5):               a = 2,   b = -5,    gm = -1/5   (v[+1] = 0)
//   L+F    (case 2):               a = 8/3, b = -16/3              (v[-1] = v[+2] = 0)
//   R+F    (case 3):               a = 8/3, b = -16/3              (v[+1] = v[-2] = 0)
//   L+R    (case 1):               a = 0,   b = -8
template <typename T>
struct Coef {
    T a, b, gp, gm;
};

template <typename T>
__host__ __device__ inline Coef<T> coef_of_code(int code)
{
    const T third8 = T(8) / T(3), third16 = T(16) / T(3), fifth = T(1) / T(5);
    switch (code & 7) {
    case 1: return {T(2), T(-5), -fifth, T(0)};
    case 2: return {T(2), T(-5), T(0), -fifth};
    case 3: case 7: return {T(0), T(-8), T(0), T(0)};
    case 5: return {third8, -third16, T(0), T(0)};
    case 6: return {third8, -third16, T(0), T(0)};
    default: return {T(1), T(-2), T(0), T(0)};  // 0 and 4: no adjacent wall
    }
}

template <typename T>
__device__ __forceinline__ T d2_perp(const Coef<T> &c, T vm2, T vm1, T v0, T vp1, T vp2)
{
    // ((gm vm2 + gp vp2) + b v0) + a (vm1 + vp1), fused in a fixed order
    T t = c.gm * vm2;
    t = fma(c.gp, vp2, t);
    t = fma(c.b, v0, t);
    return fma(c.a, vm1 + vp1, t);
}

// Along the component's own axis: standard 3-point stencil, a solid
// neighbour face holds an exact zero (no penetration at distance one).
template <typename T>
__device__ __forceinline__ T d2_own(T vm1, T v0, T vp1)
{
    return fma(T(-2), v0, vm1 + vp1);
}

// Momentum residual of one fluid face: F = nu (d2x + d2y + d2z) - (p_c - p_m) + G
template <typename T>
__device__ __forceinline__ T momentum(T d2x, T d2y, T d2z, T pc, T pm, T nu, T g)
{
    T lap = (d2x + d2y) + d2z;
    T f = fma(nu, lap, -(pc - pm));
    return f + g;
}

// Divergence of a cell from its six face values, x then y then z.
template <typename T>
__device__ __forceinline__ T divergence(T u0, T u1, T v0, T v1, T w0, T w1)
{
    return ((u1 - u0) + (v1 - v0)) + (w1 - w0);
}

// ---------------------------------------------------------------- reductions
//
// Five FP64 sums per instance and check: S_F, S_D, Q_x, Q_y, Q_z.
constexpr int kNumSums = 5;

__device__ __forceinline__ double wave_sum(double v)
{
    // fixed butterfly over the 64 lanes of a wavefront
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum of kNumSums doubles into out[0..kNumSums) by thread 0.
// scratch: __shared__ double[kNumSums * (blockDim / 64)].
__device__ __forceinline__ void block_sums(double (&acc)[kNumSums], double *scratch, double *out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < kNumSums; ++i) acc[i] = wave_sum(acc[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < kNumSums; ++i) scratch[wave * kNumSums + i] = acc[i];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kNumSums; ++i) {
            double s = 0.0;
            for (int wv = 0; wv < nwaves; ++wv) s += scratch[wv * kNumSums + i];
            out[i] = s;
        }
    }
}

__host__ __device__ inline int wrap_int(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return (int)(r < 0 ? r + n : r);
}

}  // namespace ps
