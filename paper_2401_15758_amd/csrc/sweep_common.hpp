// Per-point stencil arithmetic and region edge exchanges shared by the 1-D
// Burgers sweeps (periodic RK4 and wall-bounded RK3-TVD).  Included by the
// sweep translation units only; everything here is internal to each of them.
#pragma once
#include "internal.hpp"

// Every multiply-add is an explicit fma() and automatic contraction is off, so
// each point's rounding is fixed by the source (bitwise tiling independence).
#pragma clang fp contract(off)

namespace rp4d {
namespace {

// Nonlinear RHS at a point: -Y (Y+ - Y-)/(2dx) + nu (Y+ - 2Y + Y-)/dx^2.
template <typename T>
__device__ __forceinline__ T rhs_pt(T Y, T ym, T yp, T i2, T nd) {
    const T Dy = (yp - ym) * i2;
    const T lap = fma(T(-2), Y, yp + ym);
    return fma(nd, lap, -(Y * Dy));
}

__device__ __forceinline__ int wrap_index(long v, int n) {
    long r = v % n;
    return static_cast<int>(r < 0 ? r + n : r);
}

// Edge exchange: each thread hands over the values of its first and last point
// and receives its left neighbour's last-point values and its right
// neighbour's first-point values.  The region's end threads receive values of
// their own region (any finite values do: they lie in the halo, which the
// temporal blocking discards).
template <typename T, int W>
struct LdsExchange {
    T* sh;
    int NT, t, tl, tr;
    int buf;
    __device__ LdsExchange(T* sh_, int NT_, int t_) : sh(sh_), NT(NT_), t(t_), buf(0) {
        tl = t > 0 ? t - 1 : 0;
        tr = t < NT - 1 ? t + 1 : NT - 1;
    }
    template <int N>
    __device__ __forceinline__ void operator()(const T (&first)[N], const T (&last)[N], T (&from_left)[N],
                                               T (&from_right)[N]) {
        static_assert(N <= W, "exchange record wider than the LDS slot");
        T* B = sh + static_cast<size_t>(buf) * 2 * NT * W;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            B[t * W + i] = first[i];
            B[(NT + t) * W + i] = last[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < N; ++i) {
            from_left[i] = B[(NT + tl) * W + i];
            from_right[i] = B[tr * W + i];
        }
        buf ^= 1;
    }
};

// DPP wave shifts by one lane (lane i reads lane i - 1, resp. i + 1); the end
// lane of the shift reads zero (bound_ctrl), which spares the copy of the old
// value that a keep-own-value shift needs.  Every lane of the wave must be active.
__device__ __forceinline__ int lane_from_lower(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int lane_from_upper(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }

template <bool FromLower>
__device__ __forceinline__ double lane_shift(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    int lo = static_cast<int>(b), hi = static_cast<int>(b >> 32);
    lo = FromLower ? lane_from_lower(lo) : lane_from_upper(lo);
    hi = FromLower ? lane_from_lower(hi) : lane_from_upper(hi);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <bool FromLower>
__device__ __forceinline__ float lane_shift(float v) {
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, FromLower ? lane_from_lower(b) : lane_from_upper(b));
}

struct WaveExchange {
    template <typename T, int N>
    __device__ __forceinline__ void operator()(const T (&first)[N], const T (&last)[N], T (&from_left)[N],
                                               T (&from_right)[N]) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            from_left[i] = lane_shift<true>(last[i]);
            from_right[i] = lane_shift<false>(first[i]);
        }
    }
};

}  // namespace
}  // namespace rp4d
