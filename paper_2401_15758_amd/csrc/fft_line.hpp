// Line FFTs of the 2-D model's spectral operators (device code shared by
// fft2d.hip and the fused stage kernels of bve.hip).
//
// A line of N = 16 B complex values is transformed in padded LDS by sixteen
// threads with the four-step factorisation n = n1 + 16 n2, k = B k1 + k2:
// X[k] = sum_{n1} W16^{n1 k1} W_N^{n1 k2} sum_{n2} x[n1 + 16 n2] W_B^{n2 k2}.
// Thread n1 takes the B-point DFT over n2 (radix 4 x 4 when B = 16, radix-2
// decimation in time down to 16, 4 or an odd 3 or 5 otherwise) and the
// twiddle W_N^{n1 k2}; after a barrier, thread k2 takes
// the radix-4 x 4 16-point DFT of the contiguous block k2.  The inverse is the
// conjugate of the forward transform of the conjugate.  Storage is padded by
// one complex value per 16, which keeps both access patterns free of LDS bank
// conflicts.
#pragma once

#include "internal.hpp"

namespace rp4d {
namespace fftl {

// A multiply-add within one expression may fuse: the 2-D kernels have one
// arithmetic per operator (no tiling choices), so results stay reproducible.
#pragma clang fp contract(on)

constexpr int kLines = 8;  // lines (rows or columns) per workgroup, 16 threads each

__host__ __device__ constexpr int padded(int e) { return e + (e >> 4); }

template <typename T>
struct C2 {
    T r, i;
};

template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, T wr, T wi) {
    return C2<T>{fma(a.r, wr, -(a.i * wi)), fma(a.r, wi, a.i * wr)};
}

// In-place forward 4-point DFT of (a, b, c, d) (W4 = -i).
template <typename T>
__device__ __forceinline__ void dft4(C2<T>& a, C2<T>& b, C2<T>& c, C2<T>& d) {
    const C2<T> t0{a.r + c.r, a.i + c.i}, t1{a.r - c.r, a.i - c.i};
    const C2<T> t2{b.r + d.r, b.i + d.i}, t3{b.r - d.r, b.i - d.i};
    a = C2<T>{t0.r + t2.r, t0.i + t2.i};
    c = C2<T>{t0.r - t2.r, t0.i - t2.i};
    b = C2<T>{t1.r + t3.i, t1.i - t3.r};  // t1 - i t3
    d = C2<T>{t1.r - t3.i, t1.i + t3.r};  // t1 + i t3
}

// Forward 16-point DFT of x (natural order in, natural order out): 4 x 4 with
// n = n1 + 4 n2, k = 4 k1 + k2.
template <typename T>
__device__ __forceinline__ void fft16(C2<T> (&x)[16]) {
    // cos / sin of 2 pi m / 16
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
    constexpr double c2 = 0.70710678118654752440;
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) dft4(x[n1], x[n1 + 4], x[n1 + 8], x[n1 + 12]);
    // now x[n1 + 4 k2] = y[n1][k2]; twiddle by W16^{n1 k2} = exp(-2 pi i n1 k2 / 16)
    x[5] = cmul(x[5], T(c1), T(-s1));    // n1 = 1, k2 = 1: m = 1
    x[9] = cmul(x[9], T(c2), T(-c2));    // n1 = 1, k2 = 2: m = 2
    x[13] = cmul(x[13], T(s1), T(-c1));  // n1 = 1, k2 = 3: m = 3
    x[6] = cmul(x[6], T(c2), T(-c2));    // n1 = 2, k2 = 1: m = 2
    x[10] = C2<T>{x[10].i, -x[10].r};    // n1 = 2, k2 = 2: m = 4 (times -i)
    x[14] = cmul(x[14], T(-c2), T(-c2)); // n1 = 2, k2 = 3: m = 6
    x[7] = cmul(x[7], T(s1), T(-c1));    // n1 = 3, k2 = 1: m = 3
    x[11] = cmul(x[11], T(-c2), T(-c2)); // n1 = 3, k2 = 2: m = 6
    x[15] = cmul(x[15], T(-c1), T(s1));  // n1 = 3, k2 = 3: m = 9
    // 4-point DFTs over n1 for each k2: X[4 k1 + k2] from y[0..3][k2] at 4 k2 + n1
    C2<T> o[16];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        C2<T> a = x[4 * k2], b = x[4 * k2 + 1], c = x[4 * k2 + 2], d = x[4 * k2 + 3];
        dft4(a, b, c, d);
        o[k2] = a;
        o[4 + k2] = b;
        o[8 + k2] = c;
        o[12 + k2] = d;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = o[e];
}

// Forward B-point DFT of x in registers with W_B^m = W_N^{m N/B} (Wl:
// exp(-2 pi i m / N), m < N, in LDS).  B = 16: radix 4 x 4; B = 4: one
// radix-4 butterfly; other even B: decimation in time, the DFTs of the even
// and the odd samples combined with the twiddles W_B^k; odd B (3, 5): the
// direct sum.
template <typename T, int B>
__device__ __forceinline__ void dft_small(C2<T> (&x)[B], const C2<T>* Wl, int N) {
    if constexpr (B == 16) {
        fft16<T>(x);
    } else if constexpr (B == 4) {
        dft4(x[0], x[1], x[2], x[3]);
    } else if constexpr (B == 1) {
    } else if constexpr (B % 2 == 0) {
        constexpr int M = B / 2;
        C2<T> e[M], o[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            e[m] = x[2 * m];
            o[m] = x[2 * m + 1];
        }
        dft_small<T, M>(e, Wl, N);
        dft_small<T, M>(o, Wl, N);
        const int st = N / B;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const C2<T> w = Wl[k * st];
            const C2<T> t = cmul(o[k], w.r, w.i);
            x[k] = C2<T>{e[k].r + t.r, e[k].i + t.i};
            x[k + M] = C2<T>{e[k].r - t.r, e[k].i - t.i};
        }
    } else {
        T wr[B], wi[B];
        const int st = N / B;
#pragma unroll
        for (int m = 0; m < B; ++m) {
            wr[m] = Wl[m * st].r;
            wi[m] = Wl[m * st].i;
        }
        C2<T> y[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            T ar = x[0].r, ai = x[0].i;
#pragma unroll
            for (int n = 1; n < B; ++n) {
                const int m = (n * k) % B;
                ar = ar + (x[n].r * wr[m] - x[n].i * wi[m]);
                ai = ai + (x[n].r * wi[m] + x[n].i * wr[m]);
            }
            y[k] = C2<T>{ar, ai};
        }
#pragma unroll
        for (int k = 0; k < B; ++k) x[k] = y[k];
    }
}

// Transform the line of N = 16 B complex values at `line` (LDS, padded) in place
// with 16 threads (q = 0..15), twiddles Wl in LDS (see stage_twiddles); conj =
// true gives the unnormalised inverse.
// Every thread of the workgroup must call it (it holds a barrier).
template <typename T, int B>
__device__ __forceinline__ void line_fft(C2<T>* line, int q, bool active, const C2<T>* Wl, bool conj) {
    constexpr int N = 16 * B;
    const T sg = conj ? T(-1) : T(1);
    if (active) {
        // step 1: thread n1 = q, B-point DFT over n2 of x[q + 16 n2], then W_N^{q k2}
        C2<T> x[B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) {
            const C2<T> v = line[padded(q + 16 * n2)];
            x[n2] = C2<T>{v.r, sg * v.i};
        }
        dft_small<T, B>(x, Wl, N);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            const int m = q * k2;
            x[k2] = cmul(x[k2], Wl[m].r, Wl[m].i);
            line[padded(q + 16 * k2)] = x[k2];
        }
    }
    __syncthreads();
    // step 3: for k2 = q, q + 16, ...: 16-point DFT over n1 of block k2, to X[B k1 + k2]
    constexpr int R = (B + 15) / 16;
    C2<T> y[R][16];
    if (active) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k2 = q + 16 * r;
            if (k2 < B) {
#pragma unroll
                for (int n1 = 0; n1 < 16; ++n1) y[r][n1] = line[padded(n1 + 16 * k2)];
                fft16<T>(y[r]);
            }
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k2 = q + 16 * r;
            if (k2 < B) {
#pragma unroll
                for (int k1 = 0; k1 < 16; ++k1) line[padded(B * k1 + k2)] = C2<T>{y[r][k1].r, sg * y[r][k1].i};
            }
        }
    }
    __syncthreads();
}


// The N twiddles exp(-2 pi i m / N) (global, (re, im) pairs) of a workgroup of
// 16 kLines threads: load_twiddles issues the loads, store_twiddles writes the
// values into LDS (the caller places its own loads between the two, so that
// their latencies overlap, and a barrier before the first use).
template <int N>
constexpr int twiddles_per_thread() { return (N + 16 * kLines - 1) / (16 * kLines); }

template <typename T, int N>
__device__ __forceinline__ void load_twiddles(const T* __restrict__ W, C2<T> (&v)[twiddles_per_thread<N>()]) {
#pragma unroll
    for (int r = 0; r < twiddles_per_thread<N>(); ++r) {
        const int m = min(static_cast<int>(threadIdx.x) + r * 16 * kLines, N - 1);
        v[r] = C2<T>{W[2 * m], W[2 * m + 1]};
    }
}

template <typename T, int N>
__device__ __forceinline__ void store_twiddles(C2<T>* wl, const C2<T> (&v)[twiddles_per_thread<N>()]) {
#pragma unroll
    for (int r = 0; r < twiddles_per_thread<N>(); ++r) {
        const int m = threadIdx.x + r * 16 * kLines;
        if (m < N) wl[m] = v[r];
    }
}


// ---------------------------------------------------------------------------
// Lines transformed by one wave each (64 threads, lane q), for every side
// N = 16 B the 2-D model takes (32 to 512; factors 2, 3 and 5): self-sorting
// (Stockham) passes of radix 4 while 4 divides what is left, then radix 2, 3
// or 5 (160 = 4 4 2 5, 384 = 4 4 4 2 3); lanes past a pass's N/R butterflies
// idle.  The pass that follows sub-transforms
// of length NS takes, for each butterfly j < N/R, the R values j + r N/R,
// multiplies value r by W_N^{(j mod NS) r N/(NS R)}, transforms them and writes
// them to (j div NS) NS R + (j mod NS) + r NS.  The line is transformed in
// place: the wave reads all of it before it writes any of it, and a wave's LDS
// operations take effect in program order, so no pass needs a workgroup
// barrier -- only the compiler must keep the order (wave_sync).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int N, int R, int NS>
__device__ __forceinline__ void stockham_pass(C2<T>* line, int q, const C2<T>* Wl, bool conj_in, bool conj_out) {
    constexpr int J = N / R, U = (J + 63) / 64;
    C2<T> v[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = q + 64 * u;
        if (J % 64 == 0 || j < J) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const C2<T> x = line[padded(j + r * J)];
                v[u][r] = C2<T>{x.r, conj_in ? -x.i : x.i};
            }
        }
    }
    wave_sync();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = q + 64 * u;
        if (J % 64 == 0 || j < J) {
            const int jm = j % NS;
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const C2<T> w = Wl[jm * r * (N / (NS * R))];
                    v[u][r] = cmul(v[u][r], w.r, w.i);
                }
            }
            if constexpr (R == 4) {
                dft4(v[u][0], v[u][1], v[u][2], v[u][3]);
            } else if constexpr (R == 2) {
                const C2<T> a = v[u][0], b = v[u][1];
                v[u][0] = C2<T>{a.r + b.r, a.i + b.i};
                v[u][1] = C2<T>{a.r - b.r, a.i - b.i};
            } else {
                dft_small<T, R>(v[u], Wl, N);  // 3 or 5: the direct sum
            }
            const int base = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r)
                line[padded(base + r * NS)] = C2<T>{v[u][r].r, conj_out ? -v[u][r].i : v[u][r].i};
        }
    }
    wave_sync();
}

template <typename T, int N, int NS>
__device__ __forceinline__ void stockham_from(C2<T>* line, int q, const C2<T>* Wl, bool conj) {
    constexpr int left = N / NS;
    constexpr int R = left % 4 == 0 ? 4 : (left % 2 == 0 ? 2 : (left % 3 == 0 ? 3 : 5));
    static_assert(left % R == 0, "wave line FFTs take sides whose factors are 2, 3 and 5");
    stockham_pass<T, N, R, NS>(line, q, Wl, NS == 1 && conj, NS * R == N && conj);
    if constexpr (NS * R < N) stockham_from<T, N, NS * R>(line, q, Wl, conj);
}

// Transform the line of N complex values at `line` (LDS, padded) in place with
// the 64 lanes of one wave (q = lane), twiddles Wl (W_N^m, m < N) in LDS;
// conj = true gives the unnormalised inverse.  Only the line's own wave calls
// it; it holds no workgroup barrier.
template <typename T, int N>
__device__ __forceinline__ void line_fft_wave(C2<T>* line, int q, const C2<T>* Wl, bool conj) {
    static_assert(N >= 32 && N <= 512 && N % 16 == 0, "wave line FFTs take N = 16 B from 32 to 512");
    stockham_from<T, N, 1>(line, q, Wl, conj);
}

// Points of a wave line: lane q holds i = q + 64 u for u < wave_points<N>().
// When 64 does not divide N the last u is ragged: wave_has is false on the
// lanes past the end, where wave_point returns N - 1 so that their loads stay
// in bounds; their stores and arithmetic are skipped.
template <int N>
constexpr int wave_points() { return (N + 63) / 64; }

template <int N>
__device__ __forceinline__ bool wave_has(int q, int u) { return N % 64 == 0 || q + 64 * u < N; }

template <int N>
__device__ __forceinline__ int wave_point(int q, int u) { return wave_has<N>(q, u) ? q + 64 * u : N - 1; }

}  // namespace fftl
}  // namespace rp4d
