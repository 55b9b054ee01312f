// Periodic spectral operators of the 2-D model by fast Fourier transforms.
//
// A real operator that is diagonal in the 2-D Fourier basis with an even
// diagonal D(k_y, k_x) = D(-k_y, -k_x) (the inverse Laplacian of the vorticity
// model, Sec. 5.2 in periodic form, and the prior square root) maps two real
// fields at once: with z = a + i b, F^{-1}(D F z) = (L a) + i (L b).  So k real
// fields are transformed as ceil(k/2) complex pair fields in three passes:
//   rows:    z_j  <- DFT_x(a_j + i b_j)                 (one pass over the rows)
//   columns: for every k_x, DFT_y, times D(., k_x), inverse DFT_y
//   rows:    a_j + i b_j <- inverse DFT_x (real part to field 2p, imaginary to 2p+1)
// The 1/(nx ny) of the inverse is folded into D.
//
// Each line transform of length N = 16 B is a four-step factorisation: with
// n = n1 + 16 n2 and k = B k1 + k2, X[k] = sum_{n1} W16^{n1 k1} W_N^{n1 k2}
// sum_{n2} x[n1 + 16 n2] W_B^{n2 k2}.  Sixteen threads share a line held in
// LDS: thread n1 takes the B-point DFT over n2 (radix 4 x 4 when B = 16, a
// direct sum otherwise) and the twiddle W_N^{n1 k2}; after a barrier, thread k2
// takes the 16-point DFT over n1 of the contiguous block k2 (radix 4 x 4).  The
// inverse transform is the conjugate of the forward transform of the conjugate.
// Line storage is padded by one complex value per 16, which keeps both access
// patterns free of LDS bank conflicts.
//
// FP64 has the same peak on the vector units as on the matrix cores of this
// chip, and the radix-4 butterflies need a fraction of the multiply-adds of a
// dense 16-point DFT written as a matrix product, so the butterflies run on the
// vector units.
#include <cmath>

#include "internal.hpp"

namespace rp4d {
namespace {

#pragma clang fp contract(off)

constexpr int kLines = 8;  // lines (rows or columns) per workgroup, 16 threads each

__host__ __device__ constexpr int padded(int e) { return e + (e >> 4); }

template <typename T>
struct C2 {
    T r, i;
};

template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, T wr, T wi) {
    return C2<T>{a.r * wr - a.i * wi, a.r * wi + a.i * wr};
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

// Forward B-point DFT of x with W_B^m = W_N^{m N/B} (W holds exp(-2 pi i m / N)
// as (re, im) pairs).
template <typename T, int B>
__device__ __forceinline__ void dft_small(C2<T> (&x)[B], const T* __restrict__ W, int N) {
    if constexpr (B == 16) {
        fft16<T>(x);
    } else if constexpr (B == 4) {
        dft4(x[0], x[1], x[2], x[3]);
    } else {
        T wr[B], wi[B];
        const int st = N / B;
#pragma unroll
        for (int m = 0; m < B; ++m) {
            wr[m] = W[2 * m * st];
            wi[m] = W[2 * m * st + 1];
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
// with 16 threads (q = 0..15); conj = true gives the unnormalised inverse.
// Every thread of the workgroup must call it (it holds a barrier).
template <typename T, int B>
__device__ __forceinline__ void line_fft(C2<T>* line, int q, bool active, const T* __restrict__ W, bool conj) {
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
        dft_small<T, B>(x, W, N);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            const int m = q * k2;
            x[k2] = cmul(x[k2], W[2 * m], W[2 * m + 1]);
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

// Rows forward: pair p of k real fields (field-major, nx * ny each) -> complex
// row spectra z[p][j][kx] (interleaved re, im).
template <typename T, int B>
__global__ void __launch_bounds__(16 * kLines) fft_rows_fwd(const T* __restrict__ in, int k, int ny,
                                                            T* __restrict__ z, const T* __restrict__ W) {
    constexpr int N = 16 * B;  // nx
    __shared__ C2<T> lds[kLines * padded(N)];
    const int l = threadIdx.x >> 4, q = threadIdx.x & 15;
    const int j = blockIdx.x * kLines + l, p = blockIdx.y;
    const bool active = j < ny;
    C2<T>* line = lds + l * padded(N);
    const size_t n = static_cast<size_t>(N) * ny;
    if (active) {
        const T* a = in + (2 * p) * n + static_cast<size_t>(j) * N;
        const bool hasb = 2 * p + 1 < k;
        const T* b = a + n;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int i = q + 16 * e;
            line[padded(i)] = C2<T>{a[i], hasb ? b[i] : T(0)};
        }
    }
    __syncthreads();
    line_fft<T, B>(line, q, active, W, false);
    if (active) {
        T* zo = z + (static_cast<size_t>(p) * n + static_cast<size_t>(j) * N) * 2;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int i = q + 16 * e;
            const C2<T> v = line[padded(i)];
            zo[2 * i] = v.r;
            zo[2 * i + 1] = v.i;
        }
    }
}

// Columns: for kLines columns kx of pair p, DFT along y (length ny = 16 B),
// times D[ky][kx] (ny x nx, real), inverse DFT along y, in place in z.
template <typename T, int B>
__global__ void __launch_bounds__(16 * kLines) fft_cols(T* __restrict__ z, int nx, const T* __restrict__ D,
                                                        const T* __restrict__ W) {
    constexpr int N = 16 * B;  // ny
    __shared__ C2<T> lds[kLines * padded(N)];
    const int tid = threadIdx.x;
    const int l = tid >> 4, q = tid & 15;
    const int kx0 = blockIdx.x * kLines, p = blockIdx.y;
    const bool active = kx0 + l < nx;
    T* zp = z + static_cast<size_t>(p) * N * nx * 2;
    // load: element (j, c) of the tile, consecutive threads along c
    for (int e = tid; e < N * kLines; e += 16 * kLines) {
        const int j = e / kLines, c = e - j * kLines;
        if (kx0 + c < nx) {
            const T* s = zp + (static_cast<size_t>(j) * nx + kx0 + c) * 2;
            lds[c * padded(N) + padded(j)] = C2<T>{s[0], s[1]};
        }
    }
    __syncthreads();
    C2<T>* line = lds + l * padded(N);
    line_fft<T, B>(line, q, active, W, false);
    if (active) {
        const int kx = kx0 + l;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int ky = q + 16 * e;
            const T d = D[static_cast<size_t>(ky) * nx + kx];
            const C2<T> v = line[padded(ky)];
            line[padded(ky)] = C2<T>{v.r * d, v.i * d};
        }
    }
    __syncthreads();
    line_fft<T, B>(line, q, active, W, true);
    for (int e = tid; e < N * kLines; e += 16 * kLines) {
        const int j = e / kLines, c = e - j * kLines;
        if (kx0 + c < nx) {
            T* s = zp + (static_cast<size_t>(j) * nx + kx0 + c) * 2;
            const C2<T> v = lds[c * padded(N) + padded(j)];
            s[0] = v.r;
            s[1] = v.i;
        }
    }
}

// Rows inverse: z[p] -> fields 2p (real part) and 2p+1 (imaginary part, if any).
template <typename T, int B>
__global__ void __launch_bounds__(16 * kLines) fft_rows_inv(const T* __restrict__ z, int k, int ny,
                                                            T* __restrict__ out, const T* __restrict__ W) {
    constexpr int N = 16 * B;  // nx
    __shared__ C2<T> lds[kLines * padded(N)];
    const int l = threadIdx.x >> 4, q = threadIdx.x & 15;
    const int j = blockIdx.x * kLines + l, p = blockIdx.y;
    const bool active = j < ny;
    C2<T>* line = lds + l * padded(N);
    const size_t n = static_cast<size_t>(N) * ny;
    if (active) {
        const T* zi = z + (static_cast<size_t>(p) * n + static_cast<size_t>(j) * N) * 2;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int i = q + 16 * e;
            line[padded(i)] = C2<T>{zi[2 * i], zi[2 * i + 1]};
        }
    }
    __syncthreads();
    line_fft<T, B>(line, q, active, W, true);
    if (active) {
        T* a = out + (2 * p) * n + static_cast<size_t>(j) * N;
        const bool hasb = 2 * p + 1 < k;
        T* b = a + n;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int i = q + 16 * e;
            const C2<T> v = line[padded(i)];
            a[i] = v.r;
            if (hasb) b[i] = v.i;
        }
    }
}

#define RP4D_FFT_SIZES(X) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32)

template <typename T>
void launch_rows(bool inverse, const T* in, int k, int nx, int ny, T* z, T* out, const T* Wx, hipStream_t st) {
    const dim3 grid((ny + kLines - 1) / kLines, (k + 1) / 2), blk(16 * kLines);
    switch (nx / 16) {
#define RP4D_ROWS(b)                                                                  \
    case b:                                                                           \
        if (inverse)                                                                  \
            fft_rows_inv<T, b><<<grid, blk, 0, st>>>(z, k, ny, out, Wx);              \
        else                                                                          \
            fft_rows_fwd<T, b><<<grid, blk, 0, st>>>(in, k, ny, z, Wx);               \
        break;
        RP4D_FFT_SIZES(RP4D_ROWS)
#undef RP4D_ROWS
        default: fail(RP4D_EINVAL, "2-D grid: unsupported nx");
    }
}

template <typename T>
void launch_cols(T* z, int k, int nx, int ny, const T* D, const T* Wy, hipStream_t st) {
    const dim3 grid((nx + kLines - 1) / kLines, (k + 1) / 2), blk(16 * kLines);
    switch (ny / 16) {
#define RP4D_COLS(b) \
    case b: fft_cols<T, b><<<grid, blk, 0, st>>>(z, nx, D, Wy); break;
        RP4D_FFT_SIZES(RP4D_COLS)
#undef RP4D_COLS
        default: fail(RP4D_EINVAL, "2-D grid: unsupported ny");
    }
}

}  // namespace

bool fft_size_supported(int n) {
    if (n % 16 != 0) return false;
    switch (n / 16) {
        case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 12: case 16: case 20: case 24: case 32:
            return true;
        default:
            return false;
    }
}

template <typename T>
void launch_spectral_diag(const T* in, int k, int nx, int ny, const T* D, const T* Wx, const T* Wy, T* z, T* out,
                          hipStream_t st) {
    RP4D_REQUIRE(fft_size_supported(nx) && fft_size_supported(ny), RP4D_EINVAL,
                 "2-D grid: sides must be 16 B with B in {2,3,4,5,6,8,10,12,16,20,24,32}");
    launch_rows<T>(false, in, k, nx, ny, z, nullptr, Wx, st);
    launch_cols<T>(z, k, nx, ny, D, Wy, st);
    launch_rows<T>(true, nullptr, k, nx, ny, z, out, Wx, st);
    RP4D_HIP(hipGetLastError());
}

template void launch_spectral_diag<double>(const double*, int, int, int, const double*, const double*,
                                           const double*, double*, double*, hipStream_t);
template void launch_spectral_diag<float>(const float*, int, int, int, const float*, const float*, const float*,
                                          float*, float*, hipStream_t);

}  // namespace rp4d
