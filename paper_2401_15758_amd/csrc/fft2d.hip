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

#include "fft_line.hpp"
#include "internal.hpp"

namespace rp4d {
namespace {

// A multiply-add within one expression may fuse: the 2-D kernels have one
// arithmetic per operator (no tiling choices), so results stay reproducible.
#pragma clang fp contract(on)

using namespace fftl;

// Every kernel below issues all of its global loads (data, twiddles and, for
// the columns, the diagonal) before its first LDS store, so that one memory
// latency is paid per kernel rather than one per loop iteration.

// Rows forward: pair p of k real fields (field-major, nx * ny each) -> complex
// row spectra z[p][j][kx] (interleaved re, im).
template <typename T, int B>
__global__ void __launch_bounds__(16 * kLines) fft_rows_fwd(const T* __restrict__ in, int k, int ny,
                                                            T* __restrict__ z, const T* __restrict__ W) {
    constexpr int N = 16 * B;  // nx
    __shared__ C2<T> lds[kLines * padded(N)];
    __shared__ C2<T> wl[N];
    const int l = threadIdx.x >> 4, q = threadIdx.x & 15;
    const int j = blockIdx.x * kLines + l, p = blockIdx.y;
    const bool active = j < ny;
    C2<T>* line = lds + l * padded(N);
    const size_t n = static_cast<size_t>(N) * ny;
    C2<T> tw[twiddles_per_thread<N>()];
    load_twiddles<T, N>(W, tw);
    const bool hasb = 2 * p + 1 < k;
    const T* a = in + (2 * p) * n + static_cast<size_t>(active ? j : 0) * N;
    const T* b = hasb ? a + n : a;
    C2<T> v[B];
#pragma unroll
    for (int e = 0; e < B; ++e) {
        const int i = q + 16 * e;
        v[e] = C2<T>{a[i], b[i]};
    }
    store_twiddles<T, N>(wl, tw);
    if (active) {
#pragma unroll
        for (int e = 0; e < B; ++e) line[padded(q + 16 * e)] = C2<T>{v[e].r, hasb ? v[e].i : T(0)};
    }
    __syncthreads();
    line_fft<T, B>(line, q, active, wl, false);
    if (active) {
        T* zo = z + (static_cast<size_t>(p) * n + static_cast<size_t>(j) * N) * 2;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int i = q + 16 * e;
            const C2<T> u = line[padded(i)];
            zo[2 * i] = u.r;
            zo[2 * i + 1] = u.i;
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
    __shared__ C2<T> wl[N];
    const int tid = threadIdx.x;
    const int l = tid >> 4, q = tid & 15;
    const int kx0 = blockIdx.x * kLines, p = blockIdx.y;
    const bool active = kx0 + l < nx;
    T* zp = z + static_cast<size_t>(p) * N * nx * 2;
    // thread tid loads rows j = tid / kLines + 16 r of column kx0 + tid % kLines
    const int c = tid % kLines, jb = tid / kLines;
    const bool cok = kx0 + c < nx;
    C2<T> tw[twiddles_per_thread<N>()];
    load_twiddles<T, N>(W, tw);
    C2<T> v[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const T* s = zp + (static_cast<size_t>(jb + 16 * r) * nx + (cok ? kx0 + c : 0)) * 2;
        v[r] = C2<T>{s[0], s[1]};
    }
    // the diagonal at (ky = q + 16 e, kx0 + l), used after the forward transform
    T d[B];
    const int kx = active ? kx0 + l : 0;
#pragma unroll
    for (int e = 0; e < B; ++e) d[e] = D[static_cast<size_t>(q + 16 * e) * nx + kx];
    store_twiddles<T, N>(wl, tw);
#pragma unroll
    for (int r = 0; r < B; ++r)
        if (cok) lds[c * padded(N) + padded(jb + 16 * r)] = v[r];
    __syncthreads();
    C2<T>* line = lds + l * padded(N);
    line_fft<T, B>(line, q, active, wl, false);
    if (active) {
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int ky = q + 16 * e;
            const C2<T> u = line[padded(ky)];
            line[padded(ky)] = C2<T>{u.r * d[e], u.i * d[e]};
        }
    }
    __syncthreads();
    line_fft<T, B>(line, q, active, wl, true);
#pragma unroll
    for (int r = 0; r < B; ++r) {
        if (cok) {
            T* s = zp + (static_cast<size_t>(jb + 16 * r) * nx + kx0 + c) * 2;
            const C2<T> u = lds[c * padded(N) + padded(jb + 16 * r)];
            s[0] = u.r;
            s[1] = u.i;
        }
    }
}

// The same column pass with one wave per column (few field pairs, every
// supported ny): L columns per workgroup, loaded and stored row-wise
// (coalesced) through LDS; wave c transforms column c, scales it by the
// diagonal and transforms it back with no workgroup barrier in between.
// Columns per workgroup: 2 (22.2 ms per bve-256 k = 1 product) against 4
// (22.7 ms) and 8 (25.8 ms).
constexpr int kColWaveLines = 2;

template <typename T, int N, int L>
__global__ void __launch_bounds__(64 * L) fft_cols_w(T* __restrict__ z, int nx, const T* __restrict__ D,
                                                   const T* __restrict__ W) {
    constexpr int NT = 64 * L, P = wave_points<N>(), TW = (N + NT - 1) / NT;
    __shared__ C2<T> lds[L * padded(N)];
    __shared__ C2<T> wl[N];
    const int tid = threadIdx.x, wv = tid >> 6, q = tid & 63;
    const int kx0 = blockIdx.x * L, p = blockIdx.y;
    T* zp = z + static_cast<size_t>(p) * N * nx * 2;
    // thread tid moves rows jb + 64 r < N of column kx0 + c (c = tid % L)
    const int c = tid % L, jb = tid / L;
    const bool cok = kx0 + c < nx;
    C2<T> tw[TW];
#pragma unroll
    for (int r = 0; r < TW; ++r) {
        const int m = min(tid + r * NT, N - 1);
        tw[r] = C2<T>{W[2 * m], W[2 * m + 1]};
    }
    C2<T> v[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const T* s = zp + (static_cast<size_t>(wave_point<N>(jb, r)) * nx + (cok ? kx0 + c : 0)) * 2;
        v[r] = C2<T>{s[0], s[1]};
    }
    const bool active = kx0 + wv < nx;
    const int kx = active ? kx0 + wv : 0;
    T d[P];
#pragma unroll
    for (int u = 0; u < P; ++u) d[u] = D[static_cast<size_t>(wave_point<N>(q, u)) * nx + kx];
#pragma unroll
    for (int r = 0; r < TW; ++r) {
        const int m = tid + r * NT;
        if (m < N) wl[m] = tw[r];
    }
#pragma unroll
    for (int r = 0; r < P; ++r)
        if (cok && wave_has<N>(jb, r)) lds[c * padded(N) + padded(jb + 64 * r)] = v[r];
    __syncthreads();
    if (active) {
        C2<T>* line = lds + wv * padded(N);
        line_fft_wave<T, N>(line, q, wl, false);
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (!wave_has<N>(q, u)) continue;
            const int ky = q + 64 * u;
            const C2<T> x = line[padded(ky)];
            line[padded(ky)] = C2<T>{x.r * d[u], x.i * d[u]};
        }
        wave_sync();
        line_fft_wave<T, N>(line, q, wl, true);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < P; ++r) {
        if (cok && wave_has<N>(jb, r)) {
            T* s = zp + (static_cast<size_t>(jb + 64 * r) * nx + kx0 + c) * 2;
            const C2<T> x = lds[c * padded(N) + padded(jb + 64 * r)];
            s[0] = x.r;
            s[1] = x.i;
        }
    }
}

// Rows inverse: z[p] -> fields 2p (real part) and 2p+1 (imaginary part, if any).
template <typename T, int B>
__global__ void __launch_bounds__(16 * kLines) fft_rows_inv(const T* __restrict__ z, int k, int ny,
                                                            T* __restrict__ out, const T* __restrict__ W) {
    constexpr int N = 16 * B;  // nx
    __shared__ C2<T> lds[kLines * padded(N)];
    __shared__ C2<T> wl[N];
    const int l = threadIdx.x >> 4, q = threadIdx.x & 15;
    const int j = blockIdx.x * kLines + l, p = blockIdx.y;
    const bool active = j < ny;
    C2<T>* line = lds + l * padded(N);
    const size_t n = static_cast<size_t>(N) * ny;
    C2<T> tw[twiddles_per_thread<N>()];
    load_twiddles<T, N>(W, tw);
    const T* zi = z + (static_cast<size_t>(p) * n + static_cast<size_t>(active ? j : 0) * N) * 2;
    C2<T> v[B];
#pragma unroll
    for (int e = 0; e < B; ++e) {
        const int i = q + 16 * e;
        v[e] = C2<T>{zi[2 * i], zi[2 * i + 1]};
    }
    store_twiddles<T, N>(wl, tw);
    if (active) {
#pragma unroll
        for (int e = 0; e < B; ++e) line[padded(q + 16 * e)] = v[e];
    }
    __syncthreads();
    line_fft<T, B>(line, q, active, wl, true);
    if (active) {
        T* a = out + (2 * p) * n + static_cast<size_t>(j) * N;
        const bool hasb = 2 * p + 1 < k;
        T* b = a + n;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int i = q + 16 * e;
            const C2<T> u = line[padded(i)];
            a[i] = u.r;
            if (hasb) b[i] = u.i;
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

// Column passes with one wave per column while the grid has at most this many
// field pairs (latency-bound launches).
constexpr int kWaveColPairs = 4;

template <typename T>
void launch_cols(T* z, int k, int nx, int ny, const T* D, const T* Wy, hipStream_t st) {
    if ((k + 1) / 2 <= kWaveColPairs) {
        constexpr int L = kColWaveLines;
        const dim3 gw((nx + L - 1) / L, (k + 1) / 2), bw(64 * L);
        switch (ny / 16) {
#define RP4D_WAVE_COLS(b) \
    case b: fft_cols_w<T, 16 * b, L><<<gw, bw, 0, st>>>(z, nx, D, Wy); return;
            RP4D_FFT_SIZES(RP4D_WAVE_COLS)
#undef RP4D_WAVE_COLS
            default: fail(RP4D_EINVAL, "2-D grid: unsupported ny");
        }
    }
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

template <typename T>
void launch_fft_rows_fwd(const T* in, int k, int nx, int ny, T* z, const T* Wx, hipStream_t st) {
    launch_rows<T>(false, in, k, nx, ny, z, nullptr, Wx, st);
    RP4D_HIP(hipGetLastError());
}

template <typename T>
void launch_fft_cols(T* z, int k, int nx, int ny, const T* D, const T* Wy, hipStream_t st) {
    launch_cols<T>(z, k, nx, ny, D, Wy, st);
    RP4D_HIP(hipGetLastError());
}

template void launch_fft_rows_fwd<double>(const double*, int, int, int, double*, const double*, hipStream_t);
template void launch_fft_rows_fwd<float>(const float*, int, int, int, float*, const float*, hipStream_t);
template void launch_fft_cols<double>(double*, int, int, int, const double*, const double*, hipStream_t);
template void launch_fft_cols<float>(float*, int, int, int, const float*, const float*, hipStream_t);
template void launch_spectral_diag<double>(const double*, int, int, int, const double*, const double*,
                                           const double*, double*, double*, hipStream_t);
template void launch_spectral_diag<float>(const float*, int, int, int, const float*, const float*, const float*,
                                          float*, float*, hipStream_t);

}  // namespace rp4d
