// Dense and reduction kernels of the rp4d library (gfx950, FP64 unless noted):
//   * circulant prior square root Gamma^{1/2} (banded periodic convolution)
//   * layout conversion between row-major (n, k) and the blocked sweep layout
//   * tall-skinny Gram X^T Y and tall-skinny X * M products (deterministic)
//   * dot products with a fixed reduction tree
//   * Philox4x32-10 + Box-Muller Gaussian generator
//   * one-workgroup l x l Cholesky, triangular inverse, small GEMM and a cyclic
//     Jacobi symmetric eigensolver (l <= 128)
#include <cmath>

#include "internal.hpp"

namespace rp4d {
namespace {

__device__ __forceinline__ size_t blk_off(int j, int c, int kc, int n) {
    return (static_cast<size_t>(c / kc) * n + j) * kc + (c % kc);
}

__device__ __forceinline__ int wrapi(long v, int n) {
    long r = v % n;
    return static_cast<int>(r < 0 ? r + n : r);
}

// ---------------------------------------------------------------------------
// Gamma^{1/2}: out(j, c) = sum_{d=-Dm..Dp} g(|d|) in((j - d) mod n, c) [+ addv(j, c)]
// One workgroup per (segment of 4*blockDim outputs, vector); the input segment
// with its halo is staged in LDS; each thread slides a 4-point window.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) circ_conv_kernel(const T* in, int in_kc, T* out, int out_kc,
                                                        const double* gk, int Dm, int Dp, int n, int k,
                                                        const T* addv) {
    extern __shared__ double seg[];
    const int c = blockIdx.y;
    const int TJ = 4 * blockDim.x;
    const int j0 = blockIdx.x * TJ;
    // seg[e + 1] = in(j0 - Dp + e); seg[0] is a pad read by the last window shift
    const int len = TJ + Dm + Dp;
    for (int e = threadIdx.x; e < len; e += blockDim.x) {
        const int j = wrapi(static_cast<long>(j0) - Dp + e, n);
        seg[e + 1] = static_cast<double>(in[blk_off(j, c, in_kc, n)]);
    }
    if (threadIdx.x == 0) seg[0] = 0.0;
    __syncthreads();
    const int t = threadIdx.x;
    // output q = j0 + 4t + i needs in(q - d): seg index 4t + i - d + Dp + 1
    const int base = 4 * t + Dp + 1;
    double w0 = seg[base + Dm], w1 = seg[base + Dm + 1], w2 = seg[base + Dm + 2], w3 = seg[base + Dm + 3];
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int d = -Dm; d <= Dp; ++d) {
        const double gd = gk[d < 0 ? -d : d];
        a0 = fma(gd, w0, a0);
        a1 = fma(gd, w1, a1);
        a2 = fma(gd, w2, a2);
        a3 = fma(gd, w3, a3);
        w3 = w2;
        w2 = w1;
        w1 = w0;
        w0 = seg[base - d - 1];
    }
    const double acc[4] = {a0, a1, a2, a3};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = j0 + 4 * t + i;
        if (q < n) {
            const size_t o = blk_off(q, c, out_kc, n);
            double v = acc[i];
            if (addv) v += static_cast<double>(addv[o]);
            out[o] = static_cast<T>(v);
        }
    }
}

template <typename TI, typename TO>
__global__ void relayout_kernel(const TI* in, int in_kc, TO* out, int out_kc, int n, int k) {
    const size_t total = static_cast<size_t>(n) * k;
    for (size_t idx = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; idx < total;
         idx += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int j = static_cast<int>(idx / k), c = static_cast<int>(idx % k);
        out[blk_off(j, c, out_kc, n)] = static_cast<TO>(in[blk_off(j, c, in_kc, n)]);
    }
}

template <typename T>
__global__ void fill_kernel(T* p, size_t count, T v) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void axpby_kernel(const double* x, double alpha, double* y, double beta, size_t count) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        y[i] = beta == 0.0 ? alpha * x[i] : alpha * x[i] + beta * y[i];  // beta = 0 overwrites
}

// ---------------------------------------------------------------------------
// Tall-skinny products on FP64 MFMA (16x16x4).  Both kernels stage all of a
// workgroup's operand rows through LDS in one round of global loads, so each
// launch pays one memory latency; a workgroup owns a 64 x 64 output tile and
// its four waves 32 x 32 quadrants (2 x 2 MFMA blocks).  Operand fragments:
// lane l holds A[l%16][l/16] and B[l/16][l%16]; the FP64 accumulator element r
// of lane l is row 4r + l/16, column l%16.  LDS operands are k-major with rows
// padded by 16 elements, so the half-waves of a fragment read use disjoint
// banks.  Accumulation order is fixed by the kernel: results are deterministic.
// ---------------------------------------------------------------------------
typedef double ts_v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ ts_v4d ts_mfma(double a, double b, ts_v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int GR = 64;       // Gram: rows per block (the MFMA k dimension), multiple of 4
constexpr int TS_PAD = 16;   // LDS row padding of k-major operands (elements)
constexpr int LDW = 64 + TS_PAD;  // k-major operand: S[k * LDW + col]
constexpr int LDK = GR + 4;       // col-major operand: S[col * LDK + k]

// Offset of element (j, c) of an n-row matrix in the blocked layout with kc
// vectors per block.  Blocked layouts have power-of-two kc (shifts and masks);
// any other kc is a row-major matrix of width <= kc (checked by the launchers).
// Written without branches (the two forms agree for c < kc, so only the block
// index and the column within it are selected): a branch between a tile's
// loads splits them into basic blocks that each wait for their data.
__device__ __forceinline__ size_t ts_off(int j, int c, int kc, int n) {
    const bool p2 = (kc & (kc - 1)) == 0;
    const int blk = p2 ? (c >> __builtin_ctz(kc)) : 0;
    const int in = p2 ? (c & (kc - 1)) : c;
    return (static_cast<size_t>(blk) * n + j) * static_cast<size_t>(kc) + in;
}

// The load is unconditional (element (0, 0) stands in outside the matrix) and
// the zero is selected after it: a guarded load compiles to a branch with a
// wait for its data, which made a tile's loads one memory round trip each.
template <typename TX>
__device__ __forceinline__ double ts_ld(const TX* X, int lx, int n, int row, int col, int nrow, int ncol) {
    const bool ok = row < nrow && col < ncol;
    const double v = static_cast<double>(X[ts_off(ok ? row : 0, ok ? col : 0, lx, n)]);
    return ok ? v : 0.0;
}

// An operand block of GR rows x 64 columns in LDS.  Loaded with lanes walking
// the columns when the layout is row-major-like (lx >= 16) and the rows
// otherwise, and stored in the orientation that keeps those stores contiguous:
// k-major S[k * LDW + col] or column-major S[col * LDK + k].
struct TsBlock {
    bool colwalk;
    __device__ __forceinline__ void coords(int e, int& k, int& c) const {
        k = colwalk ? e / 64 : e % GR;
        c = colwalk ? e % 64 : e / GR;
    }
    __device__ __forceinline__ int at(int k, int c) const { return colwalk ? k * LDW + c : c * LDK + k; }
};
constexpr int TS_BLOCK_DOUBLES = GR * LDW > 64 * LDK ? GR * LDW : 64 * LDK;

// partial[chunk][i * b + j] = sum over the chunk's rows r of X(r, i0 + i) Y(r, j0 + j);
// a chunk is `rows` consecutive rows (a multiple of GR), consumed GR at a time
// with the next block's loads issued before the current block's MFMAs.
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) gram_partial_kernel(const TX* X, int lx, const TY* Y, int ly, int n, int a,
                                                           int b, int rows, double* part) {
    __shared__ double Xs[TS_BLOCK_DOUBLES];
    __shared__ double Ys[TS_BLOCK_DOUBLES];
    const int chunk = blockIdx.x;
    const int tiles_b = (b + 63) / 64;
    const int i0 = (blockIdx.y / tiles_b) * 64, j0 = (blockIdx.y % tiles_b) * 64;
    const int r0 = chunk * rows;
    const int r1 = min(n, r0 + rows);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int PER = GR * 64 / 256;
    const TsBlock bx{lx >= 16}, by{ly >= 16};
    double xv[PER], yv[PER];
    auto load = [&](int rb) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            int k, c;
            bx.coords(e, k, c);
            xv[q] = ts_ld(X, lx, n, rb + k, i0 + c, r1, a);
            by.coords(e, k, c);
            yv[q] = ts_ld(Y, ly, n, rb + k, j0 + c, r1, b);
        }
    };
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    ts_v4d acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = ts_v4d{0.0, 0.0, 0.0, 0.0};
    load(r0);
    for (int rb = r0; rb < r1; rb += GR) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            int k, c;
            bx.coords(e, k, c);
            Xs[bx.at(k, c)] = xv[q];
            by.coords(e, k, c);
            Ys[by.at(k, c)] = yv[q];
        }
        __syncthreads();
        if (rb + GR < r1) load(rb + GR);
        // C = X^T Y: A[i][k] = X(k, i), B[k][j] = Y(k, j)
#pragma unroll 4
        for (int k0 = 0; k0 < GR; k0 += 4) {
            const int kk = k0 + (lane >> 4);
            double fa[2], fb[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                fa[u] = Xs[bx.at(kk, wi + 16 * u + (lane & 15))];
                fb[u] = Ys[by.at(kk, wj + 16 * u + (lane & 15))];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) acc[u][v] = ts_mfma(fa[u], fb[v], acc[u][v]);
        }
        __syncthreads();
    }
    double* P = part + static_cast<size_t>(chunk) * a * b;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + 16 * u + 4 * r + (lane >> 4);
                const int j = j0 + wj + 16 * v + (lane & 15);
                if (i < a && j < b) P[static_cast<size_t>(i) * b + j] = acc[u][v][r];
            }
}

// ---------------------------------------------------------------------------
// BF16 Gram (an option of the sketch post-processing): the same chunked X^T Y
// with both operands rounded to bfloat16 (via FP32, round to nearest even) on
// the BF16 matrix cores, FP32 accumulation within a chunk, and the chunks
// summed in FP64 by reduce_chunks_kernel.  v_mfma_f32_16x16x16_bf16 operands,
// as measured on gfx950: lane l holds A[l%16][4(l/16) + j] and
// B[4(l/16) + j][l%16], j = 0..3; accumulator element r of lane l is
// D[4(l/16) + r][l%16].  LDS holds each operand column with its GR rows
// contiguous (a lane's four k values are one 8-byte read).
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int LDB = GR + 8;  // bf16 column stride in LDS

__device__ __forceinline__ unsigned short to_bf16(double v) {
    const float f = static_cast<float>(v);
    const unsigned u = __builtin_bit_cast(unsigned, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<unsigned short>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return static_cast<unsigned short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <typename TX, typename TY>
__global__ void __launch_bounds__(256) gram_partial_bf16_kernel(const TX* X, int lx, const TY* Y, int ly, int n,
                                                                int a, int b, int rows, double* part) {
    __shared__ __align__(16) unsigned short Xs[64 * LDB];
    __shared__ __align__(16) unsigned short Ys[64 * LDB];
    const int chunk = blockIdx.x;
    const int tiles_b = (b + 63) / 64;
    const int i0 = (blockIdx.y / tiles_b) * 64, j0 = (blockIdx.y % tiles_b) * 64;
    const int r0 = chunk * rows;
    const int r1 = min(n, r0 + rows);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int PER = GR * 64 / 256;
    const TsBlock bx{lx >= 16}, by{ly >= 16};
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int rb = r0; rb < r1; rb += GR) {
        double xv[PER], yv[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            int k, c;
            bx.coords(e, k, c);
            xv[q] = ts_ld(X, lx, n, rb + k, i0 + c, r1, a);
            by.coords(e, k, c);
            yv[q] = ts_ld(Y, ly, n, rb + k, j0 + c, r1, b);
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            int k, c;
            bx.coords(e, k, c);
            Xs[c * LDB + k] = to_bf16(xv[q]);
            by.coords(e, k, c);
            Ys[c * LDB + k] = to_bf16(yv[q]);
        }
        __syncthreads();
#pragma unroll
        for (int k0 = 0; k0 < GR; k0 += 16) {
            const int kk = k0 + 4 * (lane >> 4);
            bf16x4 fa[2], fb[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                fa[u] = *reinterpret_cast<const bf16x4*>(Xs + (wi + 16 * u + (lane & 15)) * LDB + kk);
                fb[u] = *reinterpret_cast<const bf16x4*>(Ys + (wj + 16 * u + (lane & 15)) * LDB + kk);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[u], fb[v], acc[u][v], 0, 0, 0);
        }
        __syncthreads();
    }
    double* P = part + static_cast<size_t>(chunk) * a * b;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + 16 * u + 4 * (lane >> 4) + r;
                const int j = j0 + wj + 16 * v + (lane & 15);
                if (i < a && j < b) P[static_cast<size_t>(i) * b + j] = static_cast<double>(acc[u][v][r]);
            }
}

// out[idx] = sum_c part[c][idx], c in increasing order; loads issued 16 at a time.
__global__ void reduce_chunks_kernel(const double* part, int nchunks, size_t stride, double* out) {
    const size_t idx = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
    if (idx >= stride) return;
    double s = 0.0;
    int c = 0;
    for (; c + 16 <= nchunks; c += 16) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = part[static_cast<size_t>(c + q) * stride + idx];
#pragma unroll
        for (int q = 0; q < 16; ++q) s += v[q];
    }
    for (; c < nchunks; ++c) s += part[static_cast<size_t>(c) * stride + idx];
    out[idx] = s;
}

// Rows per Gram chunk: single GR blocks up to 256 chunks, longer chunks beyond.
int gram_rows(int n) {
    const int blocks = (n + GR - 1) / GR;
    return GR * ((blocks + 255) / 256);
}

int gram_chunks(int n) { return (n + gram_rows(n) - 1) / gram_rows(n); }

// ---------------------------------------------------------------------------
// Out (n x b) = beta * C + alpha * X diag(ds) M, 64 x 64 output tiles; K (= a)
// in blocks of GR staged through LDS (one block for K <= 64), the next block's
// loads issued before the current block's MFMAs.  X's block is an operand block
// indexed (k, row); M's is k-major.
// ---------------------------------------------------------------------------
template <typename TX, typename TO>
__global__ void __launch_bounds__(256) tsmm_kernel(const TX* X, int lx, const double* M, const double* ds, int n,
                                                   int a, int b, double alpha, const TO* C, int lc, double beta,
                                                   TO* Out, int lo) {
    __shared__ double Xs[TS_BLOCK_DOUBLES];
    __shared__ double Ms[GR * LDW];
    const int r0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int PER = GR * 64 / 256;
    // X(row, k): "columns" of the operand block are rows of the output
    const TsBlock bx{lx < 16};
    double xv[PER], mv[PER];
    // every load of a block unconditional and in one basic block, so that all
    // of them are in flight together: out-of-range elements load a stand-in
    // (element 0; the scales from M when there are none) and select zero
    const bool has_ds = ds != nullptr;
    const double* dsrc = has_ds ? ds : M;
    auto load = [&](int kk) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            int k, c;
            bx.coords(e, k, c);
            xv[q] = ts_ld(X, lx, n, r0 + c, kk + k, n, a);
            const int mk = e / 64, mj = e % 64;
            const bool krow = kk + mk < a, okm = krow && j0 + mj < b;
            const double m = M[okm ? static_cast<size_t>(kk + mk) * b + j0 + mj : 0];
            const double dk = dsrc[krow ? kk + mk : 0];
            const double mm = okm ? m : 0.0;
            mv[q] = (has_ds && krow) ? mm * dk : mm;
        }
    };
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    ts_v4d acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = ts_v4d{0.0, 0.0, 0.0, 0.0};
    load(0);
    for (int kk = 0; kk < a; kk += GR) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            int k, c;
            bx.coords(e, k, c);
            Xs[bx.at(k, c)] = xv[q];
            Ms[(e / 64) * LDW + e % 64] = mv[q];
        }
        __syncthreads();
        if (kk + GR < a) load(kk + GR);
        const int kend = min(GR, a - kk);
        for (int k0 = 0; k0 < kend; k0 += 4) {
            const int k = k0 + (lane >> 4);
            double fa[2], fb[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                fa[u] = Xs[bx.at(k, wi + 16 * u + (lane & 15))];
                fb[u] = Ms[k * LDW + wj + 16 * u + (lane & 15)];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) acc[u][v] = ts_mfma(fa[u], fb[v], acc[u][v]);
        }
        __syncthreads();
    }
    // Out may alias C: every C element of the lane is read before any store, so
    // the loads go out together instead of one round trip per output
    double cv[2][2][4] = {};
    if (beta != 0.0) {  // uniform; the loads unconditional, as in ts_ld
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = r0 + wi + 16 * u + 4 * r + (lane >> 4);
                    const int col = j0 + wj + 16 * v + (lane & 15);
                    const bool ok = row < n && col < b;
                    const double c = static_cast<double>(C[ts_off(ok ? row : 0, ok ? col : 0, lc, n)]);
                    cv[u][v][r] = ok ? c : 0.0;
                }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wi + 16 * u + 4 * r + (lane >> 4);
                const int col = j0 + wj + 16 * v + (lane & 15);
                if (row < n && col < b) {
                    double val = alpha * acc[u][v][r];
                    if (beta != 0.0) val += beta * cv[u][v][r];
                    Out[ts_off(row, col, lo, n)] = static_cast<TO>(val);
                }
            }
}

// ---------------------------------------------------------------------------
// Dot product with a fixed reduction tree.
// ---------------------------------------------------------------------------
constexpr int DOT_THREADS = 256;

__global__ void __launch_bounds__(DOT_THREADS) dot_partial_kernel(const double* x, const double* y, size_t count,
                                                                  double* part) {
    __shared__ double red[DOT_THREADS];
    double s = 0.0;
    for (size_t i = blockIdx.x * static_cast<size_t>(DOT_THREADS) + threadIdx.x; i < count;
         i += static_cast<size_t>(gridDim.x) * DOT_THREADS)
        s = fma(x[i], y[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = DOT_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(DOT_THREADS) dot_final_kernel(const double* part, int nb, double* out) {
    __shared__ double red[DOT_THREADS];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += DOT_THREADS) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = DOT_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

int dot_blocks(size_t count) {
    size_t b = (count + 4 * DOT_THREADS - 1) / (4 * DOT_THREADS);
    if (b < 1) b = 1;
    if (b > 256) b = 256;
    return static_cast<int>(b);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) + Box-Muller.
// Counter (i, 0, 0, 0) under key (seed lo, seed hi) gives normals 2i and 2i+1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                             uint32_t k1) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
}

template <typename T>
__global__ void philox_normal_kernel(uint64_t seed, size_t count, T* out) {
    const size_t npairs = (count + 1) / 2;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < npairs;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        uint32_t c0 = static_cast<uint32_t>(i), c1 = static_cast<uint32_t>(i >> 32), c2 = 0, c3 = 0;
        uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            philox_round(c0, c1, c2, c3, k0, k1);
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // two uniforms in (0, 1] with 53 random bits each
        const uint64_t a = (static_cast<uint64_t>(c0) << 21) ^ (c1 >> 11);
        const uint64_t b = (static_cast<uint64_t>(c2) << 21) ^ (c3 >> 11);
        const double u1 = (static_cast<double>(a & ((1ull << 53) - 1)) + 1.0) * (1.0 / 9007199254740992.0);
        const double u2 = static_cast<double>(b & ((1ull << 53) - 1)) * (1.0 / 9007199254740992.0);
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = 6.283185307179586476925286766559 * u2;
        out[2 * i] = static_cast<T>(rad * cos(ang));
        if (2 * i + 1 < count) out[2 * i + 1] = static_cast<T>(rad * sin(ang));
    }
}

// ---------------------------------------------------------------------------
// One-workgroup l x l kernels.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) chol_kernel(double* A, int l, int* info) {
    extern __shared__ double sA[];
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < l * l; e += nt) {
        const int i = e / l, j = e % l;
        sA[e] = 0.5 * (A[i * l + j] + A[j * l + i]);
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < l; ++j) {
        if (tid == 0) {
            const double dj = sA[j * l + j];
            if (!(dj > 0.0) || !isfinite(dj))
                bad = j + 1;
            else
                sA[j * l + j] = sqrt(dj);
        }
        __syncthreads();
        if (bad) break;
        const double djj = sA[j * l + j];
        for (int i = j + 1 + tid; i < l; i += nt) sA[i * l + j] /= djj;
        __syncthreads();
        const int rem = l - j - 1;
        for (int e = tid; e < rem * rem; e += nt) {
            const int i = j + 1 + e / rem, c = j + 1 + e % rem;
            if (c <= i) sA[i * l + c] -= sA[i * l + j] * sA[c * l + j];
        }
        __syncthreads();
    }
    for (int e = tid; e < l * l; e += nt) {
        const int i = e / l, j = e % l;
        A[e] = (j <= i) ? sA[e] : 0.0;
    }
    if (tid == 0) info[0] = bad;
}

// The 64-bit value of `v` held by lane `lane` (uniform), through two 32-bit
// lane reads.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), lane));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), lane));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Cholesky factor of the symmetric part of an l x l matrix, l <= 64, on one
// wave (right-looking).  Lane i keeps row i in registers (zero past l).  Step j
// reads the pivot a(j, j) from lane j, every lane forms its entry of column j
// (the pivot's square root on the diagonal, a(i, j) / L(j, j) below it), the
// column passes through LDS, and each lane updates a(i, c) -= L(i, j) L(c, j)
// for c > j.  Entries right of a lane's diagonal also receive updates; they are
// never read and are written out as zeros.  info = first failing column + 1
// (pivot not positive or not finite), 0 on success.
__global__ void __launch_bounds__(64) chol64_kernel(double* A, int l, int* info) {
    constexpr int LD = 65;
    __shared__ double sA[64 * LD];
    __shared__ double col[64];
    const int i = threadIdx.x;
    const int li = i < l ? i : l - 1;
    // stage A through LDS: coalesced rows, every load in bounds and unconditional
    // (so they are all in flight together), entries past l replaced after the read
#pragma unroll
    for (int t = 0; t < 64; ++t) sA[t * LD + i] = A[(t < l ? t : l - 1) * l + li];
    __syncthreads();
    double a[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) a[c] = (i < l && c < l) ? 0.5 * (sA[i * LD + c] + sA[c * LD + i]) : 0.0;
    int bad = 0;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        if (j >= l || bad) continue;  // uniform: l, and the pivot read from one lane
        const double djj = readlane_f64(a[j], j);
        if (!(djj > 0.0) || !isfinite(djj)) {
            bad = j + 1;
            continue;
        }
        const double d = sqrt(djj);
        const double lij = (i == j) ? d : a[j] / d;
        a[j] = lij;
        col[i] = lij;
        __syncthreads();
#pragma unroll
        for (int c = j + 1; c < 64; ++c) a[c] = fma(-lij, col[c], a[c]);
        __syncthreads();
    }
    if (i < l) {
#pragma unroll
        for (int c = 0; c < 64; ++c)
            if (c < l) A[i * l + c] = (c <= i) ? a[c] : 0.0;
    }
    if (i == 0) info[0] = bad;
}

// X = L^{-1} for orders l <= 64 on one wave: lane c forms column c by forward
// substitution, X(r, c) = -(sum_{k<r} L(r, k) X(k, c)) / L(r, r) for r > c and
// X(c, c) = 1 / L(c, c), keeping the column in registers (zero above c, so the
// sum may run over every k < r).  L sits in LDS as 64 x 64; its rows are read at
// one address across the wave (broadcasts), and the lanes exchange nothing.
// Four partial sums shorten the dependent chain.
__global__ void __launch_bounds__(64) trinv64_kernel(const double* L, double* X, int l) {
    __shared__ __align__(16) double sL[64 * 64];
    __shared__ double rd[64];
    const int c = threadIdx.x;
    const int lc = c < l ? c : l - 1;
    // coalesced rows, every load in bounds and unconditional (all in flight
    // together).  Rows and columns past l hold clamped copies: row r < l reads
    // only k < r, and rows r >= l and lanes c >= l are never written out.
#pragma unroll
    for (int r = 0; r < 64; ++r) sL[r * 64 + c] = L[(r < l ? r : l - 1) * l + lc];
    const double dc = L[lc * l + lc];
    rd[c] = c < l ? 1.0 / dc : 0.0;
    __syncthreads();
    double x[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) {
        double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < r; ++k) s[k & 3] = fma(sL[r * 64 + k], x[k], s[k & 3]);
        const double sum = (s[0] + s[1]) + (s[2] + s[3]);
        x[r] = (r == c) ? rd[r] : (r > c ? -sum * rd[r] : 0.0);
    }
    if (c < l) {
#pragma unroll
        for (int r = 0; r < 64; ++r)
            if (r < l) X[r * l + c] = x[r];
    }
}

// chol64_kernel followed by trinv64_kernel's forward substitution in the same
// wave: the same operations in the same order, so L (written to A) and L^{-1}
// are bitwise those of the two kernels, without L's trip through global memory
// and two launches.  Lane c stores column c of L^{-1} as row c of
// LinvT = L^{-T}.  After a failed factorisation (info != 0) LinvT is untouched.
__global__ void __launch_bounds__(64) chol_invt64_kernel(double* A, int l, int* info, double* LinvT) {
    constexpr int LD = 65;
    __shared__ double sA[64 * LD];
    __shared__ double col[64];
    __shared__ double rd[64];
    const int i = threadIdx.x;
    const int li = i < l ? i : l - 1;
#pragma unroll
    for (int t = 0; t < 64; ++t) sA[t * LD + i] = A[(t < l ? t : l - 1) * l + li];
    __syncthreads();
    double a[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) a[c] = (i < l && c < l) ? 0.5 * (sA[i * LD + c] + sA[c * LD + i]) : 0.0;
    int bad = 0;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        if (j >= l || bad) continue;  // uniform: l, and the pivot read from one lane
        const double djj = readlane_f64(a[j], j);
        if (!(djj > 0.0) || !isfinite(djj)) {
            bad = j + 1;
            continue;
        }
        const double d = sqrt(djj);
        const double lij = (i == j) ? d : a[j] / d;
        a[j] = lij;
        col[i] = lij;
        __syncthreads();
#pragma unroll
        for (int c = j + 1; c < 64; ++c) a[c] = fma(-lij, col[c], a[c]);
        __syncthreads();
    }
    if (i < l) {
#pragma unroll
        for (int c = 0; c < 64; ++c)
            if (c < l) A[i * l + c] = (c <= i) ? a[c] : 0.0;
    }
    if (i == 0) info[0] = bad;
    if (bad) return;  // uniform
    // L by rows in LDS (the entries the substitution reads: k < r < l, and the
    // diagonal), then lane c forms column c of L^{-1} exactly as trinv64_kernel
#pragma unroll
    for (int c = 0; c < 64; ++c) sA[i * LD + c] = (c <= i) ? a[c] : 0.0;
    rd[i] = i < l ? 1.0 / sA[i * LD + i] : 0.0;  // L(i, i), read back: a[] takes no lane-dependent index
    __syncthreads();
    double x[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < r; ++k) s4[k & 3] = fma(sA[r * LD + k], x[k], s4[k & 3]);
        const double sum = (s4[0] + s4[1]) + (s4[2] + s4[3]);
        x[r] = (r == i) ? rd[r] : (r > i ? -sum * rd[r] : 0.0);
    }
    if (i < l) {
#pragma unroll
        for (int r = 0; r < 64; ++r)
            if (r < l) LinvT[i * l + r] = x[r];
    }
}

// X = L^{-1} with L and X both in LDS: thread c forms column c by forward
// substitution (orders with 2 l^2 doubles within the LDS budget).
__global__ void __launch_bounds__(256) trinv_lds_kernel(const double* L, double* X, int l) {
    extern __shared__ double sm[];
    double* sL = sm;
    double* sX = sm + l * l;
    for (int e = threadIdx.x; e < l * l; e += blockDim.x) sL[e] = L[e];
    __syncthreads();
    for (int c = threadIdx.x; c < l; c += blockDim.x) {
        for (int i = 0; i < l; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int q = c; q < i; ++q) s -= sL[i * l + q] * sX[q * l + c];
            sX[i * l + c] = (i < c) ? 0.0 : s / sL[i * l + i];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < l * l; e += blockDim.x) X[e] = sX[e];
}

__global__ void __launch_bounds__(256) trinv_kernel(const double* L, double* X, int l) {
    extern __shared__ double sL[];
    for (int e = threadIdx.x; e < l * l; e += blockDim.x) sL[e] = L[e];
    __syncthreads();
    for (int c = threadIdx.x; c < l; c += blockDim.x) {
        for (int i = 0; i < l; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int q = c; q < i; ++q) s -= sL[i * l + q] * X[q * l + c];
            X[i * l + c] = (i < c) ? 0.0 : s / sL[i * l + i];
        }
    }
}

__global__ void small_gemm_kernel(const double* A, int ta, const double* B, int tb, double* C, int l, double alpha) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= l * l) return;
    const int i = idx / l, j = idx % l;
    double s = 0.0;
    for (int q = 0; q < l; ++q) {
        const double av = ta ? A[q * l + i] : A[i * l + q];
        const double bv = tb ? B[j * l + q] : B[q * l + j];
        s = fma(av, bv, s);
    }
    C[idx] = alpha * s;
}

// Cyclic Jacobi (round-robin parallel ordering; rotation as in Golub & Van Loan
// sym.schur2).  The matrix is padded to even order m (a zero row/column when l
// is odd) and kept in LDS with an odd row stride.  Each round: the m/2 disjoint
// rotations are computed, then every thread applies J^T B J to its own 2x2
// blocks B = A[{p_i,q_i}, {p_j,q_j}] in place (blocks are disjoint, so one
// barrier suffices) and V <- V J on its (row, pair) items.
template <bool VLDS, bool WANTV>
__global__ void __launch_bounds__(1024) jacobi_kernel(double* A, double* evals, double* evecs, double* vwork, int l) {
    extern __shared__ double sm[];
    const int m = l + (l & 1);
    const int ld = m + 1;
    double* sA = sm;
    double* V = VLDS ? (sm + m * ld) : vwork;
    const int vld = VLDS ? ld : m;
    __shared__ double cs[64], sn[64];
    __shared__ int pp[64], qq[64];
    __shared__ int rotated;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int half = m / 2;
    for (int e = tid; e < m * m; e += nt) {
        const int i = e / m, j = e % m;
        sA[i * ld + j] = (i < l && j < l) ? 0.5 * (A[i * l + j] + A[j * l + i]) : 0.0;
    }
    __syncthreads();  // V may alias A's global storage: stage A fully first
    for (int e = tid; WANTV && e < m * m; e += nt) {
        const int i = e / m, j = e % m;
        V[i * vld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int nblk = half * half;      // 2x2 blocks of A
    const int nvit = m * half;         // (row, pair) items of V
    // Frobenius norm (invariant under the rotations).  Applying rotations leaves
    // roundoff of order eps |A|_F in every entry, so off-diagonal entries below
    // 1e-15 |A|_F are not rotated away (otherwise pairs of eigenvalues near the
    // noise level of a numerically singular Gram matrix never converge); above it
    // the relative test |a_pq| > eps sqrt(|a_pp a_qq|) applies.
    __shared__ double red[1024];
    double f2 = 0.0;
    for (int e = tid; e < m * m; e += nt) {
        const double v = sA[(e / m) * ld + (e % m)];
        f2 = fma(v, v, f2);
    }
    red[tid] = f2;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double floor_abs = 1e-15 * sqrt(red[0]);
    // this thread's 2x2-block and V items (fixed across rounds; m <= 128, nt = 1024)
    int tb_i[4], tb_j[4], tv_i[8], tv_r[8];
    int nbt = 0, nvt = 0;
    for (int e = tid; e < nblk && nbt < 4; e += nt, ++nbt) {
        tb_i[nbt] = e / half;
        tb_j[nbt] = e % half;
    }
    for (int e = tid; e < nvit && nvt < 8; e += nt, ++nvt) {
        tv_i[nvt] = e / m;
        tv_r[nvt] = e % m;
    }
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            if (tid < half) {
                // circle method: position 0 fixed, the others rotate
                const int a0 = tid, b0 = m - 1 - tid;
                int p = a0 == 0 ? 0 : ((a0 - 1 + round) % (m - 1)) + 1;
                int q = ((b0 - 1 + round) % (m - 1)) + 1;
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                double c = 1.0, s = 0.0;
                const double apq = sA[p * ld + q];
                const double app = sA[p * ld + p], aqq = sA[q * ld + q];
                if (fabs(apq) > 2.2e-16 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs && fabs(apq) > 1e-300) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double tt = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                                 : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                    rotated = 1;
                }
                cs[tid] = c;
                sn[tid] = s;
                pp[tid] = p;
                qq[tid] = q;
            }
            __syncthreads();
            for (int q8 = 0; q8 < nbt; ++q8) {
                const int bi = tb_i[q8], bj = tb_j[q8];
                const double ci = cs[bi], si = sn[bi], cj = cs[bj], sj = sn[bj];
                if (si == 0.0 && sj == 0.0) continue;
                const int pi = pp[bi], qi = qq[bi], pj = pp[bj], qj = qq[bj];
                const double b00 = sA[pi * ld + pj], b01 = sA[pi * ld + qj];
                const double b10 = sA[qi * ld + pj], b11 = sA[qi * ld + qj];
                // rows: [c -s; s c] B
                const double r00 = ci * b00 - si * b10, r01 = ci * b01 - si * b11;
                const double r10 = si * b00 + ci * b10, r11 = si * b01 + ci * b11;
                // columns: R [c s; -s c]
                sA[pi * ld + pj] = cj * r00 - sj * r01;
                sA[pi * ld + qj] = sj * r00 + cj * r01;
                sA[qi * ld + pj] = cj * r10 - sj * r11;
                sA[qi * ld + qj] = sj * r10 + cj * r11;
            }
            for (int q8 = 0; WANTV && q8 < nvt; ++q8) {
                const int i = tv_i[q8], row = tv_r[q8];
                const double s = sn[i];
                if (s == 0.0) continue;
                const double c = cs[i];
                const int p = pp[i], q = qq[i];
                const double vp = V[row * vld + p], vq = V[row * vld + q];
                V[row * vld + p] = c * vp - s * vq;
                V[row * vld + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
        if (!rotated) break;
        __syncthreads();
    }
    // sort descending (ties by index) and write out the l x l part
    for (int i = tid; i < l; i += nt) {
        const double li = sA[i * ld + i];
        int rank = 0;
        for (int j = 0; j < l; ++j) {
            const double lj = sA[j * ld + j];
            if (lj > li || (lj == li && j < i)) ++rank;
        }
        evals[rank] = li;
        if (WANTV)
            for (int row = 0; row < l; ++row) evecs[row * l + rank] = V[row * vld + i];
    }
}

// Cyclic Jacobi for orders m <= 64 (l padded to even m), the same rotations,
// ordering and stopping rule as jacobi_kernel with fewer dependent LDS trips per
// round: pair indices come from the round number in closed form, thread
// (bi, bj) owns the 2 x 2 block of pairs (bi, bj) of A and the eigenvector
// entries of rows 2bj, 2bj+1 in the columns of pair bi, so after the rotation
// parameters are published (one barrier) each thread loads its block, its V
// entries and two (c, s) pairs at once, updates them and stores (one barrier).
__device__ __forceinline__ void circle_pair(int t, int round, int m, int& p, int& q) {
    const int mm = m - 1;
    int a = t == 0 ? 0 : t - 1 + round;
    if (t != 0) a = (a >= mm ? a - mm : a) + 1;
    int b = m - 2 - t + round;
    b = (b >= mm ? b - mm : b) + 1;
    p = a < b ? a : b;
    q = a < b ? b : a;
}

template <bool WANTV>
__global__ void __launch_bounds__(1024) jacobi64_kernel(const double* A, double* evals, double* evecs, int l) {
    constexpr int LD = 65;
    __shared__ double sA[64 * LD];
    __shared__ double V[WANTV ? 64 * LD : 1];
    __shared__ double cs[32], sn[32];
    __shared__ double red[16];
    __shared__ int rotated;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = l + (l & 1), half = m / 2;
    for (int e = tid; e < m * m; e += 1024) {
        const int i = e / m, j = e % m;
        sA[i * LD + j] = (i < l && j < l) ? 0.5 * (A[i * l + j] + A[j * l + i]) : 0.0;
        if (WANTV) V[i * LD + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    // Frobenius norm (invariant under rotations): noise floor 1e-15 |A|_F
    double f2 = 0.0;
    for (int e = tid; e < m * m; e += 1024) {
        const double v = sA[(e / m) * LD + (e % m)];
        f2 = fma(v, v, f2);
    }
    for (int o = 32; o > 0; o >>= 1) f2 += __shfl_xor(f2, o);
    if (lane == 0) red[wave] = f2;
    __syncthreads();
    double fro2 = 0.0;
    for (int w = 0; w < 16; ++w) fro2 += red[w];
    const double floor_abs = 1e-15 * sqrt(fro2);
    const bool own = tid < half * half;
    const int bi = own ? tid / half : 0, bj = own ? tid % half : 0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            if (tid < half) {
                int p, q;
                circle_pair(tid, round, m, p, q);
                double c = 1.0, s = 0.0;
                const double apq = sA[p * LD + q], app = sA[p * LD + p], aqq = sA[q * LD + q];
                if (fabs(apq) > 2.2e-16 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs && fabs(apq) > 1e-300) {
                    // t = tan(theta) = sign(d) 2apq / (|d| + sqrt(d^2 + 4apq^2)), d = aqq - app (the
                    // smaller root of t^2 + 2 t d/(2apq) - 1 = 0); c = 1/sqrt(1 + t^2) from the
                    // hardware reciprocal square root and one Newton step (one sqrt and one
                    // division on the critical path instead of two and three)
                    const double d = aqq - app, e = 2.0 * apq;
                    const double r = sqrt(fma(d, d, e * e));
                    const double tt = (d >= 0.0 ? e : -e) / (fabs(d) + r);
                    const double w = fma(tt, tt, 1.0);
                    const double y = __builtin_amdgcn_rsq(w);
                    c = y * fma(-0.5 * w * y, y, 1.5);
                    s = tt * c;
                    rotated = 1;
                }
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            if (own) {
                int pi, qi, pj, qj;
                circle_pair(bi, round, m, pi, qi);
                circle_pair(bj, round, m, pj, qj);
                const double ci = cs[bi], si = sn[bi], cj = cs[bj], sj = sn[bj];
                const double b00 = sA[pi * LD + pj], b01 = sA[pi * LD + qj];
                const double b10 = sA[qi * LD + pj], b11 = sA[qi * LD + qj];
                double v0p = 0, v0q = 0, v1p = 0, v1q = 0;
                const int r0 = 2 * bj, r1 = 2 * bj + 1;
                if (WANTV) {
                    v0p = V[r0 * LD + pi];
                    v0q = V[r0 * LD + qi];
                    v1p = V[r1 * LD + pi];
                    v1q = V[r1 * LD + qi];
                }
                if (si != 0.0 || sj != 0.0) {
                    // rows: [c -s; s c] B ; columns: R [c s; -s c]
                    const double r00 = ci * b00 - si * b10, r01 = ci * b01 - si * b11;
                    const double r10 = si * b00 + ci * b10, r11 = si * b01 + ci * b11;
                    sA[pi * LD + pj] = cj * r00 - sj * r01;
                    sA[pi * LD + qj] = sj * r00 + cj * r01;
                    sA[qi * LD + pj] = cj * r10 - sj * r11;
                    sA[qi * LD + qj] = sj * r10 + cj * r11;
                }
                if (WANTV && si != 0.0) {
                    V[r0 * LD + pi] = ci * v0p - si * v0q;
                    V[r0 * LD + qi] = si * v0p + ci * v0q;
                    V[r1 * LD + pi] = ci * v1p - si * v1q;
                    V[r1 * LD + qi] = si * v1p + ci * v1q;
                }
            }
            __syncthreads();
        }
        if (!rotated) break;
        __syncthreads();
    }
    // sort descending (ties by index) and write out the l x l part
    for (int i = tid; i < l; i += 1024) {
        const double li = sA[i * LD + i];
        int rank = 0;
        for (int j = 0; j < l; ++j) {
            const double lj = sA[j * LD + j];
            if (lj > li || (lj == li && j < i)) ++rank;
        }
        evals[rank] = li;
        if (WANTV)
            for (int row = 0; row < l; ++row) evecs[row * l + rank] = V[row * LD + i];
    }
}

// Largest eigenvalue of a symmetric PSD l x l matrix G (l <= 64), padded with
// zeros to 64 x 64 (which adds only zero eigenvalues).  Normalised squarings
// B <- B^2 / max diag(B^2), each a 64 x 64 x 64 product on FP64 MFMA (one
// 16 x 16 output block per wave), concentrate B on the top eigenspace; the
// Rayleigh quotient of G at B's heaviest column is then lambda_max.  Its error
// is second order in the angle to that eigenspace.  After k squarings the
// components outside it carry weights (lambda_m / lambda_1)^(2^k), which move
// max diag(B^2) by about that much per squaring; once it changes by at most
// 1e-12 relative (after at least 6 squarings) one more squaring squares the
// weights again and the loop stops.  At most 24 squarings: then the error is at
// most ~2^-25 relative when the two largest eigenvalues nearly coincide, and
// rounding otherwise.
constexpr int LMAX_SQUARINGS = 24;
constexpr int LMAX_MIN_SQUARINGS = 6;
constexpr double LMAX_STALL_TOL = 1e-12;
typedef double lmax_v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(1024) lmax_squaring_kernel(const double* __restrict__ G, int l, double* out) {
    constexpr int M = 64, LD = 65;
    __shared__ double S[2][M * LD];
    __shared__ double w[M];
    __shared__ double scal[5];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < M * M; e += 1024) {
        const int i = e / M, j = e % M;
        S[0][i * LD + j] = (i < l && j < l) ? 0.5 * (G[i * l + j] + G[j * l + i]) : 0.0;
    }
    if (tid == 0) {
        scal[0] = 1.0;
        scal[2] = -1.0;  // largest diagonal of the previous product
        scal[3] = 0.0;   // 1: the largest diagonal has stalled
        scal[4] = 0.0;   // 1: stop after this squaring
    }
    __syncthreads();
    const int bi = wave >> 2, bj = wave & 3;   // this wave's 16 x 16 output block
    const int fr = lane >> 4, fc = lane & 15;
    int cur = 0;
    for (int it = 0; it < LMAX_SQUARINGS; ++it) {
        const double* B = S[cur];
        double* B2 = S[cur ^ 1];
        const double inv = scal[0];
        lmax_v4d acc = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < M / 4; ++ks) {
            const double a = inv * B[(bi * 16 + fc) * LD + 4 * ks + fr];
            const double b = inv * B[(4 * ks + fr) * LD + bj * 16 + fc];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        // FP64 16x16x4 accumulator: element r of lane l is row 4r + l/16, column l%16
#pragma unroll
        for (int r = 0; r < 4; ++r) B2[(bi * 16 + 4 * r + fr) * LD + bj * 16 + fc] = acc[r];
        __syncthreads();
        if (wave == 0) {
            double d = B2[lane * LD + lane];
            for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_xor(d, o));
            if (lane == 0) {
                scal[0] = d > 0.0 ? 1.0 / d : 1.0;
                if (scal[3] != 0.0)
                    scal[4] = 1.0;  // the one squaring after the stall is done
                else if (it + 1 >= LMAX_MIN_SQUARINGS && fabs(d - scal[2]) <= LMAX_STALL_TOL * d)
                    scal[3] = 1.0;
                scal[2] = d;
            }
        }
        __syncthreads();
        cur ^= 1;
        if (scal[4] != 0.0) break;  // uniform: every thread reads it after the barrier
    }
    // heaviest column of B (largest diagonal entry; lowest index on ties)
    const double* B = S[cur];
    if (wave == 0) {
        double d = B[lane * LD + lane];
        int idx = lane;
        for (int o = 32; o > 0; o >>= 1) {
            const double d2 = __shfl_xor(d, o);
            const int i2 = __shfl_xor(idx, o);
            if (d2 > d || (d2 == d && i2 < idx)) {
                d = d2;
                idx = i2;
            }
        }
        if (lane == 0) scal[1] = static_cast<double>(idx);
    }
    __syncthreads();
    const int jc = static_cast<int>(scal[1]);
    // w = G v (v = column jc of B), then v.w / v.v
    if (tid < l) {
        double acc = 0.0;
        for (int k = 0; k < l; ++k) acc = fma(0.5 * (G[tid * l + k] + G[k * l + tid]), B[k * LD + jc], acc);
        w[tid] = acc;
    }
    __syncthreads();
    if (wave == 0) {
        const double v = lane < l ? B[lane * LD + jc] : 0.0;
        double num = lane < l ? v * w[lane] : 0.0, den = v * v;
        for (int o = 32; o > 0; o >>= 1) {
            num += __shfl_xor(num, o);
            den += __shfl_xor(den, o);
        }
        if (lane == 0) out[0] = den > 0.0 ? num / den : 0.0;
    }
}

inline dim3 grid_for(size_t count, int threads = 256) {
    size_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return dim3(static_cast<unsigned>(b));
}

}  // namespace

template <typename T>
void launch_circ_conv(const T* in, int in_kc, T* out, int out_kc, const double* gk, int D, int n, int k,
                      const T* addv, hipStream_t st) {
    int Dm = D, Dp = D;
    if (2 * D + 1 > n) {  // kernel support covers the circle: each residue once
        Dm = (n - 1) / 2;
        Dp = n / 2;
    }
    int threads = 256;
    while (threads > 64 && 4 * (threads / 2) >= n) threads /= 2;
    const int TJ = 4 * threads;
    const size_t shmem = static_cast<size_t>(TJ + Dm + Dp + 1) * sizeof(double);
    RP4D_REQUIRE(shmem <= 160 * 1024, RP4D_EINVAL, "bhalf: prior kernel band too wide for LDS staging");
    if (shmem > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&circ_conv_kernel<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem));
    dim3 grid((n + TJ - 1) / TJ, k);
    circ_conv_kernel<T><<<grid, threads, shmem, st>>>(in, in_kc, out, out_kc, gk, Dm, Dp, n, k, addv);
    RP4D_HIP(hipGetLastError());
}

template <typename TI, typename TO>
void launch_relayout(const TI* in, int in_kc, TO* out, int out_kc, int n, int k, hipStream_t st) {
    relayout_kernel<TI, TO><<<grid_for(static_cast<size_t>(n) * k), 256, 0, st>>>(in, in_kc, out, out_kc, n, k);
    RP4D_HIP(hipGetLastError());
}

template <typename T>
void launch_fill(T* p, size_t count, T v, hipStream_t st) {
    if (count == 0) return;
    fill_kernel<T><<<grid_for(count), 256, 0, st>>>(p, count, v);
    RP4D_HIP(hipGetLastError());
}

void launch_axpby(const double* x, double alpha, double* y, double beta, size_t count, hipStream_t st) {
    if (count == 0) return;
    axpby_kernel<<<grid_for(count), 256, 0, st>>>(x, alpha, y, beta, count);
    RP4D_HIP(hipGetLastError());
}

size_t gram_work_doubles(int n, int a, int b) {
    return static_cast<size_t>(gram_chunks(n)) * a * b;
}

// Blocked layouts have power-of-two kc; any other leading size is a row-major
// matrix whose width must not exceed it.
static void check_ts_layout(int kc, int width) {
    RP4D_REQUIRE(kc > 0 && ((kc & (kc - 1)) == 0 || width <= kc), RP4D_EINVAL,
                 "tall-skinny product: layout width exceeds a non-power-of-two leading size");
}

template <typename TX, typename TY>
void launch_gram(const TX* X, int lx, const TY* Y, int ly, int n, int a, int b, double* C, double* work,
                 hipStream_t st) {
    check_ts_layout(lx, a);
    check_ts_layout(ly, b);
    const int nchunks = gram_chunks(n);
    dim3 grid(nchunks, ((a + 63) / 64) * ((b + 63) / 64));
    gram_partial_kernel<TX, TY><<<grid, 256, 0, st>>>(X, lx, Y, ly, n, a, b, gram_rows(n), work);
    RP4D_HIP(hipGetLastError());
    const size_t stride = static_cast<size_t>(a) * b;
    reduce_chunks_kernel<<<grid_for(stride), 256, 0, st>>>(work, nchunks, stride, C);
    RP4D_HIP(hipGetLastError());
}

template <typename TX, typename TY>
void launch_gram_bf16(const TX* X, int lx, const TY* Y, int ly, int n, int a, int b, double* C, double* work,
                      hipStream_t st) {
    check_ts_layout(lx, a);
    check_ts_layout(ly, b);
    const int nchunks = gram_chunks(n);
    dim3 grid(nchunks, ((a + 63) / 64) * ((b + 63) / 64));
    gram_partial_bf16_kernel<TX, TY><<<grid, 256, 0, st>>>(X, lx, Y, ly, n, a, b, gram_rows(n), work);
    RP4D_HIP(hipGetLastError());
    const size_t stride = static_cast<size_t>(a) * b;
    reduce_chunks_kernel<<<grid_for(stride), 256, 0, st>>>(work, nchunks, stride, C);
    RP4D_HIP(hipGetLastError());
}

template <typename TX, typename TO>
void launch_tsmm(const TX* X, int lx, const double* M, const double* dscale, int n, int a, int b, double alpha,
                 const TO* Cin, int lc, double beta, TO* Out, int lo, hipStream_t st) {
    check_ts_layout(lx, a);
    check_ts_layout(lo, b);
    if (beta != 0.0) check_ts_layout(lc, b);
    dim3 grid((n + 63) / 64, (b + 63) / 64);
    tsmm_kernel<TX, TO><<<grid, 256, 0, st>>>(X, lx, M, dscale, n, a, b, alpha, Cin, lc, beta, Out, lo);
    RP4D_HIP(hipGetLastError());
}

size_t dot_work_doubles(size_t count) { return static_cast<size_t>(dot_blocks(count)); }

void launch_dot(const double* x, const double* y, size_t count, double* out, double* work, hipStream_t st) {
    const int nb = dot_blocks(count);
    dot_partial_kernel<<<nb, DOT_THREADS, 0, st>>>(x, y, count, work);
    RP4D_HIP(hipGetLastError());
    dot_final_kernel<<<1, DOT_THREADS, 0, st>>>(work, nb, out);
    RP4D_HIP(hipGetLastError());
}

void launch_philox_normal(uint64_t seed, size_t count, double* out, hipStream_t st) {
    launch_philox_normal_t<double>(seed, count, out, st);
}

template <typename T>
void launch_philox_normal_t(uint64_t seed, size_t count, T* out, hipStream_t st) {
    if (count == 0) return;
    philox_normal_kernel<T><<<grid_for((count + 1) / 2), 256, 0, st>>>(seed, count, out);
    RP4D_HIP(hipGetLastError());
}

void launch_chol(double* A, int l, int* info, hipStream_t st) {
    RP4D_REQUIRE(l >= 1 && l <= 128, RP4D_EINVAL, "cholesky: l must be in [1, 128]");
    const size_t shmem = static_cast<size_t>(l) * l * sizeof(double);
    if (shmem > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(shmem));
    if (l <= 64) {
        chol64_kernel<<<1, 64, 0, st>>>(A, l, info);
        RP4D_HIP(hipGetLastError());
        return;
    }
    chol_kernel<<<1, 1024, shmem, st>>>(A, l, info);
    RP4D_HIP(hipGetLastError());
}

bool launch_chol_invt(double* A, int l, int* info, double* LinvT, hipStream_t st) {
    if (l < 1 || l > 64) return false;
    chol_invt64_kernel<<<1, 64, 0, st>>>(A, l, info, LinvT);
    RP4D_HIP(hipGetLastError());
    return true;
}

void launch_trinv(const double* L, double* Linv, int l, hipStream_t st) {
    RP4D_REQUIRE(l >= 1 && l <= 128, RP4D_EINVAL, "trinv: l must be in [1, 128]");
    if (l <= 64) {
        trinv64_kernel<<<1, 64, 0, st>>>(L, Linv, l);
        RP4D_HIP(hipGetLastError());
        return;
    }
    const size_t both = 2 * static_cast<size_t>(l) * l * sizeof(double);
    if (lds_fits(reinterpret_cast<const void*>(&trinv_lds_kernel), both)) {
        if (both > 64 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&trinv_lds_kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(both));
        trinv_lds_kernel<<<1, 256, both, st>>>(L, Linv, l);
        RP4D_HIP(hipGetLastError());
        return;
    }
    const size_t shmem = static_cast<size_t>(l) * l * sizeof(double);
    if (shmem > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&trinv_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(shmem));
    trinv_kernel<<<1, 256, shmem, st>>>(L, Linv, l);
    RP4D_HIP(hipGetLastError());
}

void launch_small_gemm(const double* A, int ta, const double* B, int tb, double* C, int l, double alpha,
                       hipStream_t st) {
    small_gemm_kernel<<<grid_for(static_cast<size_t>(l) * l), 256, 0, st>>>(A, ta, B, tb, C, l, alpha);
    RP4D_HIP(hipGetLastError());
}

// Whether `dyn` bytes of dynamic LDS fit beside the kernel's static LDS.
bool lds_fits(const void* fn, size_t dyn) {
    hipFuncAttributes at{};
    int dev = 0, lim = 0;
    RP4D_HIP(hipFuncGetAttributes(&at, fn));
    RP4D_HIP(hipGetDevice(&dev));
    RP4D_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
    return at.sharedSizeBytes + dyn <= static_cast<size_t>(lim);
}

void launch_sym_lmax(const double* G, int l, double* out, double* work, hipStream_t st) {
    if (l <= 64) {
        lmax_squaring_kernel<<<1, 1024, 0, st>>>(G, l, out);
        RP4D_HIP(hipGetLastError());
        return;
    }
    // larger orders: eigenvalues by the Jacobi solver, which only reads G
    // without eigenvectors (descending: out[0])
    (void)work;
    launch_jacobi_eig(const_cast<double*>(G), out, nullptr, l, st);
}

void launch_jacobi_eig(double* A, double* evals, double* evecs, int l, hipStream_t st) {
    RP4D_REQUIRE(l >= 1 && l <= 128, RP4D_EINVAL, "eigensolver: l must be in [1, 128]");
    const size_t me = static_cast<size_t>(l + (l & 1));
    const bool wantv = evecs != nullptr;
    const size_t both = 2 * me * (me + 1) * sizeof(double);
    const size_t one = me * (me + 1) * sizeof(double);
    if (me <= 64) {
        if (wantv)
            jacobi64_kernel<true><<<1, 1024, 0, st>>>(A, evals, evecs, l);
        else
            jacobi64_kernel<false><<<1, 1024, 0, st>>>(A, evals, nullptr, l);
    } else if (!wantv) {
        // eigenvalues only: V is never touched
        if (one > 64 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_kernel<true, false>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(one));
        jacobi_kernel<true, false><<<1, 1024, one, st>>>(A, evals, nullptr, nullptr, l);
    } else if (lds_fits(reinterpret_cast<const void*>(&jacobi_kernel<true, true>), both)) {
        if (both > 64 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_kernel<true, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(both));
        jacobi_kernel<true, true><<<1, 1024, both, st>>>(A, evals, evecs, nullptr, l);
    } else {
        // V in global memory reuses A's storage (l x l), which needs an even order
        RP4D_REQUIRE((l & 1) == 0, RP4D_EINVAL, "eigensolver: odd l above the LDS limit is not supported");
        if (one > 64 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_kernel<false, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(one));
        jacobi_kernel<false, true><<<1, 1024, one, st>>>(A, evals, evecs, A, l);
    }
    RP4D_HIP(hipGetLastError());
}

template void launch_circ_conv<double>(const double*, int, double*, int, const double*, int, int, int,
                                       const double*, hipStream_t);
template void launch_circ_conv<float>(const float*, int, float*, int, const double*, int, int, int, const float*,
                                      hipStream_t);
template void launch_relayout<double, double>(const double*, int, double*, int, int, int, hipStream_t);
template void launch_relayout<double, float>(const double*, int, float*, int, int, int, hipStream_t);
template void launch_relayout<float, double>(const float*, int, double*, int, int, int, hipStream_t);
template void launch_relayout<float, float>(const float*, int, float*, int, int, int, hipStream_t);
template void launch_fill<double>(double*, size_t, double, hipStream_t);
template void launch_fill<float>(float*, size_t, float, hipStream_t);
template void launch_gram_bf16<double, double>(const double*, int, const double*, int, int, int, int, double*,
                                               double*, hipStream_t);
template void launch_gram<double, double>(const double*, int, const double*, int, int, int, int, double*, double*,
                                          hipStream_t);
template void launch_gram<float, float>(const float*, int, const float*, int, int, int, int, double*, double*,
                                        hipStream_t);
template void launch_gram<double, float>(const double*, int, const float*, int, int, int, int, double*, double*,
                                         hipStream_t);
template void launch_gram<float, double>(const float*, int, const double*, int, int, int, int, double*, double*,
                                         hipStream_t);
template void launch_tsmm<double, double>(const double*, int, const double*, const double*, int, int, int, double,
                                          const double*, int, double, double*, int, hipStream_t);
template void launch_tsmm<float, double>(const float*, int, const double*, const double*, int, int, int, double,
                                         const double*, int, double, double*, int, hipStream_t);
template void launch_tsmm<double, float>(const double*, int, const double*, const double*, int, int, int, double,
                                         const float*, int, double, float*, int, hipStream_t);
template void launch_philox_normal_t<double>(uint64_t, size_t, double*, hipStream_t);
template void launch_philox_normal_t<float>(uint64_t, size_t, float*, hipStream_t);

}  // namespace rp4d
