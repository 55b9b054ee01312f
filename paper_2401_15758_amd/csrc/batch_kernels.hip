// Batched kernels for many independent problems in one launch (gfx950).
//
// Each launch reads a device array of per-problem descriptors; problems may
// differ in size (n) but share the sketch size l.  Reductions (Gram matrices,
// dot products) use one workgroup per problem and a fixed summation order, so a
// problem's result does not depend on which other problems share the batch.
#include <cmath>

#include "internal.hpp"

namespace rp4d {
namespace {

__device__ __forceinline__ size_t boff(int j, int c, int kc, int n) {
    return (static_cast<size_t>(c / kc) * n + j) * kc + (c % kc);
}

// C_p (a x b, FP64 row-major) = X_p^T Y_p over n_p rows.  Work item (problem,
// row chunk, 64 x 64 output tile): partial sums of the chunk go to d.part
// [chunk][a][b]; bgram_reduce sums the chunks in order.  The chunking depends
// only on the problem (d.rows), so results do not depend on the batch.
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) bgram_kernel(const BGram* __restrict__ desc, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const BGram d = desc[it.x];
    const TX* X = static_cast<const TX*>(d.X);
    const TY* Y = static_cast<const TY*>(d.Y);
    __shared__ double xs[16][64];
    __shared__ double ys[16][64];
    const int tid = threadIdx.x, ti = tid / 16, tj = tid % 16;
    const int tiles_b = (d.b + 63) / 64;
    const int i0 = (it.z / tiles_b) * 64, j0 = (it.z % tiles_b) * 64;
    const int r0 = it.y * d.rows, r1 = min(d.n, r0 + d.rows);
    double acc[4][4] = {};
    for (int rr = r0; rr < r1; rr += 16) {
        for (int e = tid; e < 16 * 64; e += 256) {
            const int r = e / 64, col = e % 64, row = rr + r;
            xs[r][col] = (row < r1 && i0 + col < d.a) ? static_cast<double>(X[boff(row, i0 + col, d.lx, d.n)]) : 0.0;
            ys[r][col] = (row < r1 && j0 + col < d.b) ? static_cast<double>(Y[boff(row, j0 + col, d.ly, d.n)]) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int r = 0; r < 16; ++r) {
            double xv[4], yv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                xv[q] = xs[r][ti * 4 + q];
                yv[q] = ys[r][tj * 4 + q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fma(xv[p], yv[q], acc[p][q]);
        }
        __syncthreads();
    }
    double* P = d.part + static_cast<size_t>(it.y) * d.a * d.b;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + ti * 4 + p, j = j0 + tj * 4 + q;
            if (i < d.a && j < d.b) P[static_cast<size_t>(i) * d.b + j] = acc[p][q];
        }
}

__global__ void __launch_bounds__(256) bgram_reduce_kernel(const BGram* __restrict__ desc, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const BGram d = desc[it.x];
    const int nch = (d.n + d.rows - 1) / d.rows;
    const size_t stride = static_cast<size_t>(d.a) * d.b;
    const size_t idx = static_cast<size_t>(it.y) * 256 + threadIdx.x;
    if (idx >= stride) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += d.part[static_cast<size_t>(c) * stride + idx];
    d.C[idx] = s;
}

// Out_p = beta C_p + alpha X_p diag(ds_p) M_p; item = (problem, 64-row block, 64-col block).
template <typename TX, typename TO>
__global__ void __launch_bounds__(256) btsmm_kernel(const BTsmm* __restrict__ desc, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const BTsmm d = desc[it.x];
    const TX* X = static_cast<const TX*>(d.X);
    const TO* C = static_cast<const TO*>(d.C);
    TO* Out = static_cast<TO*>(d.Out);
    __shared__ double xs[64][17];
    __shared__ double ms[16][64];
    const int r0 = it.y * 64, j0 = it.z * 64;
    const int tid = threadIdx.x, ti = tid / 16, tj = tid % 16;
    double acc[4][4] = {};
    for (int kk = 0; kk < d.a; kk += 16) {
        for (int e = tid; e < 64 * 16; e += 256) {
            const int r = e / 16, q = e % 16, row = r0 + r, col = kk + q;
            xs[r][q] = (row < d.n && col < d.a) ? static_cast<double>(X[boff(row, col, d.lx, d.n)]) : 0.0;
        }
        for (int e = tid; e < 16 * 64; e += 256) {
            const int q = e / 64, j = e % 64, i = kk + q, col = j0 + j;
            double v = (i < d.a && col < d.b) ? d.M[static_cast<size_t>(i) * d.b + col] : 0.0;
            if (d.ds && i < d.a) v *= d.ds[i];
            ms[q][j] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
            double xv[4], mv[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                xv[p] = xs[ti * 4 + p][q];
                mv[p] = ms[q][tj * 4 + p];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int s = 0; s < 4; ++s) acc[p][s] = fma(xv[p], mv[s], acc[p][s]);
        }
        __syncthreads();
    }
    // Out may alias C: read every C element of the thread before any store
    double cv[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int row = r0 + ti * 4 + p, col = j0 + tj * 4 + s;
            cv[p][s] = (d.beta != 0.0 && row < d.n && col < d.b) ? static_cast<double>(C[boff(row, col, d.lc, d.n)])
                                                                  : 0.0;
        }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int row = r0 + ti * 4 + p, col = j0 + tj * 4 + s;
            if (row < d.n && col < d.b) {
                double v = d.alpha * acc[p][s];
                if (d.beta != 0.0) v += d.beta * cv[p][s];
                Out[boff(row, col, d.lo, d.n)] = static_cast<TO>(v);
            }
        }
}

// Dense l x l per problem.
__global__ void __launch_bounds__(1024) bchol_kernel(const BSmall* __restrict__ desc, int l) {
    extern __shared__ double sA[];
    __shared__ int bad;
    const BSmall d = desc[blockIdx.x];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < l * l; e += nt) {
        const int i = e / l, j = e % l;
        sA[e] = 0.5 * (d.A[i * l + j] + d.A[j * l + i]);
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
        d.A[e] = (j <= i) ? sA[e] : 0.0;
    }
    if (tid == 0) d.info[0] = bad;
}

// XLDS: the inverse is formed in LDS (two l x l tiles) and written once;
// otherwise in place in global memory.
template <bool XLDS>
__global__ void __launch_bounds__(256) btrinv_kernel(const BSmall* __restrict__ desc, int l) {
    extern __shared__ double sL[];
    const BSmall d = desc[blockIdx.x];
    double* X = XLDS ? sL + l * l : d.B;
    for (int e = threadIdx.x; e < l * l; e += blockDim.x) sL[e] = d.A[e];
    __syncthreads();
    for (int c = threadIdx.x; c < l; c += blockDim.x) {
        for (int i = 0; i < l; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int q = c; q < i; ++q) s -= sL[i * l + q] * X[q * l + c];
            X[i * l + c] = (i < c) ? 0.0 : s / sL[i * l + i];
        }
    }
    if (XLDS) {
        __syncthreads();
        for (int e = threadIdx.x; e < l * l; e += blockDim.x) d.B[e] = X[e];
    }
}

// C = alpha op(A) op(B) (+ column scaling of the result by cs when given)
__global__ void __launch_bounds__(256) bgemm_small_kernel(const BSmall* __restrict__ desc, int l, int ta, int tb,
                                                          double alpha) {
    const BSmall d = desc[blockIdx.x];
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
        const int i = idx / l, j = idx % l;
        double s = 0.0;
        for (int q = 0; q < l; ++q) {
            const double av = ta ? d.A[q * l + i] : d.A[i * l + q];
            const double bv = tb ? d.B[j * l + q] : d.B[q * l + j];
            s = fma(av, bv, s);
        }
        d.C[idx] = alpha * s;
    }
}

// Cyclic Jacobi, one workgroup per problem (same algorithm as the single-problem
// solver: round-robin ordering, in-place 2x2 block rotations, roundoff floor).
template <bool WANTV>
__global__ void __launch_bounds__(1024) bjacobi_kernel(const BSmall* __restrict__ desc, int l) {
    extern __shared__ double sm[];
    const BSmall d = desc[blockIdx.x];
    const int m = l + (l & 1);
    const int ld = m + 1;
    double* sA = sm;
    double* V = sm + m * ld;
    __shared__ double cs[64], sn[64];
    __shared__ int pp[64], qq[64];
    __shared__ int rotated;
    __shared__ double red[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int half = m / 2;
    for (int e = tid; e < m * m; e += nt) {
        const int i = e / m, j = e % m;
        sA[i * ld + j] = (i < l && j < l) ? 0.5 * (d.A[i * l + j] + d.A[j * l + i]) : 0.0;
        if (WANTV) V[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
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
    const int nblk = half * half, nvit = m * half;
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
                const double r00 = ci * b00 - si * b10, r01 = ci * b01 - si * b11;
                const double r10 = si * b00 + ci * b10, r11 = si * b01 + ci * b11;
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
                const double vp = V[row * ld + p], vq = V[row * ld + q];
                V[row * ld + p] = c * vp - s * vq;
                V[row * ld + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
        if (!rotated) break;
        __syncthreads();
    }
    for (int i = tid; i < l; i += nt) {
        const double li = sA[i * ld + i];
        int rank = 0;
        for (int j = 0; j < l; ++j) {
            const double lj = sA[j * ld + j];
            if (lj > li || (lj == li && j < i)) ++rank;
        }
        d.C[rank] = li;  // eigenvalues
        if (WANTV)
            for (int row = 0; row < l; ++row) d.B[row * l + rank] = V[row * ld + i];
    }
}

// Per-problem dot product / max-abs with a fixed reduction order.
__global__ void __launch_bounds__(256) bdot_kernel(const BVec* __restrict__ desc, int absmax) {
    const BVec d = desc[blockIdx.x];
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < d.n; i += 256)
        s = absmax ? fmax(s, fabs(d.x[i])) : fma(d.x[i], d.y[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = absmax ? fmax(red[threadIdx.x], red[threadIdx.x + w])
                                                       : red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.out[0] = red[0];
}

// y = alpha x + beta y, alpha = alpha_h * (alpha_d ? *alpha_d : 1); items (problem, block)
__global__ void __launch_bounds__(256) baxpby_kernel(const BAxpby* __restrict__ desc, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const BAxpby d = desc[it.x];
    const double alpha = d.alpha * (d.alpha_d ? d.alpha_d[0] : 1.0);
    const size_t i0 = static_cast<size_t>(it.y) * 2048;
    for (size_t i = i0 + threadIdx.x; i < d.count && i < i0 + 2048; i += 256)
        d.y[i] = d.beta == 0.0 ? alpha * (d.x ? d.x[i] : 0.0)   // overwrite: y may hold garbage
                               : fma(alpha, d.x ? d.x[i] : 0.0, d.beta * d.y[i]);
}

// PCG updates per problem; inactive problems (converged) are skipped.
__global__ void __launch_bounds__(256) bpcg_xr_kernel(const BPcg* __restrict__ desc, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const BPcg d = desc[it.x];
    const double alpha = d.sc[0] / d.sc[1];  // rz / pq
    const int i0 = it.y * 2048;
    for (int i = i0 + threadIdx.x; i < d.n && i < i0 + 2048; i += 256) {
        d.x[i] = fma(alpha, d.p[i], d.x[i]);
        d.r[i] = fma(-alpha, d.q[i], d.r[i]);
    }
}

__global__ void __launch_bounds__(256) bpcg_p_kernel(const BPcg* __restrict__ desc, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const BPcg d = desc[it.x];
    const double beta = d.sc[2] / d.sc[0];  // rz_new / rz
    const int i0 = it.y * 2048;
    for (int i = i0 + threadIdx.x; i < d.n && i < i0 + 2048; i += 256) d.p[i] = fma(beta, d.p[i], d.z[i]);
}

__global__ void bpcg_scal_kernel(const BPcg* __restrict__ desc, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) desc[i].sc[0] = desc[i].sc[2];
}

// Nystrom shift per problem: nu = sqrt(n) eps sqrt(max(lambda_max(Y^T Y), 0)).
__global__ void bnu_kernel(const BSketch* __restrict__ desc, int np, double eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const BSketch d = desc[i];
    d.nu[0] = sqrt(static_cast<double>(d.n)) * eps * sqrt(fmax(d.ev[0], 0.0));
}

// lam = max(0, s2 - nu), D = lam/(1+lam), cs = 1/sqrt(s2), then U <- U diag(cs).
__global__ void bfinalize_kernel(const BSketch* __restrict__ desc, int l, int use_nu) {
    const BSketch d = desc[blockIdx.x];
    __shared__ double csh[128];
    const double nu = use_nu ? d.nu[0] : 0.0;
    const double smax = fmax(d.ev[0], 0.0);
    for (int i = threadIdx.x; i < l; i += blockDim.x) {
        const double s = d.ev[i];
        const bool ok = s > 1e-300 && s > 1e-30 * smax;
        const double lv = ok ? fmax(0.0, s - nu) : 0.0;
        d.lam[i] = lv;
        d.D[i] = lv / (1.0 + lv);
        csh[i] = ok ? 1.0 / sqrt(s) : 0.0;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) d.U[idx] *= csh[idx % l];
}

// Per-problem Philox4x32-10 + Box-Muller normals (same generator as the
// single-problem path); items (problem, block of 2048 pairs).
__device__ __forceinline__ void philox_round_b(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
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

__global__ void __launch_bounds__(256) bphilox_kernel(const BRand* __restrict__ desc, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const BRand d = desc[it.x];
    const size_t npairs = (d.count + 1) / 2;
    const size_t i0 = static_cast<size_t>(it.y) * 2048;
    for (size_t i = i0 + threadIdx.x; i < npairs && i < i0 + 2048; i += 256) {
        uint32_t c0 = static_cast<uint32_t>(i), c1 = static_cast<uint32_t>(i >> 32), c2 = 0, c3 = 0;
        uint32_t k0 = static_cast<uint32_t>(d.seed), k1 = static_cast<uint32_t>(d.seed >> 32);
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            philox_round_b(c0, c1, c2, c3, k0, k1);
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t a = (static_cast<uint64_t>(c0) << 21) ^ (c1 >> 11);
        const uint64_t b = (static_cast<uint64_t>(c2) << 21) ^ (c3 >> 11);
        const double u1 = (static_cast<double>(a & ((1ull << 53) - 1)) + 1.0) * (1.0 / 9007199254740992.0);
        const double u2 = static_cast<double>(b & ((1ull << 53) - 1)) * (1.0 / 9007199254740992.0);
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = 6.283185307179586476925286766559 * u2;
        d.out[2 * i] = rad * cos(ang);
        if (2 * i + 1 < d.count) d.out[2 * i + 1] = rad * sin(ang);
    }
}

// Converting copy per problem: dst(j, c) [layout dkc] = src(j, c) [layout skc]; items (problem, block)
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) bcopy_kernel(const BCopy* __restrict__ desc, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const BCopy d = desc[it.x];
    const TI* src = static_cast<const TI*>(d.src);
    TO* dst = static_cast<TO*>(d.dst);
    const size_t total = static_cast<size_t>(d.n) * d.k;
    const size_t i0 = static_cast<size_t>(it.y) * 2048;
    for (size_t idx = i0 + threadIdx.x; idx < total && idx < i0 + 2048; idx += 256) {
        const int j = static_cast<int>(idx / d.k), c = static_cast<int>(idx % d.k);
        dst[boff(j, c, d.dkc, d.n)] = d.zero ? TO(0) : static_cast<TO>(src[boff(j, c, d.skc, d.n)]);
    }
}

}  // namespace

template <typename TX, typename TY>
void launch_bgram(const BGram* d, const int4* items, int nitems, const int4* ritems, int nritems, hipStream_t st) {
    if (nitems <= 0) return;
    bgram_kernel<TX, TY><<<nitems, 256, 0, st>>>(d, items);
    RP4D_HIP(hipGetLastError());
    bgram_reduce_kernel<<<nritems, 256, 0, st>>>(d, ritems);
    RP4D_HIP(hipGetLastError());
}

template <typename TX, typename TO>
void launch_btsmm(const BTsmm* d, const int4* items, int nitems, hipStream_t st) {
    if (nitems <= 0) return;
    btsmm_kernel<TX, TO><<<nitems, 256, 0, st>>>(d, items);
    RP4D_HIP(hipGetLastError());
}

void launch_bchol(const BSmall* d, int np, int l, hipStream_t st) {
    if (np <= 0) return;
    const size_t sh = static_cast<size_t>(l) * l * sizeof(double);
    if (sh > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&bchol_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(sh));
    bchol_kernel<<<np, 1024, sh, st>>>(d, l);
    RP4D_HIP(hipGetLastError());
}

void launch_btrinv(const BSmall* d, int np, int l, hipStream_t st) {
    if (np <= 0) return;
    const size_t one = static_cast<size_t>(l) * l * sizeof(double);
    if (lds_fits(reinterpret_cast<const void*>(&btrinv_kernel<true>), 2 * one)) {
        if (2 * one > 64 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&btrinv_kernel<true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(2 * one));
        btrinv_kernel<true><<<np, 256, 2 * one, st>>>(d, l);
    } else {
        if (one > 64 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&btrinv_kernel<false>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(one));
        btrinv_kernel<false><<<np, 256, one, st>>>(d, l);
    }
    RP4D_HIP(hipGetLastError());
}

void launch_bgemm_small(const BSmall* d, int np, int l, int ta, int tb, double alpha, hipStream_t st) {
    if (np <= 0) return;
    bgemm_small_kernel<<<np, 256, 0, st>>>(d, l, ta, tb, alpha);
    RP4D_HIP(hipGetLastError());
}

void launch_bjacobi(const BSmall* d, int np, int l, bool wantv, hipStream_t st) {
    if (np <= 0) return;
    RP4D_REQUIRE(l >= 1 && l <= (wantv ? 96 : 128), RP4D_EINVAL, "batched eigensolver: l must be in [1, 96]");
    const size_t me = static_cast<size_t>(l + (l & 1));
    const size_t sh = (wantv ? 2 : 1) * me * (me + 1) * sizeof(double);
    if (wantv) {
        if (sh > 64 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&bjacobi_kernel<true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(sh));
        bjacobi_kernel<true><<<np, 1024, sh, st>>>(d, l);
    } else {
        if (sh > 64 * 1024)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&bjacobi_kernel<false>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(sh));
        bjacobi_kernel<false><<<np, 1024, sh, st>>>(d, l);
    }
    RP4D_HIP(hipGetLastError());
}

void launch_bdot(const BVec* d, int np, bool absmax, hipStream_t st) {
    if (np <= 0) return;
    bdot_kernel<<<np, 256, 0, st>>>(d, absmax ? 1 : 0);
    RP4D_HIP(hipGetLastError());
}

void launch_baxpby(const BAxpby* d, const int4* items, int nitems, hipStream_t st) {
    if (nitems <= 0) return;
    baxpby_kernel<<<nitems, 256, 0, st>>>(d, items);
    RP4D_HIP(hipGetLastError());
}

void launch_bpcg_xr(const BPcg* d, const int4* items, int nitems, hipStream_t st) {
    if (nitems <= 0) return;
    bpcg_xr_kernel<<<nitems, 256, 0, st>>>(d, items);
    RP4D_HIP(hipGetLastError());
}

void launch_bpcg_p(const BPcg* d, const int4* items, int nitems, int np, hipStream_t st) {
    if (nitems <= 0) return;
    bpcg_p_kernel<<<nitems, 256, 0, st>>>(d, items);
    RP4D_HIP(hipGetLastError());
    bpcg_scal_kernel<<<(np + 63) / 64, 64, 0, st>>>(d, np);
    RP4D_HIP(hipGetLastError());
}

void launch_bnu(const BSketch* d, int np, double eps, hipStream_t st) {
    if (np <= 0) return;
    bnu_kernel<<<(np + 63) / 64, 64, 0, st>>>(d, np, eps);
    RP4D_HIP(hipGetLastError());
}

void launch_bfinalize(const BSketch* d, int np, int l, bool use_nu, hipStream_t st) {
    if (np <= 0) return;
    RP4D_REQUIRE(l <= 128, RP4D_EINVAL, "batched finalize: l <= 128");
    bfinalize_kernel<<<np, 256, 0, st>>>(d, l, use_nu ? 1 : 0);
    RP4D_HIP(hipGetLastError());
}

void launch_bphilox(const BRand* d, const int4* items, int nitems, hipStream_t st) {
    if (nitems <= 0) return;
    bphilox_kernel<<<nitems, 256, 0, st>>>(d, items);
    RP4D_HIP(hipGetLastError());
}

template <typename TI, typename TO>
void launch_bcopy(const BCopy* d, const int4* items, int nitems, hipStream_t st) {
    if (nitems <= 0) return;
    bcopy_kernel<TI, TO><<<nitems, 256, 0, st>>>(d, items);
    RP4D_HIP(hipGetLastError());
}

template void launch_bgram<double, double>(const BGram*, const int4*, int, const int4*, int, hipStream_t);
template void launch_bgram<double, float>(const BGram*, const int4*, int, const int4*, int, hipStream_t);
template void launch_bgram<float, float>(const BGram*, const int4*, int, const int4*, int, hipStream_t);
template void launch_btsmm<double, double>(const BTsmm*, const int4*, int, hipStream_t);
template void launch_btsmm<double, float>(const BTsmm*, const int4*, int, hipStream_t);
template void launch_bcopy<double, double>(const BCopy*, const int4*, int, hipStream_t);
template void launch_bcopy<double, float>(const BCopy*, const int4*, int, hipStream_t);
template void launch_bcopy<float, double>(const BCopy*, const int4*, int, hipStream_t);
template void launch_bcopy<float, float>(const BCopy*, const int4*, int, hipStream_t);

}  // namespace rp4d
