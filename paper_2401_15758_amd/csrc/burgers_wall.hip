// Wall-bounded Burgers sweeps for gfx950: the paper's own setup of Sec. 5.1 --
// homogeneous Dirichlet walls, second-order central differences and the
// three-stage TVD Runge-Kutta method in Shu-Osher form,
//     w1 = u + h f(u),  w2 = 3/4 u + 1/4 (w1 + h f(w1)),  u+ = 1/3 u + 2/3 (w2 + h f(w2)),
// with its discrete tangent-linear (TLM) and adjoint (ADJ) sweeps.
//
// The decomposition is that of the periodic sweeps (overlapped temporal
// blocking on wave regions of 64 P points, DPP edge exchanges, KC interleaved
// vectors per region, the base trajectory recomputed into stage states on the
// fly) with two changes: region points are not wrapped, and every value at a
// point outside the n interior nodes is held at zero after each stage, which
// is exactly the wall value the stencils of the first and last node read.  A
// step consumes a stencil radius of three points, within the periodic sweeps'
// halo of 4 S + 4.  The n interior nodes sit at x_j = (j + 1)/(n + 1); node j
// is observed when (j + 1) is a multiple of obs_stride, as row (j + 1)/obs_stride - 1.
#include "internal.hpp"
#include "sweep_common.hpp"

namespace rp4d {
namespace {

// Shu-Osher combination of stage st: w_{st+1} = alpha_st u + beta_st (w_st + h f(w_st)).
template <typename T>
__device__ __forceinline__ T ssp_combine(int st, T e, T u) {
    if (st == 0) return e;
    if (st == 1) return fma(T(0.25), e, T(0.75) * u);
    return fma(static_cast<T>(2.0 / 3.0), e, static_cast<T>(1.0 / 3.0) * u);
}

__device__ __forceinline__ bool wall_obs(int g, int n, int stride) {
    return g >= 0 && g < n && ((g + 1) % stride) == 0;
}

template <int P, typename X>
__device__ __forceinline__ void fwd3_body(const FwdArgs& a, int tile_id, int t, X& xch) {
    const int n = a.n;
    const int tstart = tile_id * a.tile;
    const int tlen = min(a.tile, n - tstart);
    const double h = a.h, i2 = a.inv2dx, nd = a.nu_dx2;
    int g[P];
    bool in[P], own[P];
    double u[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = t * P + p;
        g[p] = tstart - a.halo + r;
        in[p] = g[p] >= 0 && g[p] < n;
        own[p] = in[p] && r >= a.halo && r < a.halo + tlen;
        u[p] = in[p] ? a.xin[g[p]] : 0.0;
    }
    for (int s = a.s0; s < a.s0 + a.S; ++s) {
        double w[P];
#pragma unroll
        for (int p = 0; p < P; ++p) w[p] = u[p];
#pragma unroll
        for (int st = 0; st < 3; ++st) {
            const double e0[1] = {w[0]}, e1[1] = {w[P - 1]};
            double fl[1], fr[1];
            xch(e0, e1, fl, fr);
            double wn[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const double ym = p > 0 ? w[p - 1] : fl[0];
                const double yp = p < P - 1 ? w[p + 1] : fr[0];
                const double e = fma(h, rhs_pt<double>(w[p], ym, yp, i2, nd), w[p]);
                wn[p] = in[p] ? ssp_combine<double>(st, e, u[p]) : 0.0;
            }
#pragma unroll
            for (int p = 0; p < P; ++p) w[p] = wn[p];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = w[p];
        const int s1 = s + 1;
        if (a.store != nullptr && (s1 % a.store_every) == 0) {
            const int row = s1 / a.store_every - a.store_row0;
            if (row >= 0 && row < a.store_rows) {
#pragma unroll
                for (int p = 0; p < P; ++p)
                    if (own[p]) a.store[static_cast<size_t>(row) * n + g[p]] = u[p];
            }
        }
        if ((s1 % a.obs_every) == 0) {
            const int i = s1 / a.obs_every;
            if (i >= 1 && i <= a.n_t) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (own[p] && wall_obs(g[p], n, a.obs_stride)) {
                        const size_t idx = static_cast<size_t>(i - 1) * a.n_obs + (g[p] + 1) / a.obs_stride - 1;
                        if (a.obs_out) a.obs_out[idx] = u[p];
                        if (a.innov) a.innov[idx] = (u[p] - a.y[idx]) * a.inv_sigma_o;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (own[p]) a.xout[g[p]] = u[p];
}

template <typename T, int P, int KC, typename X>
__device__ __forceinline__ void tlm3_body(const SweepArgs<T>& a, int tile_id, int grp, int t, X& xch) {
    const int n = a.n;
    const int tstart = tile_id * a.tile;
    const int tlen = min(a.tile, n - tstart);
    const T h = a.h, i2 = a.inv2dx, nd = a.nu_dx2;
    const T nd2 = T(2) * nd;
    int g[P];
    bool in[P], own[P];
    T d[P][KC];
    const T* xin = a.xin + static_cast<size_t>(grp) * n * KC;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = t * P + p;
        g[p] = tstart - a.halo + r;
        in[p] = g[p] >= 0 && g[p] < n;
        own[p] = in[p] && r >= a.halo && r < a.halo + tlen;
#pragma unroll
        for (int c = 0; c < KC; ++c) d[p][c] = in[p] ? xin[static_cast<size_t>(g[p]) * KC + c] : T(0);
    }
    auto base_at = [&](int s, int p) -> T {
        return in[p] ? static_cast<T>(a.base[static_cast<size_t>(s - a.base_row0) * n + g[p]]) : T(0);
    };
    T unext[P];
#pragma unroll
    for (int p = 0; p < P; ++p) unext[p] = base_at(a.s0, p);
    for (int s = a.s0; s < a.s0 + a.S; ++s) {
        T u[P];
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = unext[p];
        if (s + 1 < a.s0 + a.S) {
#pragma unroll
            for (int p = 0; p < P; ++p) unext[p] = base_at(s + 1, p);
        }
        T Y[P], dY[P][KC];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            Y[p] = u[p];
#pragma unroll
            for (int c = 0; c < KC; ++c) dY[p][c] = d[p][c];
        }
#pragma unroll
        for (int st = 0; st < 3; ++st) {
            T e0[1 + KC], e1[1 + KC], fl[1 + KC], fr[1 + KC];
            e0[0] = Y[0];
            e1[0] = Y[P - 1];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                e0[1 + c] = dY[0][c];
                e1[1 + c] = dY[P - 1][c];
            }
            xch(e0, e1, fl, fr);
            T Yn[P], dYn[P][KC];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const T ym = p > 0 ? Y[p - 1] : fl[0];
                const T yp = p < P - 1 ? Y[p + 1] : fr[0];
                const T Dy = (yp - ym) * i2;
                const T Yh = Y[p] * i2;
                const T ca = -Dy - nd2;
                const T cp = nd - Yh;
                const T cm = nd + Yh;
                if (st < 2) {
                    const T e = fma(h, rhs_pt<T>(Y[p], ym, yp, i2, nd), Y[p]);
                    Yn[p] = in[p] ? ssp_combine<T>(st, e, u[p]) : T(0);
                }
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    const T dm = p > 0 ? dY[p - 1][c] : fl[1 + c];
                    const T dp = p < P - 1 ? dY[p + 1][c] : fr[1 + c];
                    const T dK = fma(cm, dm, fma(cp, dp, ca * dY[p][c]));
                    const T e = fma(h, dK, dY[p][c]);
                    dYn[p][c] = in[p] ? ssp_combine<T>(st, e, d[p][c]) : T(0);
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (st < 2) Y[p] = Yn[p];
#pragma unroll
                for (int c = 0; c < KC; ++c) dY[p][c] = dYn[p][c];
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int c = 0; c < KC; ++c) d[p][c] = dY[p][c];
        const int s1 = s + 1;
        if ((s1 % a.obs_every) == 0) {
            const int i = s1 / a.obs_every;
            if (i >= 1 && i <= a.n_t) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (own[p] && wall_obs(g[p], n, a.obs_stride)) {
                        const size_t row = static_cast<size_t>(i - 1) * a.n_obs + (g[p] + 1) / a.obs_stride - 1;
#pragma unroll
                        for (int c = 0; c < KC; ++c) {
                            const int col = grp * KC + c;
                            if (col < a.k) a.z[row * a.k + col] = d[p][c] * a.inv_sigma_o;
                        }
                    }
                }
            }
        }
    }
    T* xout = a.xout + static_cast<size_t>(grp) * n * KC;
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (own[p]) {
#pragma unroll
            for (int c = 0; c < KC; ++c) xout[static_cast<size_t>(g[p]) * KC + c] = d[p][c];
        }
}

// J(Y)^T m at every point of the thread (edges of Y and m from the neighbours):
// ca m + cp m+ + cm m-, ca = -Dy - 2nu/dx^2, cp = nu/dx^2 + Y+/(2dx),
// cm = nu/dx^2 - Y-/(2dx).
template <typename T, int P, int KC>
__device__ __forceinline__ void jac_t_pts(const T (&Y)[P], T YL, T YR, const T (&m)[P][KC], const T (&ml)[KC],
                                          const T (&mr)[KC], T i2, T nd, T (&out)[P][KC]) {
    const T nd2 = T(2) * nd;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const T ym = p > 0 ? Y[p - 1] : YL;
        const T yp = p < P - 1 ? Y[p + 1] : YR;
        const T Dy = (yp - ym) * i2;
        const T ca = -Dy - nd2;
        const T cp = fma(yp, i2, nd);
        const T cm = fma(-ym, i2, nd);
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            const T mm = p > 0 ? m[p - 1][c] : ml[c];
            const T mp = p < P - 1 ? m[p + 1][c] : mr[c];
            out[p][c] = fma(cm, mm, fma(cp, mp, ca * m[p][c]));
        }
    }
}

template <typename T, int P, int KC, typename X>
__device__ __forceinline__ void adj3_body(const SweepArgs<T>& a, int tile_id, int grp, int t, X& xch) {
    const int n = a.n;
    const int tstart = tile_id * a.tile;
    const int tlen = min(a.tile, n - tstart);
    const T h = a.h, i2 = a.inv2dx, nd = a.nu_dx2;
    int g[P];
    bool in[P], own[P];
    T lam[P][KC];
    const T* xin = a.xin + static_cast<size_t>(grp) * n * KC;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = t * P + p;
        g[p] = tstart - a.halo + r;
        in[p] = g[p] >= 0 && g[p] < n;
        own[p] = in[p] && r >= a.halo && r < a.halo + tlen;
#pragma unroll
        for (int c = 0; c < KC; ++c) lam[p][c] = in[p] ? xin[static_cast<size_t>(g[p]) * KC + c] : T(0);
    }
    auto base_at = [&](int s, int p) -> T {
        return in[p] ? static_cast<T>(a.base[static_cast<size_t>(s - a.base_row0) * n + g[p]]) : T(0);
    };
    const int s_hi = a.s0 + a.S - 1;
    T unext[P];
#pragma unroll
    for (int p = 0; p < P; ++p) unext[p] = base_at(s_hi, p);
    for (int s = s_hi; s >= a.s0; --s) {
        // observation forcing at state index s+1, before transposing step s -> s+1
        const int s1 = s + 1;
        if ((s1 % a.obs_every) == 0) {
            const int i = s1 / a.obs_every;
            if (i >= 1 && i <= a.n_t) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (wall_obs(g[p], n, a.obs_stride)) {
                        const size_t row = static_cast<size_t>(i - 1) * a.n_obs + (g[p] + 1) / a.obs_stride - 1;
#pragma unroll
                        for (int c = 0; c < KC; ++c) {
                            const int col = grp * KC + c;
                            if (col < a.k) lam[p][c] = fma(a.w[row * a.k + col], a.inv_sigma_o, lam[p][c]);
                        }
                    }
                }
            }
        }
        T u[P];
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = unext[p];
        if (s - 1 >= a.s0) {
#pragma unroll
            for (int p = 0; p < P; ++p) unext[p] = base_at(s - 1, p);
        }
        // stage inputs Y1 = u, Y2 = w1, Y3 = w2 of step s and their edge neighbours
        T Ys[3][P], YL[3], YR[3];
#pragma unroll
        for (int p = 0; p < P; ++p) Ys[0][p] = u[p];
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const T e0[1] = {Ys[st][0]}, e1[1] = {Ys[st][P - 1]};
            T fl[1], fr[1];
            xch(e0, e1, fl, fr);
            YL[st] = fl[0];
            YR[st] = fr[0];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const T ym = p > 0 ? Ys[st][p - 1] : YL[st];
                const T yp = p < P - 1 ? Ys[st][p + 1] : YR[st];
                const T e = fma(h, rhs_pt<T>(Ys[st][p], ym, yp, i2, nd), Ys[st][p]);
                Ys[st + 1][p] = in[p] ? ssp_combine<T>(st, e, u[p]) : T(0);
            }
        }
        // mu2 = 2/3 (lam + h J(Y3)^T lam); Y3's edges travel with lam's
        T ml[KC], mr[KC], th[P][KC], mu2[P][KC], mu1[P][KC];
        {
            T e0[1 + KC], e1[1 + KC], fl[1 + KC], fr[1 + KC];
            e0[0] = Ys[2][0];
            e1[0] = Ys[2][P - 1];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                e0[1 + c] = lam[0][c];
                e1[1 + c] = lam[P - 1][c];
            }
            xch(e0, e1, fl, fr);
            YL[2] = fl[0];
            YR[2] = fr[0];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                ml[c] = fl[1 + c];
                mr[c] = fr[1 + c];
            }
        }
        jac_t_pts<T, P, KC>(Ys[2], YL[2], YR[2], lam, ml, mr, i2, nd, th);
        const T c23 = static_cast<T>(2.0 / 3.0);
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int c = 0; c < KC; ++c) mu2[p][c] = in[p] ? c23 * fma(h, th[p][c], lam[p][c]) : T(0);
        // mu1 = 1/4 (mu2 + h J(Y2)^T mu2)
        {
            T e0[KC], e1[KC];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                e0[c] = mu2[0][c];
                e1[c] = mu2[P - 1][c];
            }
            xch(e0, e1, ml, mr);
        }
        jac_t_pts<T, P, KC>(Ys[1], YL[1], YR[1], mu2, ml, mr, i2, nd, th);
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int c = 0; c < KC; ++c) mu1[p][c] = in[p] ? T(0.25) * fma(h, th[p][c], mu2[p][c]) : T(0);
        // lam <- lam/3 + 3/4 mu2 + mu1 + h J(Y1)^T mu1
        {
            T e0[KC], e1[KC];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                e0[c] = mu1[0][c];
                e1[c] = mu1[P - 1][c];
            }
            xch(e0, e1, ml, mr);
        }
        jac_t_pts<T, P, KC>(Ys[0], YL[0], YR[0], mu1, ml, mr, i2, nd, th);
        const T c13 = static_cast<T>(1.0 / 3.0);
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const T v = fma(h, th[p][c], mu1[p][c]) + fma(T(0.75), mu2[p][c], c13 * lam[p][c]);
                lam[p][c] = in[p] ? v : T(0);
            }
    }
    T* xout = a.xout + static_cast<size_t>(grp) * n * KC;
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (own[p]) {
#pragma unroll
            for (int c = 0; c < KC; ++c) xout[static_cast<size_t>(g[p]) * KC + c] = lam[p][c];
        }
}

template <int P>
__global__ void __launch_bounds__(256) burgers_fwd3_wave_kernel(FwdArgs a, int ntiles) {
    const int tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= ntiles) return;  // the whole wave leaves
    WaveExchange x;
    fwd3_body<P>(a, tile, threadIdx.x & 63, x);
}

template <typename T, int P, int KC>
__global__ void __launch_bounds__(256) burgers_tlm3_wave_kernel(SweepArgs<T> a, int ngroups, int nitems) {
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= nitems) return;
    WaveExchange x;
    tlm3_body<T, P, KC>(a, item / ngroups, item % ngroups, threadIdx.x & 63, x);
}

template <typename T, int P, int KC>
__global__ void __launch_bounds__(256) burgers_adj3_wave_kernel(SweepArgs<T> a, int ngroups, int nitems) {
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= nitems) return;
    WaveExchange x;
    adj3_body<T, P, KC>(a, item / ngroups, item % ngroups, threadIdx.x & 63, x);
}

void check_wall_tiling(const Tiling& t, int n, int halo, int S) {
    RP4D_REQUIRE(t.threads == 64 || t.threads == 128 || t.threads == 256, RP4D_EINVAL,
                 "wall sweep tiling: wave regions take 64, 128 or 256 threads per workgroup");
    RP4D_REQUIRE(t.tile >= 1 && t.tile <= n, RP4D_EINVAL, "wall sweep tiling: tile out of range");
    RP4D_REQUIRE(S >= 1 && halo >= 4 * S + 4, RP4D_EINVAL, "wall sweep tiling: halo too small for steps per launch");
    RP4D_REQUIRE(64L * t.ppt >= static_cast<long>(t.tile) + 2L * halo, RP4D_EINVAL,
                 "wall sweep tiling: wave region (64 ppt) smaller than tile + 2 * halo");
}

template <typename T, int P, int KC>
void launch_wall_one(int mode, const SweepArgs<T>& a, int ngroups, int nitems, int threads, hipStream_t st) {
    const int wpg = threads / 64;
    dim3 grid((nitems + wpg - 1) / wpg), block(threads);
    if (mode == MODE_TLM)
        burgers_tlm3_wave_kernel<T, P, KC><<<grid, block, 0, st>>>(a, ngroups, nitems);
    else
        burgers_adj3_wave_kernel<T, P, KC><<<grid, block, 0, st>>>(a, ngroups, nitems);
}

}  // namespace

void launch_wall_fwd(const FwdArgs& a, const Tiling& t, hipStream_t st) {
    check_wall_tiling(t, a.n, a.halo, a.S);
    const int ntiles = (a.n + t.tile - 1) / t.tile;
    const int wpg = t.threads / 64;
    dim3 grid((ntiles + wpg - 1) / wpg), block(t.threads);
    switch (t.ppt) {
        case 1: burgers_fwd3_wave_kernel<1><<<grid, block, 0, st>>>(a, ntiles); break;
        case 2: burgers_fwd3_wave_kernel<2><<<grid, block, 0, st>>>(a, ntiles); break;
        case 4: burgers_fwd3_wave_kernel<4><<<grid, block, 0, st>>>(a, ntiles); break;
        case 8: burgers_fwd3_wave_kernel<8><<<grid, block, 0, st>>>(a, ntiles); break;
        default: fail(RP4D_EINVAL, "wall sweep tiling: unsupported points per thread for fwd");
    }
    RP4D_HIP(hipGetLastError());
}

template <typename T>
void launch_wall_sweep(int mode, const SweepArgs<T>& a, const Tiling& t, int ngroups, hipStream_t st) {
    check_wall_tiling(t, a.n, a.halo, a.S);
    RP4D_REQUIRE(mode == MODE_TLM || mode == MODE_ADJ, RP4D_EINVAL, "wall sweep: bad mode");
    const int nitems = ((a.n + t.tile - 1) / t.tile) * ngroups;
    switch (t.ppt * 100 + t.kc) {
        case 101: launch_wall_one<T, 1, 1>(mode, a, ngroups, nitems, t.threads, st); break;
        case 102: launch_wall_one<T, 1, 2>(mode, a, ngroups, nitems, t.threads, st); break;
        case 201: launch_wall_one<T, 2, 1>(mode, a, ngroups, nitems, t.threads, st); break;
        case 202: launch_wall_one<T, 2, 2>(mode, a, ngroups, nitems, t.threads, st); break;
        case 401: launch_wall_one<T, 4, 1>(mode, a, ngroups, nitems, t.threads, st); break;
        case 402: launch_wall_one<T, 4, 2>(mode, a, ngroups, nitems, t.threads, st); break;
        default: fail(RP4D_EINVAL, "wall sweep tiling: unsupported (points per thread, vectors per group)");
    }
    RP4D_HIP(hipGetLastError());
}

template void launch_wall_sweep<double>(int, const SweepArgs<double>&, const Tiling&, int, hipStream_t);
template void launch_wall_sweep<float>(int, const SweepArgs<float>&, const Tiling&, int, hipStream_t);

}  // namespace rp4d
