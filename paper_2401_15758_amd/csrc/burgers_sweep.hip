// Burgers RK4 sweeps for gfx950: nonlinear forward (FWD), block tangent-linear
// (TLM) and block discrete adjoint (ADJ), Sec. 2.1 eq. (model) and the discrete
// Runge-Kutta TLM/ADJ used in Sec. 5.1.
//
// Decomposition.  A launch advances S steps.  Workgroup (tile, group) owns the
// grid points [tile*T, tile*T + T) of the vectors in `group` (KC vectors,
// interleaved per grid point) and computes an extended region of
// T + 2*halo points (periodic wrap), halo >= 4 S + 4: every RK4 step consumes a
// stencil radius of one point per stage, so after S steps the owned points are
// exact (overlapped temporal blocking).  Between launches the block state lives
// in HBM in the blocked layout [group][point][KC]; inside a launch it lives in
// registers: thread t holds P consecutive points of the region for the KC vectors
// and exchanges only its two edge points with its neighbours, once per RK stage.
// The base trajectory u_s is read once per step per point (shared by the KC
// vectors) and the nonlinear stage states Y_1..Y_4 are recomputed from it on the
// fly.
//
// Two region shapes share the same per-point arithmetic (the bodies below are
// templated on the exchange):
//  * workgroup regions: the whole workgroup covers one region and the edge
//    values travel through LDS (double-buffered, one barrier per exchange);
//  * wave regions: every 64-lane wave is an independent region of 64 P points
//    and the edge values move between neighbouring lanes with DPP wave shifts,
//    so a stage needs neither LDS nor a barrier.  The waves of a workgroup are
//    different vector groups of the same tile, so their base-trajectory loads
//    hit the same cache lines.
#include "internal.hpp"
#include "sweep_common.hpp"

// Every multiply-add of the sweeps is written as an explicit fma() and automatic
// contraction is off, so the rounding of each grid point's update is fixed by
// the source alone: results are bitwise independent of the tiling (points per
// thread, vectors per group, tile length, steps per launch) and of checkpointing.
#pragma clang fp contract(off)

namespace rp4d {
namespace {

// RK4 stage offsets for Y2, Y3, Y4 and weights.
__device__ __forceinline__ double rk_c(int st) { return st < 2 ? 0.5 : 1.0; }
__device__ __forceinline__ double rk_b(int st) { return (st == 0 || st == 3) ? (1.0 / 6.0) : (1.0 / 3.0); }

// Thread t of a region holds region points t*P .. t*P+P-1.
template <int P, typename X>
__device__ __forceinline__ void fwd_body(const FwdArgs& a, int tile_id, int t, X& xch) {
    const int n = a.n;
    const int tstart = tile_id * a.tile;
    const int tlen = min(a.tile, n - tstart);
    const double h = a.h, i2 = a.inv2dx, nd = a.nu_dx2;

    int g[P];
    bool own[P];
    double u[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = t * P + p;
        g[p] = wrap_index(static_cast<long>(tstart) - a.halo + r, n);
        own[p] = (r >= a.halo) && (r < a.halo + tlen);
        u[p] = a.xin[g[p]];
    }
    for (int s = a.s0; s < a.s0 + a.S; ++s) {
        double Y[P], acc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            Y[p] = u[p];
            acc[p] = 0.0;
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const double e0[1] = {Y[0]}, e1[1] = {Y[P - 1]};
            double fl[1], fr[1];
            xch(e0, e1, fl, fr);
            const double Yl = fl[0], Yr = fr[0];
            double Yn[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const double ym = p > 0 ? Y[p - 1] : Yl;
                const double yp = p < P - 1 ? Y[p + 1] : Yr;
                const double K = rhs_pt<double>(Y[p], ym, yp, i2, nd);
                acc[p] = fma(rk_b(st), K, acc[p]);
                if (st < 3) Yn[p] = fma(rk_c(st) * h, K, u[p]);
            }
            if (st < 3) {
#pragma unroll
                for (int p = 0; p < P; ++p) Y[p] = Yn[p];
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = fma(h, acc[p], u[p]);
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
                    if (own[p] && (g[p] % a.obs_stride) == 0) {
                        const size_t idx = static_cast<size_t>(i - 1) * a.n_obs + g[p] / a.obs_stride;
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

template <int P>
__global__ void __launch_bounds__(1024) burgers_fwd_kernel(FwdArgs a) {
    extern __shared__ double sh_fwd[];
    LdsExchange<double, 1> x(sh_fwd, blockDim.x, threadIdx.x);
    fwd_body<P>(a, blockIdx.x, threadIdx.x, x);
}

// Wave regions: wave w of workgroup b is tile b * (blockDim.x / 64) + w.
template <int P>
__global__ void __launch_bounds__(256) burgers_fwd_wave_kernel(FwdArgs a, int ntiles) {
    const int tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= ntiles) return;  // the whole wave leaves
    WaveExchange x;
    fwd_body<P>(a, tile, threadIdx.x & 63, x);
}

// Batched: work item (problem, tile) from `items`, arguments per problem.
template <int P>
__global__ void __launch_bounds__(1024) burgers_fwd_batched_kernel(const FwdArgs* __restrict__ args,
                                                                   const int4* __restrict__ items) {
    extern __shared__ double sh_fwd[];
    const int4 it = items[blockIdx.x];
    const FwdArgs a = args[it.x];  // private copy: no aliasing with the kernel's stores
    LdsExchange<double, 1> x(sh_fwd, blockDim.x, threadIdx.x);
    fwd_body<P>(a, it.y, threadIdx.x, x);
}

// Instances holding P*KC >= 8 point-vectors per thread are limited to 512
// threads per workgroup so that they get 256 VGPRs instead of spilling.
template <int P, int KC>
constexpr int sweep_max_threads() { return P * KC >= 8 ? 512 : 1024; }

template <typename T, int P, int KC, typename X>
__device__ __forceinline__ void tlm_body(const SweepArgs<T>& a, int tile_id, int grp, int t, X& xch) {
    const int n = a.n;
    const int tstart = tile_id * a.tile;
    const int tlen = min(a.tile, n - tstart);
    const T h = a.h, i2 = a.inv2dx, nd = a.nu_dx2;
    const T nd2 = T(2) * nd;

    int g[P];
    bool own[P];
    T d[P][KC];
    const T* xin = a.xin + static_cast<size_t>(grp) * n * KC;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = t * P + p;
        g[p] = wrap_index(static_cast<long>(tstart) - a.halo + r, n);
        own[p] = (r >= a.halo) && (r < a.halo + tlen);
#pragma unroll
        for (int c = 0; c < KC; ++c) d[p][c] = xin[static_cast<size_t>(g[p]) * KC + c];
    }
    T unext[P];
#pragma unroll
    for (int p = 0; p < P; ++p) unext[p] = static_cast<T>(a.base[static_cast<size_t>(a.s0 - a.base_row0) * n + g[p]]);

    for (int s = a.s0; s < a.s0 + a.S; ++s) {
        T u[P];
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = unext[p];
        if (s + 1 < a.s0 + a.S) {
#pragma unroll
            for (int p = 0; p < P; ++p)
                unext[p] = static_cast<T>(a.base[static_cast<size_t>(s + 1 - a.base_row0) * n + g[p]]);
        }
        T Y[P], dY[P][KC], acc[P][KC];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            Y[p] = u[p];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                dY[p][c] = d[p][c];
                acc[p][c] = T(0);
            }
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            // base and perturbation edges travel together
            T e0[1 + KC], e1[1 + KC], fl[1 + KC], fr[1 + KC];
            e0[0] = Y[0];
            e1[0] = Y[P - 1];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                e0[1 + c] = dY[0][c];
                e1[1 + c] = dY[P - 1][c];
            }
            xch(e0, e1, fl, fr);
            const T Yl = fl[0], Yr = fr[0];
            T dl[KC], dr[KC];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                dl[c] = fl[1 + c];
                dr[c] = fr[1 + c];
            }
            const T cb = static_cast<T>(rk_b(st));
            const T ch = static_cast<T>(rk_c(st)) * h;
            T Yn[P], dYn[P][KC];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const T ym = p > 0 ? Y[p - 1] : Yl;
                const T yp = p < P - 1 ? Y[p + 1] : Yr;
                const T Dy = (yp - ym) * i2;
                const T Yh = Y[p] * i2;
                // J(Y) d = ca d + cp d+ + cm d-  (coefficients shared by the KC vectors)
                const T ca = -Dy - nd2;
                const T cp = nd - Yh;
                const T cm = nd + Yh;
                if (st < 3) {
                    const T K = rhs_pt<T>(Y[p], ym, yp, i2, nd);
                    Yn[p] = fma(ch, K, u[p]);
                }
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    const T dm = p > 0 ? dY[p - 1][c] : dl[c];
                    const T dp = p < P - 1 ? dY[p + 1][c] : dr[c];
                    const T dK = fma(cm, dm, fma(cp, dp, ca * dY[p][c]));
                    acc[p][c] = fma(cb, dK, acc[p][c]);
                    if (st < 3) dYn[p][c] = fma(ch, dK, d[p][c]);
                }
            }
            if (st < 3) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    Y[p] = Yn[p];
#pragma unroll
                    for (int c = 0; c < KC; ++c) dY[p][c] = dYn[p][c];
                }
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int c = 0; c < KC; ++c) d[p][c] = fma(h, acc[p][c], d[p][c]);
        const int s1 = s + 1;
        if ((s1 % a.obs_every) == 0) {
            const int i = s1 / a.obs_every;
            if (i >= 1 && i <= a.n_t) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (own[p] && (g[p] % a.obs_stride) == 0) {
                        const size_t row = static_cast<size_t>(i - 1) * a.n_obs + g[p] / a.obs_stride;
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

template <typename T, int P, int KC, typename X>
__device__ __forceinline__ void adj_body(const SweepArgs<T>& a, int tile_id, int grp, int t, X& xch) {
    const int n = a.n;
    const int tstart = tile_id * a.tile;
    const int tlen = min(a.tile, n - tstart);
    const T h = a.h, i2 = a.inv2dx, nd = a.nu_dx2;
    const T nd2 = T(2) * nd;

    int g[P];
    bool own[P];
    T lam[P][KC];
    const T* xin = a.xin + static_cast<size_t>(grp) * n * KC;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int r = t * P + p;
        g[p] = wrap_index(static_cast<long>(tstart) - a.halo + r, n);
        own[p] = (r >= a.halo) && (r < a.halo + tlen);
#pragma unroll
        for (int c = 0; c < KC; ++c) lam[p][c] = xin[static_cast<size_t>(g[p]) * KC + c];
    }
    const int s_hi = a.s0 + a.S - 1;
    T unext[P];
#pragma unroll
    for (int p = 0; p < P; ++p) unext[p] = static_cast<T>(a.base[static_cast<size_t>(s_hi - a.base_row0) * n + g[p]]);

    for (int s = s_hi; s >= a.s0; --s) {
        // observation forcing at state index s+1, before transposing step s -> s+1
        const int s1 = s + 1;
        if ((s1 % a.obs_every) == 0) {
            const int i = s1 / a.obs_every;
            if (i >= 1 && i <= a.n_t) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if ((g[p] % a.obs_stride) == 0) {
                        const size_t row = static_cast<size_t>(i - 1) * a.n_obs + g[p] / a.obs_stride;
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
            for (int p = 0; p < P; ++p)
                unext[p] = static_cast<T>(a.base[static_cast<size_t>(s - 1 - a.base_row0) * n + g[p]]);
        }
        // nonlinear stage states Y1..Y4 of step s (recomputed) and their edge neighbours
        T Ys[4][P], YL[4], YR[4];
#pragma unroll
        for (int p = 0; p < P; ++p) Ys[0][p] = u[p];
#pragma unroll
        for (int st = 0; st < 3; ++st) {
            {
                const T e0[1] = {Ys[st][0]}, e1[1] = {Ys[st][P - 1]};
                T fl[1], fr[1];
                xch(e0, e1, fl, fr);
                YL[st] = fl[0];
                YR[st] = fr[0];
            }
            const T ch = static_cast<T>(rk_c(st)) * h;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const T ym = p > 0 ? Ys[st][p - 1] : YL[st];
                const T yp = p < P - 1 ? Ys[st][p + 1] : YR[st];
                const T K = rhs_pt<T>(Ys[st][p], ym, yp, i2, nd);
                Ys[st + 1][p] = fma(ch, K, u[p]);
            }
        }
        // reverse stages: mu_i = adjoint of dK_i, theta_i = J(Y_i)^T mu_i
        T mu[P][KC], lu[P][KC];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                mu[p][c] = (h / T(6)) * lam[p][c];
                lu[p][c] = lam[p][c];
            }
#pragma unroll
        for (int st = 3; st >= 0; --st) {
            T ml[KC], mr[KC];
            if (st == 3) {
                // the last stage state's edges travel with the first adjoint stage
                T e0[1 + KC], e1[1 + KC], fl[1 + KC], fr[1 + KC];
                e0[0] = Ys[3][0];
                e1[0] = Ys[3][P - 1];
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    e0[1 + c] = mu[0][c];
                    e1[1 + c] = mu[P - 1][c];
                }
                xch(e0, e1, fl, fr);
                YL[3] = fl[0];
                YR[3] = fr[0];
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    ml[c] = fl[1 + c];
                    mr[c] = fr[1 + c];
                }
            } else {
                T e0[KC], e1[KC];
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    e0[c] = mu[0][c];
                    e1[c] = mu[P - 1][c];
                }
                xch(e0, e1, ml, mr);
            }
            // coefficients of the next mu: mu_{st} = a_lam * lam + a_th * theta
            const T a_lam = st == 1 ? h / T(6) : h / T(3);
            const T a_th = st == 3 ? h : h * T(0.5);
            T mun[P][KC];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const T ym = p > 0 ? Ys[st][p - 1] : YL[st];
                const T yp = p < P - 1 ? Ys[st][p + 1] : YR[st];
                const T Dy = (yp - ym) * i2;
                // J(Y)^T mu = ca mu + cp mu+ + cm mu-, with ca = -Dy - 2nu/dx^2,
                // cp = nu/dx^2 + Y+/(2dx), cm = nu/dx^2 - Y-/(2dx)
                const T ca = -Dy - nd2;
                const T cp = fma(yp, i2, nd);
                const T cm = fma(-ym, i2, nd);
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    const T mm = p > 0 ? mu[p - 1][c] : ml[c];
                    const T mp = p < P - 1 ? mu[p + 1][c] : mr[c];
                    const T th = fma(cm, mm, fma(cp, mp, ca * mu[p][c]));
                    lu[p][c] += th;
                    if (st > 0) mun[p][c] = fma(a_th, th, a_lam * lam[p][c]);
                }
            }
            if (st > 0) {
#pragma unroll
                for (int p = 0; p < P; ++p)
#pragma unroll
                    for (int c = 0; c < KC; ++c) mu[p][c] = mun[p][c];
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int c = 0; c < KC; ++c) lam[p][c] = lu[p][c];
    }
    T* xout = a.xout + static_cast<size_t>(grp) * n * KC;
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (own[p]) {
#pragma unroll
            for (int c = 0; c < KC; ++c) xout[static_cast<size_t>(g[p]) * KC + c] = lam[p][c];
        }
}

template <typename T, int P, int KC>
__global__ void __launch_bounds__((sweep_max_threads<P, KC>())) burgers_tlm_kernel(SweepArgs<T> a) {
    extern __shared__ __align__(16) unsigned char sh_raw[];
    LdsExchange<T, 1 + KC> x(reinterpret_cast<T*>(sh_raw), blockDim.x, threadIdx.x);
    tlm_body<T, P, KC>(a, blockIdx.x, blockIdx.y, threadIdx.x, x);
}

template <typename T, int P, int KC>
__global__ void __launch_bounds__((sweep_max_threads<P, KC>())) burgers_adj_kernel(SweepArgs<T> a) {
    extern __shared__ __align__(16) unsigned char sh_raw[];
    LdsExchange<T, 1 + KC> x(reinterpret_cast<T*>(sh_raw), blockDim.x, threadIdx.x);
    adj_body<T, P, KC>(a, blockIdx.x, blockIdx.y, threadIdx.x, x);
}

// Wave regions: wave item = blockIdx.x * (blockDim.x / 64) + wave index, with
// tile = item / ngroups and group = item % ngroups, so that the waves of one
// workgroup share a tile.
template <typename T, int P, int KC>
__global__ void __launch_bounds__(256) burgers_tlm_wave_kernel(SweepArgs<T> a, int ngroups, int nitems) {
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= nitems) return;  // the whole wave leaves
    WaveExchange x;
    tlm_body<T, P, KC>(a, item / ngroups, item % ngroups, threadIdx.x & 63, x);
}

template <typename T, int P, int KC>
__global__ void __launch_bounds__(256) burgers_adj_wave_kernel(SweepArgs<T> a, int ngroups, int nitems) {
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= nitems) return;
    WaveExchange x;
    adj_body<T, P, KC>(a, item / ngroups, item % ngroups, threadIdx.x & 63, x);
}

// Batched sweeps: one launch covers the current interval of every problem of a
// batch; work item (problem, tile, group) from `items`, arguments per problem.
template <typename T, int P, int KC>
__global__ void __launch_bounds__((sweep_max_threads<P, KC>()))
    burgers_tlm_batched_kernel(const SweepArgs<T>* __restrict__ args, const int4* __restrict__ items) {
    extern __shared__ __align__(16) unsigned char sh_raw[];
    const int4 it = items[blockIdx.x];
    const SweepArgs<T> a = args[it.x];
    LdsExchange<T, 1 + KC> x(reinterpret_cast<T*>(sh_raw), blockDim.x, threadIdx.x);
    tlm_body<T, P, KC>(a, it.y, it.z, threadIdx.x, x);
}

template <typename T, int P, int KC>
__global__ void __launch_bounds__((sweep_max_threads<P, KC>()))
    burgers_adj_batched_kernel(const SweepArgs<T>* __restrict__ args, const int4* __restrict__ items) {
    extern __shared__ __align__(16) unsigned char sh_raw[];
    const int4 it = items[blockIdx.x];
    const SweepArgs<T> a = args[it.x];
    LdsExchange<T, 1 + KC> x(reinterpret_cast<T*>(sh_raw), blockDim.x, threadIdx.x);
    adj_body<T, P, KC>(a, it.y, it.z, threadIdx.x, x);
}

// Batched wave regions: one work item (problem, tile, group) per 64-lane wave.
template <int P>
__global__ void __launch_bounds__(256) burgers_fwd_wave_batched_kernel(const FwdArgs* __restrict__ args,
                                                                       const int4* __restrict__ items, int nitems) {
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= nitems) return;  // the whole wave leaves
    const int4 it = items[item];
    const FwdArgs a = args[it.x];
    WaveExchange x;
    fwd_body<P>(a, it.y, threadIdx.x & 63, x);
}

template <typename T, int P, int KC>
__global__ void __launch_bounds__(256) burgers_tlm_wave_batched_kernel(const SweepArgs<T>* __restrict__ args,
                                                                       const int4* __restrict__ items, int nitems) {
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= nitems) return;
    const int4 it = items[item];
    const SweepArgs<T> a = args[it.x];
    WaveExchange x;
    tlm_body<T, P, KC>(a, it.y, it.z, threadIdx.x & 63, x);
}

template <typename T, int P, int KC>
__global__ void __launch_bounds__(256) burgers_adj_wave_batched_kernel(const SweepArgs<T>* __restrict__ args,
                                                                       const int4* __restrict__ items, int nitems) {
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= nitems) return;
    const int4 it = items[item];
    const SweepArgs<T> a = args[it.x];
    WaveExchange x;
    adj_body<T, P, KC>(a, it.y, it.z, threadIdx.x & 63, x);
}

void check_tiling(const Tiling& t, int n, int halo, int S) {
    RP4D_REQUIRE(t.xch == XCH_LDS || t.xch == XCH_WAVE, RP4D_EINVAL, "sweep tiling: unknown exchange");
    if (t.xch == XCH_WAVE)
        RP4D_REQUIRE(t.threads == 64 || t.threads == 128 || t.threads == 256, RP4D_EINVAL,
                     "sweep tiling: wave regions take 64, 128 or 256 threads per workgroup");
    RP4D_REQUIRE(t.threads >= 64 && t.threads <= 1024 && t.threads % 64 == 0, RP4D_EINVAL,
                 "sweep tiling: threads must be a multiple of 64 in [64, 1024]");
    RP4D_REQUIRE(t.tile >= 1 && t.tile <= n, RP4D_EINVAL, "sweep tiling: tile out of range");
    RP4D_REQUIRE(halo >= 4 * S + 4, RP4D_EINVAL, "sweep tiling: halo too small for steps per launch");
    const long region = static_cast<long>(t.xch == XCH_WAVE ? 64 : t.threads) * t.ppt;
    RP4D_REQUIRE(region >= static_cast<long>(t.tile) + 2L * halo, RP4D_EINVAL,
                 "sweep tiling: region (threads per region * ppt) smaller than tile + 2 * halo");
}

}  // namespace

void launch_burgers_fwd(const FwdArgs& a, const Tiling& t, hipStream_t st) {
    if (a.wall) {
        launch_wall_fwd(a, t, st);
        return;
    }
    check_tiling(t, a.n, a.halo, a.S);
    const int ntiles = (a.n + t.tile - 1) / t.tile;
    if (t.xch == XCH_WAVE) {
        const int wpg = t.threads / 64;
        dim3 grid((ntiles + wpg - 1) / wpg), block(t.threads);
        switch (t.ppt) {
            case 1: burgers_fwd_wave_kernel<1><<<grid, block, 0, st>>>(a, ntiles); break;
            case 2: burgers_fwd_wave_kernel<2><<<grid, block, 0, st>>>(a, ntiles); break;
            case 4: burgers_fwd_wave_kernel<4><<<grid, block, 0, st>>>(a, ntiles); break;
            case 8: burgers_fwd_wave_kernel<8><<<grid, block, 0, st>>>(a, ntiles); break;
            default: fail(RP4D_EINVAL, "sweep tiling: unsupported points per thread for fwd");
        }
        RP4D_HIP(hipGetLastError());
        return;
    }
    dim3 grid(ntiles), block(t.threads);
    const size_t shmem = 2 * 2 * static_cast<size_t>(t.threads) * sizeof(double);
    switch (t.ppt) {
        case 1: burgers_fwd_kernel<1><<<grid, block, shmem, st>>>(a); break;
        case 2: burgers_fwd_kernel<2><<<grid, block, shmem, st>>>(a); break;
        case 4: burgers_fwd_kernel<4><<<grid, block, shmem, st>>>(a); break;
        case 8: burgers_fwd_kernel<8><<<grid, block, shmem, st>>>(a); break;
        default: fail(RP4D_EINVAL, "sweep tiling: unsupported points per thread for fwd");
    }
    RP4D_HIP(hipGetLastError());
}

template <typename T, int P, int KC>
static void launch_one_wave(int mode, const SweepArgs<T>& a, int ngroups, int nitems, int threads, hipStream_t st) {
    const int wpg = threads / 64;
    dim3 grid((nitems + wpg - 1) / wpg), block(threads);
    if (mode == MODE_TLM)
        burgers_tlm_wave_kernel<T, P, KC><<<grid, block, 0, st>>>(a, ngroups, nitems);
    else
        burgers_adj_wave_kernel<T, P, KC><<<grid, block, 0, st>>>(a, ngroups, nitems);
}

template <typename T, int P, int KC>
static void launch_one(int mode, const SweepArgs<T>& a, dim3 grid, dim3 block, size_t shmem, hipStream_t st) {
    RP4D_REQUIRE((static_cast<int>(block.x) <= sweep_max_threads<P, KC>()), RP4D_EINVAL,
                 "sweep tiling: too many threads for this (points per thread, vectors per group)");
    if (mode == MODE_TLM) {
        if (shmem > 64 * 1024)
            RP4D_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&burgers_tlm_kernel<T, P, KC>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem)));
        burgers_tlm_kernel<T, P, KC><<<grid, block, shmem, st>>>(a);
    } else {
        if (shmem > 64 * 1024)
            RP4D_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&burgers_adj_kernel<T, P, KC>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem)));
        burgers_adj_kernel<T, P, KC><<<grid, block, shmem, st>>>(a);
    }
}

template <typename T>
void launch_burgers_sweep(int mode, const SweepArgs<T>& a, const Tiling& t, int ngroups, hipStream_t st) {
    if (a.wall) {
        launch_wall_sweep<T>(mode, a, t, ngroups, st);
        return;
    }
    check_tiling(t, a.n, a.halo, a.S);
    RP4D_REQUIRE(mode == MODE_TLM || mode == MODE_ADJ, RP4D_EINVAL, "sweep: bad mode");
    const int ntiles = (a.n + t.tile - 1) / t.tile;
    if (t.xch == XCH_WAVE) {
        const int nitems = ntiles * ngroups;
        switch (t.ppt * 100 + t.kc) {
            case 101: launch_one_wave<T, 1, 1>(mode, a, ngroups, nitems, t.threads, st); break;
            case 102: launch_one_wave<T, 1, 2>(mode, a, ngroups, nitems, t.threads, st); break;
            case 104: launch_one_wave<T, 1, 4>(mode, a, ngroups, nitems, t.threads, st); break;
            case 201: launch_one_wave<T, 2, 1>(mode, a, ngroups, nitems, t.threads, st); break;
            case 202: launch_one_wave<T, 2, 2>(mode, a, ngroups, nitems, t.threads, st); break;
            case 204: launch_one_wave<T, 2, 4>(mode, a, ngroups, nitems, t.threads, st); break;
            case 401: launch_one_wave<T, 4, 1>(mode, a, ngroups, nitems, t.threads, st); break;
            case 402: launch_one_wave<T, 4, 2>(mode, a, ngroups, nitems, t.threads, st); break;
            case 801: launch_one_wave<T, 8, 1>(mode, a, ngroups, nitems, t.threads, st); break;
            default: fail(RP4D_EINVAL, "sweep tiling: unsupported (points per thread, vectors per group) for wave regions");
        }
        RP4D_HIP(hipGetLastError());
        return;
    }
    dim3 grid(ntiles, ngroups), block(t.threads);
    const size_t shmem = 2 * 2 * static_cast<size_t>(t.threads) * (1 + t.kc) * sizeof(T);
    RP4D_REQUIRE(shmem <= 160 * 1024, RP4D_EINVAL, "sweep tiling: LDS exchange buffer too large");
    const int key = t.ppt * 100 + t.kc;
    switch (key) {
        case 101: launch_one<T, 1, 1>(mode, a, grid, block, shmem, st); break;
        case 102: launch_one<T, 1, 2>(mode, a, grid, block, shmem, st); break;
        case 104: launch_one<T, 1, 4>(mode, a, grid, block, shmem, st); break;
        case 201: launch_one<T, 2, 1>(mode, a, grid, block, shmem, st); break;
        case 202: launch_one<T, 2, 2>(mode, a, grid, block, shmem, st); break;
        case 204: launch_one<T, 2, 4>(mode, a, grid, block, shmem, st); break;
        case 401: launch_one<T, 4, 1>(mode, a, grid, block, shmem, st); break;
        case 402: launch_one<T, 4, 2>(mode, a, grid, block, shmem, st); break;
        case 404: launch_one<T, 4, 4>(mode, a, grid, block, shmem, st); break;
        case 108: launch_one<T, 1, 8>(mode, a, grid, block, shmem, st); break;
        case 208: launch_one<T, 2, 8>(mode, a, grid, block, shmem, st); break;
        default: fail(RP4D_EINVAL, "sweep tiling: unsupported (points per thread, vectors per group)");
    }
    RP4D_HIP(hipGetLastError());
}

void launch_burgers_fwd_batched(const FwdArgs* args, const int4* items, int nitems, const Tiling& t, hipStream_t st) {
    if (nitems <= 0) return;
    if (t.xch == XCH_WAVE) {
        RP4D_REQUIRE(t.threads == 64 || t.threads == 128 || t.threads == 256, RP4D_EINVAL,
                     "batched fwd: wave regions take 64, 128 or 256 threads per workgroup");
        const int wpg = t.threads / 64;
        const dim3 grid((nitems + wpg - 1) / wpg);
        switch (t.ppt) {
            case 1: burgers_fwd_wave_batched_kernel<1><<<grid, t.threads, 0, st>>>(args, items, nitems); break;
            case 2: burgers_fwd_wave_batched_kernel<2><<<grid, t.threads, 0, st>>>(args, items, nitems); break;
            case 4: burgers_fwd_wave_batched_kernel<4><<<grid, t.threads, 0, st>>>(args, items, nitems); break;
            case 8: burgers_fwd_wave_batched_kernel<8><<<grid, t.threads, 0, st>>>(args, items, nitems); break;
            default: fail(RP4D_EINVAL, "batched fwd: unsupported points per thread");
        }
        RP4D_HIP(hipGetLastError());
        return;
    }
    const size_t shmem = 2 * 2 * static_cast<size_t>(t.threads) * sizeof(double);
    switch (t.ppt) {
        case 1: burgers_fwd_batched_kernel<1><<<nitems, t.threads, shmem, st>>>(args, items); break;
        case 2: burgers_fwd_batched_kernel<2><<<nitems, t.threads, shmem, st>>>(args, items); break;
        case 4: burgers_fwd_batched_kernel<4><<<nitems, t.threads, shmem, st>>>(args, items); break;
        case 8: burgers_fwd_batched_kernel<8><<<nitems, t.threads, shmem, st>>>(args, items); break;
        default: fail(RP4D_EINVAL, "batched fwd: unsupported points per thread");
    }
    RP4D_HIP(hipGetLastError());
}

template <typename T, int P, int KC>
static void launch_one_wave_batched(int mode, const SweepArgs<T>* args, const int4* items, int nitems, int threads,
                                    hipStream_t st) {
    const int wpg = threads / 64;
    const dim3 grid((nitems + wpg - 1) / wpg);
    if (mode == MODE_TLM)
        burgers_tlm_wave_batched_kernel<T, P, KC><<<grid, threads, 0, st>>>(args, items, nitems);
    else
        burgers_adj_wave_batched_kernel<T, P, KC><<<grid, threads, 0, st>>>(args, items, nitems);
}

template <typename T, int P, int KC>
static void launch_one_batched(int mode, const SweepArgs<T>* args, const int4* items, int nitems, int threads,
                               size_t shmem, hipStream_t st) {
    RP4D_REQUIRE((threads <= sweep_max_threads<P, KC>()), RP4D_EINVAL,
                 "batched sweep: too many threads for this (points per thread, vectors per group)");
    if (mode == MODE_TLM) {
        if (shmem > 64 * 1024)
            RP4D_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&burgers_tlm_batched_kernel<T, P, KC>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem)));
        burgers_tlm_batched_kernel<T, P, KC><<<nitems, threads, shmem, st>>>(args, items);
    } else {
        if (shmem > 64 * 1024)
            RP4D_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&burgers_adj_batched_kernel<T, P, KC>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem)));
        burgers_adj_batched_kernel<T, P, KC><<<nitems, threads, shmem, st>>>(args, items);
    }
}

template <typename T>
void launch_burgers_sweep_batched(int mode, const SweepArgs<T>* args, const int4* items, int nitems, const Tiling& t,
                                  hipStream_t st) {
    if (nitems <= 0) return;
    RP4D_REQUIRE(mode == MODE_TLM || mode == MODE_ADJ, RP4D_EINVAL, "batched sweep: bad mode");
    if (t.xch == XCH_WAVE) {
        RP4D_REQUIRE(t.threads == 64 || t.threads == 128 || t.threads == 256, RP4D_EINVAL,
                     "batched sweep: wave regions take 64, 128 or 256 threads per workgroup");
        switch (t.ppt * 100 + t.kc) {
            case 101: launch_one_wave_batched<T, 1, 1>(mode, args, items, nitems, t.threads, st); break;
            case 102: launch_one_wave_batched<T, 1, 2>(mode, args, items, nitems, t.threads, st); break;
            case 104: launch_one_wave_batched<T, 1, 4>(mode, args, items, nitems, t.threads, st); break;
            case 201: launch_one_wave_batched<T, 2, 1>(mode, args, items, nitems, t.threads, st); break;
            case 202: launch_one_wave_batched<T, 2, 2>(mode, args, items, nitems, t.threads, st); break;
            case 204: launch_one_wave_batched<T, 2, 4>(mode, args, items, nitems, t.threads, st); break;
            case 401: launch_one_wave_batched<T, 4, 1>(mode, args, items, nitems, t.threads, st); break;
            case 402: launch_one_wave_batched<T, 4, 2>(mode, args, items, nitems, t.threads, st); break;
            default: fail(RP4D_EINVAL, "batched sweep: unsupported (points per thread, vectors per group) for wave regions");
        }
        RP4D_HIP(hipGetLastError());
        return;
    }
    RP4D_REQUIRE(t.xch == XCH_LDS, RP4D_EINVAL, "batched sweep: unknown exchange");
    const size_t shmem = 2 * 2 * static_cast<size_t>(t.threads) * (1 + t.kc) * sizeof(T);
    RP4D_REQUIRE(shmem <= 160 * 1024, RP4D_EINVAL, "batched sweep: LDS exchange buffer too large");
    switch (t.ppt * 100 + t.kc) {
        case 101: launch_one_batched<T, 1, 1>(mode, args, items, nitems, t.threads, shmem, st); break;
        case 102: launch_one_batched<T, 1, 2>(mode, args, items, nitems, t.threads, shmem, st); break;
        case 104: launch_one_batched<T, 1, 4>(mode, args, items, nitems, t.threads, shmem, st); break;
        case 108: launch_one_batched<T, 1, 8>(mode, args, items, nitems, t.threads, shmem, st); break;
        case 201: launch_one_batched<T, 2, 1>(mode, args, items, nitems, t.threads, shmem, st); break;
        case 202: launch_one_batched<T, 2, 2>(mode, args, items, nitems, t.threads, shmem, st); break;
        case 204: launch_one_batched<T, 2, 4>(mode, args, items, nitems, t.threads, shmem, st); break;
        case 401: launch_one_batched<T, 4, 1>(mode, args, items, nitems, t.threads, shmem, st); break;
        case 402: launch_one_batched<T, 4, 2>(mode, args, items, nitems, t.threads, shmem, st); break;
        default: fail(RP4D_EINVAL, "batched sweep: unsupported (points per thread, vectors per group)");
    }
    RP4D_HIP(hipGetLastError());
}

template void launch_burgers_sweep_batched<double>(int, const SweepArgs<double>*, const int4*, int, const Tiling&,
                                                   hipStream_t);
template void launch_burgers_sweep_batched<float>(int, const SweepArgs<float>*, const int4*, int, const Tiling&,
                                                  hipStream_t);
template void launch_burgers_sweep<double>(int, const SweepArgs<double>&, const Tiling&, int, hipStream_t);
template void launch_burgers_sweep<float>(int, const SweepArgs<float>&, const Tiling&, int, hipStream_t);

}  // namespace rp4d
