// C ABI of the rp4d library: handles, block sweeps (FWD/TLM/ADJ/Hessian),
// sketches (Nystrom Alg. 2, RandSVD Alg. 1), PCG, Gauss-Newton step.
// Every numerical step runs in the kernels of this library; the host code only
// sequences launches on the context stream and reads back control scalars.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace rp4d {

static thread_local std::string g_last_error;

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void DevBuf::ensure(size_t b) {
    if (b <= bytes && p != nullptr) return;
    release();
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        p = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        fail(RP4D_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

KernelTimer::KernelTimer(rp4d_ctx* ctx, int k, double fl) : c(ctx), kind(k), flops(fl) {
    if (!c->timing) return;
    if (c->event_pool.empty()) {
        hipEvent_t e;
        RP4D_HIP(hipEventCreate(&e));
        c->event_pool.push_back(e);
    }
    a = c->event_pool.back();
    c->event_pool.pop_back();
    RP4D_HIP(hipEventRecord(a, c->stream));
}

KernelTimer::~KernelTimer() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (c->event_pool.empty()) {
        if (hipEventCreate(&b) != hipSuccess) {
            c->event_pool.push_back(a);
            return;
        }
    } else {
        b = c->event_pool.back();
        c->event_pool.pop_back();
    }
    if (hipEventRecord(b, c->stream) != hipSuccess) {
        c->event_pool.push_back(a);
        c->event_pool.push_back(b);
        return;
    }
    c->pending.push_back(rp4d_ctx::Pending{kind, a, b, flops});
}

namespace {

// Resolve recorded event pairs into the per-class statistics (synchronises).
void resolve_timing(rp4d_ctx* c) {
    if (c->pending.empty()) return;
    RP4D_HIP(hipStreamSynchronize(c->stream));
    for (auto& pe : c->pending) {
        float ms = 0.f;
        RP4D_HIP(hipEventElapsedTime(&ms, pe.a, pe.b));
        c->launches[pe.kind] += 1;
        c->ms[pe.kind] += ms;
        c->flops[pe.kind] += pe.flops;
        c->event_pool.push_back(pe.a);
        c->event_pool.push_back(pe.b);
    }
    c->pending.clear();
}

// Algorithmic flops per owned grid point and step, counted from the sweep
// kernels' source (sub/mul/add = 1, fma = 2): per vector and shared base part.
//   TLM vector: 4 stages x (dK 5 + acc 2) + 3 x dY 2 + update 2 = 36
//   TLM base:   4 x (Dy 2, Y/2dx 1, 3 coefficients 3) + 3 x (RHS 6 + stage 2) = 48
//   ADJ vector: mu 1 + 4 x (theta 5 + sum 1) + 3 x next mu 3 = 34
//   ADJ base:   3 x (RHS 8 + stage 2) + 4 x (Dy 2 + 3 coefficients 5) = 58
constexpr double FL_TLM_VEC = 36.0, FL_TLM_BASE = 48.0;
constexpr double FL_ADJ_VEC = 34.0, FL_ADJ_BASE = 58.0;
constexpr double FL_FWD = 48.0;

template <typename F>
int guarded(F&& f) {
    try {
        f();
        g_last_error.clear();
        return RP4D_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return RP4D_EINVAL;
    } catch (...) {
        g_last_error = "unknown error";
        return RP4D_EINVAL;
    }
}

// ---------------------------------------------------------------------------
// small device helpers for PCG / GN control scalars
// ---------------------------------------------------------------------------
enum { SC_RZ = 0, SC_PQ, SC_RZN, SC_RR, SC_BB, SC_T0, SC_T1, SC_T2, SC_COUNT };

__global__ void pcg_update_xr(double* x, double* r, const double* p, const double* q, const double* sc, int n) {
    const double alpha = sc[SC_RZ] / sc[SC_PQ];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        x[i] = fma(alpha, p[i], x[i]);
        r[i] = fma(-alpha, q[i], r[i]);
    }
}

__global__ void pcg_update_p(double* p, const double* z, const double* sc, int n) {
    const double beta = sc[SC_RZN] / sc[SC_RZ];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = fma(beta, p[i], z[i]);
}

__global__ void scal_copy(double* sc, int dst, int src) { sc[dst] = sc[src]; }

__global__ void absmax_kernel(const double* x, int n, double* out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(x[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// lam = max(0, s2 - nu) (s2 descending), D = lam/(1+lam), cs = 1/sqrt(s2) (0 where s2 is negligible)
__global__ void sketch_finalize(const double* s2, const double* nu_ptr, double nu_host, int l, double* lam,
                                double* D, double* cs) {
    const int i = threadIdx.x;
    if (i >= l) return;
    const double nu = nu_ptr ? nu_ptr[0] : nu_host;
    const double smax = fmax(s2[0], 0.0);
    const double s = s2[i];
    const bool ok = s > 1e-300 && s > 1e-30 * smax;
    const double lv = ok ? fmax(0.0, s - nu) : 0.0;
    lam[i] = lv;
    D[i] = lv / (1.0 + lv);
    cs[i] = ok ? 1.0 / sqrt(s) : 0.0;
}

__global__ void scale_cols(double* A, int l, const double* cs) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < l * l) A[idx] *= cs[idx % l];
}

__global__ void transpose_small(const double* A, double* B, int l) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < l * l) B[(idx % l) * l + idx / l] = A[idx];
}

inline int nblk(long count, int t = 256) {
    long b = (count + t - 1) / t;
    return static_cast<int>(std::max(1L, std::min(b, 4096L)));
}

// ---------------------------------------------------------------------------
// problem helpers
// ---------------------------------------------------------------------------
void set_device(const rp4d_ctx* c) { RP4D_HIP(hipSetDevice(c->device)); }

hipStream_t stream_of(const rp4d_problem* p) { return p->ctx->stream; }

void sync(const rp4d_problem* p) { RP4D_HIP(hipStreamSynchronize(stream_of(p))); }

double read_scalar(const rp4d_problem* p, const double* dptr) {
    double v = 0.0;
    RP4D_HIP(hipMemcpyAsync(&v, dptr, sizeof(double), hipMemcpyDeviceToHost, stream_of(p)));
    sync(p);
    return v;
}

Tiling heuristic_tiling(int n, int k) {
    Tiling t;
    t.kc = 1;
    const int groups = (k + t.kc - 1) / t.kc;
    const int tmin = std::min(n, 128);
    int tiles = std::max(1, (512 + groups - 1) / groups);
    tiles = std::min(tiles, std::max(1, (n + tmin - 1) / tmin));
    int T = (n + tiles - 1) / tiles;
    T = std::min(T, 3200);
    int S = static_cast<int>(std::floor((0.3 * T - 8.0) / 8.0));
    S = std::max(1, std::min(S, 32));
    const int R = T + 2 * (4 * S + 4);
    t.ppt = R > 2048 ? 4 : (R > 512 ? 2 : 1);
    t.threads = ((R + t.ppt - 1) / t.ppt + 63) / 64 * 64;
    if (t.threads > 1024) {
        t.ppt = 4;
        t.threads = ((R + 3) / 4 + 63) / 64 * 64;
    }
    t.tile = T;
    t.steps = S;
    return t;
}

Tiling tiling_for(const rp4d_problem* p, int mode, int dtype, int k) {
    Tiling t = heuristic_tiling(p->n, k);
    for (auto key : {std::make_tuple(mode, dtype, k), std::make_tuple(0, dtype, k), std::make_tuple(mode, dtype, 0),
                     std::make_tuple(0, dtype, 0)}) {
        auto it = p->tiling.find(key);
        if (it != p->tiling.end()) {
            const Tiling& o = it->second;
            if (o.ppt > 0) t.ppt = o.ppt;
            if (o.kc > 0) t.kc = o.kc;
            if (o.threads > 0) t.threads = o.threads;
            if (o.tile > 0) t.tile = o.tile;
            if (o.steps > 0) t.steps = o.steps;
            break;
        }
    }
    return t;
}

Tiling fwd_tiling(const rp4d_problem* p) {
    Tiling t = heuristic_tiling(p->n, 1);
    // the single nonlinear state: fewer, larger tiles amortise launches better
    if (p->n >= 1024) {
        const int tiles = std::max(1, p->n / 512);
        t.tile = (p->n + tiles - 1) / tiles;
        t.steps = std::max(1, std::min(32, static_cast<int>((0.3 * t.tile - 8.0) / 8.0)));
        const int R = t.tile + 2 * (4 * t.steps + 4);
        t.ppt = R > 2048 ? 8 : (R > 512 ? 2 : 1);
        t.threads = ((R + t.ppt - 1) / t.ppt + 63) / 64 * 64;
    }
    if (t.ppt == 8 && t.threads > 1024) t.threads = 1024;
    return t;
}

void check_traj(const rp4d_problem* p, const rp4d_traj* tr) {
    RP4D_REQUIRE(tr != nullptr && tr->p == p, RP4D_EINVAL, "trajectory does not belong to this problem");
    RP4D_REQUIRE(tr->valid, RP4D_ESTATE, "trajectory not computed: call rp4d_fwd first");
}

// Run the nonlinear model over steps [s_from, s_to) starting from state x (n),
// storing u_s for s % store_every == 0 at store rows s/store_every - store_row0.
void run_fwd(rp4d_problem* p, const double* x, int s_from, int s_to, double* store, int store_every, int store_row0,
             int store_rows, double* innov, double* obs_out) {
    const int n = p->n;
    hipStream_t st = stream_of(p);
    Tiling t = fwd_tiling(p);
    p->ws_red.ensure(std::max<size_t>(p->ws_red.bytes, 2 * n * sizeof(double) + 64));
    double* bufA = p->ws_red.as<double>();
    double* bufB = bufA + n;
    launch_relayout<double, double>(x, 1, bufA, 1, n, 1, st);
    double* in = bufA;
    double* out = bufB;
    FwdArgs a{};
    a.store = store;
    a.store_every = store_every;
    a.store_row0 = store_row0;
    a.store_rows = store_rows;
    a.n = n;
    a.h = p->d.dt;
    a.inv2dx = p->inv2dx;
    a.nu_dx2 = p->nu_dx2;
    a.tile = t.tile;
    a.halo = 4 * t.steps + 4;
    a.obs_stride = p->d.obs_stride;
    a.obs_every = p->d.obs_every;
    a.n_obs = p->n_obs;
    a.n_t = p->n_t;
    a.inv_sigma_o = 1.0 / p->d.sigma_o;
    a.y = p->has_data ? p->y.as<double>() : nullptr;
    a.innov = p->has_data ? innov : nullptr;
    a.obs_out = obs_out;
    for (int s0 = s_from; s0 < s_to; s0 += t.steps) {
        a.s0 = s0;
        a.S = std::min(t.steps, s_to - s0);
        a.xin = in;
        a.xout = out;
        {
            KernelTimer kt(p->ctx, RP4D_K_FWD, FL_FWD * a.S * static_cast<double>(n));
            launch_burgers_fwd(a, t, st);
        }
        std::swap(in, out);
    }
}

// TLM of k vectors: x0 blocked (kc) in buf0, z out (n_t, n_obs, k).
template <typename T>
void run_tlm(rp4d_problem* p, const rp4d_traj* tr, int k, const Tiling& t, T* buf0, T* buf1, T* z) {
    const int n = p->n;
    hipStream_t st = stream_of(p);
    const int groups = (k + t.kc - 1) / t.kc;
    SweepArgs<T> a{};
    a.n = n;
    a.h = static_cast<T>(p->d.dt);
    a.inv2dx = static_cast<T>(p->inv2dx);
    a.nu_dx2 = static_cast<T>(p->nu_dx2);
    a.tile = t.tile;
    a.halo = 4 * t.steps + 4;
    a.k = k;
    a.obs_stride = p->d.obs_stride;
    a.obs_every = p->d.obs_every;
    a.n_obs = p->n_obs;
    a.n_t = p->n_t;
    a.inv_sigma_o = static_cast<T>(1.0 / p->d.sigma_o);
    a.z = z;
    T* in = buf0;
    T* out = buf1;
    const int C = tr->C;
    const int seglen = C == 1 ? std::max(1, p->s_last) : C;  // full storage: one segment
    for (int seg0 = 0; seg0 < p->s_last; seg0 += seglen) {
        const int seg1 = std::min(p->s_last, seg0 + seglen);
        if (C == 1) {
            a.base = tr->states.as<double>();
            a.base_row0 = 0;
        } else {
            // recompute u_{seg0 .. seg1-1} from the checkpoint at seg0
            const int rows = seg1 - seg0 + 1;
            p->ws_seg.ensure(static_cast<size_t>(C + 1) * n * sizeof(double));
            double* seg = p->ws_seg.as<double>();
            const double* ck = tr->states.as<double>() + static_cast<size_t>(seg0 / C) * n;
            launch_relayout<double, double>(ck, 1, seg, 1, n, 1, st);
            if (seg1 - seg0 > 1) run_fwd(p, ck, seg0, seg1 - 1, seg, 1, seg0, rows, nullptr, nullptr);
            a.base = seg;
            a.base_row0 = seg0;
        }
        for (int s0 = seg0; s0 < seg1; s0 += t.steps) {
            a.s0 = s0;
            a.S = std::min(t.steps, seg1 - s0);
            a.xin = in;
            a.xout = out;
            {
                KernelTimer kt(p->ctx, RP4D_K_TLM,
                               static_cast<double>(a.S) * n * (FL_TLM_VEC * k + FL_TLM_BASE));
                launch_burgers_sweep<T>(MODE_TLM, a, t, groups, st);
            }
            std::swap(in, out);
        }
    }
}

// ADJ of k vectors with forcing w (n_t, n_obs, k); result lambda_0 (blocked kc) returned pointer.
template <typename T>
T* run_adj(rp4d_problem* p, const rp4d_traj* tr, int k, const Tiling& t, T* buf0, T* buf1, const T* w) {
    const int n = p->n;
    hipStream_t st = stream_of(p);
    const int groups = (k + t.kc - 1) / t.kc;
    launch_fill<T>(buf0, static_cast<size_t>(groups) * t.kc * n, T(0), st);
    SweepArgs<T> a{};
    a.n = n;
    a.h = static_cast<T>(p->d.dt);
    a.inv2dx = static_cast<T>(p->inv2dx);
    a.nu_dx2 = static_cast<T>(p->nu_dx2);
    a.tile = t.tile;
    a.halo = 4 * t.steps + 4;
    a.k = k;
    a.obs_stride = p->d.obs_stride;
    a.obs_every = p->d.obs_every;
    a.n_obs = p->n_obs;
    a.n_t = p->n_t;
    a.inv_sigma_o = static_cast<T>(1.0 / p->d.sigma_o);
    a.w = w;
    T* in = buf0;
    T* out = buf1;
    const int C = tr->C;
    const int seglen = C == 1 ? std::max(1, p->s_last) : C;  // full storage: one segment
    const int nseg = (p->s_last + seglen - 1) / seglen;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int seg0 = sg * seglen;
        const int seg1 = std::min(p->s_last, seg0 + seglen);
        if (C == 1) {
            a.base = tr->states.as<double>();
            a.base_row0 = 0;
        } else {
            const int rows = seg1 - seg0 + 1;
            p->ws_seg.ensure(static_cast<size_t>(C + 1) * n * sizeof(double));
            double* seg = p->ws_seg.as<double>();
            const double* ck = tr->states.as<double>() + static_cast<size_t>(seg0 / C) * n;
            launch_relayout<double, double>(ck, 1, seg, 1, n, 1, st);
            if (seg1 - seg0 > 1) run_fwd(p, ck, seg0, seg1 - 1, seg, 1, seg0, rows, nullptr, nullptr);
            a.base = seg;
            a.base_row0 = seg0;
        }
        // intervals from the top of the segment down
        int s_hi = seg1;
        while (s_hi > seg0) {
            const int Sc = std::min(t.steps, s_hi - seg0);
            a.s0 = s_hi - Sc;
            a.S = Sc;
            a.xin = in;
            a.xout = out;
            {
                KernelTimer kt(p->ctx, RP4D_K_ADJ,
                               static_cast<double>(a.S) * n * (FL_ADJ_VEC * k + FL_ADJ_BASE));
                launch_burgers_sweep<T>(MODE_ADJ, a, t, groups, st);
            }
            std::swap(in, out);
            s_hi -= Sc;
        }
    }
    return in;
}

// Gamma^{1/2} on k vectors.  Spectral form when few Fourier modes survive:
// T = F^T in (r x k), out = F diag(lam) T (+ addv); otherwise the banded
// periodic convolution with the square-root kernel.
template <typename T>
void bhalf_into(rp4d_problem* p, int k, const T* in, int in_kc, T* out, int out_kc, const T* addv) {
    hipStream_t st = stream_of(p);
    if (p->spec) {
        const int r = p->r, n = p->n;
        const size_t need = static_cast<size_t>(r) * k + gram_work_doubles(n, r, k);
        p->ws_bh.ensure(need * sizeof(double));
        double* Tm = p->ws_bh.as<double>();
        double* gw = Tm + static_cast<size_t>(r) * k;
        KernelTimer kt(p->ctx, RP4D_K_BHALF, 4.0 * n * static_cast<double>(r) * k);
        launch_gram<double, T>(p->F.as<double>(), r, in, in_kc, n, r, k, Tm, gw, st);
        launch_tsmm<double, T>(p->F.as<double>(), r, Tm, p->lamF.as<double>(), n, r, k, 1.0, addv, out_kc,
                               addv ? 1.0 : 0.0, out, out_kc, st);
        return;
    }
    const int band = std::min(2 * p->D + 1, p->n);
    KernelTimer kt(p->ctx, RP4D_K_BHALF, 2.0 * p->n * static_cast<double>(k) * band);
    launch_circ_conv<T>(in, in_kc, out, out_kc, p->gk.as<double>(), p->D, p->n, k, addv, st);
}

template <typename T>
struct SweepWork {
    T* s0;
    T* s1;
    T* obs;
    Tiling tt, ta;  // TLM and ADJ tilings
};

template <typename T>
SweepWork<T> sweep_work(rp4d_problem* p, int k, int dtype) {
    SweepWork<T> w{};
    w.tt = tiling_for(p, MODE_TLM, dtype, k);
    w.ta = tiling_for(p, MODE_ADJ, dtype, k);
    const int kcmax = std::max(w.tt.kc, w.ta.kc);
    const int groups = (k + kcmax - 1) / kcmax + 1;  // covers the padding of either layout
    const size_t blk = static_cast<size_t>(groups) * kcmax * p->n * sizeof(T);
    p->ws_s0.ensure(blk);
    p->ws_s1.ensure(blk);
    p->ws_obs.ensure(static_cast<size_t>(p->m) * k * sizeof(T));
    w.s0 = p->ws_s0.as<T>();
    w.s1 = p->ws_s1.as<T>();
    w.obs = p->ws_obs.as<T>();
    return w;
}

template <typename T>
void tlm_impl(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* Z) {
    SweepWork<T> w = sweep_work<T>(p, k, sizeof(T) == 8 ? RP4D_F64 : RP4D_F32);
    const int groups = (k + w.tt.kc - 1) / w.tt.kc;
    if (groups * w.tt.kc != k) launch_fill<T>(w.s0, static_cast<size_t>(groups) * w.tt.kc * p->n, T(0), stream_of(p));
    bhalf_into<T>(p, k, V, k, w.s0, w.tt.kc, nullptr);
    run_tlm<T>(p, tr, k, w.tt, w.s0, w.s1, Z);
}

template <typename T>
void adj_impl(rp4d_problem* p, const rp4d_traj* tr, int k, const T* W, T* U, const T* addv) {
    SweepWork<T> w = sweep_work<T>(p, k, sizeof(T) == 8 ? RP4D_F64 : RP4D_F32);
    T* lam = run_adj<T>(p, tr, k, w.ta, w.s0, w.s1, W);
    bhalf_into<T>(p, k, lam, w.ta.kc, U, k, addv);
}

template <typename T>
void hessian_impl(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* HV, bool add_identity) {
    SweepWork<T> w = sweep_work<T>(p, k, sizeof(T) == 8 ? RP4D_F64 : RP4D_F32);
    const int groups = (k + w.tt.kc - 1) / w.tt.kc;
    if (groups * w.tt.kc != k) launch_fill<T>(w.s0, static_cast<size_t>(groups) * w.tt.kc * p->n, T(0), stream_of(p));
    bhalf_into<T>(p, k, V, k, w.s0, w.tt.kc, nullptr);
    run_tlm<T>(p, tr, k, w.tt, w.s0, w.s1, w.obs);
    T* lam = run_adj<T>(p, tr, k, w.ta, w.s0, w.s1, w.obs);
    bhalf_into<T>(p, k, lam, w.ta.kc, HV, k, add_identity ? V : nullptr);
    p->cnt.hv_columns += k;
}

void hessian_dispatch(rp4d_problem* p, const rp4d_traj* tr, int k, const void* V, void* HV, int dtype, bool add_id) {
    if (dtype == RP4D_F64)
        hessian_impl<double>(p, tr, k, static_cast<const double*>(V), static_cast<double*>(HV), add_id);
    else if (dtype == RP4D_F32)
        hessian_impl<float>(p, tr, k, static_cast<const float*>(V), static_cast<float*>(HV), add_id);
    else
        fail(RP4D_EINVAL, "dtype must be RP4D_F64 or RP4D_F32");
}

void check_common(const rp4d_problem* p, int k, const void* a, const void* b) {
    RP4D_REQUIRE(p != nullptr, RP4D_EINVAL, "null problem");
    RP4D_REQUIRE(k >= 1 && k <= 4096, RP4D_EINVAL, "k must be in [1, 4096]");
    RP4D_REQUIRE(a != nullptr && b != nullptr, RP4D_EINVAL, "null buffer");
}

}  // namespace
}  // namespace rp4d

rp4d_ctx::~rp4d_ctx() {
    for (auto& pe : pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (auto e : event_pool) (void)hipEventDestroy(e);
}

using namespace rp4d;

// ===========================================================================
// ABI
// ===========================================================================
extern "C" {

const char* rp4d_last_error(void) { return g_last_error.c_str(); }

const char* rp4d_version(void) { return "rp4d 0.1 (gfx950)"; }

int rp4d_ctx_create(int device, void* hip_stream, rp4d_ctx** out) {
    return guarded([&] {
        RP4D_REQUIRE(out != nullptr, RP4D_EINVAL, "null output handle");
        int ndev = 0;
        RP4D_HIP(hipGetDeviceCount(&ndev));
        RP4D_REQUIRE(device >= 0 && device < ndev, RP4D_EINVAL, "no such HIP device");
        auto* c = new rp4d_ctx();
        c->device = device;
        c->stream = static_cast<hipStream_t>(hip_stream);
        *out = c;
    });
}

int rp4d_ctx_destroy(rp4d_ctx* ctx) {
    return guarded([&] { delete ctx; });
}

int rp4d_ctx_set_stream(rp4d_ctx* ctx, void* hip_stream) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr, RP4D_EINVAL, "null context");
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    });
}

int rp4d_problem_create(rp4d_ctx* ctx, const rp4d_problem_desc* desc, rp4d_problem** out) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr && desc != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        set_device(ctx);
        const rp4d_problem_desc& d = *desc;
        RP4D_REQUIRE(d.model == RP4D_BURGERS1D, RP4D_EINVAL, "model not supported by this library build");
        RP4D_REQUIRE(d.nx >= 8 && d.nx <= (1 << 22), RP4D_EINVAL, "nx out of range");
        RP4D_REQUIRE(d.nsteps >= 1 && d.obs_every >= 1 && d.obs_stride >= 1 && d.obs_stride <= d.nx, RP4D_EINVAL,
                     "bad window / observation layout");
        RP4D_REQUIRE(d.nsteps / d.obs_every >= 1, RP4D_EINVAL, "window has no observation step");
        RP4D_REQUIRE(d.dt > 0 && d.nu >= 0 && d.sigma_o > 0 && d.sigma_b > 0 && d.L_b > 0, RP4D_EINVAL,
                     "bad physical parameters");
        const double dx = 1.0 / d.nx;
        RP4D_REQUIRE(4.0 * d.nu * d.dt / (dx * dx) <= 2.785, RP4D_EUNSTABLE,
                     "time step outside the RK4 diffusive stability interval (4 nu dt/dx^2 > 2.785)");
        RP4D_REQUIRE(10.0 * d.dt / dx <= 2.8, RP4D_EUNSTABLE,
                     "time step outside the RK4 advective stability interval for |u| <= 10");
        auto* p = new rp4d_problem();
        try {
            p->ctx = ctx;
            p->d = d;
            p->n = d.nx;
            p->n_obs = (d.nx + d.obs_stride - 1) / d.obs_stride;
            p->n_t = d.nsteps / d.obs_every;
            p->m = p->n_obs * p->n_t;
            p->s_last = p->n_t * d.obs_every;
            p->dx = dx;
            p->inv2dx = 1.0 / (2.0 * dx);
            p->nu_dx2 = d.nu / (dx * dx);
            if (p->d.ckpt_every < 1) p->d.ckpt_every = 1;
            // Gaussian square-root kernel g(d) = sigma_b a exp(-(d dx)^2 / L^2),
            // a^2 = dx / (L sqrt(pi/2)); truncated where g/g(0) < 2^-60.
            const double L = d.L_b;
            const double a = std::sqrt(dx / (L * std::sqrt(M_PI / 2.0)));
            const int Dt = static_cast<int>(std::ceil(std::sqrt(60.0 * std::log(2.0)) * L / dx));
            p->D = std::min(Dt, d.nx / 2);
            std::vector<double> g(p->D + 1);
            for (int i = 0; i <= p->D; ++i) {
                const double r = i * dx;
                g[i] = d.sigma_b * a * std::exp(-(r * r) / (L * L));
            }
            p->gk.ensure(g.size() * sizeof(double));
            RP4D_HIP(hipMemcpy(p->gk.p, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice));
            // Spectral form: the circulant's eigenvalues are the DFT of the kernel,
            // ~ exp(-pi^2 kappa^2 L^2) of the largest, below 2^-60 beyond
            // kappa_max = sqrt(60 ln 2)/(pi L); keep kappa <= kappa_max + 2 when that
            // is a small fraction of the grid.
            const int K = static_cast<int>(std::ceil(std::sqrt(60.0 * std::log(2.0)) / (M_PI * L))) + 2;
            if (2 * K + 1 <= d.nx / 4) {
                const int n = d.nx, r = 2 * K + 1;
                std::vector<double> Fh(static_cast<size_t>(n) * r), lh(r);
                std::vector<double> full(n);
                for (int i = 0; i < n; ++i) {
                    const int dd = std::min(i, n - i);
                    const double rr = dd * dx;
                    full[i] = d.sigma_b * a * std::exp(-(rr * rr) / (L * L));
                }
                auto cosn = [n](long q) { return std::cos(2.0 * M_PI * static_cast<double>(q % n) / n); };
                auto sinn = [n](long q) { return std::sin(2.0 * M_PI * static_cast<double>(q % n) / n); };
                const double c0 = 1.0 / std::sqrt(static_cast<double>(n)), c1 = std::sqrt(2.0 / n);
                for (int kap = 0; kap <= K; ++kap) {
                    double s = 0.0;
                    for (int i = 0; i < n; ++i) s += full[i] * cosn(static_cast<long>(kap) * i);
                    if (kap == 0) {
                        lh[0] = s;
                    } else {
                        lh[2 * kap - 1] = s;
                        lh[2 * kap] = s;
                    }
                }
                for (int j = 0; j < n; ++j) {
                    double* row = Fh.data() + static_cast<size_t>(j) * r;
                    row[0] = c0;
                    for (int kap = 1; kap <= K; ++kap) {
                        row[2 * kap - 1] = c1 * cosn(static_cast<long>(kap) * j);
                        row[2 * kap] = c1 * sinn(static_cast<long>(kap) * j);
                    }
                }
                p->spec = true;
                p->r = r;
                p->F.ensure(Fh.size() * sizeof(double));
                p->lamF.ensure(lh.size() * sizeof(double));
                RP4D_HIP(hipMemcpy(p->F.p, Fh.data(), Fh.size() * sizeof(double), hipMemcpyHostToDevice));
                RP4D_HIP(hipMemcpy(p->lamF.p, lh.data(), lh.size() * sizeof(double), hipMemcpyHostToDevice));
            }
            p->xb.ensure(p->n * sizeof(double));
            p->y.ensure(static_cast<size_t>(p->m) * sizeof(double));
            p->ws_scal.ensure(64 * sizeof(double));
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
    });
}

int rp4d_problem_destroy(rp4d_problem* p) {
    return guarded([&] {
        if (p) {
            set_device(p->ctx);
            (void)hipStreamSynchronize(p->ctx->stream);
        }
        delete p;
    });
}

int rp4d_problem_dims(const rp4d_problem* p, int* n, int* n_obs, int* n_t) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr, RP4D_EINVAL, "null problem");
        if (n) *n = p->n;
        if (n_obs) *n_obs = p->n_obs;
        if (n_t) *n_t = p->n_t;
    });
}

int rp4d_problem_set_data(rp4d_problem* p, const double* xb, const double* y) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && xb != nullptr && y != nullptr, RP4D_EINVAL, "null argument");
        set_device(p->ctx);
        launch_relayout<double, double>(xb, 1, p->xb.as<double>(), 1, p->n, 1, stream_of(p));
        launch_relayout<double, double>(y, 1, p->y.as<double>(), 1, p->m, 1, stream_of(p));
        p->has_data = true;
    });
}

int rp4d_traj_create(rp4d_problem* p, rp4d_traj** out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        set_device(p->ctx);
        auto* t = new rp4d_traj();
        try {
            t->p = p;
            t->C = p->d.ckpt_every;
            t->rows = p->s_last / t->C + 1;
            t->states.ensure(static_cast<size_t>(t->rows) * p->n * sizeof(double));
            t->innov.ensure(2 * static_cast<size_t>(p->m) * sizeof(double));
        } catch (...) {
            delete t;
            throw;
        }
        *out = t;
    });
}

int rp4d_traj_destroy(rp4d_traj* t) {
    return guarded([&] {
        if (t && t->p) {
            set_device(t->p->ctx);
            (void)hipStreamSynchronize(t->p->ctx->stream);
        }
        delete t;
    });
}

int rp4d_fwd(rp4d_problem* p, const double* x0, rp4d_traj* tr, double* J_obs) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && x0 != nullptr && tr != nullptr && tr->p == p, RP4D_EINVAL, "bad argument");
        set_device(p->ctx);
        hipStream_t st = stream_of(p);
        double* rows = tr->states.as<double>();
        launch_relayout<double, double>(x0, 1, rows, 1, p->n, 1, st);  // row 0 = x0
        double* innov = tr->innov.as<double>();
        double* obs = innov + p->m;
        run_fwd(p, x0, 0, p->s_last, rows, tr->C, 0, tr->rows, innov, obs);
        tr->valid = true;
        tr->has_innov = p->has_data;
        p->cnt.fwd += 1;
        if (J_obs != nullptr) {
            RP4D_REQUIRE(p->has_data, RP4D_ESTATE, "J requested but data not set");
            double* sc = p->ws_scal.as<double>();
            p->ws_red.ensure(std::max<size_t>(p->ws_red.bytes, (2 * p->n + 512) * sizeof(double)));
            launch_dot(innov, innov, p->m, sc + SC_T0, p->ws_red.as<double>() + 2 * p->n, st);
            const double s = read_scalar(p, sc + SC_T0);
            RP4D_REQUIRE(std::isfinite(s), RP4D_ENONFINITE, "non-finite innovations (state blew up or bad input)");
            *J_obs = 0.5 * s;
        }
    });
}

int rp4d_observe(rp4d_problem* p, const rp4d_traj* tr, double* y_out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && y_out != nullptr, RP4D_EINVAL, "null argument");
        check_traj(p, tr);
        set_device(p->ctx);
        launch_relayout<double, double>(tr->innov.as<double>() + p->m, 1, y_out, 1, p->m, 1, stream_of(p));
    });
}

int rp4d_bhalf(rp4d_problem* p, int k, const void* V, void* U, int dtype) {
    return guarded([&] {
        check_common(p, k, V, U);
        set_device(p->ctx);
        if (dtype == RP4D_F64)
            bhalf_into<double>(p, k, static_cast<const double*>(V), k, static_cast<double*>(U), k, nullptr);
        else if (dtype == RP4D_F32)
            bhalf_into<float>(p, k, static_cast<const float*>(V), k, static_cast<float*>(U), k, nullptr);
        else
            fail(RP4D_EINVAL, "bad dtype");
    });
}

int rp4d_tlm(rp4d_problem* p, const rp4d_traj* tr, int k, const void* V, void* Z, int dtype) {
    return guarded([&] {
        check_common(p, k, V, Z);
        check_traj(p, tr);
        set_device(p->ctx);
        if (dtype == RP4D_F64)
            tlm_impl<double>(p, tr, k, static_cast<const double*>(V), static_cast<double*>(Z));
        else if (dtype == RP4D_F32)
            tlm_impl<float>(p, tr, k, static_cast<const float*>(V), static_cast<float*>(Z));
        else
            fail(RP4D_EINVAL, "bad dtype");
    });
}

int rp4d_adj(rp4d_problem* p, const rp4d_traj* tr, int k, const void* W, void* U, int dtype) {
    return guarded([&] {
        check_common(p, k, W, U);
        check_traj(p, tr);
        set_device(p->ctx);
        if (dtype == RP4D_F64)
            adj_impl<double>(p, tr, k, static_cast<const double*>(W), static_cast<double*>(U), nullptr);
        else if (dtype == RP4D_F32)
            adj_impl<float>(p, tr, k, static_cast<const float*>(W), static_cast<float*>(U), nullptr);
        else
            fail(RP4D_EINVAL, "bad dtype");
    });
}

int rp4d_hessian_block(rp4d_problem* p, const rp4d_traj* tr, int k, const void* V, void* HV, int dtype,
                       int add_identity) {
    return guarded([&] {
        check_common(p, k, V, HV);
        RP4D_REQUIRE(V != HV, RP4D_EINVAL, "V and HV must not alias");
        check_traj(p, tr);
        set_device(p->ctx);
        hessian_dispatch(p, tr, k, V, HV, dtype, add_identity != 0);
    });
}

int rp4d_gradient(rp4d_problem* p, const rp4d_traj* tr, const double* v, double* g) {
    return guarded([&] {
        check_common(p, 1, v, g);
        check_traj(p, tr);
        RP4D_REQUIRE(tr->has_innov, RP4D_ESTATE, "trajectory has no innovations: set data before rp4d_fwd");
        set_device(p->ctx);
        adj_impl<double>(p, tr, 1, tr->innov.as<double>(), g, v);
        p->cnt.adj_online += 1;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// sketches
// ---------------------------------------------------------------------------
namespace rp4d {
namespace {

// All scratch of a sketch of size l on an n-point problem with m observations.
struct Scratch {
    double *Om, *Yd, *Y2, *S1, *S2, *S3, *S4, *ev, *lam, *D, *cs, *gw, *nu;
    void *Omt, *Yt, *Wt;
    int* info;
};

Scratch sketch_scratch(rp4d_problem* p, int l, int dtype) {
    const size_t n = p->n, m = p->m;
    const size_t es = dtype == RP4D_F64 ? 8 : 4;
    const size_t nl = n * l, ml = m * l, ll = static_cast<size_t>(l) * l;
    const size_t gw = std::max(gram_work_doubles(p->n, l, l), gram_work_doubles(p->m, l, l));
    const size_t dbl = 2 * nl + 2 * std::max(nl, ml) + 4 * ll + 4 * static_cast<size_t>(l) + gw + 8;
    const size_t typed = (nl + std::max(nl, ml) + nl) * es;
    p->ws_blk.ensure(dbl * 8 + typed + 64);
    Scratch s{};
    double* b = p->ws_blk.as<double>();
    s.Om = b;
    b += nl;
    s.Yd = b;
    b += std::max(nl, ml);
    s.Y2 = b;
    b += std::max(nl, ml);
    s.S1 = b;
    b += nl;  // also used as an n x l FP64 buffer
    s.S2 = b;
    b += ll;
    s.S3 = b;
    b += ll;
    s.S4 = b;
    b += ll;
    s.ev = b;
    b += ll;
    s.lam = b;
    b += l;
    s.D = b;
    b += l;
    s.cs = b;
    b += l;
    s.nu = b;
    b += l;
    s.gw = b;
    b += gw;
    unsigned char* tb = reinterpret_cast<unsigned char*>(b + 8);
    s.Omt = tb;
    tb += nl * es;
    s.Yt = tb;
    tb += std::max(nl, ml) * es;
    s.Wt = tb;
    s.info = reinterpret_cast<int*>(b);
    return s;
}

int read_info(rp4d_problem* p, const int* info) {
    int v = 0;
    RP4D_HIP(hipMemcpyAsync(&v, info, sizeof(int), hipMemcpyDeviceToHost, stream_of(p)));
    sync(p);
    return v;
}

void copy_host(rp4d_problem* p, void* dst, const void* src, size_t bytes) {
    RP4D_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream_of(p)));
    sync(p);
}

// Y0 = H Omega in `dtype`, returned as FP64 in s.Yd (n x l).
void sketch_misfit_hessian(rp4d_problem* p, const rp4d_traj* tr, int l, int dtype, Scratch& s) {
    hipStream_t st = stream_of(p);
    if (dtype == RP4D_F64) {
        hessian_dispatch(p, tr, l, s.Om, s.Yd, RP4D_F64, false);
    } else {
        launch_relayout<double, float>(s.Om, l, static_cast<float*>(s.Omt), l, p->n, l, st);
        hessian_dispatch(p, tr, l, s.Omt, s.Yt, RP4D_F32, false);
        launch_relayout<float, double>(static_cast<const float*>(s.Yt), l, s.Yd, l, p->n, l, st);
    }
}

void build_nystrom(rp4d_problem* p, const rp4d_traj* tr, int l, int dtype, Scratch& s, rp4d_precond* pc) {
    hipStream_t st = stream_of(p);
    const int n = p->n;
    sketch_misfit_hessian(p, tr, l, dtype, s);                       // step 2: Y = H Omega
    // step 3: nu = sqrt(n) eps ||Y||_2, ||Y||_2^2 = lambda_max(Y^T Y)
    launch_gram<double, double>(s.Yd, l, s.Yd, l, n, l, l, s.S2, s.gw, st);
    launch_jacobi_eig(s.S2, s.lam, nullptr, l, st);
    double ymax2 = 0.0;
    copy_host(p, &ymax2, s.lam, sizeof(double));
    const double eps = dtype == RP4D_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23);
    double nu = std::sqrt(static_cast<double>(n)) * eps * std::sqrt(std::max(ymax2, 0.0));
    RP4D_REQUIRE(std::isfinite(nu), RP4D_ENONFINITE, "non-finite sketch");
    bool ok = false;
    for (int attempt = 0; attempt <= 3; ++attempt) {
        // step 4: Y <- Y + nu Omega ; step 5: C = Omega^T Y, L = chol((C + C^T)/2)
        launch_relayout<double, double>(s.Yd, 1, s.Y2, 1, n * l, 1, st);
        launch_axpby(s.Om, nu, s.Y2, 1.0, static_cast<size_t>(n) * l, st);
        launch_gram<double, double>(s.Om, l, s.Y2, l, n, l, l, s.S2, s.gw, st);
        launch_chol(s.S2, l, s.info, st);
        if (read_info(p, s.info) == 0) {
            ok = true;
            break;
        }
        nu *= 10.0;
    }
    RP4D_REQUIRE(ok, RP4D_ENOTSPD, "Nystrom core matrix not positive definite after shift retries");
    // step 6-7: W = L^{-1} Y^T ; W W^T = L^{-1} (Y^T Y) L^{-T}; eig -> U, Sigma^2
    launch_trinv(s.S2, s.S3, l, st);                                  // S3 = L^{-1}
    launch_gram<double, double>(s.Y2, l, s.Y2, l, n, l, l, s.S4, s.gw, st);  // S4 = Y^T Y
    launch_small_gemm(s.S3, 0, s.S4, 0, s.S2, l, 1.0, st);            // S2 = L^{-1} Y^T Y
    launch_small_gemm(s.S2, 0, s.S3, 1, s.S4, l, 1.0, st);            // S4 = S2 L^{-T}
    launch_jacobi_eig(s.S4, s.ev, s.S2, l, st);                       // ev = Sigma^2, S2 = U
    sketch_finalize<<<1, 128, 0, st>>>(s.ev, nullptr, nu, l, s.lam, s.D, s.cs);
    RP4D_HIP(hipGetLastError());
    // V_hat = W^T U Sigma^{-1} = Y L^{-T} U Sigma^{-1}
    scale_cols<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S2, l, s.cs);
    launch_small_gemm(s.S3, 1, s.S2, 0, s.S4, l, 1.0, st);            // S4 = L^{-T} U Sigma^{-1}
    pc->V.ensure(static_cast<size_t>(n) * l * sizeof(double));
    launch_tsmm<double, double>(s.Y2, l, s.S4, nullptr, n, l, l, 1.0, nullptr, 0, 0.0, pc->V.as<double>(), l, st);
    pc->nu = nu;
}

// One Cholesky-QR pass on Y (rows x l, FP64, in s.Yd): G = Y^T Y + shift I = L L^T,
// Y <- Y L^{-T}.  Returns the Cholesky info (0 = success; Y untouched otherwise).
int cholqr_pass(rp4d_problem* p, int rows, int l, Scratch& s, double shift) {
    hipStream_t st = stream_of(p);
    launch_gram<double, double>(s.Yd, l, s.Yd, l, rows, l, l, s.S2, s.gw, st);
    if (shift > 0) {
        std::vector<double> eye(static_cast<size_t>(l) * l, 0.0);
        for (int i = 0; i < l; ++i) eye[static_cast<size_t>(i) * l + i] = shift;
        RP4D_HIP(hipMemcpyAsync(s.S4, eye.data(), eye.size() * sizeof(double), hipMemcpyHostToDevice, st));
        launch_axpby(s.S4, 1.0, s.S2, 1.0, static_cast<size_t>(l) * l, st);
        sync(p);  // the host staging vector must outlive the copy
    }
    launch_chol(s.S2, l, s.info, st);
    const int info = read_info(p, s.info);
    if (info != 0) return info;
    launch_trinv(s.S2, s.S3, l, st);
    transpose_small<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S3, s.S4, l);  // S4 = L^{-T}
    RP4D_HIP(hipGetLastError());
    launch_tsmm<double, double>(s.Yd, l, s.S4, nullptr, rows, l, l, 1.0, nullptr, 0, 0.0, s.Y2, l, st);
    launch_relayout<double, double>(s.Y2, 1, s.Yd, 1, rows * l, 1, st);
    return 0;
}

// Thin QR of Y (rows x l) by CholeskyQR2; if the Gram matrix is numerically
// indefinite, shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa, Yamamoto,
// Yanagisawa 2020): one pass with shift 11 (rows l + l(l+1)) u ||Y||_2^2, then two
// plain passes.  Q overwrites s.Yd.
void cholqr2(rp4d_problem* p, int rows, int l, Scratch& s) {
    hipStream_t st = stream_of(p);
    if (cholqr_pass(p, rows, l, s, 0.0) == 0) {
        RP4D_REQUIRE(cholqr_pass(p, rows, l, s, 0.0) == 0, RP4D_ENOTSPD, "RandSVD: Cholesky QR second pass failed");
        return;
    }
    launch_gram<double, double>(s.Yd, l, s.Yd, l, rows, l, l, s.S2, s.gw, st);
    launch_jacobi_eig(s.S2, s.lam, nullptr, l, st);
    double ymax2 = 0.0;
    copy_host(p, &ymax2, s.lam, sizeof(double));
    const double sh = 11.0 * (static_cast<double>(rows) * l + l * (l + 1.0)) * std::ldexp(1.0, -53) * ymax2;
    RP4D_REQUIRE(cholqr_pass(p, rows, l, s, std::max(sh, 1e-300)) == 0, RP4D_ENOTSPD,
                 "RandSVD: shifted Cholesky QR failed");
    RP4D_REQUIRE(cholqr_pass(p, rows, l, s, 0.0) == 0, RP4D_ENOTSPD, "RandSVD: Cholesky QR pass failed");
    RP4D_REQUIRE(cholqr_pass(p, rows, l, s, 0.0) == 0, RP4D_ENOTSPD, "RandSVD: Cholesky QR pass failed");
}

void build_randsvd(rp4d_problem* p, const rp4d_traj* tr, int l, int dtype, Scratch& s, rp4d_precond* pc) {
    hipStream_t st = stream_of(p);
    const int n = p->n, m = p->m;
    // step 2: Y = A Omega (m x l)
    if (dtype == RP4D_F64) {
        tlm_impl<double>(p, tr, l, s.Om, s.Yd);
    } else {
        launch_relayout<double, float>(s.Om, l, static_cast<float*>(s.Omt), l, n, l, st);
        tlm_impl<float>(p, tr, l, static_cast<const float*>(s.Omt), static_cast<float*>(s.Yt));
        launch_relayout<float, double>(static_cast<const float*>(s.Yt), l, s.Yd, l, m, l, st);
    }
    // step 3: thin QR (CholeskyQR2 in FP64)
    cholqr2(p, m, l, s);
    // step 4: W^T = A^T Q (n x l)
    if (dtype == RP4D_F64) {
        adj_impl<double>(p, tr, l, s.Yd, s.S1, nullptr);
    } else {
        launch_relayout<double, float>(s.Yd, l, static_cast<float*>(s.Yt), l, m, l, st);
        adj_impl<float>(p, tr, l, static_cast<const float*>(s.Yt), static_cast<float*>(s.Wt), nullptr);
        launch_relayout<float, double>(static_cast<const float*>(s.Wt), l, s.S1, l, n, l, st);
    }
    // step 5: thin SVD of W via eig(W W^T): V_hat = W^T U Sigma^{-1}, Lambda = Sigma^2
    launch_gram<double, double>(s.S1, l, s.S1, l, n, l, l, s.S2, s.gw, st);
    launch_jacobi_eig(s.S2, s.ev, s.S3, l, st);
    sketch_finalize<<<1, 128, 0, st>>>(s.ev, nullptr, 0.0, l, s.lam, s.D, s.cs);
    RP4D_HIP(hipGetLastError());
    scale_cols<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S3, l, s.cs);
    pc->V.ensure(static_cast<size_t>(n) * l * sizeof(double));
    launch_tsmm<double, double>(s.S1, l, s.S3, nullptr, n, l, l, 1.0, nullptr, 0, 0.0, pc->V.as<double>(), l, st);
    pc->nu = 0.0;
}

void precond_apply_impl(rp4d_problem* p, const rp4d_precond* pc, int k, const double* R, double* Z) {
    hipStream_t st = stream_of(p);
    const int n = p->n, l = pc->ell;
    p->ws_red.ensure(std::max<size_t>(p->ws_red.bytes,
                                      (2 * static_cast<size_t>(n) + 512 + static_cast<size_t>(l) * k +
                                       gram_work_doubles(n, l, k)) * sizeof(double)));
    double* T = p->ws_red.as<double>() + 2 * n + 512;
    double* gw = T + static_cast<size_t>(l) * k;
    // T = V^T R (l x k); Z = R - V diag(D) T
    launch_gram<double, double>(pc->V.as<double>(), l, R, k, n, l, k, T, gw, st);
    launch_tsmm<double, double>(pc->V.as<double>(), l, T, pc->Dg.as<double>(), n, l, k, -1.0, R, k, 1.0, Z, k, st);
}

}  // namespace
}  // namespace rp4d

extern "C" {

int rp4d_build_precond(rp4d_problem* p, const rp4d_traj* tr, int method, int ell, uint64_t seed,
                       const double* omega, int sketch_dtype, rp4d_precond** out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        check_traj(p, tr);
        RP4D_REQUIRE(method == RP4D_NYSTROM || method == RP4D_RANDSVD, RP4D_EINVAL, "unknown sketch method");
        RP4D_REQUIRE(ell >= 1 && ell <= 128 && ell <= p->n, RP4D_EINVAL, "ell must be in [1, min(128, n)]");
        RP4D_REQUIRE(sketch_dtype == RP4D_F64 || sketch_dtype == RP4D_F32, RP4D_EINVAL, "bad sketch dtype");
        set_device(p->ctx);
        hipStream_t st = stream_of(p);
        Scratch s = sketch_scratch(p, ell, sketch_dtype);
        if (omega)
            launch_relayout<double, double>(omega, 1, s.Om, 1, p->n * ell, 1, st);
        else
            launch_philox_normal(seed, static_cast<size_t>(p->n) * ell, s.Om, st);
        auto* pc = new rp4d_precond();
        try {
            pc->p = p;
            pc->ell = ell;
            if (method == RP4D_NYSTROM)
                build_nystrom(p, tr, ell, sketch_dtype, s, pc);
            else
                build_randsvd(p, tr, ell, sketch_dtype, s, pc);
            pc->Dg.ensure(static_cast<size_t>(ell) * sizeof(double));
            launch_relayout<double, double>(s.D, 1, pc->Dg.as<double>(), 1, ell, 1, st);
            pc->lam.resize(ell);
            copy_host(p, pc->lam.data(), s.lam, ell * sizeof(double));
            for (double v : pc->lam) RP4D_REQUIRE(std::isfinite(v), RP4D_ENONFINITE, "non-finite sketch eigenvalues");
        } catch (...) {
            delete pc;
            throw;
        }
        p->cnt.tlm_offline += ell;
        p->cnt.adj_offline += ell;
        p->cnt.sketches += 1;
        *out = pc;
    });
}

int rp4d_precond_destroy(rp4d_precond* pc) {
    return guarded([&] {
        if (pc && pc->p) {
            set_device(pc->p->ctx);
            (void)hipStreamSynchronize(pc->p->ctx->stream);
        }
        delete pc;
    });
}

int rp4d_precond_info(const rp4d_precond* pc, int* ell, double* lambda_host, double* nu_host) {
    return guarded([&] {
        RP4D_REQUIRE(pc != nullptr, RP4D_EINVAL, "null preconditioner");
        if (ell) *ell = pc->ell;
        if (lambda_host) std::memcpy(lambda_host, pc->lam.data(), pc->lam.size() * sizeof(double));
        if (nu_host) *nu_host = pc->nu;
    });
}

int rp4d_precond_basis(const rp4d_precond* pc, double* V_out) {
    return guarded([&] {
        RP4D_REQUIRE(pc != nullptr && V_out != nullptr, RP4D_EINVAL, "null argument");
        set_device(pc->p->ctx);
        launch_relayout<double, double>(pc->V.as<double>(), 1, V_out, 1, pc->p->n * pc->ell, 1, stream_of(pc->p));
    });
}

int rp4d_precond_apply(const rp4d_precond* pc, int k, const double* R, double* Z) {
    return guarded([&] {
        RP4D_REQUIRE(pc != nullptr, RP4D_EINVAL, "null preconditioner");
        check_common(pc->p, k, R, Z);
        set_device(pc->p->ctx);
        precond_apply_impl(pc->p, pc, k, R, Z);
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// PCG and Gauss-Newton
// ---------------------------------------------------------------------------
namespace rp4d {
namespace {

void pcg_impl(rp4d_problem* p, const rp4d_traj* tr, const rp4d_precond* pc, const double* b, double* x,
              double rtol, int maxit, rp4d_pcg_info* info, bool true_res, rp4d::DevBuf& vecs) {
    hipStream_t st = stream_of(p);
    const int n = p->n;
    vecs.ensure(5 * static_cast<size_t>(n) * sizeof(double) + 1024 * sizeof(double));
    double* r = vecs.as<double>();
    double* z = r + n;
    double* pv = z + n;
    double* q = pv + n;
    double* red = q + n + n;  // 1024 doubles of reduction scratch
    double* sc = p->ws_scal.as<double>();
    if (maxit <= 0) maxit = n;
    launch_fill<double>(x, n, 0.0, st);
    launch_relayout<double, double>(b, 1, r, 1, n, 1, st);
    if (pc)
        precond_apply_impl(p, pc, 1, r, z);
    else
        launch_relayout<double, double>(r, 1, z, 1, n, 1, st);
    launch_relayout<double, double>(z, 1, pv, 1, n, 1, st);
    launch_dot(r, z, n, sc + SC_RZ, red, st);
    launch_dot(b, b, n, sc + SC_BB, red, st);
    const double bnorm = std::sqrt(read_scalar(p, sc + SC_BB));
    RP4D_REQUIRE(std::isfinite(bnorm), RP4D_ENONFINITE, "non-finite right-hand side");
    double rnorm = bnorm;
    int it = 0;
    bool conv = bnorm == 0.0 || rnorm <= rtol * bnorm;
    while (!conv && it < maxit) {
        hessian_dispatch(p, tr, 1, pv, q, RP4D_F64, true);
        launch_dot(pv, q, n, sc + SC_PQ, red, st);
        pcg_update_xr<<<nblk(n), 256, 0, st>>>(x, r, pv, q, sc, n);
        RP4D_HIP(hipGetLastError());
        ++it;
        launch_dot(r, r, n, sc + SC_RR, red, st);
        rnorm = std::sqrt(read_scalar(p, sc + SC_RR));
        RP4D_REQUIRE(std::isfinite(rnorm), RP4D_ENONFINITE, "non-finite PCG residual");
        if (rnorm <= rtol * bnorm) {
            conv = true;
            break;
        }
        if (pc)
            precond_apply_impl(p, pc, 1, r, z);
        else
            launch_relayout<double, double>(r, 1, z, 1, n, 1, st);
        launch_dot(r, z, n, sc + SC_RZN, red, st);
        pcg_update_p<<<nblk(n), 256, 0, st>>>(pv, z, sc, n);
        RP4D_HIP(hipGetLastError());
        scal_copy<<<1, 1, 0, st>>>(sc, SC_RZ, SC_RZN);
        RP4D_HIP(hipGetLastError());
    }
    p->cnt.tlm_online += it;
    p->cnt.adj_online += it;
    if (info) {
        info->iters = it;
        info->converged = conv ? 1 : 0;
        info->relres = bnorm > 0 ? rnorm / bnorm : 0.0;
        info->true_relres = -1.0;
    }
    if (true_res && info) {
        hessian_dispatch(p, tr, 1, x, q, RP4D_F64, true);
        launch_axpby(b, 1.0, q, -1.0, n, st);  // q = b - (I+H)x
        launch_dot(q, q, n, sc + SC_T1, red, st);
        const double tr2 = read_scalar(p, sc + SC_T1);
        info->true_relres = bnorm > 0 ? std::sqrt(tr2) / bnorm : 0.0;
    }
    if (!conv) fail(RP4D_ENOCONV, "PCG reached maxit before the tolerance");
}

double kappa_impl(rp4d_problem* p, const rp4d_traj* tr, const rp4d_precond* pc, const double* v,
                  rp4d::DevBuf& vecs) {
    hipStream_t st = stream_of(p);
    const int n = p->n;
    vecs.ensure(5 * static_cast<size_t>(n) * sizeof(double) + 1024 * sizeof(double));
    double* z = vecs.as<double>();
    double* q = z + n;
    double* red = z + 5 * static_cast<size_t>(n);
    double* sc = p->ws_scal.as<double>();
    // normalise v
    launch_dot(v, v, n, sc + SC_T0, red, st);
    const double vn = std::sqrt(read_scalar(p, sc + SC_T0));
    RP4D_REQUIRE(vn > 0 && std::isfinite(vn), RP4D_EINVAL, "kappa_re: zero or non-finite test vector");
    double* vu = q + n;
    launch_fill<double>(vu, n, 0.0, st);
    launch_axpby(v, 1.0 / vn, vu, 0.0, n, st);
    precond_apply_impl(p, pc, 1, vu, z);
    hessian_dispatch(p, tr, 1, z, q, RP4D_F64, true);
    launch_dot(q, q, n, sc + SC_T0, red, st);
    return std::sqrt(read_scalar(p, sc + SC_T0));
}

}  // namespace
}  // namespace rp4d

namespace {
rp4d::DevBuf& pcg_buf(rp4d_problem* p) { return p->ws_pcg; }
}  // namespace

extern "C" {

int rp4d_pcg_solve(rp4d_problem* p, const rp4d_traj* tr, const rp4d_precond* pc, const double* b, double* x,
                   double rtol, int maxit, rp4d_pcg_info* info) {
    return guarded([&] {
        check_common(p, 1, b, x);
        check_traj(p, tr);
        RP4D_REQUIRE(pc == nullptr || pc->p == p, RP4D_EINVAL, "preconditioner belongs to another problem");
        RP4D_REQUIRE(rtol >= 0, RP4D_EINVAL, "rtol must be >= 0");
        set_device(p->ctx);
        pcg_impl(p, tr, pc, b, x, rtol, maxit, info, true, pcg_buf(p));
    });
}

int rp4d_kappa_re(rp4d_problem* p, const rp4d_traj* tr, const rp4d_precond* pc, const double* v, double* kappa) {
    return guarded([&] {
        check_common(p, 1, v, kappa);
        check_traj(p, tr);
        RP4D_REQUIRE(pc != nullptr && pc->p == p, RP4D_EINVAL, "bad preconditioner");
        set_device(p->ctx);
        *kappa = kappa_impl(p, tr, pc, v, pcg_buf(p));
    });
}

int rp4d_gn_state_create(rp4d_problem* p, rp4d_gn_state** out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        RP4D_REQUIRE(p->has_data, RP4D_ESTATE, "set data before creating a GN state");
        set_device(p->ctx);
        auto* s = new rp4d_gn_state();
        try {
            s->p = p;
            const size_t nb = p->n * sizeof(double);
            s->v.ensure(nb);
            s->x.ensure(nb);
            s->dv.ensure(nb);
            s->g.ensure(nb);
            s->b.ensure(nb);
            hipStream_t st = stream_of(p);
            launch_fill<double>(s->v.as<double>(), p->n, 0.0, st);
            launch_fill<double>(s->dv.as<double>(), p->n, 0.0, st);
            launch_relayout<double, double>(p->xb.as<double>(), 1, s->x.as<double>(), 1, p->n, 1, st);
            int rc = rp4d_traj_create(p, &s->traj);
            RP4D_REQUIRE(rc == RP4D_OK, rc, g_last_error);
        } catch (...) {
            delete s;
            throw;
        }
        *out = s;
    });
}

int rp4d_gn_state_destroy(rp4d_gn_state* s) {
    return guarded([&] {
        if (!s) return;
        if (s->pc) rp4d_precond_destroy(s->pc);
        if (s->traj) rp4d_traj_destroy(s->traj);
        delete s;
    });
}

int rp4d_gn_state_get(const rp4d_gn_state* s, double* v, double* x) {
    return guarded([&] {
        RP4D_REQUIRE(s != nullptr, RP4D_EINVAL, "null state");
        set_device(s->p->ctx);
        if (v) launch_relayout<double, double>(s->v.as<double>(), 1, v, 1, s->p->n, 1, stream_of(s->p));
        if (x) launch_relayout<double, double>(s->x.as<double>(), 1, x, 1, s->p->n, 1, stream_of(s->p));
    });
}

int rp4d_gn_state_last_step(const rp4d_gn_state* s, double* dv) {
    return guarded([&] {
        RP4D_REQUIRE(s != nullptr && dv != nullptr, RP4D_EINVAL, "null argument");
        set_device(s->p->ctx);
        launch_relayout<double, double>(s->dv.as<double>(), 1, dv, 1, s->p->n, 1, stream_of(s->p));
    });
}

int rp4d_gn_step(rp4d_problem* p, rp4d_gn_state* s, const rp4d_gn_opts* o, rp4d_gn_info* info) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && s != nullptr && o != nullptr && s->p == p, RP4D_EINVAL, "bad argument");
        RP4D_REQUIRE(o->sketch == RP4D_NYSTROM || o->sketch == RP4D_RANDSVD || o->sketch == RP4D_NOPREC, RP4D_EINVAL,
                     "unknown sketch method");
        set_device(p->ctx);
        hipStream_t st = stream_of(p);
        const int n = p->n;
        double* sc = p->ws_scal.as<double>();
        rp4d::DevBuf& vecs = pcg_buf(p);
        vecs.ensure(5 * static_cast<size_t>(n) * sizeof(double) + 1024 * sizeof(double));
        double* red = vecs.as<double>() + 5 * static_cast<size_t>(n);
        // 1. FWD at x, J
        double Jobs = 0.0;
        int rc = rp4d_fwd(p, s->x.as<double>(), s->traj, &Jobs);
        RP4D_REQUIRE(rc == RP4D_OK, rc, g_last_error);
        launch_dot(s->v.as<double>(), s->v.as<double>(), n, sc + SC_T2, red, st);
        const double vv = read_scalar(p, sc + SC_T2);
        // 2. gradient g = v + A^T d
        adj_impl<double>(p, s->traj, 1, s->traj->innov.as<double>(), s->g.as<double>(), s->v.as<double>());
        p->cnt.adj_online += 1;
        absmax_kernel<<<1, 256, 0, st>>>(s->g.as<double>(), n, sc + SC_T1);
        RP4D_HIP(hipGetLastError());
        const double ginf = read_scalar(p, sc + SC_T1);
        RP4D_REQUIRE(std::isfinite(ginf), RP4D_ENONFINITE, "non-finite gradient");
        // 3. b = -g
        launch_fill<double>(s->b.as<double>(), n, 0.0, st);
        launch_axpby(s->g.as<double>(), -1.0, s->b.as<double>(), 0.0, n, st);
        rp4d_gn_info inf{};
        inf.J = 0.5 * vv + Jobs;
        inf.gnorm_inf = ginf;
        inf.kappa_re = -1.0;
        // 4-5. reuse test or sketch
        const rp4d_precond* use = nullptr;
        if (o->sketch != RP4D_NOPREC) {
            if (s->pc && o->reuse_eps > 0) {
                const double* vh = o->vhat;
                double* tmpv = nullptr;
                if (!vh) {
                    tmpv = s->dv.as<double>();  // dv is overwritten by the PCG below
                    launch_philox_normal(o->seed ^ 0x5DEECE66DULL, n, tmpv, st);
                    vh = tmpv;
                }
                inf.kappa_re = kappa_impl(p, s->traj, s->pc, vh, vecs);
                if (inf.kappa_re < o->reuse_eps) {
                    use = s->pc;
                    inf.reused = 1;
                    p->cnt.reuses += 1;
                }
            }
            if (!use) {
                if (s->pc) {
                    rp4d_precond_destroy(s->pc);
                    s->pc = nullptr;
                }
                rc = rp4d_build_precond(p, s->traj, o->sketch, o->ell, o->seed, o->omega, o->sketch_dtype, &s->pc);
                RP4D_REQUIRE(rc == RP4D_OK, rc, g_last_error);
                use = s->pc;
                inf.sketched = 1;
            }
        }
        // 6. PCG
        rp4d_pcg_info pi{};
        int pcg_rc = RP4D_OK;
        try {
            pcg_impl(p, s->traj, use, s->b.as<double>(), s->dv.as<double>(), o->rtol, o->maxit, &pi, false, vecs);
        } catch (const Error& e) {
            if (e.code != RP4D_ENOCONV) throw;
            pcg_rc = e.code;
        }
        inf.pcg_iters = pi.iters;
        inf.pcg_converged = pi.converged;
        inf.pcg_relres = pi.relres;
        // 7. v <- v + dv ; x = x_b + Gamma^{1/2} v
        launch_axpby(s->dv.as<double>(), 1.0, s->v.as<double>(), 1.0, n, st);
        bhalf_into<double>(p, 1, s->v.as<double>(), 1, s->x.as<double>(), 1, p->xb.as<double>());
        if (info) *info = inf;
        if (pcg_rc != RP4D_OK) fail(pcg_rc, "PCG reached maxit before the tolerance (step applied)");
    });
}

int rp4d_gn_state_reset(rp4d_gn_state* s) {
    return guarded([&] {
        RP4D_REQUIRE(s != nullptr, RP4D_EINVAL, "null state");
        rp4d_problem* p = s->p;
        set_device(p->ctx);
        hipStream_t st = stream_of(p);
        launch_fill<double>(s->v.as<double>(), p->n, 0.0, st);
        launch_fill<double>(s->dv.as<double>(), p->n, 0.0, st);
        launch_relayout<double, double>(p->xb.as<double>(), 1, s->x.as<double>(), 1, p->n, 1, st);
        if (s->pc) {
            rp4d_precond_destroy(s->pc);
            s->pc = nullptr;
        }
    });
}

int rp4d_problem_synthesize(rp4d_problem* p, const double* x_true, const double* xi, const double* eta,
                            double* xb_out, double* y_out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && x_true && xi && eta && xb_out && y_out, RP4D_EINVAL, "null argument");
        set_device(p->ctx);
        hipStream_t st = stream_of(p);
        bhalf_into<double>(p, 1, xi, 1, xb_out, 1, x_true);
        run_fwd(p, x_true, 0, p->s_last, nullptr, 1, 0, 0, nullptr, y_out);
        launch_axpby(eta, p->d.sigma_o, y_out, 1.0, p->m, st);
    });
}

int rp4d_ctx_set_timing(rp4d_ctx* ctx, int enable) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr, RP4D_EINVAL, "null context");
        set_device(ctx);
        resolve_timing(ctx);
        ctx->timing = enable != 0;
        for (int i = 0; i < RP4D_K_COUNT; ++i) {
            ctx->launches[i] = 0;
            ctx->ms[i] = 0.0;
            ctx->flops[i] = 0.0;
        }
    });
}

int rp4d_ctx_kernel_stats(rp4d_ctx* ctx, int kind, long long* launches, double* total_ms, double* alg_flops) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr && kind >= 0 && kind < RP4D_K_COUNT, RP4D_EINVAL, "bad argument");
        set_device(ctx);
        resolve_timing(ctx);
        if (launches) *launches = ctx->launches[kind];
        if (total_ms) *total_ms = ctx->ms[kind];
        if (alg_flops) *alg_flops = ctx->flops[kind];
    });
}

int rp4d_counters_get(const rp4d_problem* p, rp4d_counters* out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        *out = p->cnt;
    });
}

int rp4d_counters_reset(rp4d_problem* p) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr, RP4D_EINVAL, "null problem");
        p->cnt = rp4d_counters{};
    });
}

int rp4d_philox_normal(rp4d_ctx* ctx, uint64_t seed, size_t count, double* out) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        set_device(ctx);
        launch_philox_normal(seed, count, out, ctx->stream);
    });
}

int rp4d_set_sweep_tiling(rp4d_problem* p, int mode, int dtype, int k, int ppt, int kc, int threads, int tile,
                          int steps) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr, RP4D_EINVAL, "null problem");
        RP4D_REQUIRE(mode == 0 || mode == MODE_TLM || mode == MODE_ADJ, RP4D_EINVAL, "bad sweep mode");
        Tiling t;
        t.ppt = ppt;
        t.kc = kc;
        t.threads = threads;
        t.tile = tile;
        t.steps = steps;
        if (ppt <= 0 && kc <= 0 && threads <= 0 && tile <= 0 && steps <= 0)
            p->tiling.erase(std::make_tuple(mode, dtype, k));
        else
            p->tiling[std::make_tuple(mode, dtype, k)] = t;
    });
}

int rp4d_get_sweep_tiling(const rp4d_problem* p, int mode, int dtype, int k, int* ppt, int* kc, int* threads,
                          int* tile, int* steps) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr, RP4D_EINVAL, "null problem");
        Tiling t = tiling_for(p, mode == 0 ? MODE_TLM : mode, dtype, k > 0 ? k : 1);
        if (ppt) *ppt = t.ppt;
        if (kc) *kc = t.kc;
        if (threads) *threads = t.threads;
        if (tile) *tile = t.tile;
        if (steps) *steps = t.steps;
    });
}

}  // extern "C"
