// C ABI of the rp4d library: handles, block sweeps (FWD/TLM/ADJ/Hessian),
// sketches (Nystrom Alg. 2, RandSVD Alg. 1), PCG, Gauss-Newton step.
// Every numerical step runs in the kernels of this library; the host code only
// sequences launches on the context stream and reads back control scalars.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <tuple>
#include <type_traits>

#include <limits>
#include <map>
#include <mutex>

#include "batch_plan.hpp"
#include "internal.hpp"

namespace rp4d {

static thread_local std::string g_last_error;

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

thread_local std::shared_ptr<HbmAcct> tl_acct;

void DevBuf::ensure(size_t b) {
    if (b <= bytes && p != nullptr) return;
    if (borrowed) {
        if (b == 0) return;
        fail(RP4D_ENOMEM, "no-allocation call: a workspace exceeds its scratch view");
    }
    std::shared_ptr<HbmAcct> a = acct ? acct : tl_acct;
    release();
    if (b == 0) return;
    if (a && a->budget > 0 && a->used.load() + static_cast<long long>(b) > a->budget)
        fail(RP4D_ENOMEM, "context HBM budget exceeded: " + std::to_string(a->used.load()) + " bytes held, " +
                              std::to_string(b) + " more asked, budget " + std::to_string(a->budget));
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        p = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        fail(RP4D_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
    acct = a;
    if (acct) acct->used += static_cast<long long>(b);
}

void DevBuf::release() {
    if (p && !borrowed) {
        (void)hipFree(p);
        if (acct) acct->used -= static_cast<long long>(bytes);
    }
    p = nullptr;
    bytes = 0;
    borrowed = false;
    acct.reset();
}

namespace {
hipEvent_t pooled_event(rp4d_ctx* c) {
    if (c->event_pool.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
}

// Record the closing event of a pair opened with `a` and queue it for resolution.
void close_pair(rp4d_ctx* c, int kind, hipEvent_t a, double flops, long long nl) {
    hipEvent_t b = pooled_event(c);
    if (b == nullptr) {
        c->event_pool.push_back(a);
        return;
    }
    if (hipEventRecord(b, c->stream) != hipSuccess) {
        c->event_pool.push_back(a);
        c->event_pool.push_back(b);
        return;
    }
    c->pending.push_back(rp4d_ctx::Pending{kind, a, b, flops, nl});
}
}  // namespace

KernelTimer::KernelTimer(rp4d_ctx* ctx, int k, double fl) : c(ctx), kind(k), flops(fl) {
    if (!c->timing || c->capturing) return;
    if (c->span_open[kind]) {  // counted by the enclosing span
        c->span_launches[kind] += 1;
        c->span_flops[kind] += fl;
        return;
    }
    a = pooled_event(c);
    if (a == nullptr) RP4D_HIP(hipErrorOutOfMemory);
    RP4D_HIP(hipEventRecord(a, c->stream));
}

KernelTimer::~KernelTimer() {
    if (!a) return;
    close_pair(c, kind, a, flops, 1);
}

SpanTimer::SpanTimer(rp4d_ctx* ctx, int k) : c(ctx), kind(k) {
    if (c->timing != 2 || c->capturing || c->span_open[kind]) return;
    a = pooled_event(c);
    if (a == nullptr) RP4D_HIP(hipErrorOutOfMemory);
    RP4D_HIP(hipEventRecord(a, c->stream));
    c->span_open[kind] = true;
    c->span_launches[kind] = 0;
    c->span_flops[kind] = 0.0;
}

SpanTimer::~SpanTimer() {
    if (!a) return;
    c->span_open[kind] = false;
    close_pair(c, kind, a, c->span_flops[kind], c->span_launches[kind]);
}

namespace {

// Resolve recorded event pairs into the per-class statistics (synchronises).
void resolve_timing(rp4d_ctx* c) {
    if (c->pending.empty()) return;
    RP4D_HIP(hipStreamSynchronize(c->stream));
    for (auto& pe : c->pending) {
        float ms = 0.f;
        RP4D_HIP(hipEventElapsedTime(&ms, pe.a, pe.b));
        c->launches[pe.kind] += pe.nlaunch;
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
    struct ClearAcct {
        ClearAcct() { tl_acct.reset(); }
        ~ClearAcct() { tl_acct.reset(); }
    } clear_acct;
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
enum { SC_RZ = 0, SC_PQ, SC_RZN, SC_RR, SC_BB, SC_T0, SC_T1, SC_T2, SC_DD, SC_VV, SC_GI, SC_COUNT };
static_assert(SC_COUNT <= 16, "per-problem scalar block of the batched path holds 16");

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

// nu = scale * sqrt(max(lambda_max, 0)) with scale = sqrt(n) eps (Alg. 2's shift).
__global__ void nystrom_nu_kernel(const double* lmax, double scale, double* nu) {
    nu[0] = scale * sqrt(fmax(lmax[0], 0.0));
}

__global__ void scale_scalar(double* v, double f) { v[0] *= f; }

// y += a x with a read from device memory (same rounding as axpby with beta = 1).
__global__ void axpy_dev(const double* x, const double* a, double* y, size_t count) {
    const double alpha = a[0], beta = 1.0;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        y[i] = alpha * x[i] + beta * y[i];
}

// out = v / sqrt(sc[0]) (same rounding as axpby with alpha = 1 / sqrt(sc[0]), beta = 0).
__global__ void scale_inv_sqrt(const double* v, const double* sc, double* out, int n) {
    const double alpha = 1.0 / sqrt(sc[0]);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = alpha * v[i];
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
void set_device(const rp4d_ctx* c) {
    RP4D_HIP(hipSetDevice(c->device));
    (void)hipGetLastError();  // drop errors left by calls outside this library
    tl_acct = c->acct;        // allocations of this call count against c's budget
}

hipStream_t stream_of(const rp4d_problem* p) { return p->ctx->stream; }

// Destruction waits for all work on the object's device and reads nothing
// outside the object, so owners and children may be destroyed in any order
// (a language runtime's finaliser may not respect ownership).
void quiesce_device(int device) {
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    (void)hipGetLastError();
}

void sync(const rp4d_problem* p) { RP4D_HIP(hipStreamSynchronize(stream_of(p))); }

double read_scalar(const rp4d_problem* p, const double* dptr) {
    double v = 0.0;
    RP4D_HIP(hipMemcpyAsync(&v, dptr, sizeof(double), hipMemcpyDeviceToHost, stream_of(p)));
    sync(p);
    return v;
}

// Tiling of a sweep with no tuned one set: wave regions in the shapes the
// tiling search picked for burgers-4096 -- single vectors 2 points per lane,
// 13 steps per launch, 16 owned points per 128-point region; blocks 4 points x
// 2 vectors per lane, 15 steps, 128 owned of 256 -- with the tiles balanced
// over n (a region may wrap a small ring more than once).
Tiling heuristic_tiling(int n, int k) {
    Tiling t;
    t.xch = XCH_WAVE;
    t.threads = 64;
    if (k == 1) {
        t.ppt = 2;
        t.kc = 1;
        t.steps = 13;
    } else {
        t.ppt = 4;
        t.kc = 2;
        t.steps = 15;
    }
    const int room = 64 * t.ppt - 2 * (4 * t.steps + 4);
    const int tiles = std::max(1, (n + room - 1) / room);
    t.tile = (n + tiles - 1) / tiles;
    return t;
}

// Wall-bounded sweeps run on wave regions: 4 points per lane (256-point
// regions), 12 steps per launch (halo 52), tiles of up to 152 points, two
// vectors per group for blocks.
Tiling wall_tiling(int n, int k) {
    Tiling t;
    t.xch = XCH_WAVE;
    t.ppt = 4;
    t.kc = k >= 2 ? 2 : 1;
    t.threads = 64;
    t.steps = 12;
    t.tile = std::min(n, 64 * t.ppt - 2 * (4 * t.steps + 4));
    return t;
}

Tiling tiling_for(const rp4d_problem* p, int mode, int dtype, int k) {
    Tiling t = p->wall ? wall_tiling(p->n, k) : heuristic_tiling(p->n, k);
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
            if (o.xch > 0) t.xch = o.xch;
            break;
        }
    }
    return t;
}

Tiling fwd_tiling(const rp4d_problem* p) {
    Tiling t = p->wall ? wall_tiling(p->n, 1) : heuristic_tiling(p->n, 1);
    // the single nonlinear state: fewer, larger tiles amortise launches better
    if (p->n >= 1024 && !p->wall) {
        t.xch = XCH_LDS;
        const int tiles = std::max(1, p->n / 512);
        t.tile = (p->n + tiles - 1) / tiles;
        t.steps = std::max(1, std::min(32, static_cast<int>((0.3 * t.tile - 8.0) / 8.0)));
        const int R = t.tile + 2 * (4 * t.steps + 4);
        t.ppt = R > 2048 ? 8 : (R > 512 ? 2 : 1);
        t.threads = ((R + t.ppt - 1) / t.ppt + 63) / 64 * 64;
    }
    if (t.ppt == 8 && t.threads > 1024) t.threads = 1024;
    auto it = p->tiling.find(std::make_tuple(static_cast<int>(RP4D_MODE_FWD), static_cast<int>(RP4D_F64), 1));
    if (it != p->tiling.end()) {
        const Tiling& o = it->second;
        if (o.ppt > 0) t.ppt = o.ppt;
        if (o.threads > 0) t.threads = o.threads;
        if (o.tile > 0) t.tile = o.tile;
        if (o.steps > 0) t.steps = o.steps;
        if (o.xch > 0) t.xch = o.xch;
    }
    t.kc = 1;
    return t;
}

void check_traj(const rp4d_problem* p, const rp4d_traj* tr) {
    RP4D_REQUIRE(tr != nullptr && tr->p == p, RP4D_EINVAL, "trajectory does not belong to this problem");
    RP4D_REQUIRE(tr->valid, RP4D_ESTATE, "trajectory not computed: call rp4d_fwd first");
}

// Run the nonlinear model over steps [s_from, s_to) starting from state x (n),
// storing u_s for s % store_every == 0 at store rows s/store_every - store_row0.
FwdArgs fwd_args(const rp4d_problem* p, const Tiling& t, double* store, int store_every, int store_row0,
                 int store_rows, double* innov, double* obs_out) {
    FwdArgs a{};
    a.store = store;
    a.store_every = store_every;
    a.store_row0 = store_row0;
    a.store_rows = store_rows;
    a.n = p->n;
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
    a.wall = p->wall ? 1 : 0;
    return a;
}

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
    FwdArgs a = fwd_args(p, t, store, store_every, store_row0, store_rows, innov, obs_out);
    SpanTimer span(p->ctx, RP4D_K_FWD);
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

// The planned FWD (every row stored) over [0, s_last) from x0 into tr, on the
// current stream; its launches are enqueued by fwd_plan_need / fwd_plan_finish.
// The ping-pong states and the scratch at 2n.. of ws_red belong to it until it
// is finished.
void fwd_plan_start(rp4d_problem* p, const double* x0, rp4d_traj* tr) {
    RP4D_REQUIRE(tr->C == 1 && !p->bve, RP4D_ESTATE, "planned FWD needs the 1-D model with every row stored");
    rp4d_ctx* c = p->ctx;
    FwdPlan& f = p->fwd_plan;
    const int n = p->n;
    f.st = stream_of(p);
    f.t = fwd_tiling(p);
    p->ws_red.ensure(std::max<size_t>(p->ws_red.bytes, (2 * static_cast<size_t>(n) + 1024) * sizeof(double)));
    f.in = p->ws_red.as<double>();
    f.out = f.in + n;
    double* innov = tr->innov.as<double>();
    f.a = fwd_args(p, f.t, tr->states.as<double>(), 1, 0, tr->rows, innov, innov + p->m);
    launch_relayout<double, double>(x0, 1, tr->states.as<double>(), 1, n, 1, f.st);  // row 0 = x0
    launch_relayout<double, double>(x0, 1, f.in, 1, n, 1, f.st);
    f.span = nullptr;
    if (c->timing && !c->capturing) {
        f.span = pooled_event(c);
        if (f.span == nullptr) RP4D_HIP(hipErrorOutOfMemory);
        RP4D_HIP(hipEventRecord(f.span, f.st));
    }
    f.tr = tr;
    f.s_next = 0;
    f.s_to = p->s_last;
    f.enq_row = 0;
    f.marked_row = -1;
    f.waited_row = -1;
    f.waited_st = nullptr;
    f.launches = 0;
    f.next_ev = 0;
    f.last_ev = nullptr;
    f.active = true;
    tr->valid = true;
    tr->has_innov = p->has_data;
    p->cnt.fwd += 1;
}

// Enqueue planned FWD launches until rows 0..row are covered, then mark the
// point with an event on the FWD's stream.
void fwd_plan_enqueue(rp4d_problem* p, int row) {
    FwdPlan& f = p->fwd_plan;
    while (f.s_next < f.s_to && f.enq_row < row) {
        f.a.s0 = f.s_next;
        f.a.S = std::min(f.t.steps, f.s_to - f.s_next);
        f.a.xin = f.in;
        f.a.xout = f.out;
        launch_burgers_fwd(f.a, f.t, f.st);
        f.launches += 1;
        f.s_next += f.a.S;
        f.enq_row = f.s_next;
        std::swap(f.in, f.out);
    }
    if (f.marked_row >= f.enq_row) return;
    if (f.next_ev == static_cast<int>(f.ev.size())) {
        hipEvent_t e = nullptr;
        RP4D_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        f.ev.push_back(e);
    }
    f.last_ev = f.ev[f.next_ev++];  // one event per mark within a plan
    RP4D_HIP(hipEventRecord(f.last_ev, f.st));
    f.marked_row = f.enq_row;
}

// A sweep on stream st is about to read rows 0..row of tr: if tr is being
// produced by the planned FWD, enqueue it far enough and make st wait.  The
// first mark covers one FWD launch past the rows asked for (the sweep starts
// early); later marks run FWD_PLAN_AHEAD launches past them, so that the next
// sweep launches find their rows marked already: fewer events and waits to
// enqueue, and the host stays ahead of the device.
constexpr int FWD_PLAN_AHEAD = 3;

void fwd_plan_need(rp4d_problem* p, const rp4d_traj* tr, int row, hipStream_t st) {
    FwdPlan& f = p->fwd_plan;
    if (!f.active || f.tr != tr) return;
    row = std::min(row, f.s_to);
    if (f.marked_row < row) fwd_plan_enqueue(p, row + (f.marked_row < 0 ? 1 : FWD_PLAN_AHEAD) * f.t.steps);
    if (st == f.st) return;
    if (f.waited_st != st) {
        f.waited_st = st;
        f.waited_row = -1;
    }
    if (f.waited_row >= row) return;
    RP4D_HIP(hipStreamWaitEvent(st, f.last_ev, 0));
    f.waited_row = f.marked_row;
}

// Enqueue the rest of the planned FWD (on its stream) and close its timing span.
void fwd_plan_finish(rp4d_problem* p) {
    FwdPlan& f = p->fwd_plan;
    if (!f.active) return;
    fwd_plan_enqueue(p, f.s_to);
    if (f.span) {
        rp4d_ctx* c = p->ctx;
        hipStream_t keep = c->stream;
        c->stream = f.st;
        close_pair(c, RP4D_K_FWD, f.span, FL_FWD * f.s_to * static_cast<double>(p->n), f.launches);
        c->stream = keep;
        f.span = nullptr;
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
    a.wall = p->wall ? 1 : 0;
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
        SpanTimer span(p->ctx, k == 1 ? RP4D_K_TLM1 : RP4D_K_TLM);
        for (int s0 = seg0; s0 < seg1; s0 += t.steps) {
            a.s0 = s0;
            a.S = std::min(t.steps, seg1 - s0);
            a.xin = in;
            a.xout = out;
            if (C == 1) fwd_plan_need(p, tr, s0 + a.S - 1, st);  // the launch reads u_s0 .. u_{s0+S-1}
            {
                KernelTimer kt(p->ctx, k == 1 ? RP4D_K_TLM1 : RP4D_K_TLM,
                               static_cast<double>(a.S) * n * (FL_TLM_VEC * k + FL_TLM_BASE));
                launch_burgers_sweep<T>(MODE_TLM, a, t, groups, st);
            }
            std::swap(in, out);
        }
    }
    if (p->after_tlm && st != p->ctx->side) {
        auto f = std::move(p->after_tlm);
        p->after_tlm = nullptr;
        f();
    }
}

// ADJ of k vectors with forcing w (n_t, n_obs, k); result lambda_0 (blocked kc) returned pointer.
template <typename T>
T* run_adj(rp4d_problem* p, const rp4d_traj* tr, int k, const Tiling& t, T* buf0, T* buf1, const T* w) {
    const int n = p->n;
    hipStream_t st = stream_of(p);
    const int groups = (k + t.kc - 1) / t.kc;
    fwd_plan_need(p, tr, p->s_last, st);  // the backward sweep starts at the last row
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
    a.wall = p->wall ? 1 : 0;
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
        SpanTimer span(p->ctx, k == 1 ? RP4D_K_ADJ1 : RP4D_K_ADJ);
        int s_hi = seg1;
        while (s_hi > seg0) {
            const int Sc = std::min(t.steps, s_hi - seg0);
            a.s0 = s_hi - Sc;
            a.S = Sc;
            a.xin = in;
            a.xout = out;
            {
                KernelTimer kt(p->ctx, k == 1 ? RP4D_K_ADJ1 : RP4D_K_ADJ,
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
    if (p->bve) {
        bve_bhalf<T>(p, k, in, in_kc, out, out_kc, addv);
        return;
    }
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
    if (p->bve) {
        bve_tlm<T>(p, tr, k, V, Z);
        return;
    }
    SweepWork<T> w = sweep_work<T>(p, k, sizeof(T) == 8 ? RP4D_F64 : RP4D_F32);
    const int groups = (k + w.tt.kc - 1) / w.tt.kc;
    if (groups * w.tt.kc != k) launch_fill<T>(w.s0, static_cast<size_t>(groups) * w.tt.kc * p->n, T(0), stream_of(p));
    bhalf_into<T>(p, k, V, k, w.s0, w.tt.kc, nullptr);
    run_tlm<T>(p, tr, k, w.tt, w.s0, w.s1, Z);
}

template <typename T>
void adj_impl(rp4d_problem* p, const rp4d_traj* tr, int k, const T* W, T* U, const T* addv) {
    if (p->bve) {
        bve_adj<T>(p, tr, k, W, U, addv);
        return;
    }
    SweepWork<T> w = sweep_work<T>(p, k, sizeof(T) == 8 ? RP4D_F64 : RP4D_F32);
    T* lam = run_adj<T>(p, tr, k, w.ta, w.s0, w.s1, W);
    bhalf_into<T>(p, k, lam, w.ta.kc, U, k, addv);
}

template <typename T>
void hessian_impl(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* HV, bool add_identity) {
    if (p->bve) {
        bve_hessian<T>(p, tr, k, V, HV, add_identity);
        p->cnt.hv_columns += k;
        return;
    }
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

void fwd_impl(rp4d_problem* p, const double* x0, rp4d_traj* tr) {
    hipStream_t st = stream_of(p);
    double* rows = tr->states.as<double>();
    double* innov = tr->innov.as<double>();
    double* obs = innov + p->m;
    if (p->bve) {
        bve_fwd(p, x0, tr, innov, obs);
    } else {
        launch_relayout<double, double>(x0, 1, rows, 1, p->n, 1, st);  // row 0 = x0
        run_fwd(p, x0, 0, p->s_last, rows, tr->C, 0, tr->rows, innov, obs);
    }
    tr->valid = true;
    tr->has_innov = p->has_data;
    p->cnt.fwd += 1;
}

}  // namespace
}  // namespace rp4d

rp4d_ctx::~rp4d_ctx() {
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    for (auto& pe : pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (auto e : event_pool) (void)hipEventDestroy(e);
}

using namespace rp4d;

namespace {
rp4d_problem* create_bve(rp4d_ctx* ctx, const rp4d_problem_desc& d) {
    RP4D_REQUIRE(d.nx == d.ny && fft_size_supported(d.nx), RP4D_EINVAL,
                 "2-D grid must be square with side 16 B, B in {2,3,4,5,6,8,10,12,16,20,24,32}");
    RP4D_REQUIRE(d.nsteps >= 1 && d.obs_every >= 1 && d.obs_stride >= 1 && d.obs_stride <= d.nx, RP4D_EINVAL,
                 "bad window / observation layout");
    RP4D_REQUIRE(d.nsteps / d.obs_every >= 1, RP4D_EINVAL, "window has no observation step");
    RP4D_REQUIRE(d.dt > 0 && d.nu >= 0 && d.sigma_o > 0 && d.sigma_b > 0 && d.L_b > 0, RP4D_EINVAL,
                 "bad physical parameters");
    RP4D_REQUIRE(d.ckpt_every <= 1, RP4D_EINVAL, "the 2-D model stores the full trajectory (ckpt_every 0 or 1)");
    const double dx = 1.0 / d.nx;
    RP4D_REQUIRE(8.0 * d.nu * d.dt / (dx * dx) <= 2.785, RP4D_EUNSTABLE,
                 "time step outside the RK4 diffusive stability interval (8 nu dt/dx^2 > 2.785)");
    auto* p = new rp4d_problem();
    try {
        p->ctx = ctx;
        p->d = d;
        p->d.ckpt_every = 1;
        p->n = d.nx * d.ny;
        const int nox = (d.nx + d.obs_stride - 1) / d.obs_stride, noy = (d.ny + d.obs_stride - 1) / d.obs_stride;
        p->n_obs = nox * noy;
        p->n_t = d.nsteps / d.obs_every;
        p->m = p->n_obs * p->n_t;
        p->s_last = p->n_t * d.obs_every;
        p->dx = dx;
        bve_setup(p);
        p->xb.ensure(p->n * sizeof(double));
        p->y.ensure(static_cast<size_t>(p->m) * sizeof(double));
        p->ws_scal.ensure(64 * sizeof(double));
    } catch (...) {
        delete p;
        throw;
    }
    return p;
}
}  // namespace

// The paper's Burgers setup (Sec. 5.1): n interior nodes of (0, 1) with
// Dirichlet walls, dx = 1/(n + 1), RK3-TVD, observations at nodes j with
// (j + 1) a multiple of obs_stride, prior Gamma^{1/2} = (alpha I - beta Lap*)^{-1}.
rp4d_problem* create_wall(rp4d_ctx* ctx, const rp4d_problem_desc& d) {
    RP4D_REQUIRE(d.nx >= 8 && d.nx <= 16384, RP4D_EINVAL, "wall model: nx must be in [8, 16384]");
    RP4D_REQUIRE(d.nsteps >= 1 && d.obs_every >= 1 && d.obs_stride >= 1 && d.obs_stride <= d.nx, RP4D_EINVAL,
                 "bad window / observation layout");
    RP4D_REQUIRE(d.nsteps / d.obs_every >= 1, RP4D_EINVAL, "window has no observation step");
    RP4D_REQUIRE(d.dt > 0 && d.nu >= 0 && d.sigma_o > 0 && d.prior_alpha > 0 && d.prior_beta >= 0, RP4D_EINVAL,
                 "bad physical parameters (wall model: prior_alpha > 0, prior_beta >= 0)");
    const double dx = 1.0 / (d.nx + 1);
    RP4D_REQUIRE(4.0 * d.nu * d.dt / (dx * dx) <= 2.51, RP4D_EUNSTABLE,
                 "time step outside the RK3-TVD diffusive stability interval (4 nu dt/dx^2 > 2.51)");
    RP4D_REQUIRE(10.0 * d.dt / dx <= 1.7, RP4D_EUNSTABLE,
                 "time step outside the RK3-TVD advective stability interval for |u| <= 10");
    auto* p = new rp4d_problem();
    try {
        p->ctx = ctx;
        p->d = d;
        p->wall = true;
        p->n = d.nx;
        p->n_obs = d.nx / d.obs_stride;
        p->n_t = d.nsteps / d.obs_every;
        p->m = p->n_obs * p->n_t;
        p->s_last = p->n_t * d.obs_every;
        p->dx = dx;
        p->inv2dx = 1.0 / (2.0 * dx);
        p->nu_dx2 = d.nu / (dx * dx);
        if (p->d.ckpt_every < 1) p->d.ckpt_every = 1;
        // (alpha I - beta Lap*) is diagonalised by the orthonormal sine basis
        // S_ij = sqrt(2/(n+1)) sin((i+1)(j+1) pi/(n+1)), eigenvalues
        // alpha + 4 beta sin^2((j+1) pi/(2(n+1))): Gamma^{1/2} = S diag(1/eig) S,
        // applied by the spectral path with all n modes.
        const int n = d.nx;
        const long per = 2L * (n + 1);
        std::vector<double> Fh(static_cast<size_t>(n) * n), lh(n);
        const double c = std::sqrt(2.0 / (n + 1));
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const long q = (static_cast<long>(i + 1) * (j + 1)) % per;
                Fh[static_cast<size_t>(i) * n + j] = c * std::sin(M_PI * static_cast<double>(q) / (n + 1));
            }
        for (int j = 0; j < n; ++j) {
            const double sj = std::sin(M_PI * (j + 1) / (2.0 * (n + 1)));
            lh[j] = 1.0 / (d.prior_alpha + 4.0 * d.prior_beta * sj * sj);
        }
        p->spec = true;
        p->r = n;
        p->F.ensure(Fh.size() * sizeof(double));
        p->lamF.ensure(lh.size() * sizeof(double));
        RP4D_HIP(hipMemcpyAsync(p->F.p, Fh.data(), Fh.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        RP4D_HIP(hipMemcpyAsync(p->lamF.p, lh.data(), lh.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        RP4D_HIP(hipStreamSynchronize(ctx->stream));  // the host staging vectors go out of scope
        p->xb.ensure(p->n * sizeof(double));
        p->y.ensure(static_cast<size_t>(p->m) * sizeof(double));
        p->ws_scal.ensure(64 * sizeof(double));
    } catch (...) {
        delete p;
        throw;
    }
    return p;
}

// ===========================================================================
// ABI
// ===========================================================================
// ---------------------------------------------------------------------------
// Static scratch of the no-allocation entry point (rp4d_hessian_block_noalloc).
// Each device holds its own copy of `scratch` for the life of the process; host
// code reaches a device's copy only through the address hipGetSymbolAddress
// returned for it (the array's name on the host is a stand-in, not a device
// address).  The address is resolved once per device, with that device current,
// when the first context on the device is created.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

void resolve_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return;
    void* ptr = nullptr;
    RP4D_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    RP4D_REQUIRE(ptr != nullptr, RP4D_EHIP, "no device address for the static scratch");
    g_scratch_ptr[device] = ptr;
}

void* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}
}  // namespace

extern "C" {

const char* rp4d_last_error(void) { return g_last_error.c_str(); }

const char* rp4d_version(void) { return "rp4d 0.1 (gfx950)"; }

int rp4d_ctx_create(int device, void* hip_stream, size_t hbm_budget_bytes, rp4d_ctx** out) {
    return guarded([&] {
        RP4D_REQUIRE(out != nullptr, RP4D_EINVAL, "null output handle");
        int ndev = 0;
        RP4D_HIP(hipGetDeviceCount(&ndev));
        RP4D_REQUIRE(device >= 0 && device < ndev, RP4D_EINVAL, "no such HIP device");
        RP4D_HIP(hipSetDevice(device));
        resolve_scratch(device);
        RP4D_REQUIRE(hbm_budget_bytes <= static_cast<size_t>(std::numeric_limits<long long>::max()), RP4D_EINVAL,
                     "HBM budget out of range");
        auto* c = new rp4d_ctx();
        c->device = device;
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->acct->budget = static_cast<long long>(hbm_budget_bytes);
        *out = c;
    });
}

int rp4d_ctx_hbm(const rp4d_ctx* ctx, size_t* used, size_t* budget) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr, RP4D_EINVAL, "null context");
        if (used) *used = static_cast<size_t>(std::max(0LL, ctx->acct->used.load()));
        if (budget) *budget = static_cast<size_t>(ctx->acct->budget);
    });
}

int rp4d_ctx_destroy(rp4d_ctx* ctx) {
    return guarded([&] {
        if (ctx) quiesce_device(ctx->device);
        delete ctx;
    });
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
        RP4D_REQUIRE(d.model == RP4D_BURGERS1D || d.model == RP4D_BVE2D || d.model == RP4D_BURGERS1D_WALL,
                     RP4D_EINVAL, "unknown model");
        if (d.model == RP4D_BVE2D) {
            *out = create_bve(ctx, d);
            return;
        }
        if (d.model == RP4D_BURGERS1D_WALL) {
            *out = create_wall(ctx, d);
            return;
        }
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
            RP4D_HIP(hipMemcpyAsync(p->gk.p, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
            RP4D_HIP(hipStreamSynchronize(ctx->stream));
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
                RP4D_HIP(hipMemcpyAsync(p->F.p, Fh.data(), Fh.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
                RP4D_HIP(hipMemcpyAsync(p->lamF.p, lh.data(), lh.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
                RP4D_HIP(hipStreamSynchronize(ctx->stream));  // Fh, lh are freed at the end of this block
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
        if (p) quiesce_device(p->device);
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

int rp4d_problem_set_id(rp4d_problem* p, uint64_t id) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr, RP4D_EINVAL, "null problem");
        p->id = id;
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
            if (p->bve) t->stages.ensure(bve_traj_stage_bytes(p));
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
        if (t) quiesce_device(t->device);
        delete t;
    });
}

int rp4d_fwd(rp4d_problem* p, const double* x0, rp4d_traj* tr, double* J_obs) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && x0 != nullptr && tr != nullptr && tr->p == p, RP4D_EINVAL, "bad argument");
        set_device(p->ctx);
        hipStream_t st = stream_of(p);
        double* innov = tr->innov.as<double>();
        fwd_impl(p, x0, tr);
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

int rp4d_hessian_block_noalloc(rp4d_problem* p, const rp4d_traj* tr, int k, const void* V, void* HV, int dtype,
                               int add_identity) {
    return guarded([&] {
        check_common(p, k, V, HV);
        RP4D_REQUIRE(V != HV, RP4D_EINVAL, "V and HV must not alias");
        check_traj(p, tr);
        RP4D_REQUIRE(!p->bve, RP4D_EINVAL, "no-allocation Hessian: 1-D models only");
        RP4D_REQUIRE(dtype == RP4D_F64 || dtype == RP4D_F32, RP4D_EINVAL, "dtype must be RP4D_F64 or RP4D_F32");
        set_device(p->ctx);
        unsigned char* base = static_cast<unsigned char*>(scratch_of(p->ctx->device));
        RP4D_REQUIRE(base != nullptr, RP4D_ESTATE, "no-allocation Hessian: scratch not resolved for this device");
        // the workspaces hessian_impl asks for, carved out of the scratch
        const size_t es = dtype == RP4D_F64 ? 8 : 4;
        const Tiling tt = tiling_for(p, MODE_TLM, dtype, k), ta = tiling_for(p, MODE_ADJ, dtype, k);
        const int kcmax = std::max(tt.kc, ta.kc);
        const size_t blk = static_cast<size_t>((k + kcmax - 1) / kcmax + 1) * kcmax * p->n * es;
        const size_t obs = static_cast<size_t>(p->m) * k * es;
        const size_t bh = p->spec ? (static_cast<size_t>(p->r) * k + gram_work_doubles(p->n, p->r, k)) * 8 : 0;
        const size_t seg = tr->C > 1 ? static_cast<size_t>(tr->C + 1) * p->n * 8 : 0;
        const size_t red = tr->C > 1 ? 2 * static_cast<size_t>(p->n) * 8 + 64 : 0;
        DevBuf* bufs[6] = {&p->ws_s0, &p->ws_s1, &p->ws_obs, &p->ws_bh, &p->ws_seg, &p->ws_red};
        const size_t need[6] = {blk, blk, obs, bh, seg, red};
        size_t total = 0;
        for (size_t b : need) total += ring_round(b);
        RP4D_REQUIRE(total <= kScratchBytes, RP4D_EINVAL,
                     "no-allocation Hessian: workspaces of " + std::to_string(total) +
                         " bytes exceed the 64 MiB scratch (smaller k or n)");
        // swap views of the scratch in for the problem's own workspaces; put them
        // back on every exit.  Timing events are suspended (their pool may create).
        struct Borrow {
            DevBuf view[6];
            DevBuf** slots;
            rp4d_ctx* c;
            int timing;
            ~Borrow() {
                for (int i = 0; i < 6; ++i) slots[i]->swap(view[i]);
                for (auto& v : view) v.release();
                c->timing = timing;
            }
        } g{{}, bufs, p->ctx, p->ctx->timing};
        size_t off = 0;
        for (int i = 0; i < 6; ++i) {
            g.view[i].p = need[i] ? base + off : nullptr;
            g.view[i].bytes = need[i];
            g.view[i].borrowed = true;
            off += ring_round(need[i]);
        }
        for (int i = 0; i < 6; ++i) bufs[i]->swap(g.view[i]);
        p->ctx->timing = 0;
        hessian_dispatch(p, tr, k, V, HV, dtype, add_identity != 0);
    });
}

int rp4d_bve_inv_laplacian(rp4d_problem* p, int k, const void* in, void* out, int dtype) {
    return guarded([&] {
        check_common(p, k, in, out);
        RP4D_REQUIRE(p->bve != nullptr, RP4D_EINVAL, "inverse Laplacian needs a 2-D problem");
        set_device(p->ctx);
        if (dtype == RP4D_F64)
            bve_inv_laplacian<double>(p, k, static_cast<const double*>(in), static_cast<double*>(out));
        else if (dtype == RP4D_F32)
            bve_inv_laplacian<float>(p, k, static_cast<const float*>(in), static_cast<float*>(out));
        else
            fail(RP4D_EINVAL, "bad dtype");
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

void nystrom_core(rp4d_problem* p, int l, double eps, Scratch& s, rp4d_precond* pc, bool fast = false);
void lmp_factor_fast(rp4d_problem* p, int l, const double* Wt, Scratch& s, rp4d_precond* pc);

void build_nystrom(rp4d_problem* p, const rp4d_traj* tr, int l, int dtype, Scratch& s, rp4d_precond* pc,
                   bool fast = false) {
    sketch_misfit_hessian(p, tr, l, dtype, s);                       // Y = H Omega
    nystrom_core(p, l, dtype == RP4D_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23), s, pc, fast);
}

// A Gram of the sketch post-processing that feeds an eigenvalue estimate or an
// eigendecomposition (FP64 X, Y): FP64, or BF16 when the context asks for it.
void eigen_gram(rp4d_problem* p, const double* X, int lx, const double* Y, int ly, int n, int a, int b, double* C,
                double* work) {
    if (p->ctx->gram_dtype == RP4D_BF16)
        launch_gram_bf16<double, double>(X, lx, Y, ly, n, a, b, C, work, stream_of(p));
    else
        launch_gram<double, double>(X, lx, Y, ly, n, a, b, C, work, stream_of(p));
}

// Nystrom approximation (Alg. 2) from its sketch: Omega (n x l) in s.Om and Y = H Omega in s.Yd, both
// row-major with leading size l; eps is the unit roundoff of the sketch sweeps.
// Writes pc->V and s.lam, s.D, s.nu; with `fast` the factored form of the
// preconditioner instead (lmp_factor_fast on B, no eigendecomposition).
void nystrom_core(rp4d_problem* p, int l, double eps, Scratch& s, rp4d_precond* pc, bool fast) {
    hipStream_t st = stream_of(p);
    const int n = p->n;
    // shift nu = sqrt(n) eps ||Y||_2, ||Y||_2^2 = lambda_max(Y^T Y)
    eigen_gram(p, s.Yd, l, s.Yd, l, n, l, l, s.S2, s.gw);
    {
        KernelTimer kt(p->ctx, RP4D_K_EIG, 0.0);
        launch_sym_lmax(s.S2, l, s.lam, s.S3, st);
    }
    // nu stays on the device (s.nu); a non-finite sketch surfaces as a failed
    // Cholesky factorisation below
    nystrom_nu_kernel<<<1, 1, 0, st>>>(s.lam, std::sqrt(static_cast<double>(n)) * eps, s.nu);
    RP4D_HIP(hipGetLastError());
    bool ok = false, fused = false;
    for (int attempt = 0; attempt <= 3; ++attempt) {
        // shifted sketch Y_nu = Y + nu Omega, core C = Omega^T Y_nu = L L^T (symmetrised)
        launch_relayout<double, double>(s.Yd, 1, s.Y2, 1, n * l, 1, st);
        const size_t cnt = static_cast<size_t>(n) * l;
        axpy_dev<<<nblk(static_cast<long>(cnt)), 256, 0, st>>>(s.Om, s.nu, s.Y2, cnt);
        RP4D_HIP(hipGetLastError());
        launch_gram<double, double>(s.Om, l, s.Y2, l, n, l, l, s.S2, s.gw, st);
        fused = launch_chol_invt(s.S2, l, s.info, s.S4, st);  // S2 = L, and S4 = L^{-T} if fused
        if (!fused) launch_chol(s.S2, l, s.info, st);
        if (read_info(p, s.info) == 0) {
            ok = true;
            break;
        }
        scale_scalar<<<1, 1, 0, st>>>(s.nu, 10.0);
        RP4D_HIP(hipGetLastError());
    }
    RP4D_REQUIRE(ok, RP4D_ENOTSPD, "Nystrom core matrix not positive definite after shift retries (or non-finite sketch)");
    // B = Y_nu L^{-T} (n x l), B B^T the shifted approximant; B^T B = U Sigma^2 U^T.  Forming B before the
    // Gram keeps the error at eps cond(L) |B|^2 (the Gram of Y between two
    // triangular inverses would square cond(L)).
    if (!fused) {
        launch_trinv(s.S2, s.S3, l, st);                                  // S3 = L^{-1}
        transpose_small<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S3, s.S4, l);  // S4 = L^{-T}
        RP4D_HIP(hipGetLastError());
    }
    launch_tsmm<double, double>(s.Y2, l, s.S4, nullptr, n, l, l, 1.0, nullptr, 0, 0.0, s.S1, l, st);  // S1 = B
    if (fast) {
        lmp_factor_fast(p, l, s.S1, s, pc);
        return;
    }
    eigen_gram(p, s.S1, l, s.S1, l, n, l, l, s.S4, s.gw);   // S4 = B^T B
    {
        KernelTimer kt(p->ctx, RP4D_K_EIG, 0.0);
        launch_jacobi_eig(s.S4, s.ev, s.S2, l, st);                       // ev = Sigma^2, S2 = U
    }
    sketch_finalize<<<1, 128, 0, st>>>(s.ev, s.nu, 0.0, l, s.lam, s.D, s.cs);
    RP4D_HIP(hipGetLastError());
    // V_hat = B U Sigma^{-1}
    scale_cols<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S2, l, s.cs);
    pc->V.ensure(static_cast<size_t>(n) * l * sizeof(double));
    launch_tsmm<double, double>(s.S1, l, s.S2, nullptr, n, l, l, 1.0, nullptr, 0, 0.0, pc->V.as<double>(), l, st);
}

// One Cholesky-QR pass on Y (rows x l, FP64, in s.Yd): G = Y^T Y + shift I = L L^T,
// Y <- Y L^{-T}.  Returns the Cholesky info (0 = success; Y untouched otherwise).
// With Rinv (l x l) the pass's R^{-1} = L^{-T} is accumulated: Rinv <- L^{-T}
// on the first pass, Rinv <- Rinv L^{-T} after it, so that Q = Y_in Rinv; with
// Rout (l x l) the factor itself: Rout <- L^T, then Rout <- L^T Rout, so that
// Y_in = Q Rout.
int cholqr_pass(rp4d_problem* p, int rows, int l, Scratch& s, double shift, double* Rinv = nullptr,
                bool first = true, double* Rout = nullptr) {
    hipStream_t st = stream_of(p);
    launch_gram<double, double>(s.Yd, l, s.Yd, l, rows, l, l, s.S2, s.gw, st);
    if (shift > 0) {
        std::vector<double> eye(static_cast<size_t>(l) * l, 0.0);
        for (int i = 0; i < l; ++i) eye[static_cast<size_t>(i) * l + i] = shift;
        RP4D_HIP(hipMemcpyAsync(s.S4, eye.data(), eye.size() * sizeof(double), hipMemcpyHostToDevice, st));
        launch_axpby(s.S4, 1.0, s.S2, 1.0, static_cast<size_t>(l) * l, st);
        sync(p);  // the host staging vector must outlive the copy
    }
    const bool fused = launch_chol_invt(s.S2, l, s.info, s.S4, st);  // S2 = L, and S4 = L^{-T} if fused
    if (!fused) launch_chol(s.S2, l, s.info, st);
    const int info = read_info(p, s.info);
    if (info != 0) return info;
    if (!fused) {
        launch_trinv(s.S2, s.S3, l, st);
        transpose_small<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S3, s.S4, l);  // S4 = L^{-T}
        RP4D_HIP(hipGetLastError());
    }
    launch_tsmm<double, double>(s.Yd, l, s.S4, nullptr, rows, l, l, 1.0, nullptr, 0, 0.0, s.Y2, l, st);
    launch_relayout<double, double>(s.Y2, 1, s.Yd, 1, rows * l, 1, st);
    if (Rinv && first) {
        launch_relayout<double, double>(s.S4, 1, Rinv, 1, l * l, 1, st);
    } else if (Rinv) {
        launch_small_gemm(Rinv, 0, s.S4, 0, s.S3, l, 1.0, st);
        launch_relayout<double, double>(s.S3, 1, Rinv, 1, l * l, 1, st);
    }
    if (Rout && first) {
        transpose_small<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S2, Rout, l);  // L^T
        RP4D_HIP(hipGetLastError());
    } else if (Rout) {
        launch_small_gemm(s.S2, 1, Rout, 0, s.S3, l, 1.0, st);  // L^T Rout
        launch_relayout<double, double>(s.S3, 1, Rout, 1, l * l, 1, st);
    }
    return 0;
}

// Thin QR of Y (rows x l) by CholeskyQR2; if the Gram matrix is numerically
// indefinite, shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa, Yamamoto,
// Yanagisawa 2020): one pass with shift 11 (rows l + l(l+1)) u ||Y||_2^2, then two
// plain passes.  Q overwrites s.Yd; Rinv (nullable, l x l) receives R^{-1} and
// Rout (nullable, l x l) receives R.
void cholqr2(rp4d_problem* p, int rows, int l, Scratch& s, double* Rinv = nullptr, double* Rout = nullptr) {
    hipStream_t st = stream_of(p);
    if (cholqr_pass(p, rows, l, s, 0.0, Rinv, true, Rout) == 0) {
        RP4D_REQUIRE(cholqr_pass(p, rows, l, s, 0.0, Rinv, false, Rout) == 0, RP4D_ENOTSPD,
                     "sketch: Cholesky QR second pass failed");
        return;
    }
    launch_gram<double, double>(s.Yd, l, s.Yd, l, rows, l, l, s.S2, s.gw, st);
    {
        KernelTimer kt(p->ctx, RP4D_K_EIG, 0.0);
        launch_sym_lmax(s.S2, l, s.lam, s.S3, st);
    }
    double ymax2 = 0.0;
    copy_host(p, &ymax2, s.lam, sizeof(double));
    const double sh = 11.0 * (static_cast<double>(rows) * l + l * (l + 1.0)) * std::ldexp(1.0, -53) * ymax2;
    RP4D_REQUIRE(cholqr_pass(p, rows, l, s, std::max(sh, 1e-300), Rinv, true, Rout) == 0, RP4D_ENOTSPD,
                 "sketch: shifted Cholesky QR failed");
    RP4D_REQUIRE(cholqr_pass(p, rows, l, s, 0.0, Rinv, false, Rout) == 0, RP4D_ENOTSPD,
                 "sketch: Cholesky QR pass failed");
    RP4D_REQUIRE(cholqr_pass(p, rows, l, s, 0.0, Rinv, false, Rout) == 0, RP4D_ENOTSPD,
                 "sketch: Cholesky QR pass failed");
}

void build_randsvd(rp4d_problem* p, const rp4d_traj* tr, int l, int dtype, Scratch& s, rp4d_precond* pc,
                   bool fast = false) {
    hipStream_t st = stream_of(p);
    const int n = p->n, m = p->m;
    // Y = A Omega (m x l)
    if (dtype == RP4D_F64) {
        tlm_impl<double>(p, tr, l, s.Om, s.Yd);
    } else {
        launch_relayout<double, float>(s.Om, l, static_cast<float*>(s.Omt), l, n, l, st);
        tlm_impl<float>(p, tr, l, static_cast<const float*>(s.Omt), static_cast<float*>(s.Yt));
        launch_relayout<float, double>(static_cast<const float*>(s.Yt), l, s.Yd, l, m, l, st);
    }
    // thin QR Y = Q R (CholeskyQR2 in FP64)
    cholqr2(p, m, l, s);
    // W^T = A^T Q (n x l)
    if (dtype == RP4D_F64) {
        adj_impl<double>(p, tr, l, s.Yd, s.S1, nullptr);
    } else {
        launch_relayout<double, float>(s.Yd, l, static_cast<float*>(s.Yt), l, m, l, st);
        adj_impl<float>(p, tr, l, static_cast<const float*>(s.Yt), static_cast<float*>(s.Wt), nullptr);
        launch_relayout<float, double>(static_cast<const float*>(s.Wt), l, s.S1, l, n, l, st);
    }
    if (fast) {
        lmp_factor_fast(p, l, s.S1, s, pc);
        launch_fill<double>(s.nu, 1, 0.0, st);
        return;
    }
    // thin SVD of W via eig(W W^T): V_hat = W^T U Sigma^{-1}, Lambda = Sigma^2
    eigen_gram(p, s.S1, l, s.S1, l, n, l, l, s.S2, s.gw);
    {
        KernelTimer kt(p->ctx, RP4D_K_EIG, 0.0);
        launch_jacobi_eig(s.S2, s.ev, s.S3, l, st);
    }
    sketch_finalize<<<1, 128, 0, st>>>(s.ev, nullptr, 0.0, l, s.lam, s.D, s.cs);
    RP4D_HIP(hipGetLastError());
    scale_cols<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S3, l, s.cs);
    pc->V.ensure(static_cast<size_t>(n) * l * sizeof(double));
    launch_tsmm<double, double>(s.S1, l, s.S3, nullptr, n, l, l, 1.0, nullptr, 0, 0.0, pc->V.as<double>(), l, st);
    launch_fill<double>(s.nu, 1, 0.0, st);
}

__global__ void add_identity(double* G, int l) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < l) G[static_cast<size_t>(i) * l + i] += 1.0;
}

// Factored limited-memory preconditioner of a sketch H_hat = W^T W, W^T (n x l)
// FP64 row-major: (I + W^T W)^{-1} = I - W^T (I + W W^T)^{-1} W (eq. (randsvdsv))
// = I - F F^T with F = W^T K^{-T}, I + W W^T = K K^T.  pc->V = F, pc->Dg = 1, so
// the apply of eq. (woodbury) is unchanged.  I + W W^T has eigenvalues >= 1
// (its Cholesky factorisation cannot fail on the finite sketches that reach
// here), and no eigendecomposition is formed.
void lmp_factor_fast(rp4d_problem* p, int l, const double* Wt, Scratch& s, rp4d_precond* pc) {
    hipStream_t st = stream_of(p);
    const int n = p->n;
    launch_gram<double, double>(Wt, l, Wt, l, n, l, l, s.S4, s.gw, st);     // W W^T
    add_identity<<<nblk(l), 256, 0, st>>>(s.S4, l);
    RP4D_HIP(hipGetLastError());
    if (!launch_chol_invt(s.S4, l, s.info, s.S2, st)) {                       // K, and K^{-T}
        launch_chol(s.S4, l, s.info, st);
        launch_trinv(s.S4, s.S3, l, st);                                     // K^{-1}
        transpose_small<<<nblk(static_cast<long>(l) * l), 256, 0, st>>>(s.S3, s.S2, l);  // K^{-T}
        RP4D_HIP(hipGetLastError());
    }
    pc->V.ensure(static_cast<size_t>(n) * l * sizeof(double));
    launch_tsmm<double, double>(Wt, l, s.S2, nullptr, n, l, l, 1.0, nullptr, 0, 0.0, pc->V.as<double>(), l, st);
    pc->Dg.ensure(static_cast<size_t>(l) * sizeof(double));
    launch_fill<double>(pc->Dg.as<double>(), l, 1.0, st);
    pc->fast = true;
}

// Seed of the Gaussian block drawn by extension r of the adaptive sketch, and of
// its kappa_sk test vector.
inline uint64_t adaptive_seed(uint64_t seed, int r) { return seed + 0x9E3779B97F4A7C15ULL * static_cast<uint64_t>(r); }
inline uint64_t adaptive_vseed(uint64_t seed) { return seed ^ 0xD1B54A32D192ED03ULL; }

// Device buffers of one kappa_sk evaluation for sketches of up to L columns.
struct KappaWork {
    double *G, *Gi, *Gt;  // L x L each
    double *vu, *u, *q;   // n each: unit test vector, u, (I + H) u
    double *red, *tv, *zv;  // 1024 dot partials, L, L
    double* gw;           // Gram partials
};

// Unit test vector of kappa_sk into w.vu: vtest normalised, or a Philox draw.
void kappa_test_vector(rp4d_problem* p, const double* vtest, uint64_t vseed, const KappaWork& w) {
    hipStream_t st = stream_of(p);
    const int n = p->n;
    double* sc = p->ws_scal.as<double>();
    if (vtest)
        launch_relayout<double, double>(vtest, 1, w.u, 1, n, 1, st);
    else
        launch_philox_normal(vseed, n, w.u, st);
    launch_dot(w.u, w.u, n, sc + SC_T0, w.red, st);
    scale_inv_sqrt<<<nblk(n), 256, 0, st>>>(w.u, sc + SC_T0, w.vu, n);
    RP4D_HIP(hipGetLastError());
}

// kappa_sk = |(I + H) u| with u = v - W^T (I + W W^T)^{-1} W v (eq. (condtext),
// (randsvdsv)) for H_hat = W^T W, W^T (n x c) with leading size ld.  One
// single-vector Hessian product (counted offline) and one scalar read.
double kappa_sk_dev(rp4d_problem* p, const rp4d_traj* tr, const double* Wt, int ld, int c, const KappaWork& w,
                    int* info) {
    hipStream_t st = stream_of(p);
    const int n = p->n;
    double* sc = p->ws_scal.as<double>();
    launch_gram<double, double>(Wt, ld, Wt, ld, n, c, c, w.G, w.gw, st);  // G = W W^T (c x c)
    add_identity<<<nblk(c), 256, 0, st>>>(w.G, c);
    RP4D_HIP(hipGetLastError());
    launch_chol(w.G, c, info, st);                                        // I + W W^T = Lc Lc^T (SPD)
    launch_trinv(w.G, w.Gi, c, st);                                       // Gi = Lc^{-1}
    launch_small_gemm(w.Gi, 1, w.Gi, 0, w.Gt, c, 1.0, st);                // Gt = (I + W W^T)^{-1}
    launch_gram<double, double>(Wt, ld, w.vu, 1, n, c, 1, w.tv, w.gw, st);  // tv = W v
    launch_tsmm<double, double>(w.Gt, c, w.tv, nullptr, c, c, 1, 1.0, nullptr, 0, 0.0, w.zv, 1, st);
    launch_tsmm<double, double>(Wt, ld, w.zv, nullptr, n, c, 1, -1.0, w.vu, 1, 1.0, w.u, 1, st);
    hessian_dispatch(p, tr, 1, w.u, w.q, RP4D_F64, true);                 // (I + H) u
    p->cnt.tlm_offline += 1;
    p->cnt.adj_offline += 1;
    launch_dot(w.q, w.q, n, sc + SC_T1, w.red, st);
    const double kappa = std::sqrt(read_scalar(p, sc + SC_T1));
    RP4D_REQUIRE(std::isfinite(kappa), RP4D_ENONFINITE, "adaptive sketch: non-finite kappa_sk");
    return kappa;
}

// Adaptive RandSVD (Sec. 3.1.2, Alg. 4) into pc.  The accumulated basis Q (m x c)
// and W^T = A^T Q (n x c) are kept row-major with leading size l_max; a new
// block of b columns is drawn (or read from omega's columns [c, c + b)), swept
// by the block TLM, orthogonalised against Q twice, factored by Cholesky QR,
// swept back by the block ADJ and appended.  kappa_sk (eq. (condtext)) uses
// (I + W^T W)^{-1} = I - W^T (I + W W^T)^{-1} W (eq. (randsvdsv)) and one
// single-vector Hessian product; the loop stops once kappa_sk <= eps_sk or the
// next block would pass l_max.  The final thin SVD of W is the eigen-
// decomposition of W W^T, V_hat = W^T U Sigma^{-1}.  Host waits: the Cholesky
// QR checks and one scalar read per kappa_sk.
void build_randsvd_adaptive(rp4d_problem* p, const rp4d_traj* tr, const rp4d_adaptive_opts& o, rp4d_precond* pc,
                            rp4d_adaptive_info* info) {
    hipStream_t st = stream_of(p);
    const int n = p->n, m = p->m, L = o.ell_max;
    Scratch s = sketch_scratch(p, L, RP4D_F64);  // blocks of up to L columns, ell-sized results up to L
    const size_t ll = static_cast<size_t>(L) * L;
    const size_t gw = std::max(gram_work_doubles(n, L, L), gram_work_doubles(m, L, L));
    p->ws_ad.ensure((static_cast<size_t>(m) * L + static_cast<size_t>(n) * L + 3 * ll + 3 * static_cast<size_t>(n) +
                     1024 + 4 * static_cast<size_t>(L) + gw + 64) * sizeof(double));
    double* Qa = p->ws_ad.as<double>();            // m x L
    double* Wt = Qa + static_cast<size_t>(m) * L;  // n x L
    KappaWork kw{};
    kw.G = Wt + static_cast<size_t>(n) * L;        // L x L
    kw.Gi = kw.G + ll;
    kw.Gt = kw.Gi + ll;
    kw.vu = kw.Gt + ll;                            // n
    kw.u = kw.vu + n;
    kw.q = kw.u + n;
    kw.red = kw.q + n;                             // 1024 (dot-product partials)
    kw.tv = kw.red + 1024;                         // L
    kw.zv = kw.tv + L;                             // L
    kw.gw = kw.zv + 2 * L;                         // Gram partials
    double* G = kw.G;
    double* Gi = kw.Gi;
    double* Gt = kw.Gt;
    double* agw = kw.gw;
    kappa_test_vector(p, o.vtest, adaptive_vseed(o.seed), kw);
    int c = 0, r = 0, nk = 0;
    double kappa = 0.0;
    for (;;) {
        const int b = r == 0 ? o.ell0 : o.ell_hat;
        if (o.omega)
            launch_relayout<double, double>(o.omega + c, L, s.Om, b, n, b, st);
        else
            launch_philox_normal(adaptive_seed(o.seed, r), static_cast<size_t>(n) * b, s.Om, st);
        tlm_impl<double>(p, tr, b, s.Om, s.Yd);                        // Y = A Omega (m x b)
        for (int pass = 0; c > 0 && pass < 2; ++pass) {                // Y <- Y - Q (Q^T Y)
            launch_gram<double, double>(Qa, L, s.Yd, b, m, c, b, Gt, agw, st);
            launch_tsmm<double, double>(Qa, L, Gt, nullptr, m, c, b, -1.0, s.Yd, b, 1.0, s.Yd, b, st);
        }
        cholqr2(p, m, b, s);                                            // Y = Q_hat R
        adj_impl<double>(p, tr, b, s.Yd, s.S1, nullptr);                // W_hat^T = A^T Q_hat (n x b)
        launch_relayout<double, double>(s.Yd, b, Qa + c, L, m, b, st);
        launch_relayout<double, double>(s.S1, b, Wt + c, L, n, b, st);
        c += b;
        ++r;
        p->cnt.tlm_offline += b;
        p->cnt.adj_offline += b;
        kappa = kappa_sk_dev(p, tr, Wt, L, c, kw, s.info);
        if (info && nk < 16) info->kappa[nk] = kappa;
        ++nk;
        if (kappa <= o.eps_sk || c + o.ell_hat > L) break;
    }
    // thin SVD of W: W W^T = U Sigma^2 U^T, V_hat = W^T U Sigma^{-1}, Lambda = Sigma^2
    launch_gram<double, double>(Wt, L, Wt, L, n, c, c, G, agw, st);
    {
        KernelTimer kt(p->ctx, RP4D_K_EIG, 0.0);
        launch_jacobi_eig(G, s.ev, Gi, c, st);
    }
    sketch_finalize<<<1, 128, 0, st>>>(s.ev, nullptr, 0.0, c, s.lam, s.D, s.cs);
    RP4D_HIP(hipGetLastError());
    scale_cols<<<nblk(static_cast<long>(c) * c), 256, 0, st>>>(Gi, c, s.cs);
    pc->V.ensure(static_cast<size_t>(n) * c * sizeof(double));
    launch_tsmm<double, double>(Wt, L, Gi, nullptr, n, c, c, 1.0, nullptr, 0, 0.0, pc->V.as<double>(), c, st);
    launch_fill<double>(s.nu, 1, 0.0, st);
    pc->p = p;
    pc->ell = c;
    pc->host_ok = false;
    pc->Dg.ensure(static_cast<size_t>(c) * sizeof(double));
    launch_relayout<double, double>(s.D, 1, pc->Dg.as<double>(), 1, c, 1, st);
    pc->lamd.ensure(static_cast<size_t>(c + 1) * sizeof(double));
    launch_relayout<double, double>(s.lam, 1, pc->lamd.as<double>(), 1, c, 1, st);
    launch_relayout<double, double>(s.nu, 1, pc->lamd.as<double>() + c, 1, 1, 1, st);
    p->cnt.sketches += 1;
    if (info) {
        info->ell = c;
        info->nkappa = nk;
        info->kappa_sk = kappa;
    }
}

void precond_apply_impl(rp4d_problem* p, const rp4d_precond* pc, int k, const double* R, double* Z);

// Adaptive Nystrom (Sec. 3.1.2: the Nystrom form of the adaptive loop of
// Alg. 4) into pc.  Each round draws the next Gaussian block (or reads omega's
// columns [c, c + b)), sweeps only that block (Y_hat = H Omega_hat, one block
// Hessian product), appends both to the accumulated Omega and Y (n x l_max,
// leading size l_max) and forms Alg. 2 on all c columns; kappa_sk (eq.
// (condtext)) applies the new preconditioner (eq. (woodbury)) to v and then
// I + H.  The loop stops once kappa_sk <= eps_sk or the next block would pass
// l_max.  FP64.  Host waits: the Nystrom Cholesky check and one scalar read
// per round.
void build_nystrom_adaptive(rp4d_problem* p, const rp4d_traj* tr, const rp4d_adaptive_opts& o, rp4d_precond* pc,
                            rp4d_adaptive_info* info) {
    hipStream_t st = stream_of(p);
    const int n = p->n, L = o.ell_max;
    Scratch s = sketch_scratch(p, L, RP4D_F64);
    const size_t nL = static_cast<size_t>(n) * L;
    p->ws_ad.ensure((2 * nL + 3 * static_cast<size_t>(n) + 1024 + 64) * sizeof(double));
    double* Oa = p->ws_ad.as<double>();  // n x L: Omega
    double* Ya = Oa + nL;                // n x L: H Omega
    KappaWork kw{};
    kw.vu = Ya + nL;
    kw.u = kw.vu + n;
    kw.q = kw.u + n;
    kw.red = kw.q + n;
    kappa_test_vector(p, o.vtest, adaptive_vseed(o.seed), kw);
    double* sc = p->ws_scal.as<double>();
    const double eps = std::ldexp(1.0, -52);
    pc->p = p;
    pc->host_ok = false;
    int c = 0, r = 0, nk = 0;
    double kappa = 0.0;
    for (;;) {
        const int b = r == 0 ? o.ell0 : o.ell_hat;
        if (o.omega)
            launch_relayout<double, double>(o.omega + c, L, s.Om, b, n, b, st);
        else
            launch_philox_normal(adaptive_seed(o.seed, r), static_cast<size_t>(n) * b, s.Om, st);
        hessian_dispatch(p, tr, b, s.Om, s.Yd, RP4D_F64, false);        // Y_hat = H Omega_hat
        launch_relayout<double, double>(s.Om, b, Oa + c, L, n, b, st);
        launch_relayout<double, double>(s.Yd, b, Ya + c, L, n, b, st);
        c += b;
        ++r;
        p->cnt.tlm_offline += b;
        p->cnt.adj_offline += b;
        // Alg. 2 on the c columns so far
        launch_relayout<double, double>(Oa, L, s.Om, c, n, c, st);
        launch_relayout<double, double>(Ya, L, s.Yd, c, n, c, st);
        nystrom_core(p, c, eps, s, pc);
        pc->ell = c;
        pc->Dg.ensure(static_cast<size_t>(c) * sizeof(double));
        launch_relayout<double, double>(s.D, 1, pc->Dg.as<double>(), 1, c, 1, st);
        // kappa_sk = |(I + H) (I + H_hat)^{-1} v|
        precond_apply_impl(p, pc, 1, kw.vu, kw.u);
        hessian_dispatch(p, tr, 1, kw.u, kw.q, RP4D_F64, true);
        p->cnt.tlm_offline += 1;
        p->cnt.adj_offline += 1;
        launch_dot(kw.q, kw.q, n, sc + SC_T1, kw.red, st);
        kappa = std::sqrt(read_scalar(p, sc + SC_T1));
        RP4D_REQUIRE(std::isfinite(kappa), RP4D_ENONFINITE, "adaptive sketch: non-finite kappa_sk");
        if (info && nk < 16) info->kappa[nk] = kappa;
        ++nk;
        if (kappa <= o.eps_sk || c + o.ell_hat > L) break;
    }
    pc->lamd.ensure(static_cast<size_t>(c + 1) * sizeof(double));
    launch_relayout<double, double>(s.lam, 1, pc->lamd.as<double>(), 1, c, 1, st);
    launch_relayout<double, double>(s.nu, 1, pc->lamd.as<double>() + c, 1, 1, 1, st);
    p->cnt.sketches += 1;
    if (info) {
        info->ell = c;
        info->nkappa = nk;
        info->kappa_sk = kappa;
    }
}

void check_adaptive_opts(const rp4d_problem* p, const rp4d_adaptive_opts& o) {
    RP4D_REQUIRE(o.ell0 >= 1 && o.ell_hat >= 1 && o.ell_max >= o.ell0 && o.ell_max <= 128 && o.ell_max <= p->n,
                 RP4D_EINVAL, "adaptive sketch: need 1 <= ell0 <= ell_max <= min(128, n) and ell_hat >= 1");
    RP4D_REQUIRE(o.ell_max <= p->m, RP4D_EINVAL, "adaptive sketch: ell_max must not exceed the number of observations");
    RP4D_REQUIRE(o.eps_sk > 0 && std::isfinite(o.eps_sk), RP4D_EINVAL, "adaptive sketch: eps_sk must be positive");
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

// Keep D = lambda/(1+lambda), Lambda_hat and nu of a sketch in the preconditioner.
void keep_eigs(rp4d_problem* p, int ell, const Scratch& s, rp4d_precond* pc) {
    hipStream_t st = stream_of(p);
    pc->Dg.ensure(static_cast<size_t>(ell) * sizeof(double));
    launch_relayout<double, double>(s.D, 1, pc->Dg.as<double>(), 1, ell, 1, st);
    pc->lamd.ensure(static_cast<size_t>(ell + 1) * sizeof(double));
    launch_relayout<double, double>(s.lam, 1, pc->lamd.as<double>(), 1, ell, 1, st);
    launch_relayout<double, double>(s.nu, 1, pc->lamd.as<double>() + ell, 1, 1, 1, st);
}

// Sketch and factor into `pc` (its buffers are reused when large enough).
// Everything is enqueued on the problem stream; the only host wait is the
// Nystrom core's Cholesky check.  Host copies of the eigenvalues and the shift
// are fetched on demand (fetch_host).
void build_precond_into(rp4d_problem* p, const rp4d_traj* tr, int method, int ell, uint64_t seed,
                        const double* omega, int sketch_dtype, rp4d_precond* pc, bool fast = false) {
    RP4D_REQUIRE(method == RP4D_NYSTROM || method == RP4D_RANDSVD, RP4D_EINVAL, "unknown sketch method");
    RP4D_REQUIRE(ell >= 1 && ell <= 128 && ell <= p->n, RP4D_EINVAL, "ell must be in [1, min(128, n)]");
    RP4D_REQUIRE(sketch_dtype == RP4D_F64 || sketch_dtype == RP4D_F32, RP4D_EINVAL, "bad sketch dtype");
    hipStream_t st = stream_of(p);
    Scratch s = sketch_scratch(p, ell, sketch_dtype);
    if (omega)
        launch_relayout<double, double>(omega, 1, s.Om, 1, p->n * ell, 1, st);
    else
        launch_philox_normal(seed, static_cast<size_t>(p->n) * ell, s.Om, st);
    pc->p = p;
    pc->ell = ell;
    pc->host_ok = false;
    pc->fast = false;
    if (method == RP4D_NYSTROM)
        build_nystrom(p, tr, ell, sketch_dtype, s, pc, fast);
    else
        build_randsvd(p, tr, ell, sketch_dtype, s, pc, fast);
    p->cnt.tlm_offline += ell;
    p->cnt.adj_offline += ell;
    p->cnt.sketches += 1;
    if (fast) return;
    keep_eigs(p, ell, s, pc);
}

// Nystrom approximation from a caller-supplied sketch: Omega (n x l) and
// Y = H Omega (n x l), device, row-major, FP64.
void build_nystrom_from_sketch(rp4d_problem* p, int ell, const double* omega, const double* Y, rp4d_precond* pc) {
    RP4D_REQUIRE(ell >= 1 && ell <= 128 && ell <= p->n, RP4D_EINVAL, "ell must be in [1, min(128, n)]");
    hipStream_t st = stream_of(p);
    Scratch s = sketch_scratch(p, ell, RP4D_F64);
    launch_relayout<double, double>(omega, 1, s.Om, 1, p->n * ell, 1, st);
    launch_relayout<double, double>(Y, 1, s.Yd, 1, p->n * ell, 1, st);
    pc->p = p;
    pc->ell = ell;
    pc->host_ok = false;
    pc->fast = false;
    nystrom_core(p, ell, std::ldexp(1.0, -52), s, pc);
    keep_eigs(p, ell, s, pc);
}

// Host copies of Lambda_hat and nu (one copy and wait after each build).
void fetch_host(const rp4d_precond* pc) {
    if (pc->host_ok) return;
    RP4D_REQUIRE(!pc->fast, RP4D_ESTATE, "factored preconditioner: no eigenvalues were formed");
    std::vector<double> h(static_cast<size_t>(pc->ell) + 1);
    RP4D_HIP(hipMemcpyAsync(h.data(), pc->lamd.p, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                            stream_of(pc->p)));
    sync(pc->p);
    for (double v : h) RP4D_REQUIRE(std::isfinite(v), RP4D_ENONFINITE, "non-finite sketch eigenvalues");
    pc->lam.assign(h.begin(), h.begin() + pc->ell);
    pc->nu = h[pc->ell];
    pc->host_ok = true;
}

}  // namespace
}  // namespace rp4d

extern "C" {

int rp4d_build_precond(rp4d_problem* p, const rp4d_traj* tr, int method, int ell, uint64_t seed,
                       const double* omega, int sketch_dtype, rp4d_precond** out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        check_traj(p, tr);
        set_device(p->ctx);
        auto* pc = new rp4d_precond();
        try {
            build_precond_into(p, tr, method, ell, seed, omega, sketch_dtype, pc);
            fetch_host(pc);
        } catch (...) {
            delete pc;
            throw;
        }
        *out = pc;
    });
}

int rp4d_build_precond_from_sketch(rp4d_problem* p, int ell, const double* omega, const double* Y,
                                   rp4d_precond** out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && omega != nullptr && Y != nullptr && out != nullptr, RP4D_EINVAL,
                     "null argument");
        set_device(p->ctx);
        auto* pc = new rp4d_precond();
        try {
            build_nystrom_from_sketch(p, ell, omega, Y, pc);
            fetch_host(pc);
        } catch (...) {
            delete pc;
            throw;
        }
        *out = pc;
    });
}

int rp4d_build_precond_adaptive(rp4d_problem* p, const rp4d_traj* tr, const rp4d_adaptive_opts* o,
                                rp4d_precond** out, rp4d_adaptive_info* info) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && o != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        check_traj(p, tr);
        check_adaptive_opts(p, *o);
        set_device(p->ctx);
        auto* pc = new rp4d_precond();
        try {
            build_randsvd_adaptive(p, tr, *o, pc, info);
            fetch_host(pc);
        } catch (...) {
            delete pc;
            throw;
        }
        *out = pc;
    });
}

int rp4d_build_precond_nystrom_adaptive(rp4d_problem* p, const rp4d_traj* tr, const rp4d_adaptive_opts* o,
                                        rp4d_precond** out, rp4d_adaptive_info* info) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && o != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        check_traj(p, tr);
        check_adaptive_opts(p, *o);
        set_device(p->ctx);
        auto* pc = new rp4d_precond();
        try {
            build_nystrom_adaptive(p, tr, *o, pc, info);
            fetch_host(pc);
        } catch (...) {
            delete pc;
            throw;
        }
        *out = pc;
    });
}

int rp4d_precond_destroy(rp4d_precond* pc) {
    return guarded([&] {
        if (pc) quiesce_device(pc->device);
        delete pc;
    });
}

int rp4d_precond_info(const rp4d_precond* pc, int* ell, double* lambda_host, double* nu_host) {
    return guarded([&] {
        RP4D_REQUIRE(pc != nullptr, RP4D_EINVAL, "null preconditioner");
        if (ell) *ell = pc->ell;
        if (lambda_host || nu_host) {
            set_device(pc->p->ctx);
            fetch_host(pc);
        }
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

// Exchange the problem's sweep workspaces with their side-stream copies.
void swap_side_workspaces(rp4d_problem* p) {
    p->ws_s0.swap(p->side_s0);
    p->ws_s1.swap(p->side_s1);
    p->ws_obs.swap(p->side_obs);
    p->ws_bh.swap(p->side_bh);
    p->ws_seg.swap(p->side_seg);
    p->ws_red.swap(p->side_red);
}

// Enqueue the work `f` on the context's side stream after everything already on
// the main stream, with the problem's side workspaces swapped in (the kernels
// capture the buffer addresses at launch); ev_join marks its completion.
template <typename F>
void on_side_lane(rp4d_problem* p, F&& f) {
    rp4d_ctx* c = p->ctx;
    if (!c->side) {
        RP4D_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        RP4D_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        RP4D_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
    hipStream_t main = c->stream;
    RP4D_HIP(hipEventRecord(c->ev_fork, main));
    RP4D_HIP(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    auto swap_all = [p]() { swap_side_workspaces(p); };
    swap_all();
    c->stream = c->side;
    try {
        f();
    } catch (...) {
        c->stream = main;
        swap_all();
        throw;
    }
    c->stream = main;
    swap_all();
    RP4D_HIP(hipEventRecord(c->ev_join, c->side));
}

// Enqueue `f` on the side stream after the work already there (no wait on the
// main stream), with the side workspaces swapped in; ev_join marks its end.
template <typename F>
void continue_on_side(rp4d_problem* p, F&& f) {
    rp4d_ctx* c = p->ctx;
    RP4D_REQUIRE(c->side != nullptr, RP4D_ESTATE, "no side stream to continue on");
    hipStream_t main = c->stream;
    auto swap_all = [p]() { swap_side_workspaces(p); };
    swap_all();
    c->stream = c->side;
    try {
        f();
    } catch (...) {
        c->stream = main;
        swap_all();
        throw;
    }
    c->stream = main;
    swap_all();
    RP4D_HIP(hipEventRecord(c->ev_join, c->side));
}

inline uint64_t singleview_psi_seed(uint64_t seed) { return seed ^ 0x2545F4914F6CDD1DULL; }

void check_singleview_opts(const rp4d_problem* p, rp4d_singleview_opts& o) {
    if (o.ell2 == 0) o.ell2 = std::min(2 * o.ell1 + 1, p->m);
    RP4D_REQUIRE(o.ell1 >= 1 && o.ell1 <= 128 && o.ell1 <= p->n && o.ell1 <= p->m, RP4D_EINVAL,
                 "SingleView: ell1 must be in [1, min(128, n, m)]");
    RP4D_REQUIRE(o.ell2 >= o.ell1 && o.ell2 <= p->m, RP4D_EINVAL, "SingleView: need ell1 <= ell2 <= m");
    RP4D_REQUIRE(o.sketch_dtype == RP4D_F64 || o.sketch_dtype == RP4D_F32, RP4D_EINVAL, "bad sketch dtype");
}

// SingleView (Sec. 3.1.1, Alg. 3) into pc.  The co-range sketch Z = A^T Psi
// (n x l2) needs nothing from the range sketch, so on the 1-D model it runs on
// the side stream (with the side sweep workspaces) while the main stream forms
// Y = A Omega (m x l1), its Cholesky-QR basis Q_Y, M = Psi^T Q_Y (l2 x l1) and
// M's Cholesky-QR factors Q_M, R_M^{-1}.  Then P = Q_M R_M^{-T} (l2 x l1) and
// W^T = Z P (n x l1), i.e. W = R_M^{-1} (Z Q_M)^T; the thin SVD of W comes from
// the eigendecomposition of W W^T: V_hat = W^T U Sigma^{-1}, Lambda = Sigma^2.
// Host waits: the Cholesky-QR checks.
void build_singleview(rp4d_problem* p, const rp4d_traj* tr, const rp4d_singleview_opts& o, rp4d_precond* pc) {
    hipStream_t st = stream_of(p);
    const int n = p->n, m = p->m, l1 = o.ell1, l2 = o.ell2;
    const bool f64 = o.sketch_dtype == RP4D_F64;
    Scratch s = sketch_scratch(p, l1, o.sketch_dtype);
    const size_t gw = std::max({gram_work_doubles(m, l2, l1), gram_work_doubles(m, l1, l1),
                                gram_work_doubles(n, l1, l1), gram_work_doubles(l2, l1, l1)});
    const size_t ml2 = static_cast<size_t>(m) * l2, nl2 = static_cast<size_t>(n) * l2;
    const size_t l21 = static_cast<size_t>(l2) * l1;
    const size_t typed = f64 ? 0 : (ml2 + nl2) * sizeof(float);
    p->ws_ad.ensure((ml2 + nl2 + 2 * l21 + static_cast<size_t>(l1) * l1 + gw + 64) * sizeof(double) + typed);
    double* Psi = p->ws_ad.as<double>();  // m x l2
    double* Z = Psi + ml2;                // n x l2
    double* Mb = Z + nl2;                 // l2 x l1
    double* P = Mb + l21;                 // l2 x l1
    double* Rinv = P + l21;               // l1 x l1
    s.gw = Rinv + static_cast<size_t>(l1) * l1;
    float* Psit = reinterpret_cast<float*>(s.gw + gw + 64);
    float* Zt = Psit + ml2;
    // Gaussian Omega (n x l1) and Psi (m x l2)
    if (o.omega)
        launch_relayout<double, double>(o.omega, 1, s.Om, 1, n * l1, 1, st);
    else
        launch_philox_normal(o.seed, static_cast<size_t>(n) * l1, s.Om, st);
    if (o.psi)
        launch_relayout<double, double>(o.psi, 1, Psi, 1, m * l2, 1, st);
    else
        launch_philox_normal(singleview_psi_seed(o.seed), ml2, Psi, st);
    // co-range sketch Z = A^T Psi beside the range sketch Y = A Omega
    auto corange = [&]() {
        hipStream_t zs = stream_of(p);
        if (f64) {
            adj_impl<double>(p, tr, l2, Psi, Z, nullptr);
        } else {
            launch_relayout<double, float>(Psi, l2, Psit, l2, m, l2, zs);
            adj_impl<float>(p, tr, l2, Psit, Zt, nullptr);
            launch_relayout<float, double>(Zt, l2, Z, l2, n, l2, zs);
        }
    };
    const bool lane = !o.serial && p->bve == nullptr;
    if (lane)
        on_side_lane(p, corange);
    else
        corange();
    if (f64) {
        tlm_impl<double>(p, tr, l1, s.Om, s.Yd);
    } else {
        launch_relayout<double, float>(s.Om, l1, static_cast<float*>(s.Omt), l1, n, l1, st);
        tlm_impl<float>(p, tr, l1, static_cast<const float*>(s.Omt), static_cast<float*>(s.Yt));
        launch_relayout<float, double>(static_cast<const float*>(s.Yt), l1, s.Yd, l1, m, l1, st);
    }
    cholqr2(p, m, l1, s);                                                        // Y = Q_Y R_Y
    launch_gram<double, double>(Psi, l2, s.Yd, l1, m, l2, l1, Mb, s.gw, st);   // M = Psi^T Q_Y
    launch_relayout<double, double>(Mb, 1, s.Yd, 1, l2 * l1, 1, st);
    cholqr2(p, l2, l1, s, Rinv);                                                 // M = Q_M R_M
    transpose_small<<<nblk(static_cast<long>(l1) * l1), 256, 0, st>>>(Rinv, s.S4, l1);  // S4 = R_M^{-T}
    RP4D_HIP(hipGetLastError());
    launch_tsmm<double, double>(s.Yd, l1, s.S4, nullptr, l2, l1, l1, 1.0, nullptr, 0, 0.0, P, l1, st);
    if (lane) RP4D_HIP(hipStreamWaitEvent(st, p->ctx->ev_join, 0));
    // W^T = Z Q_M R_M^{-T} (n x l1); thin SVD of W by eig(W W^T)
    launch_tsmm<double, double>(Z, l2, P, nullptr, n, l2, l1, 1.0, nullptr, 0, 0.0, s.S1, l1, st);
    launch_gram<double, double>(s.S1, l1, s.S1, l1, n, l1, l1, s.S2, s.gw, st);
    {
        KernelTimer kt(p->ctx, RP4D_K_EIG, 0.0);
        launch_jacobi_eig(s.S2, s.ev, s.S3, l1, st);
    }
    sketch_finalize<<<1, 128, 0, st>>>(s.ev, nullptr, 0.0, l1, s.lam, s.D, s.cs);
    RP4D_HIP(hipGetLastError());
    scale_cols<<<nblk(static_cast<long>(l1) * l1), 256, 0, st>>>(s.S3, l1, s.cs);
    pc->V.ensure(static_cast<size_t>(n) * l1 * sizeof(double));
    launch_tsmm<double, double>(s.S1, l1, s.S3, nullptr, n, l1, l1, 1.0, nullptr, 0, 0.0, pc->V.as<double>(), l1, st);
    launch_fill<double>(s.nu, 1, 0.0, st);
    pc->p = p;
    pc->ell = l1;
    pc->host_ok = false;
    pc->Dg.ensure(static_cast<size_t>(l1) * sizeof(double));
    launch_relayout<double, double>(s.D, 1, pc->Dg.as<double>(), 1, l1, 1, st);
    pc->lamd.ensure(static_cast<size_t>(l1 + 1) * sizeof(double));
    launch_relayout<double, double>(s.lam, 1, pc->lamd.as<double>(), 1, l1, 1, st);
    launch_relayout<double, double>(s.nu, 1, pc->lamd.as<double>() + l1, 1, 1, 1, st);
    p->cnt.tlm_offline += l1;
    p->cnt.adj_offline += l2;
    p->cnt.sketches += 1;
}

// Largest co-range sketch of an adaptive SingleView run: the initial l2 plus
// l2_hat for every extension that fits within l1_max.
int sv_adaptive_l2max(const rp4d_sv_adaptive_opts& o) {
    return o.ell2 + o.ell2_hat * ((o.ell1_max - o.ell1) / o.ell1_hat);
}

void check_sv_adaptive_opts(const rp4d_problem* p, rp4d_sv_adaptive_opts& o) {
    if (o.ell2 == 0) o.ell2 = std::min(2 * o.ell1 + 1, p->m);
    if (o.ell2_hat == 0) o.ell2_hat = 2 * o.ell1_hat;
    RP4D_REQUIRE(o.ell1 >= 1 && o.ell1_hat >= 1 && o.ell1_max >= o.ell1 && o.ell1_max <= 128 &&
                     o.ell1_max <= p->n && o.ell1_max <= p->m,
                 RP4D_EINVAL, "adaptive SingleView: need 1 <= ell1 <= ell1_max <= min(128, n, m) and ell1_hat >= 1");
    RP4D_REQUIRE(o.ell2 >= o.ell1 && o.ell2_hat >= o.ell1_hat, RP4D_EINVAL,
                 "adaptive SingleView: need ell2 >= ell1 and ell2_hat >= ell1_hat");
    RP4D_REQUIRE(sv_adaptive_l2max(o) <= p->m, RP4D_EINVAL,
                 "adaptive SingleView: the largest co-range sketch exceeds the number of observations");
    RP4D_REQUIRE(o.eps_sk > 0 && std::isfinite(o.eps_sk), RP4D_EINVAL, "adaptive sketch: eps_sk must be positive");
    RP4D_REQUIRE(!o.qr_update || o.ell1_max + o.ell2_hat <= std::max(p->n, p->m), RP4D_EINVAL,
                 "adaptive SingleView: the QR update needs ell1_max + ell2_hat <= max(n, m)");
}

// Thin QR of M = Psi^T Q_Y kept across the rounds of the adaptive SingleView.
// The first round factors M by Cholesky QR2.  Later rounds follow Alg. 6 with
// A1 = Psi^T, A2 = Psi_hat^T, B1 = Q_Y (c1o old columns), B2 = Q_hat (b1 new
// columns) and Q1 R1 = A1 B1 the previous factors.  Its first two thin QRs are
// taken together, as the thin QR of [R1; A2 B1]: Alg. 6 first factors
// A2 B1 = Q2 R2, which changes the Q factor of the stack by diag(I, Q2) only,
// and A2 B1 is wider than tall whenever b2 < c1o.  Then Q3 = diag(Q1, I) Q3',
// P1 = [A1; A2] B2, P2 = P1 - Q3 (Q3^T P1) = Q4 R4, Q5 = [Q3 Q4] and
// R5 = [R3, Q3^T P1; 0, R4].  Q_M (c2 x c1) and R_M (c1 x c1) stay in Qm, Rm
// with leading size L1; R4 and P1 are scratch.
void sv_qr_update(rp4d_problem* p, Scratch& s, int m, int c1o, int c2o, int b1, int b2, int L1, int L2,
                  const double* Pa, const double* Ph, const double* Qa, double* X, double* Qm, double* Rm,
                  double* Qt, double* Tt, double* Rs, double* R4, double* P1, double* gwk) {
    hipStream_t st = stream_of(p);
    const int c1 = c1o + b1, c2 = c2o + b2;
    if (c1o == 0) {
        launch_gram<double, double>(Pa, L2, Qa, L1, m, c2, c1, X, gwk, st);     // M (c2 x c1)
        launch_relayout<double, double>(X, 1, s.Yd, 1, c2 * c1, 1, st);
        cholqr2(p, c2, c1, s, nullptr, Rs);
        launch_relayout<double, double>(s.Yd, c1, Qm, L1, c2, c1, st);
        launch_relayout<double, double>(Rs, c1, Rm, L1, c1, c1, st);
        return;
    }
    // [R1; A2 B1] ((c1o + b2) x c1o) = Q3' R3
    launch_gram<double, double>(Ph, b2, Qa, L1, m, b2, c1o, X, gwk, st);         // A2 B1 (b2 x c1o)
    launch_relayout<double, double>(Rm, L1, s.Yd, c1o, c1o, c1o, st);
    launch_relayout<double, double>(X, c1o, s.Yd + static_cast<size_t>(c1o) * c1o, c1o, b2, c1o, st);
    cholqr2(p, c1o + b2, c1o, s, nullptr, Rs);                                    // s.Yd = Q3', Rs = R3
    // Q3 = diag(Q1, I) Q3' (c2 x c1o)
    launch_tsmm<double, double>(Qm, L1, s.Yd, nullptr, c2o, c1o, c1o, 1.0, nullptr, 0, 0.0, Qt, L1, st);
    launch_relayout<double, double>(s.Yd + static_cast<size_t>(c1o) * c1o, c1o, Qt + static_cast<size_t>(c2o) * L1,
                                    L1, b2, c1o, st);
    // P1 = [A1; A2] B2 (c2 x b1), T = Q3^T P1, P2 = P1 - Q3 T = Q4 R4
    launch_gram<double, double>(Pa, L2, Qa + c1o, L1, m, c2, b1, P1, gwk, st);
    launch_gram<double, double>(Qt, L1, P1, b1, c2, c1o, b1, Tt, gwk, st);
    launch_tsmm<double, double>(Qt, L1, Tt, nullptr, c2, c1o, b1, -1.0, P1, b1, 1.0, P1, b1, st);
    launch_relayout<double, double>(P1, 1, s.Yd, 1, c2 * b1, 1, st);
    cholqr2(p, c2, b1, s, nullptr, R4);                                           // s.Yd = Q4
    // Q5 = [Q3 Q4], R5 = [R3, T; 0, R4]
    launch_relayout<double, double>(Qt, L1, Qm, L1, c2, c1o, st);
    launch_relayout<double, double>(s.Yd, b1, Qm + c1o, L1, c2, b1, st);
    launch_fill<double>(Rm + static_cast<size_t>(c1o) * L1, static_cast<size_t>(b1) * L1, 0.0, st);
    launch_relayout<double, double>(Rs, c1o, Rm, L1, c1o, c1o, st);
    launch_relayout<double, double>(Tt, b1, Rm + c1o, L1, c1o, b1, st);
    launch_relayout<double, double>(R4, b1, Rm + static_cast<size_t>(c1o) * L1 + c1o, L1, b1, b1, st);
}

// Adaptive SingleView (Sec. 3.1.2, Alg. 5) into pc.  Each round draws
// Omega_hat (n x b1) and Psi_hat (m x b2); Z_hat = A^T Psi_hat runs on the side
// stream (1-D model) beside Y_hat = A Omega_hat, which is orthogonalised twice
// against the accumulated Q_Y and factored by Cholesky QR.  Q_Y (m x c1),
// Psi (m x c2) and Z (n x c2) grow by the new blocks; M = Psi^T Q_Y is
// refactored by Cholesky QR2 (its QR from scratch, which the algorithm allows
// beside the update of Alg. 6) and W^T = Z Q_M R_M^{-T} (n x c1) is formed
// anew; kappa_sk (eq. (condtext)) decides whether to extend.  FP64.
void build_singleview_adaptive(rp4d_problem* p, const rp4d_traj* tr, const rp4d_sv_adaptive_opts& o,
                               rp4d_precond* pc, rp4d_adaptive_info* info) {
    hipStream_t st = stream_of(p);
    const int n = p->n, m = p->m, L1 = o.ell1_max, L2 = sv_adaptive_l2max(o);
    const int B2 = std::max(o.ell2, o.ell2_hat);
    Scratch s = sketch_scratch(p, L1, RP4D_F64);
    const size_t ll = static_cast<size_t>(L1) * L1, l21 = static_cast<size_t>(L2) * L1;
    const size_t gw = std::max({gram_work_doubles(m, L2, L1), gram_work_doubles(m, L1, L1),
                                gram_work_doubles(n, L1, L1), gram_work_doubles(L2, L1, L1),
                                gram_work_doubles(n, L1, 1)});
    const size_t mL1 = static_cast<size_t>(m) * L1, nL1 = static_cast<size_t>(n) * L1;
    const size_t mL2 = static_cast<size_t>(m) * L2, nL2 = static_cast<size_t>(n) * L2;
    const size_t mB2 = static_cast<size_t>(m) * B2, nB2 = static_cast<size_t>(n) * B2;
    p->ws_ad.ensure((mL1 + mL2 + nL2 + mB2 + nB2 + 4 * l21 + 7 * ll + nL1 + 3 * static_cast<size_t>(n) + 1024 +
                     4 * static_cast<size_t>(L1) + gw + 64) * sizeof(double));
    double* Qa = p->ws_ad.as<double>();  // m x L1: Q_Y
    double* Pa = Qa + mL1;               // m x L2: Psi
    double* Za = Pa + mL2;               // n x L2: Z
    double* Ph = Za + nL2;               // m x B2: Psi_hat
    double* Zh = Ph + mB2;               // n x B2: Z_hat
    double* Mb = Zh + nB2;               // L2 x L1
    double* P = Mb + l21;                // L2 x L1: Q_M R_M^{-T}
    double* Rinv = P + l21;              // L1 x L1
    double* Wt = Rinv + ll;              // n x L1: W^T
    KappaWork kw{};
    kw.G = Wt + nL1;
    kw.Gi = kw.G + ll;
    kw.Gt = kw.Gi + ll;
    kw.vu = kw.Gt + ll;
    kw.u = kw.vu + n;
    kw.q = kw.u + n;
    kw.red = kw.q + n;
    kw.tv = kw.red + 1024;
    kw.zv = kw.tv + L1;
    kw.gw = kw.zv + 2 * L1;
    s.gw = kw.gw;
    // QR update (Alg. 6) state: Q_M (L2 x L1) and R_M (L1 x L1), leading size L1
    double* Qm = kw.gw + gw + 64;
    double* Rm = Qm + l21;
    double* Qt = Rm + ll;                // L2 x L1: Q3
    double* Tt = Qt + l21;               // L1 x L1: Q3^T P1
    double* Rs = Tt + ll;                // L1 x L1: R from Cholesky QR
    kappa_test_vector(p, o.vtest, adaptive_vseed(o.seed), kw);
    const bool lane = !o.serial && p->bve == nullptr;
    int c1 = 0, c2 = 0, r = 0, nk = 0;
    double kappa = 0.0;
    for (;;) {
        const int b1 = r == 0 ? o.ell1 : o.ell1_hat;
        const int b2 = r == 0 ? o.ell2 : o.ell2_hat;
        // new test blocks
        if (o.omega)
            launch_relayout<double, double>(o.omega + c1, L1, s.Om, b1, n, b1, st);
        else
            launch_philox_normal(adaptive_seed(o.seed, r), static_cast<size_t>(n) * b1, s.Om, st);
        if (o.psi)
            launch_relayout<double, double>(o.psi + c2, L2, Ph, b2, m, b2, st);
        else
            launch_philox_normal(adaptive_seed(singleview_psi_seed(o.seed), r), static_cast<size_t>(m) * b2, Ph, st);
        launch_relayout<double, double>(Ph, b2, Pa + c2, L2, m, b2, st);
        // Z_hat = A^T Psi_hat (appended to Z) beside Y_hat = A Omega_hat
        const int zc = c2;
        auto corange = [&]() {
            adj_impl<double>(p, tr, b2, Ph, Zh, nullptr);
            launch_relayout<double, double>(Zh, b2, Za + zc, L2, n, b2, stream_of(p));
        };
        if (lane)
            on_side_lane(p, corange);
        else
            corange();
        tlm_impl<double>(p, tr, b1, s.Om, s.Yd);
        for (int pass = 0; c1 > 0 && pass < 2; ++pass) {                  // Y <- Y - Q_Y (Q_Y^T Y)
            launch_gram<double, double>(Qa, L1, s.Yd, b1, m, c1, b1, kw.Gt, kw.gw, st);
            launch_tsmm<double, double>(Qa, L1, kw.Gt, nullptr, m, c1, b1, -1.0, s.Yd, b1, 1.0, s.Yd, b1, st);
        }
        cholqr2(p, m, b1, s);                                              // Y = Q_hat R
        launch_relayout<double, double>(s.Yd, b1, Qa + c1, L1, m, b1, st);
        c1 += b1;
        c2 += b2;
        ++r;
        p->cnt.tlm_offline += b1;
        p->cnt.adj_offline += b2;
        // M = Psi^T Q_Y = Q_M R_M (c2 x c1), P = Q_M R_M^{-T}
        if (!o.qr_update) {
            launch_gram<double, double>(Pa, L2, Qa, L1, m, c2, c1, Mb, kw.gw, st);
            launch_relayout<double, double>(Mb, 1, s.Yd, 1, c2 * c1, 1, st);
            cholqr2(p, c2, c1, s, Rinv);
            transpose_small<<<nblk(static_cast<long>(c1) * c1), 256, 0, st>>>(Rinv, s.S4, c1);
            RP4D_HIP(hipGetLastError());
            launch_tsmm<double, double>(s.Yd, c1, s.S4, nullptr, c2, c1, c1, 1.0, nullptr, 0, 0.0, P, c1, st);
        } else {
            sv_qr_update(p, s, m, c1 - b1, c2 - b2, b1, b2, L1, L2, Pa, Ph, Qa, Mb, Qm, Rm, Qt, Tt, Rs, Rinv, P, kw.gw);
            // P = Q_M R_M^{-T}: R_M^T is lower triangular and its inverse is R_M^{-T}
            launch_relayout<double, double>(Rm, L1, Rs, c1, c1, c1, st);
            transpose_small<<<nblk(static_cast<long>(c1) * c1), 256, 0, st>>>(Rs, s.S2, c1);
            RP4D_HIP(hipGetLastError());
            launch_trinv(s.S2, s.S4, c1, st);
            launch_tsmm<double, double>(Qm, L1, s.S4, nullptr, c2, c1, c1, 1.0, nullptr, 0, 0.0, P, c1, st);
        }
        if (lane) RP4D_HIP(hipStreamWaitEvent(st, p->ctx->ev_join, 0));
        // W^T = Z Q_M R_M^{-T} (n x c1)
        launch_tsmm<double, double>(Za, L2, P, nullptr, n, c2, c1, 1.0, nullptr, 0, 0.0, Wt, L1, st);
        kappa = kappa_sk_dev(p, tr, Wt, L1, c1, kw, s.info);
        if (info && nk < 16) info->kappa[nk] = kappa;
        ++nk;
        if (kappa <= o.eps_sk || c1 + o.ell1_hat > L1) break;
    }
    // thin SVD of W: W W^T = U Sigma^2 U^T, V_hat = W^T U Sigma^{-1}, Lambda = Sigma^2
    launch_gram<double, double>(Wt, L1, Wt, L1, n, c1, c1, kw.G, kw.gw, st);
    {
        KernelTimer kt(p->ctx, RP4D_K_EIG, 0.0);
        launch_jacobi_eig(kw.G, s.ev, kw.Gi, c1, st);
    }
    sketch_finalize<<<1, 128, 0, st>>>(s.ev, nullptr, 0.0, c1, s.lam, s.D, s.cs);
    RP4D_HIP(hipGetLastError());
    scale_cols<<<nblk(static_cast<long>(c1) * c1), 256, 0, st>>>(kw.Gi, c1, s.cs);
    pc->V.ensure(static_cast<size_t>(n) * c1 * sizeof(double));
    launch_tsmm<double, double>(Wt, L1, kw.Gi, nullptr, n, c1, c1, 1.0, nullptr, 0, 0.0, pc->V.as<double>(), c1, st);
    launch_fill<double>(s.nu, 1, 0.0, st);
    pc->p = p;
    pc->ell = c1;
    pc->host_ok = false;
    pc->Dg.ensure(static_cast<size_t>(c1) * sizeof(double));
    launch_relayout<double, double>(s.D, 1, pc->Dg.as<double>(), 1, c1, 1, st);
    pc->lamd.ensure(static_cast<size_t>(c1 + 1) * sizeof(double));
    launch_relayout<double, double>(s.lam, 1, pc->lamd.as<double>(), 1, c1, 1, st);
    launch_relayout<double, double>(s.nu, 1, pc->lamd.as<double>() + c1, 1, 1, 1, st);
    p->cnt.sketches += 1;
    if (info) {
        info->ell = c1;
        info->nkappa = nk;
        info->kappa_sk = kappa;
    }
}

// Capture the work `f` enqueues on the context stream into an executable graph
// (recorded on a library-owned stream; nothing runs during capture).
struct GraphExec {
    hipGraphExec_t ex = nullptr;
    GraphExec() = default;
    GraphExec(const GraphExec&) = delete;
    GraphExec& operator=(const GraphExec&) = delete;
    void reset() {
        if (ex) (void)hipGraphExecDestroy(ex);
        ex = nullptr;
    }
    ~GraphExec() { reset(); }
};

template <typename F>
void capture(rp4d_ctx* c, F&& f, GraphExec& out, bool instantiate = true) {
    if (!c->cap_stream) RP4D_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t orig = c->stream;
    RP4D_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    c->stream = c->cap_stream;
    c->capturing = true;
    hipGraph_t g = nullptr;
    try {
        f();
    } catch (...) {
        (void)hipStreamEndCapture(c->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        c->stream = orig;
        c->capturing = false;
        throw;
    }
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = orig;
    c->capturing = false;
    RP4D_HIP(e);
    if (!instantiate) {
        (void)hipGraphDestroy(g);
        return;
    }
    const hipError_t e2 = hipGraphInstantiate(&out.ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    RP4D_HIP(e2);
}

// snap (host, SC_COUNT doubles, nullable) receives the whole scalar block at the
// first read, so that callers get values they enqueued earlier without a wait
// of their own.
void pcg_impl(rp4d_problem* p, const rp4d_traj* tr, const rp4d_precond* pc, const double* b, double* x,
              double rtol, int maxit, rp4d_pcg_info* info, bool true_res, rp4d::DevBuf& vecs,
              double* snap = nullptr) {
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
    // One iteration: q = (I+H)p, alpha, x, r, |r|^2, then speculatively z = P r,
    // beta and the next p (unused once |r| meets the tolerance).  The stream is
    // read at each launch so that the same body can be captured into a graph.
    auto body = [&]() {
        hessian_dispatch(p, tr, 1, pv, q, RP4D_F64, true);
        hipStream_t s = stream_of(p);
        launch_dot(pv, q, n, sc + SC_PQ, red, s);
        pcg_update_xr<<<nblk(n), 256, 0, s>>>(x, r, pv, q, sc, n);
        RP4D_HIP(hipGetLastError());
        launch_dot(r, r, n, sc + SC_RR, red, s);
        if (pc)
            precond_apply_impl(p, pc, 1, r, z);
        else
            launch_relayout<double, double>(r, 1, z, 1, n, 1, s);
        launch_dot(r, z, n, sc + SC_RZN, red, s);
        pcg_update_p<<<nblk(n), 256, 0, s>>>(pv, z, sc, n);
        RP4D_HIP(hipGetLastError());
        scal_copy<<<1, 1, 0, s>>>(sc, SC_RZ, SC_RZN);
        RP4D_HIP(hipGetLastError());
    };
    // The first iteration is enqueued before |b| reaches the host, so that one
    // wait returns |b|, the first residual and (with snap) the caller's scalars.
    // With b = 0 its output is discarded: x = 0 after no iteration.
    body();
    double hs[SC_COUNT];
    double* h = snap ? snap : hs;
    RP4D_HIP(hipMemcpyAsync(h, sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(p);
    const double bnorm = std::sqrt(h[SC_BB]);
    RP4D_REQUIRE(!snap || std::isfinite(snap[SC_DD]), RP4D_ENONFINITE,
                 "non-finite innovations (state blew up or bad input)");
    RP4D_REQUIRE(!snap || std::isfinite(snap[SC_GI]), RP4D_ENONFINITE, "non-finite gradient");
    RP4D_REQUIRE(std::isfinite(bnorm), RP4D_ENONFINITE, "non-finite right-hand side");
    double rnorm = bnorm;
    int it = 0;
    bool conv = true;
    if (bnorm == 0.0 || bnorm <= rtol * bnorm) {
        // b = 0, or rtol >= 1: x_0 = 0 already meets the tolerance, and the
        // speculative first iteration is discarded
        launch_fill<double>(x, n, 0.0, st);
        p->cnt.hv_columns -= 1;
    } else {
        it = 1;
        rnorm = std::sqrt(h[SC_RR]);
        RP4D_REQUIRE(std::isfinite(rnorm), RP4D_ENONFINITE, "non-finite PCG residual");
        conv = rnorm <= rtol * bnorm;
    }
    // Long solves replay the body as a graph from the third iteration on (the
    // first two run eagerly and size every workspace the body touches).
    GraphExec gx;
    while (!conv && it < maxit) {
        if (p->ctx->graphs && it >= 2) {
            if (!gx.ex) {
                const long long hv = p->cnt.hv_columns;
                capture(p->ctx, body, gx);
                p->cnt.hv_columns = hv;
            }
            RP4D_HIP(hipGraphLaunch(gx.ex, st));
            p->cnt.hv_columns += 1;
        } else {
            body();
        }
        ++it;
        rnorm = std::sqrt(read_scalar(p, sc + SC_RR));
        RP4D_REQUIRE(std::isfinite(rnorm), RP4D_ENONFINITE, "non-finite PCG residual");
        if (rnorm <= rtol * bnorm) conv = true;
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
    // normalise v on the device (|v|^2 in SC_T0), then |(I + H) P v_hat|^2 in SC_T1
    launch_dot(v, v, n, sc + SC_T0, red, st);
    double* vu = q + n;
    scale_inv_sqrt<<<nblk(n), 256, 0, st>>>(v, sc + SC_T0, vu, n);
    RP4D_HIP(hipGetLastError());
    precond_apply_impl(p, pc, 1, vu, z);
    hessian_dispatch(p, tr, 1, z, q, RP4D_F64, true);
    launch_dot(q, q, n, sc + SC_T1, red, st);
    double h[2];
    RP4D_HIP(hipMemcpyAsync(h, sc + SC_T0, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(p);
    RP4D_REQUIRE(h[0] > 0 && std::isfinite(h[0]), RP4D_EINVAL, "kappa_re: zero or non-finite test vector");
    return std::sqrt(h[1]);
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
        quiesce_device(s->device);
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

int rp4d_build_precond_singleview(rp4d_problem* p, const rp4d_traj* tr, const rp4d_singleview_opts* o,
                                  rp4d_precond** out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && o != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        check_traj(p, tr);
        rp4d_singleview_opts so = *o;
        check_singleview_opts(p, so);
        set_device(p->ctx);
        auto* pc = new rp4d_precond();
        try {
            build_singleview(p, tr, so, pc);
            fetch_host(pc);
        } catch (...) {
            delete pc;
            throw;
        }
        *out = pc;
    });
}

int rp4d_build_precond_singleview_adaptive(rp4d_problem* p, const rp4d_traj* tr, const rp4d_sv_adaptive_opts* o,
                                           rp4d_precond** out, rp4d_adaptive_info* info) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && o != nullptr && out != nullptr, RP4D_EINVAL, "null argument");
        check_traj(p, tr);
        rp4d_sv_adaptive_opts so = *o;
        check_sv_adaptive_opts(p, so);
        set_device(p->ctx);
        auto* pc = new rp4d_precond();
        try {
            build_singleview_adaptive(p, tr, so, pc, info);
            fetch_host(pc);
        } catch (...) {
            delete pc;
            throw;
        }
        *out = pc;
    });
}

constexpr double kArmijoC = 1e-4;
constexpr int kArmijoTrials = 20;

int rp4d_gn_step(rp4d_problem* p, rp4d_gn_state* s, const rp4d_gn_opts* o, rp4d_gn_info* info) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && s != nullptr && o != nullptr && s->p == p, RP4D_EINVAL, "bad argument");
        RP4D_REQUIRE(o->sketch == RP4D_NYSTROM || o->sketch == RP4D_RANDSVD || o->sketch == RP4D_NOPREC ||
                         o->sketch == RP4D_RANDSVD_ADAPTIVE || o->sketch == RP4D_SINGLEVIEW ||
                         o->sketch == RP4D_SINGLEVIEW_ADAPTIVE || o->sketch == RP4D_NYSTROM_ADAPTIVE,
                     RP4D_EINVAL, "unknown sketch method");
        RP4D_REQUIRE(o->solve == RP4D_SOLVE_PCG || (o->solve == RP4D_SOLVE_SKETCH && o->sketch != RP4D_NOPREC),
                     RP4D_EINVAL, "solve must be RP4D_SOLVE_PCG, or RP4D_SOLVE_SKETCH with a sketch");
        rp4d_sv_adaptive_opts sao{};
        if (o->sketch == RP4D_SINGLEVIEW_ADAPTIVE) {
            sao = rp4d_sv_adaptive_opts{o->ell, o->ell2, o->ell_hat, o->ell2_hat, o->ell_max, o->eps_sk, o->seed,
                                        o->omega, o->psi, o->vhat, 0};
            check_sv_adaptive_opts(p, sao);
        }
        rp4d_adaptive_opts ao{};
        if (o->sketch == RP4D_RANDSVD_ADAPTIVE || o->sketch == RP4D_NYSTROM_ADAPTIVE) {
            ao = rp4d_adaptive_opts{o->ell, o->ell_hat, o->ell_max, o->eps_sk, o->seed, o->omega, o->vhat};
            check_adaptive_opts(p, ao);
        }
        rp4d_singleview_opts so{};
        if (o->sketch == RP4D_SINGLEVIEW) {
            so = rp4d_singleview_opts{o->ell, o->ell2, o->seed, o->omega, o->psi, o->sketch_dtype, 0};
            check_singleview_opts(p, so);
        }
        set_device(p->ctx);
        hipStream_t st = stream_of(p);
        const int n = p->n;
        double* sc = p->ws_scal.as<double>();
        rp4d::DevBuf& vecs = pcg_buf(p);
        vecs.ensure(5 * static_cast<size_t>(n) * sizeof(double) + 1024 * sizeof(double));
        double* red = vecs.as<double>() + 5 * static_cast<size_t>(n);
        // 2-3. gradient g = v + A^T d and b = -g.  The 1-D model runs them on the
        // side stream with the side workspaces, overlapping the sketch below.
        const bool overlap = p->bve == nullptr;
        auto gradient = [&]() {
            hipStream_t gs = stream_of(p);
            adj_impl<double>(p, s->traj, 1, s->traj->innov.as<double>(), s->g.as<double>(), s->v.as<double>());
            absmax_kernel<<<1, 256, 0, gs>>>(s->g.as<double>(), n, sc + SC_GI);
            RP4D_HIP(hipGetLastError());
            launch_fill<double>(s->b.as<double>(), n, 0.0, gs);
            launch_axpby(s->g.as<double>(), -1.0, s->b.as<double>(), 0.0, n, gs);
        };
        // 1. FWD at x; |d|^2 and |v|^2 stay on the device until the join below.
        // With a Nystrom or RandSVD sketch on the 1-D model (every row stored)
        // the FWD runs on the side stream and the sketch's TLM sweep on the main
        // stream follows it: the TLM's host loop enqueues the FWD launches a few
        // launches ahead of its own and waits for their rows by events, so the
        // two overlap on the device; the ADJ sweep waits for the last row.  The
        // dot products of the cost and the gradient follow the FWD on the side
        // stream, enqueued once the TLM has been.
        const bool pipelined = overlap && s->traj->C == 1 &&
                               (o->sketch == RP4D_NYSTROM || o->sketch == RP4D_RANDSVD ||
                                o->sketch == RP4D_NYSTROM_ADAPTIVE || o->sketch == RP4D_RANDSVD_ADAPTIVE);
        struct PipeGuard {  // on any exit: no pending hook or plan, and the main stream after the side's work
            rp4d_problem* p;
            bool on = false;
            ~PipeGuard() {
                if (!on) return;
                p->after_tlm = nullptr;
                FwdPlan& f = p->fwd_plan;
                if (f.active && f.s_next < f.s_to) f.tr->valid = false;  // left unfinished
                if (f.span) p->ctx->event_pool.push_back(f.span);       // timing span never closed
                f.span = nullptr;
                f.active = false;
                // join everything enqueued on the side stream so far: planned FWD
                // launches enqueued after on_side_lane recorded ev_join must not
                // outlive the step (a later main-stream FWD reuses the trajectory)
                rp4d_ctx* c = p->ctx;
                if (c->side) (void)hipEventRecord(c->ev_join, c->side);
                (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
            }
        } guard{p};
        if (pipelined) {
            on_side_lane(p, [&]() { fwd_plan_start(p, s->x.as<double>(), s->traj); });
            guard.on = true;
            RP4D_REQUIRE(s->traj->has_innov, RP4D_ESTATE, "data not set");
            p->after_tlm = [&]() {
                continue_on_side(p, [&]() {
                    hipStream_t fs = stream_of(p);
                    fwd_plan_finish(p);
                    double* fred = p->ws_red.as<double>() + 2 * static_cast<size_t>(n);  // sized by the plan
                    launch_dot(s->traj->innov.as<double>(), s->traj->innov.as<double>(), p->m, sc + SC_DD, fred, fs);
                    launch_dot(s->v.as<double>(), s->v.as<double>(), n, sc + SC_VV, fred, fs);
                    gradient();
                });
            };
        } else {
            int rc = rp4d_fwd(p, s->x.as<double>(), s->traj, nullptr);
            RP4D_REQUIRE(rc == RP4D_OK, rc, g_last_error);
            RP4D_REQUIRE(s->traj->has_innov, RP4D_ESTATE, "data not set");
            launch_dot(s->traj->innov.as<double>(), s->traj->innov.as<double>(), p->m, sc + SC_DD, red, st);
            launch_dot(s->v.as<double>(), s->v.as<double>(), n, sc + SC_VV, red, st);
            if (overlap) {
                on_side_lane(p, gradient);
            } else {
                gradient();
            }
        }
        p->cnt.adj_online += 1;
        rp4d_gn_info inf{};
        inf.kappa_re = -1.0;
        inf.kappa_sk = -1.0;
        // 4-5. reuse test or sketch
        const rp4d_precond* use = nullptr;
        if (o->sketch != RP4D_NOPREC) {
            if (s->pc_live && o->reuse_eps > 0) {
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
                // rebuild in place: the object and its device buffers persist
                s->pc_live = false;
                if (!s->pc) s->pc = new rp4d_precond();
                s->pc->fast = false;
                if (o->sketch == RP4D_RANDSVD_ADAPTIVE) {
                    rp4d_adaptive_info ai{};
                    build_randsvd_adaptive(p, s->traj, ao, s->pc, &ai);
                    inf.kappa_sk = ai.kappa_sk;
                } else if (o->sketch == RP4D_NYSTROM_ADAPTIVE) {
                    rp4d_adaptive_info ai{};
                    build_nystrom_adaptive(p, s->traj, ao, s->pc, &ai);
                    inf.kappa_sk = ai.kappa_sk;
                } else if (o->sketch == RP4D_SINGLEVIEW) {
                    build_singleview(p, s->traj, so, s->pc);
                } else if (o->sketch == RP4D_SINGLEVIEW_ADAPTIVE) {
                    rp4d_adaptive_info ai{};
                    build_singleview_adaptive(p, s->traj, sao, s->pc, &ai);
                    inf.kappa_sk = ai.kappa_sk;
                } else {
                    // SketchPrec only needs the operator: the factored form unless the
                    // eigendecomposition is asked for; SketchSolv keeps Alg. 1/2's form
                    const bool fast = o->solve == RP4D_SOLVE_PCG && !o->exact_lmp;
                    build_precond_into(p, s->traj, o->sketch, o->ell, o->seed, o->omega, o->sketch_dtype, s->pc,
                                       fast);
                }
                s->pc_live = true;
                use = s->pc;
                inf.sketched = 1;
            }
        }
        // join the gradient; J and |g|_inf arrive with PCG's first scalar read
        if (p->after_tlm) {  // no TLM sweep ran on the main stream
            auto f = std::move(p->after_tlm);
            p->after_tlm = nullptr;
            f();
        }
        if (overlap) RP4D_HIP(hipStreamWaitEvent(st, p->ctx->ev_join, 0));
        p->fwd_plan.active = false;
        guard.on = false;
        double sch[SC_COUNT];
        // 6. direction: PCG (SketchPrec) or one application of eq. (woodbury)
        // (SketchSolv, eq. (dxsol) in the v-form: dv = (I + H_hat)^{-1} b)
        rp4d_pcg_info pi{};
        int pcg_rc = RP4D_OK;
        if (o->solve == RP4D_SOLVE_SKETCH) {
            precond_apply_impl(p, use, 1, s->b.as<double>(), s->dv.as<double>());
            RP4D_HIP(hipMemcpyAsync(sch, sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
            sync(p);
            RP4D_REQUIRE(std::isfinite(sch[SC_GI]), RP4D_ENONFINITE, "non-finite gradient");
            pi.converged = 1;
            pi.relres = -1.0;
        } else {
            try {
                pcg_impl(p, s->traj, use, s->b.as<double>(), s->dv.as<double>(), o->rtol, o->maxit, &pi, false,
                         vecs, sch);
            } catch (const Error& e) {
                if (e.code != RP4D_ENOCONV) throw;
                pcg_rc = e.code;
            }
        }
        inf.J = 0.5 * sch[SC_VV] + 0.5 * sch[SC_DD];
        inf.gnorm_inf = sch[SC_GI];
        inf.pcg_iters = pi.iters;
        inf.pcg_converged = pi.converged;
        inf.pcg_relres = pi.relres;
        inf.sketch_ell = use ? use->ell : 0;
        // 7. step length: alpha = 1, or Armijo backtracking on the v-form cost
        // J(v + alpha dv) <= J(v) + c alpha g.dv (c = 1e-4; alpha halved, at
        // most 20 trials, the last one taken if none passes; a trial whose state
        // blows up counts as failed).  Each trial is one FWD on the step's
        // trajectory; b and x serve as the trial v and x.
        double alpha = 1.0;
        int trials = 0;
        if (o->line_search) {
            double* vt = s->b.as<double>();
            double* xt = s->x.as<double>();
            launch_dot(s->g.as<double>(), s->dv.as<double>(), n, sc + SC_T2, red, st);
            const double slope = read_scalar(p, sc + SC_T2);
            for (trials = 1;; ++trials) {
                launch_relayout<double, double>(s->v.as<double>(), 1, vt, 1, n, 1, st);
                launch_axpby(s->dv.as<double>(), alpha, vt, 1.0, n, st);
                bhalf_into<double>(p, 1, vt, 1, xt, 1, p->xb.as<double>());
                double jo = 0.0;
                const int frc = rp4d_fwd(p, xt, s->traj, &jo);
                RP4D_REQUIRE(frc == RP4D_OK || frc == RP4D_ENONFINITE, frc, g_last_error);
                double J = std::numeric_limits<double>::infinity();
                if (frc == RP4D_OK) {
                    launch_dot(vt, vt, n, sc + SC_T2, red, st);
                    J = 0.5 * read_scalar(p, sc + SC_T2) + jo;
                }
                if (J <= inf.J + kArmijoC * alpha * slope || trials == kArmijoTrials) break;
                alpha *= 0.5;
            }
        }
        inf.alpha = alpha;
        inf.ls_trials = trials;
        // 8. v <- v + alpha dv ; x = x_b + Gamma^{1/2} v
        launch_axpby(s->dv.as<double>(), alpha, s->v.as<double>(), 1.0, n, st);
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
        s->pc_live = false;  // the object and its buffers stay for the next build
    });
}

int rp4d_problem_synthesize(rp4d_problem* p, const double* x_true, const double* xi, const double* eta,
                            double* xb_out, double* y_out) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr && x_true && xi && eta && xb_out && y_out, RP4D_EINVAL, "null argument");
        set_device(p->ctx);
        hipStream_t st = stream_of(p);
        bhalf_into<double>(p, 1, xi, 1, xb_out, 1, x_true);
        if (p->bve)
            bve_fwd(p, x_true, nullptr, nullptr, y_out);
        else
            run_fwd(p, x_true, 0, p->s_last, nullptr, 1, 0, 0, nullptr, y_out);
        launch_axpby(eta, p->d.sigma_o, y_out, 1.0, p->m, st);
    });
}

int rp4d_ctx_set_timing(rp4d_ctx* ctx, int enable) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr, RP4D_EINVAL, "null context");
        set_device(ctx);
        RP4D_REQUIRE(enable >= 0 && enable <= 2, RP4D_EINVAL, "timing mode must be 0, 1 or 2");
        resolve_timing(ctx);
        ctx->timing = enable;
        for (int i = 0; i < RP4D_K_COUNT; ++i) {
            ctx->launches[i] = 0;
            ctx->ms[i] = 0.0;
            ctx->flops[i] = 0.0;
        }
    });
}

int rp4d_ctx_set_graphs(rp4d_ctx* ctx, int enable) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr, RP4D_EINVAL, "null context");
        ctx->graphs = enable != 0;
    });
}

int rp4d_ctx_set_gram_precision(rp4d_ctx* ctx, int dtype) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr, RP4D_EINVAL, "null context");
        RP4D_REQUIRE(dtype == RP4D_F64 || dtype == RP4D_BF16, RP4D_EINVAL, "Gram precision: RP4D_F64 or RP4D_BF16");
        ctx->gram_dtype = dtype;
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
                          int steps, int xch) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr, RP4D_EINVAL, "null problem");
        RP4D_REQUIRE(mode == 0 || mode == MODE_TLM || mode == MODE_ADJ || mode == RP4D_MODE_FWD, RP4D_EINVAL,
                     "bad sweep mode");
        if (mode == RP4D_MODE_FWD) {
            dtype = RP4D_F64;
            k = 1;
            kc = 1;
        }
        Tiling t;
        t.ppt = ppt;
        t.kc = kc;
        t.threads = threads;
        t.tile = tile;
        t.steps = steps;
        t.xch = xch > 0 ? xch : 0;
        if (ppt <= 0 && kc <= 0 && threads <= 0 && tile <= 0 && steps <= 0 && xch <= 0)
            p->tiling.erase(std::make_tuple(mode, dtype, k));
        else
            p->tiling[std::make_tuple(mode, dtype, k)] = t;
    });
}

int rp4d_get_sweep_tiling(const rp4d_problem* p, int mode, int dtype, int k, int* ppt, int* kc, int* threads,
                          int* tile, int* steps, int* xch) {
    return guarded([&] {
        RP4D_REQUIRE(p != nullptr, RP4D_EINVAL, "null problem");
        Tiling t = mode == RP4D_MODE_FWD ? fwd_tiling(p) : tiling_for(p, mode == 0 ? MODE_TLM : mode, dtype, k > 0 ? k : 1);
        if (ppt) *ppt = t.ppt;
        if (kc) *kc = t.kc;
        if (threads) *threads = t.threads;
        if (tile) *tile = t.tile;
        if (steps) *steps = t.steps;
        if (xch) *xch = t.xch;
    });
}

}  // extern "C"

// ===========================================================================
// Batches: many independent Burgers problems advanced together.  Every phase
// is one launch (or one fused launch per time interval for the sweeps) over all
// problems; per-problem arguments travel as descriptor arrays staged through a
// pinned host ring.
// ===========================================================================
struct rp4d_batch {
    int device = rp4d::construction_device();
    rp4d_ctx* ctx = nullptr;
    std::vector<rp4d_problem*> probs;
    // staging ring: pinned host memory mirrored into device memory
    char* host = nullptr;
    rp4d::DevBuf dev;
    size_t cap = 0, off = 0;
    rp4d::DevBuf scal;  // 16 doubles per problem of batch scalars
    // [mode-1][dtype] overrides (ppt, kc, threads, steps, xch; <= 0: default)
    rp4d::Tiling bt[2][2] = {{{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}}, {{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}}};
    // [mode-1][dtype] overrides of the single-vector sweeps (gradient, PCG products)
    rp4d::Tiling bt1[2][2] = {{{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}}, {{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}}};
    rp4d::Tiling bt_fwd = {0, 0, 0, 0, 0, 0};  // forward-sweep overrides
    // Staging for graph capture of the lock-step PCG body (gmode != 0): instead
    // of the ring, tables go to offsets of a device arena.  gmode 1 sizes them
    // (the graph of that pass is discarded); gmode 2 records them in arena_host
    // at addresses in arena_dev, and they are copied there after the capture.
    int gmode = 0;
    std::vector<char> arena_host;
    rp4d::DevBuf arena_dev;
    size_t arena_off = 0;
    ~rp4d_batch() {
        if (host) (void)hipHostFree(host);
    }
};

namespace rp4d {
namespace {

// Descriptor tables are staged through a pinned host ring and its device copy
// (ring placement: batch_plan.hpp).  stage() places the tables that one set of
// launches reads as one group, enqueues their copies and returns their device
// addresses; the caller enqueues those launches before it stages anything
// else, so no table outlives the next group.
inline void ring_copy(rp4d_batch* b, size_t at, const void* src, size_t bytes) {
    if (bytes == 0) return;
    char* h = b->host + at;
    std::memcpy(h, src, bytes);
    RP4D_HIP(hipMemcpyAsync(b->dev.as<char>() + at, h, bytes, hipMemcpyHostToDevice, b->ctx->stream));
}

// Arena staging (graph capture): the tables of the body at consecutive
// offsets.  The sizing pass only advances the offset; the recording pass
// copies each table into arena_host at its offset and returns its address in
// arena_dev, which the sizing pass made large enough (tables may hold the
// addresses of tables staged before them, so they are built against the final
// arena).
inline char* arena_put(rp4d_batch* b, const void* src, size_t bytes, size_t rounded) {
    const size_t at = b->arena_off;
    b->arena_off += rounded;
    if (b->gmode == 2) {
        RP4D_REQUIRE(b->arena_off <= b->arena_dev.bytes, RP4D_ESTATE,
                     "batched PCG graph: the body staged more tables than on its sizing pass");
        if (b->arena_host.size() < b->arena_off) b->arena_host.resize(b->arena_off);
        if (bytes) std::memcpy(b->arena_host.data() + at, src, bytes);
    }
    return b->arena_dev.as<char>() + at;  // not valid on the sizing pass (that graph is discarded)
}

template <typename... V>
std::tuple<typename V::value_type*...> stage(rp4d_batch* b, const V&... v) {
    const size_t sizes[] = {ring_round(v.size() * sizeof(typename V::value_type))...};
    if (b->gmode != 0) {
        int q = 0;
        auto put = [&](const auto& vec) {
            typedef typename std::decay_t<decltype(vec)>::value_type E;
            char* d = arena_put(b, vec.data(), vec.size() * sizeof(E), sizes[q++]);
            return vec.empty() ? nullptr : reinterpret_cast<E*>(d);
        };
        return std::tuple<typename V::value_type*...>{put(v)...};
    }
    size_t total = 0;
    for (size_t x : sizes) total += x;
    const RingPlace r = ring_place_group(b->off, b->cap, total);
    RP4D_REQUIRE(r.fits, RP4D_ENOMEM, "batch staging ring too small for the descriptor tables of one launch");
    if (r.drain) RP4D_HIP(hipStreamSynchronize(b->ctx->stream));
    size_t at = r.first;
    int q = 0;
    auto put = [&](const auto& vec) {
        typedef typename std::decay_t<decltype(vec)>::value_type E;
        E* d = vec.empty() ? nullptr : reinterpret_cast<E*>(b->dev.as<char>() + at);
        ring_copy(b, at, vec.data(), vec.size() * sizeof(E));
        at += sizes[q++];
        return d;
    };
    std::tuple<typename V::value_type*...> out{put(v)...};
    b->off = r.next;
    return out;
}

template <typename T>
T* stage1(rp4d_batch* b, const std::vector<T>& v) {
    return std::get<0>(stage(b, v));
}

// Work items (problem, block) covering count_p elements per problem in blocks of 2048.
std::vector<int4> elem_items(const std::vector<size_t>& counts) {
    std::vector<int4> it;
    for (size_t p = 0; p < counts.size(); ++p)
        for (size_t blk = 0; blk * 2048 < counts[p]; ++blk) it.push_back(make_int4(static_cast<int>(p), static_cast<int>(blk), 0, 0));
    return it;
}

// Batched sweep tilings.  Defaults: wave regions (64 ppt points per wave, one
// work item per wave), 12 steps per launch (single-vector sweeps: 4 points per
// lane, 16 steps, the best of a search over wave and workgroup regions on
// batch-64's PCG product); overrides per (mode, dtype) and for the forward
// sweep through rp4d_batch_set_tiling, and for single-vector sweeps (k = 1)
// through rp4d_batch_set_tiling_k, which take precedence there.
inline bool tiling_set(const Tiling& o) { return o.ppt > 0 || o.kc > 0 || o.threads > 0 || o.steps > 0 || o.xch > 0; }

Tiling batch_tiling(const rp4d_batch* b, int mode, int dtype, bool fwd, int k = 0) {
    Tiling t;
    t.xch = XCH_WAVE;
    t.threads = 256;
    t.steps = 12;
    t.kc = 1;
    t.ppt = 2;
    const Tiling* o = &b->bt_fwd;
    if (!fwd) {
        const int d = dtype == RP4D_F64 ? 0 : 1;
        t.ppt = 4;
        t.kc = k == 1 ? 1 : 2;
        if (k == 1) t.steps = 16;
        o = (k == 1 && tiling_set(b->bt1[mode - 1][d])) ? &b->bt1[mode - 1][d] : &b->bt[mode - 1][d];
    }
    if (o->ppt > 0) t.ppt = o->ppt;
    if (o->kc > 0 && !fwd) t.kc = o->kc;
    if (o->threads > 0) t.threads = o->threads;
    if (o->steps > 0) t.steps = o->steps;
    if (o->xch > 0) t.xch = o->xch;
    return t;
}


// Batched Gram matrices: each descriptor's chunking and partial-sum buffer come
// from its problem (rows per chunk depend on n only); `owner[i]` is the problem
// whose ws_bg holds descriptor i's partials (one Gram per problem per call).
template <typename TX, typename TY>
void batch_gram(rp4d_batch* b, std::vector<BGram> gd, const std::vector<rp4d_problem*>& owner) {
    std::vector<int4> items, ritems;
    for (size_t i = 0; i < gd.size(); ++i) {
        BGram& g = gd[i];
        g.rows = std::max(64, ((g.n + 15) / 16 + 15) / 16 * 16);
        const int nch = (g.n + g.rows - 1) / g.rows;
        const size_t need = static_cast<size_t>(nch) * g.a * g.b * sizeof(double);
        rp4d_problem* p = owner[i];
        p->ws_bg.ensure(std::max(p->ws_bg.bytes, need));
        g.part = p->ws_bg.as<double>();
        const int tiles = ((g.a + 63) / 64) * ((g.b + 63) / 64);
        for (int c = 0; c < nch; ++c)
            for (int t = 0; t < tiles; ++t) items.push_back(make_int4(static_cast<int>(i), c, t, 0));
        const size_t stride = static_cast<size_t>(g.a) * g.b;
        for (size_t blk = 0; blk * 256 < stride; ++blk) ritems.push_back(make_int4(static_cast<int>(i), static_cast<int>(blk), 0, 0));
    }
    if (gd.empty()) return;
    auto [dgd, dit, drit] = stage(b, gd, items, ritems);
    launch_bgram<TX, TY>(dgd, dit, static_cast<int>(items.size()), drit, static_cast<int>(ritems.size()),
                         b->ctx->stream);
}

void check_batch_traj(const rp4d_problem* p, const rp4d_traj* tr) {
    check_traj(p, tr);
    RP4D_REQUIRE(tr->C == 1, RP4D_EINVAL, "batched sweeps need full trajectory storage (ckpt_every <= 1)");
}

// The planner's view of a batch problem and its stored trajectory.
BatchProb batch_prob(const rp4d_problem* p, const rp4d_traj* tr) {
    BatchProb q{};
    q.n = p->n;
    q.s_last = p->s_last;
    q.dt = p->d.dt;
    q.inv2dx = p->inv2dx;
    q.nu_dx2 = p->nu_dx2;
    q.obs_stride = p->d.obs_stride;
    q.obs_every = p->d.obs_every;
    q.n_obs = p->n_obs;
    q.n_t = p->n_t;
    q.sigma_o = p->d.sigma_o;
    q.traj = tr->states.as<double>();
    q.traj_rows = tr->rows;
    return q;
}

// Run f(j0, j1) over chunks of the nl time intervals of a batched sweep (or
// FWD) whose argument blocks and work items take at most a quarter of the
// staging ring, so that each chunk is one staged group.
template <typename F>
void for_interval_chunks(rp4d_batch* b, const std::vector<BatchProb>& bp, const Tiling& t, int groups,
                         size_t arg_bytes, F&& f) {
    const int nl = batch_intervals(bp, t);
    std::vector<int> ntile(bp.size()), nlp(bp.size());
    for (size_t i = 0; i < bp.size(); ++i) {
        ntile[i] = (bp[i].n + batch_tile(t, bp[i].n) - 1) / batch_tile(t, bp[i].n);
        nlp[i] = (bp[i].s_last + t.steps - 1) / t.steps;
    }
    auto items_of = [&](int j) {
        long c = 0;
        for (size_t i = 0; i < bp.size(); ++i)
            if (j < nlp[i]) c += static_cast<long>(ntile[i]) * groups;
        return c;
    };
    const std::vector<int> cuts = interval_chunks(nl, arg_bytes * bp.size() + 2 * kRingAlign, items_of, b->cap / 4);
    for (size_t c = 0; c + 1 < cuts.size(); ++c) f(cuts[c], cuts[c + 1]);
}

// Fused FWD of every problem in `sel` (indices into b->probs): u_0 = x0[i].
void batch_fwd_run(rp4d_batch* b, const std::vector<int>& sel, const std::vector<const double*>& x0,
                   const std::vector<rp4d_traj*>& trajs) {
    hipStream_t st = b->ctx->stream;
    const Tiling t = batch_tiling(b, MODE_TLM, RP4D_F64, true);
    const int np = static_cast<int>(sel.size());
    std::vector<double*> bufA(np), bufB(np);
    for (int i = 0; i < np; ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        p->ws_red.ensure(std::max<size_t>(p->ws_red.bytes, (2 * static_cast<size_t>(p->n) + 512) * sizeof(double)));
        bufA[i] = p->ws_red.as<double>();
        bufB[i] = bufA[i] + p->n;
    }
    // initial state and trajectory row 0
    {
        std::vector<BCopy> cd;
        std::vector<size_t> cnt;
        for (int i = 0; i < np; ++i) {
            rp4d_problem* p = b->probs[sel[i]];
            cd.push_back(BCopy{x0[i], bufA[i], p->n, 1, 1, 1, 0});
            cd.push_back(BCopy{x0[i], trajs[i]->states.as<double>(), p->n, 1, 1, 1, 0});
            cnt.push_back(p->n);
            cnt.push_back(p->n);
        }
        auto it = elem_items(cnt);
        auto [d_cd, d_it] = stage(b, cd, it);
        launch_bcopy<double, double>(d_cd, d_it, static_cast<int>(it.size()), st);
    }
    std::vector<BatchProb> bp(np);
    for (int i = 0; i < np; ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        bp[i] = batch_prob(p, trajs[i]);
        bp[i].y = p->has_data ? p->y.as<double>() : nullptr;
        bp[i].innov = p->has_data ? trajs[i]->innov.as<double>() : nullptr;
        bp[i].obs_out = trajs[i]->innov.as<double>() + p->m;
    }
    for_interval_chunks(b, bp, t, 1, sizeof(FwdArgs), [&](int j0, int j1) {
        const IntervalTables<FwdArgs> tb = plan_fwd(bp, t, bufA, bufB, j0, j1, FL_FWD);
        auto [dargs, ditems] = stage(b, tb.args, tb.items);
        const int4* dit = reinterpret_cast<const int4*>(ditems);
        for (int j = j0; j < j1; ++j) {
            const int q = j - j0;
            KernelTimer kt(b->ctx, RP4D_K_FWD, tb.flops[q]);
            launch_burgers_fwd_batched(dargs + tb.aoff[q], dit + tb.off[q], tb.off[q + 1] - tb.off[q], t, st);
        }
    });
    for (int i = 0; i < np; ++i) {
        trajs[i]->valid = true;
        trajs[i]->has_innov = b->probs[sel[i]]->has_data;
        b->probs[sel[i]]->cnt.fwd += 1;
    }
}

// Fused TLM (mode MODE_TLM) or ADJ sweeps of k vectors for the problems in sel.
// TLM: in[i] holds Gamma^{1/2} V (blocked kc), z[i] receives (n_t, n_obs, k).
// ADJ: forcing w[i]; returns the buffer holding lambda_0 for each problem.
template <typename T>
std::vector<T*> batch_sweep_run(rp4d_batch* b, int mode, const std::vector<int>& sel,
                                const std::vector<const rp4d_traj*>& trajs, int k, const Tiling& t,
                                const std::vector<T*>& buf0, const std::vector<T*>& buf1,
                                const std::vector<T*>& z, const std::vector<const T*>& w) {
    hipStream_t st = b->ctx->stream;
    const int np = static_cast<int>(sel.size());
    const int groups = (k + t.kc - 1) / t.kc;
    if (mode == MODE_ADJ) {
        std::vector<BCopy> cd;
        std::vector<size_t> cnt;
        for (int i = 0; i < np; ++i) {
            rp4d_problem* p = b->probs[sel[i]];
            cd.push_back(BCopy{nullptr, buf0[i], p->n, groups * t.kc, 1, 1, 1});
            cnt.push_back(static_cast<size_t>(p->n) * groups * t.kc);
        }
        auto it = elem_items(cnt);
        auto [d_cd, d_it] = stage(b, cd, it);
        launch_bcopy<T, T>(d_cd, d_it, static_cast<int>(it.size()), st);
    }
    std::vector<BatchProb> bp(np);
    for (int i = 0; i < np; ++i) bp[i] = batch_prob(b->probs[sel[i]], trajs[i]);
    const double fv = mode == MODE_TLM ? FL_TLM_VEC : FL_ADJ_VEC, fb = mode == MODE_TLM ? FL_TLM_BASE : FL_ADJ_BASE;
    for_interval_chunks(b, bp, t, groups, sizeof(SweepArgs<T>), [&](int j0, int j1) {
        const IntervalTables<SweepArgs<T>> tb = plan_sweep<T>(mode, bp, k, t, buf0, buf1, z, w, j0, j1, fv, fb);
        auto [dargs, ditems] = stage(b, tb.args, tb.items);
        const int4* dit = reinterpret_cast<const int4*>(ditems);
        for (int j = j0; j < j1; ++j) {
            const int q = j - j0;
            KernelTimer kt(b->ctx, mode == MODE_TLM ? RP4D_K_TLM : RP4D_K_ADJ, tb.flops[q]);
            launch_burgers_sweep_batched<T>(mode, dargs + tb.aoff[q], dit + tb.off[q], tb.off[q + 1] - tb.off[q], t,
                                            st);
        }
    });
    return sweep_result<T>(bp, t, buf0, buf1);
}

// Gamma^{1/2} for every selected problem: out[i] (layout out_kc) = Gamma^{1/2} in[i]
// (layout in_kc) (+ addv[i]).  Spectral problems in one batched Gram + GEMM pair.
template <typename T>
void batch_bhalf(rp4d_batch* b, const std::vector<int>& sel, int k, const std::vector<const T*>& in, int in_kc,
                 const std::vector<T*>& out, int out_kc, const std::vector<const T*>& addv) {
    hipStream_t st = b->ctx->stream;
    std::vector<BGram> gd;
    std::vector<rp4d_problem*> gown;
    std::vector<BTsmm> md;
    std::vector<int4> items;
    for (size_t i = 0; i < sel.size(); ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        if (!p->spec) {
            bhalf_into<T>(p, k, in[i], in_kc, out[i], out_kc, addv[i]);
            continue;
        }
        p->ws_bh.ensure(std::max<size_t>(p->ws_bh.bytes, static_cast<size_t>(p->r) * k * sizeof(double)));
        double* Tm = p->ws_bh.as<double>();
        gd.push_back(BGram{p->F.as<double>(), in[i], Tm, p->n, p->r, k, p->r, in_kc, 0, nullptr});
        gown.push_back(p);
        const int pi = static_cast<int>(md.size());
        md.push_back(BTsmm{p->F.as<double>(), Tm, p->lamF.as<double>(), addv[i], out[i], p->n, p->r, k, p->r, out_kc,
                           out_kc, 1.0, addv[i] ? 1.0 : 0.0});
        for (int rb = 0; rb * 64 < p->n; ++rb)
            for (int cb = 0; cb * 64 < k; ++cb) items.push_back(make_int4(pi, rb, cb, 0));
    }
    if (gd.empty()) return;
    batch_gram<double, T>(b, gd, gown);
    auto [d_md, d_items] = stage(b, md, items);
    launch_btsmm<double, T>(d_md, d_items, static_cast<int>(items.size()), st);
}

// Workspace of the batched block sweeps of problem p for k vectors.
template <typename T>
void batch_ensure_ws(rp4d_problem* p, int k, int kc) {
    const size_t blk = static_cast<size_t>((k + kc - 1) / kc + 1) * kc * p->n * sizeof(T);
    p->ws_s0.ensure(std::max(p->ws_s0.bytes, blk));
    p->ws_s1.ensure(std::max(p->ws_s1.bytes, blk));
    p->ws_obs.ensure(std::max(p->ws_obs.bytes, static_cast<size_t>(p->m) * k * sizeof(T)));
}

// HV[i] = (add_identity ? V[i] : 0) + H_i V[i] for the selected problems.
template <typename T>
void batch_hessian(rp4d_batch* b, const std::vector<int>& sel, const std::vector<const rp4d_traj*>& trajs, int k,
                   const std::vector<const T*>& V, const std::vector<T*>& HV, bool add_identity) {
    hipStream_t st = b->ctx->stream;
    const int dt = sizeof(T) == 8 ? RP4D_F64 : RP4D_F32;
    Tiling tt = batch_tiling(b, MODE_TLM, dt, false, k), ta = batch_tiling(b, MODE_ADJ, dt, false, k);
    while (tt.kc > 1 && tt.kc > k) tt.kc /= 2;   // no padded vectors for small k
    while (ta.kc > 1 && ta.kc > k) ta.kc /= 2;
    const int np = static_cast<int>(sel.size());
    std::vector<T*> s0(np), s1(np), obs(np);
    std::vector<const T*> cobs(np), none(np, nullptr);
    for (int i = 0; i < np; ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        batch_ensure_ws<T>(p, k, std::max(tt.kc, ta.kc));
        s0[i] = p->ws_s0.as<T>();
        s1[i] = p->ws_s1.as<T>();
        obs[i] = p->ws_obs.as<T>();
        cobs[i] = obs[i];
    }
    const int gt = (k + tt.kc - 1) / tt.kc;
    if (gt * tt.kc != k) {
        std::vector<BCopy> cd;
        std::vector<size_t> cnt;
        for (int i = 0; i < np; ++i) {
            cd.push_back(BCopy{nullptr, s0[i], b->probs[sel[i]]->n, gt * tt.kc, 1, 1, 1});
            cnt.push_back(static_cast<size_t>(b->probs[sel[i]]->n) * gt * tt.kc);
        }
        auto it = elem_items(cnt);
        auto [d_cd, d_it] = stage(b, cd, it);
        launch_bcopy<T, T>(d_cd, d_it, static_cast<int>(it.size()), st);
    }
    batch_bhalf<T>(b, sel, k, V, k, s0, tt.kc, none);
    batch_sweep_run<T>(b, MODE_TLM, sel, trajs, k, tt, s0, s1, obs, none);
    std::vector<T*> lam = batch_sweep_run<T>(b, MODE_ADJ, sel, trajs, k, ta, s0, s1, obs, cobs);
    std::vector<const T*> clam(lam.begin(), lam.end());
    std::vector<const T*> add(np, nullptr);
    if (add_identity) add = V;
    batch_bhalf<T>(b, sel, k, clam, ta.kc, HV, k, add);
    for (int i = 0; i < np; ++i) b->probs[sel[i]]->cnt.hv_columns += k;
}

// Batched gradient g[i] = v[i] + A_i^T d_i (FP64, one ADJ sweep per problem).
void batch_gradient(rp4d_batch* b, const std::vector<int>& sel, const std::vector<const rp4d_traj*>& trajs,
                    const std::vector<const double*>& v, const std::vector<double*>& g) {
    const Tiling ta = batch_tiling(b, MODE_ADJ, RP4D_F64, false, 1);
    Tiling t1 = ta;
    t1.kc = 1;
    const int np = static_cast<int>(sel.size());
    std::vector<double*> s0(np), s1(np);
    std::vector<const double*> w(np), none(np, nullptr);
    for (int i = 0; i < np; ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        batch_ensure_ws<double>(p, 1, 1);
        s0[i] = p->ws_s0.as<double>();
        s1[i] = p->ws_s1.as<double>();
        w[i] = trajs[i]->innov.as<double>();
    }
    std::vector<double*> lam = batch_sweep_run<double>(b, MODE_ADJ, sel, trajs, 1, t1, s0, s1, {}, w);
    std::vector<const double*> clam(lam.begin(), lam.end());
    batch_bhalf<double>(b, sel, 1, clam, 1, g, 1, v);
    for (int i = 0; i < np; ++i) b->probs[sel[i]]->cnt.adj_online += 1;
}

// Batched preconditioner application z = P_i r (k = 1); pcs[i] may be null (copy).
void batch_precond_apply(rp4d_batch* b, const std::vector<int>& sel, const std::vector<const rp4d_precond*>& pcs,
                         const std::vector<const double*>& r, const std::vector<double*>& z) {
    hipStream_t st = b->ctx->stream;
    std::vector<BGram> gd;
    std::vector<rp4d_problem*> gown;
    std::vector<BTsmm> md;
    std::vector<int4> items;
    std::vector<BCopy> cd;
    std::vector<size_t> cnt;
    for (size_t i = 0; i < sel.size(); ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        const rp4d_precond* pc = pcs[i];
        if (!pc) {
            cd.push_back(BCopy{r[i], z[i], p->n, 1, 1, 1, 0});
            cnt.push_back(p->n);
            continue;
        }
        const int l = pc->ell;
        p->ws_red.ensure(std::max<size_t>(p->ws_red.bytes, (2 * static_cast<size_t>(p->n) + 512 + l) * sizeof(double)));
        double* T = p->ws_red.as<double>() + 2 * p->n + 512;
        gd.push_back(BGram{pc->V.as<double>(), r[i], T, p->n, l, 1, l, 1, 0, nullptr});
        gown.push_back(p);
        const int pi = static_cast<int>(md.size());
        md.push_back(BTsmm{pc->V.as<double>(), T, pc->Dg.as<double>(), r[i], z[i], p->n, l, 1, l, 1, 1, -1.0, 1.0});
        for (int rb = 0; rb * 64 < p->n; ++rb) items.push_back(make_int4(pi, rb, 0, 0));
    }
    if (!cd.empty()) {
        auto it = elem_items(cnt);
        auto [d_cd, d_it] = stage(b, cd, it);
        launch_bcopy<double, double>(d_cd, d_it, static_cast<int>(it.size()), st);
    }
    if (!gd.empty()) {
        batch_gram<double, double>(b, gd, gown);
        auto [d_md, d_items] = stage(b, md, items);
        launch_btsmm<double, double>(d_md, d_items, static_cast<int>(items.size()), st);
    }
}

// Batched dot products into the batch scalar array slot `slot` of each problem.
void batch_dot(rp4d_batch* b, const std::vector<int>& sel, const std::vector<const double*>& x,
               const std::vector<const double*>& y, int slot, bool absmax = false) {
    std::vector<BVec> vd;
    for (size_t i = 0; i < sel.size(); ++i)
        vd.push_back(BVec{x[i], y[i], b->scal.as<double>() + 16 * sel[i] + slot, b->probs[sel[i]]->n});
    launch_bdot(stage1(b, vd), static_cast<int>(vd.size()), absmax, b->ctx->stream);
}

std::vector<double> batch_read_scal(rp4d_batch* b) {
    std::vector<double> h(16 * b->probs.size());
    RP4D_HIP(hipMemcpyAsync(h.data(), b->scal.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, b->ctx->stream));
    RP4D_HIP(hipStreamSynchronize(b->ctx->stream));
    return h;
}

void batch_axpby(rp4d_batch* b, std::vector<BAxpby> ad) {
    std::vector<size_t> cnt;
    for (auto& a : ad) cnt.push_back(a.count);
    auto it = elem_items(cnt);
    auto [d_ad, d_it] = stage(b, ad, it);
    launch_baxpby(d_ad, d_it, static_cast<int>(it.size()), b->ctx->stream);
}

// Capture a batched body that stages descriptor tables: a first capture sizes
// its tables (its graph is discarded unlaunched), the second records them
// against the device arena, and one copy moves them there before any replay.
// The stream must be idle (no earlier graph still reading the arena).
template <typename F>
void capture_batch(rp4d_batch* b, F&& f, GraphExec& out) {
    struct Mode {
        rp4d_batch* b;
        ~Mode() { b->gmode = 0; }
    } mode{b};
    b->arena_off = 0;
    b->gmode = 1;
    {
        GraphExec sizing;
        capture(b->ctx, f, sizing, false);
    }
    b->arena_dev.ensure(std::max<size_t>(b->arena_off, 256));
    b->arena_host.assign(b->arena_off, 0);
    b->arena_off = 0;
    b->gmode = 2;
    capture(b->ctx, f, out, true);
    RP4D_HIP(hipMemcpyAsync(b->arena_dev.p, b->arena_host.data(), b->arena_off, hipMemcpyHostToDevice,
                            b->ctx->stream));
    RP4D_HIP(hipStreamSynchronize(b->ctx->stream));
}

// Batched lockstep PCG (FP64) on (I + H_i) x_i = b_i; returns per-problem iterations.
std::vector<int> batch_pcg(rp4d_batch* b, const std::vector<int>& sel, const std::vector<const rp4d_traj*>& trajs,
                           const std::vector<const rp4d_precond*>& pcs, const std::vector<const double*>& rhs,
                           const std::vector<double*>& x, double rtol, int maxit, std::vector<int>& conv,
                           std::vector<double>* relres = nullptr) {
    hipStream_t st = b->ctx->stream;
    const int np = static_cast<int>(sel.size());
    std::vector<double*> r(np), z(np), pv(np), q(np);
    std::vector<BPcg> pd(np);
    for (int i = 0; i < np; ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        p->ws_pcg.ensure(std::max<size_t>(p->ws_pcg.bytes, (5 * static_cast<size_t>(p->n) + 1024) * sizeof(double)));
        r[i] = p->ws_pcg.as<double>();
        z[i] = r[i] + p->n;
        pv[i] = z[i] + p->n;
        q[i] = pv[i] + p->n;
        pd[i] = BPcg{x[i], r[i], pv[i], q[i], z[i], b->scal.as<double>() + 16 * sel[i], p->n};
    }
    {
        std::vector<BAxpby> ad;
        for (int i = 0; i < np; ++i) {
            ad.push_back(BAxpby{nullptr, x[i], static_cast<size_t>(b->probs[sel[i]]->n), 0.0, nullptr, 0.0});
            ad.push_back(BAxpby{rhs[i], r[i], static_cast<size_t>(b->probs[sel[i]]->n), 1.0, nullptr, 0.0});
        }
        batch_axpby(b, ad);
    }
    std::vector<const double*> cr(r.begin(), r.end()), cz(z.begin(), z.end()), cp(pv.begin(), pv.end()),
        cq(q.begin(), q.end());
    batch_precond_apply(b, sel, pcs, cr, z);
    {
        std::vector<BAxpby> ad;
        for (int i = 0; i < np; ++i) ad.push_back(BAxpby{z[i], pv[i], static_cast<size_t>(b->probs[sel[i]]->n), 1.0, nullptr, 0.0});
        batch_axpby(b, ad);
    }
    batch_dot(b, sel, cr, cz, SC_RZ);
    batch_dot(b, sel, rhs, rhs, SC_BB);
    std::vector<double> sc = batch_read_scal(b);
    std::vector<double> bnorm(np);
    std::vector<int> iters(np, 0);
    conv.assign(np, 0);
    if (relres) relres->assign(np, 0.0);
    std::vector<int> act;
    for (int i = 0; i < np; ++i) {
        bnorm[i] = std::sqrt(sc[16 * sel[i] + SC_BB]);
        RP4D_REQUIRE(std::isfinite(bnorm[i]), RP4D_ENONFINITE, "non-finite right-hand side in batch");
        if (bnorm[i] == 0.0 || bnorm[i] <= rtol * bnorm[i])
            conv[i] = 1;  // b = 0 or rtol >= 1: x_0 = 0 meets the tolerance
        else
            act.push_back(i);
    }
    if (maxit <= 0) {
        maxit = 1;
        for (int i = 0; i < np; ++i) maxit = std::max(maxit, b->probs[sel[i]]->n);
    }
    // One iteration for the active problems A: q = (I+H)p, alpha, x, r, |r|^2,
    // then speculatively z = P r, r.z and the next p (unused by problems whose
    // |r| meets the tolerance).  The stream is read at each launch, so the same
    // body can be captured into a graph.
    auto body = [&](const std::vector<int>& A) {
        hipStream_t s = b->ctx->stream;
        std::vector<int> asel;
        std::vector<const rp4d_traj*> atr;
        std::vector<const double*> ap, ar;
        std::vector<double*> aq, az;
        std::vector<const rp4d_precond*> apc;
        std::vector<BPcg> apd;
        std::vector<size_t> cnt;
        for (int i : A) {
            asel.push_back(sel[i]);
            atr.push_back(trajs[i]);
            ap.push_back(pv[i]);
            aq.push_back(q[i]);
            ar.push_back(r[i]);
            az.push_back(z[i]);
            apc.push_back(pcs[i]);
            apd.push_back(pd[i]);
            cnt.push_back(b->probs[sel[i]]->n);
        }
        batch_hessian<double>(b, asel, atr, 1, ap, aq, true);
        std::vector<const double*> caq(aq.begin(), aq.end()), caz(az.begin(), az.end());
        batch_dot(b, asel, ap, caq, SC_PQ);
        const auto items = elem_items(cnt);
        {
            auto [dpd, dit] = stage(b, apd, items);
            launch_bpcg_xr(dpd, dit, static_cast<int>(items.size()), s);
        }
        batch_dot(b, asel, ar, ar, SC_RR);
        batch_precond_apply(b, asel, apc, ar, az);
        batch_dot(b, asel, ar, caz, SC_RZN);
        auto [dpd, dit] = stage(b, apd, items);
        launch_bpcg_p(dpd, dit, static_cast<int>(items.size()), static_cast<int>(apd.size()), s);
    };
    // With graphs on, iterations after the first (which sizes every workspace
    // the body touches) replay the body captured for the current active set; a
    // change of the set captures it again.
    const bool use_graph = b->ctx->graphs;
    GraphExec gx;
    std::vector<int> gact;
    for (int it = 0; it < maxit && !act.empty(); ++it) {
        if (use_graph && it >= 1) {
            if (!gx.ex || gact != act) {
                gx.reset();
                std::vector<long long> hv(np);
                for (int i = 0; i < np; ++i) hv[i] = b->probs[sel[i]]->cnt.hv_columns;
                capture_batch(b, [&] { body(act); }, gx);
                for (int i = 0; i < np; ++i) b->probs[sel[i]]->cnt.hv_columns = hv[i];
                gact = act;
            }
            RP4D_HIP(hipGraphLaunch(gx.ex, st));
            for (int i : act) b->probs[sel[i]]->cnt.hv_columns += 1;
        } else {
            body(act);
        }
        std::vector<double> s2 = batch_read_scal(b);
        std::vector<int> still;
        for (int i : act) {
            iters[i] += 1;
            const double rn = std::sqrt(s2[16 * sel[i] + SC_RR]);
            RP4D_REQUIRE(std::isfinite(rn), RP4D_ENONFINITE, "non-finite PCG residual in batch");
            if (relres) (*relres)[i] = rn / bnorm[i];
            if (rn <= rtol * bnorm[i])
                conv[i] = 1;
            else
                still.push_back(i);
        }
        act = still;
    }
    for (int i = 0; i < np; ++i) {
        b->probs[sel[i]]->cnt.tlm_online += iters[i];
        b->probs[sel[i]]->cnt.adj_online += iters[i];
    }
    return iters;
}

// Batched Nystrom sketches (Alg. 2) for the selected problems (uniform l), Omega
// from Philox with seed ^ problem index.  Returns new preconditioners.
std::vector<rp4d_precond*> batch_nystrom(rp4d_batch* b, const std::vector<int>& sel,
                                          const std::vector<const rp4d_traj*>& trajs, int l, uint64_t seed, int dtype) {
    hipStream_t st = b->ctx->stream;
    const int np = static_cast<int>(sel.size());
    std::vector<Scratch> S(np);
    for (int i = 0; i < np; ++i) S[i] = sketch_scratch(b->probs[sel[i]], l, dtype);
    // Omega
    {
        std::vector<BRand> rd;
        std::vector<size_t> cnt;
        for (int i = 0; i < np; ++i) {
            const size_t c = static_cast<size_t>(b->probs[sel[i]]->n) * l;
            rd.push_back(BRand{S[i].Om, c, seed ^ (0x9E3779B97F4A7C15ULL * (b->probs[sel[i]]->id + 1))});
            cnt.push_back((c + 1) / 2);
        }
        auto it = elem_items(cnt);
        auto [d_rd, d_it] = stage(b, rd, it);
        launch_bphilox(d_rd, d_it, static_cast<int>(it.size()), st);
    }
    auto copyall = [&](auto tag_in, auto tag_out, auto src, auto dst, bool rows_m) {
        using TI = decltype(tag_in);
        using TO = decltype(tag_out);
        std::vector<BCopy> cd;
        std::vector<size_t> cnt;
        for (int i = 0; i < np; ++i) {
            rp4d_problem* p = b->probs[sel[i]];
            const int rows = rows_m ? p->m : p->n;
            cd.push_back(BCopy{src(i), dst(i), rows, l, l, l, 0});
            cnt.push_back(static_cast<size_t>(rows) * l);
        }
        auto it = elem_items(cnt);
        auto [d_cd, d_it] = stage(b, cd, it);
        launch_bcopy<TI, TO>(d_cd, d_it, static_cast<int>(it.size()), st);
    };
    // Y0 = H Omega (data-misfit part) in the sketch precision, kept as FP64 in Yd
    if (dtype == RP4D_F64) {
        std::vector<const double*> om(np);
        std::vector<double*> y(np);
        for (int i = 0; i < np; ++i) {
            om[i] = S[i].Om;
            y[i] = S[i].Yd;
        }
        batch_hessian<double>(b, sel, trajs, l, om, y, false);
    } else {
        copyall(double(), float(), [&](int i) { return static_cast<const void*>(S[i].Om); },
                [&](int i) { return S[i].Omt; }, false);
        std::vector<const float*> om(np);
        std::vector<float*> y(np);
        for (int i = 0; i < np; ++i) {
            om[i] = static_cast<const float*>(S[i].Omt);
            y[i] = static_cast<float*>(S[i].Yt);
        }
        batch_hessian<float>(b, sel, trajs, l, om, y, false);
        copyall(float(), double(), [&](int i) { return static_cast<const void*>(S[i].Yt); },
                [&](int i) { return static_cast<void*>(S[i].Yd); }, false);
    }
    std::vector<BSmall> sm(np);
    std::vector<BSketch> sk(np);
    std::vector<BGram> gd(np);
    std::vector<rp4d_problem*> owners(np);
    for (int i = 0; i < np; ++i) owners[i] = b->probs[sel[i]];
    // nu = sqrt(n) eps ||Y||_2
    for (int i = 0; i < np; ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        gd[i] = BGram{S[i].Yd, S[i].Yd, S[i].S2, p->n, l, l, l, l, 0, nullptr};
        sm[i] = BSmall{S[i].S2, nullptr, S[i].ev, nullptr};
        sk[i] = BSketch{S[i].ev, S[i].nu, S[i].lam, S[i].D, S[i].S2, p->n};
    }
    batch_gram<double, double>(b, gd, owners);
    launch_bjacobi(stage1(b, sm), np, l, false, st);
    const double eps = dtype == RP4D_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23);
    launch_bnu(stage1(b, sk), np, eps, st);
    // shifted core matrix and its Cholesky factor, with tenfold shift retries
    std::vector<int> todo(np);
    for (int i = 0; i < np; ++i) todo[i] = i;
    for (int attempt = 0; attempt <= 3 && !todo.empty(); ++attempt) {
        std::vector<BAxpby> ad;
        std::vector<BGram> cg;
        std::vector<BSmall> cs;
        for (int i : todo) {
            rp4d_problem* p = b->probs[sel[i]];
            const size_t c = static_cast<size_t>(p->n) * l;
            ad.push_back(BAxpby{S[i].Yd, S[i].Y2, c, 1.0, nullptr, 0.0});
            ad.push_back(BAxpby{S[i].Om, S[i].Y2, c, 1.0, S[i].nu, 1.0});
            cg.push_back(BGram{S[i].Om, S[i].Y2, S[i].S2, p->n, l, l, l, l, 0, nullptr});
            cs.push_back(BSmall{S[i].S2, nullptr, nullptr, S[i].info});
        }
        // two passes so that Y2 = Yd is complete before the shift is added
        std::vector<BAxpby> a1, a2;
        for (size_t q = 0; q < ad.size(); q += 2) {
            a1.push_back(ad[q]);
            a2.push_back(ad[q + 1]);
        }
        batch_axpby(b, a1);
        batch_axpby(b, a2);
        std::vector<rp4d_problem*> cown;
        for (int i : todo) cown.push_back(b->probs[sel[i]]);
        batch_gram<double, double>(b, cg, cown);
        launch_bchol(stage1(b, cs), static_cast<int>(cs.size()), l, st);
        std::vector<int> failed;
        std::vector<int> infos(todo.size(), 0);
        for (size_t q = 0; q < todo.size(); ++q)
            RP4D_HIP(hipMemcpyAsync(&infos[q], S[todo[q]].info, sizeof(int), hipMemcpyDeviceToHost, st));
        RP4D_HIP(hipStreamSynchronize(st));
        for (size_t q = 0; q < todo.size(); ++q)
            if (infos[q] != 0) failed.push_back(todo[q]);
        for (int i : failed) {
            std::vector<BAxpby> sc1{BAxpby{nullptr, S[i].nu, 1, 0.0, nullptr, 10.0}};
            batch_axpby(b, sc1);
        }
        todo = failed;
    }
    RP4D_REQUIRE(todo.empty(), RP4D_ENOTSPD, "Nystrom core matrix not positive definite after shift retries (batch)");
    // W W^T = L^{-1} (Y^T Y) L^{-T}; eig; V = Y L^{-T} U Sigma^{-1}
    std::vector<BSmall> t1(np), g1(np), g2(np), ej(np), g3(np);
    std::vector<BGram> yy(np);
    std::vector<BTsmm> vm(np);
    std::vector<int4> vit;
    std::vector<rp4d_precond*> out(np, nullptr);
    for (int i = 0; i < np; ++i) {
        rp4d_problem* p = b->probs[sel[i]];
        t1[i] = BSmall{S[i].S2, S[i].S3, nullptr, nullptr};         // S3 = L^{-1}
        yy[i] = BGram{S[i].Y2, S[i].Y2, S[i].S4, p->n, l, l, l, l, 0, nullptr};  // S4 = Y^T Y
        g1[i] = BSmall{S[i].S3, S[i].S4, S[i].S2, nullptr};         // S2 = L^{-1} Y^T Y
        g2[i] = BSmall{S[i].S2, S[i].S3, S[i].S4, nullptr};         // S4 = S2 L^{-T}
        ej[i] = BSmall{S[i].S4, S[i].S2, S[i].ev, nullptr};         // ev, U = S2
        g3[i] = BSmall{S[i].S3, S[i].S2, S[i].S4, nullptr};         // S4 = L^{-T} U Sigma^{-1}
        auto* pc = new rp4d_precond();
        pc->p = p;
        pc->ell = l;
        pc->V.ensure(static_cast<size_t>(p->n) * l * sizeof(double));
        pc->Dg.ensure(static_cast<size_t>(l) * sizeof(double));
        out[i] = pc;
        vm[i] = BTsmm{S[i].Y2, S[i].S4, nullptr, nullptr, pc->V.p, p->n, l, l, l, l, l, 1.0, 0.0};
        for (int rb = 0; rb * 64 < p->n; ++rb)
            for (int cb = 0; cb * 64 < l; ++cb) vit.push_back(make_int4(i, rb, cb, 0));
    }
    try {
        launch_btrinv(stage1(b, t1), np, l, st);
        batch_gram<double, double>(b, yy, owners);
        launch_bgemm_small(stage1(b, g1), np, l, 0, 0, 1.0, st);
        launch_bgemm_small(stage1(b, g2), np, l, 0, 1, 1.0, st);
        launch_bjacobi(stage1(b, ej), np, l, true, st);
        launch_bfinalize(stage1(b, sk), np, l, true, st);  // lam, D and U <- U diag(1/sigma)
        launch_bgemm_small(stage1(b, g3), np, l, 1, 0, 1.0, st);
        auto [d_vm, d_vit] = stage(b, vm, vit);
        launch_btsmm<double, double>(d_vm, d_vit, static_cast<int>(vit.size()), st);
        std::vector<double> nuh(np);
        for (int i = 0; i < np; ++i) {
            launch_relayout<double, double>(S[i].D, 1, out[i]->Dg.as<double>(), 1, l, 1, st);
            out[i]->lam.resize(l);
            RP4D_HIP(hipMemcpyAsync(out[i]->lam.data(), S[i].lam, l * sizeof(double), hipMemcpyDeviceToHost, st));
            RP4D_HIP(hipMemcpyAsync(&nuh[i], S[i].nu, sizeof(double), hipMemcpyDeviceToHost, st));
        }
        RP4D_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < np; ++i) {
            out[i]->nu = nuh[i];
            out[i]->host_ok = true;
            for (double v : out[i]->lam) RP4D_REQUIRE(std::isfinite(v), RP4D_ENONFINITE, "non-finite sketch (batch)");
            b->probs[sel[i]]->cnt.tlm_offline += l;
            b->probs[sel[i]]->cnt.adj_offline += l;
            b->probs[sel[i]]->cnt.sketches += 1;
        }
    } catch (...) {
        for (auto* pc : out) delete pc;
        throw;
    }
    return out;
}

}  // namespace
}  // namespace rp4d

extern "C" {

int rp4d_batch_create(rp4d_ctx* ctx, int nprob, rp4d_problem* const* probs, rp4d_batch** out) {
    return guarded([&] {
        RP4D_REQUIRE(ctx != nullptr && out != nullptr && probs != nullptr && nprob >= 1, RP4D_EINVAL, "bad argument");
        set_device(ctx);
        auto* b = new rp4d_batch();
        try {
            b->ctx = ctx;
            for (int i = 0; i < nprob; ++i) {
                RP4D_REQUIRE(probs[i] != nullptr && probs[i]->ctx == ctx, RP4D_EINVAL,
                             "batch problems must share the context");
                RP4D_REQUIRE(probs[i]->d.model == RP4D_BURGERS1D, RP4D_EINVAL, "batches hold Burgers problems");
                b->probs.push_back(probs[i]);
            }
            b->cap = 32u << 20;
            RP4D_HIP(hipHostMalloc(reinterpret_cast<void**>(&b->host), b->cap, hipHostMallocDefault));
            b->dev.ensure(b->cap);
            b->scal.ensure(16 * sizeof(double) * nprob);
        } catch (...) {
            delete b;
            throw;
        }
        *out = b;
    });
}

int rp4d_batch_destroy(rp4d_batch* b) {
    return guarded([&] {
        if (b) quiesce_device(b->device);
        delete b;
    });
}

int rp4d_batch_set_tiling(rp4d_batch* b, int mode, int dtype, int ppt, int kc, int threads, int steps, int xch) {
    return rp4d_batch_set_tiling_k(b, mode, dtype, 0, ppt, kc, threads, steps, xch);
}

int rp4d_batch_set_tiling_k(rp4d_batch* b, int mode, int dtype, int k, int ppt, int kc, int threads, int steps,
                            int xch) {
    return guarded([&] {
        RP4D_REQUIRE(b != nullptr && (mode == MODE_TLM || mode == MODE_ADJ || mode == RP4D_MODE_FWD) &&
                         (dtype == RP4D_F64 || dtype == RP4D_F32), RP4D_EINVAL, "bad argument");
        RP4D_REQUIRE(k == 0 || (k == 1 && mode != RP4D_MODE_FWD && kc <= 1), RP4D_EINVAL,
                     "batched tiling: k is 0 (every sweep) or 1 (single-vector TLM/ADJ sweeps, kc <= 1)");
        RP4D_REQUIRE(xch <= 0 || xch == XCH_LDS || xch == XCH_WAVE, RP4D_EINVAL,
                     "batched sweeps: workgroup (1) or wave (2) regions");
        const int d = dtype == RP4D_F64 ? 0 : 1;
        Tiling& t = mode == RP4D_MODE_FWD ? b->bt_fwd : (k == 1 ? b->bt1[mode - 1][d] : b->bt[mode - 1][d]);
        t.ppt = ppt;
        t.kc = kc;
        t.threads = threads;
        t.steps = steps;
        t.xch = xch > 0 ? xch : 0;
    });
}

int rp4d_batch_fwd(rp4d_batch* b, const double* const* x0, rp4d_traj* const* trajs, double* J_obs) {
    return guarded([&] {
        RP4D_REQUIRE(b != nullptr && x0 != nullptr && trajs != nullptr, RP4D_EINVAL, "null argument");
        set_device(b->ctx);
        const int np = static_cast<int>(b->probs.size());
        std::vector<int> sel(np);
        std::vector<const double*> xs(np);
        std::vector<rp4d_traj*> tr(np);
        for (int i = 0; i < np; ++i) {
            sel[i] = i;
            xs[i] = x0[i];
            tr[i] = trajs[i];
            RP4D_REQUIRE(tr[i] && tr[i]->p == b->probs[i] && tr[i]->C == 1, RP4D_EINVAL,
                         "batch trajectories must match the problems and store every state");
        }
        batch_fwd_run(b, sel, xs, tr);
        if (J_obs) {
            std::vector<const double*> in(np);
            for (int i = 0; i < np; ++i) {
                RP4D_REQUIRE(b->probs[i]->has_data, RP4D_ESTATE, "J requested but data not set");
                in[i] = tr[i]->innov.as<double>();
            }
            std::vector<BVec> vd;
            for (int i = 0; i < np; ++i) vd.push_back(BVec{in[i], in[i], b->scal.as<double>() + 16 * i + SC_T0, b->probs[i]->m});
            launch_bdot(stage1(b, vd), np, false, b->ctx->stream);
            std::vector<double> sc = batch_read_scal(b);
            for (int i = 0; i < np; ++i) J_obs[i] = 0.5 * sc[16 * i + SC_T0];
        }
    });
}

int rp4d_batch_hessian_block(rp4d_batch* b, rp4d_traj* const* trajs, int k, const void* const* V, void* const* HV,
                             int dtype, int add_identity) {
    return guarded([&] {
        RP4D_REQUIRE(b != nullptr && trajs != nullptr && V != nullptr && HV != nullptr && k >= 1 && k <= 4096,
                     RP4D_EINVAL, "bad argument");
        set_device(b->ctx);
        const int np = static_cast<int>(b->probs.size());
        std::vector<int> sel(np);
        std::vector<const rp4d_traj*> tr(np);
        for (int i = 0; i < np; ++i) {
            sel[i] = i;
            tr[i] = trajs[i];
            check_batch_traj(b->probs[i], tr[i]);
            RP4D_REQUIRE(V[i] != nullptr && HV[i] != nullptr && V[i] != HV[i], RP4D_EINVAL, "bad block pointer");
        }
        if (dtype == RP4D_F64) {
            std::vector<const double*> v(np);
            std::vector<double*> h(np);
            for (int i = 0; i < np; ++i) {
                v[i] = static_cast<const double*>(V[i]);
                h[i] = static_cast<double*>(HV[i]);
            }
            batch_hessian<double>(b, sel, tr, k, v, h, add_identity != 0);
        } else if (dtype == RP4D_F32) {
            std::vector<const float*> v(np);
            std::vector<float*> h(np);
            for (int i = 0; i < np; ++i) {
                v[i] = static_cast<const float*>(V[i]);
                h[i] = static_cast<float*>(HV[i]);
            }
            batch_hessian<float>(b, sel, tr, k, v, h, add_identity != 0);
        } else {
            fail(RP4D_EINVAL, "bad dtype");
        }
    });
}

int rp4d_batch_gn_step(rp4d_batch* b, rp4d_gn_state* const* states, const rp4d_gn_opts* o, rp4d_gn_info* infos) {
    return guarded([&] {
        RP4D_REQUIRE(b != nullptr && states != nullptr && o != nullptr, RP4D_EINVAL, "null argument");
        RP4D_REQUIRE(o->solve == RP4D_SOLVE_PCG, RP4D_EINVAL, "batched GN step: SketchPrec (PCG) only");
        RP4D_REQUIRE(o->sketch == RP4D_NYSTROM || o->sketch == RP4D_NOPREC, RP4D_EINVAL,
                     "batched GN step supports Nystrom sketches or no preconditioner");
        RP4D_REQUIRE(o->omega == nullptr, RP4D_EINVAL, "batched GN step draws Omega on the device (omega must be NULL)");
        set_device(b->ctx);
        hipStream_t st = b->ctx->stream;
        const int np = static_cast<int>(b->probs.size());
        std::vector<int> sel(np);
        std::vector<rp4d_traj*> tr(np);
        std::vector<const rp4d_traj*> ctr(np);
        std::vector<const double*> x(np), v(np), xb(np), g(np);
        std::vector<double*> gm(np), bm(np), dv(np), vm(np), xm(np);
        for (int i = 0; i < np; ++i) {
            rp4d_gn_state* s = states[i];
            RP4D_REQUIRE(s != nullptr && s->p == b->probs[i], RP4D_EINVAL, "GN state does not match the batch problem");
            RP4D_REQUIRE(s->traj->C == 1, RP4D_EINVAL, "batched GN step needs full trajectory storage");
            sel[i] = i;
            tr[i] = s->traj;
            ctr[i] = s->traj;
            x[i] = s->x.as<double>();
            v[i] = s->v.as<double>();
            xb[i] = b->probs[i]->xb.as<double>();
            gm[i] = s->g.as<double>();
            g[i] = gm[i];
            bm[i] = s->b.as<double>();
            dv[i] = s->dv.as<double>();
            vm[i] = s->v.as<double>();
            xm[i] = s->x.as<double>();
        }
        std::vector<rp4d_gn_info> inf(np);
        // 1. FWD, J
        batch_fwd_run(b, sel, x, tr);
        {
            std::vector<BVec> vd;
            for (int i = 0; i < np; ++i) {
                const double* in = tr[i]->innov.as<double>();
                vd.push_back(BVec{in, in, b->scal.as<double>() + 16 * i + SC_T0, b->probs[i]->m});
                vd.push_back(BVec{v[i], v[i], b->scal.as<double>() + 16 * i + SC_T2, b->probs[i]->n});
            }
            launch_bdot(stage1(b, vd), static_cast<int>(vd.size()), false, st);
        }
        // 2. gradient, |g|_inf, b = -g
        batch_gradient(b, sel, ctr, v, gm);
        batch_dot(b, sel, g, g, SC_T1, true);
        {
            std::vector<BAxpby> ad;
            for (int i = 0; i < np; ++i) ad.push_back(BAxpby{g[i], bm[i], static_cast<size_t>(b->probs[i]->n), -1.0, nullptr, 0.0});
            batch_axpby(b, ad);
        }
        std::vector<double> sc = batch_read_scal(b);
        for (int i = 0; i < np; ++i) {
            inf[i].J = 0.5 * sc[16 * i + SC_T2] + 0.5 * sc[16 * i + SC_T0];
            inf[i].gnorm_inf = sc[16 * i + SC_T1];
            inf[i].kappa_re = -1.0;
            inf[i].kappa_sk = -1.0;
            RP4D_REQUIRE(std::isfinite(inf[i].J) && std::isfinite(inf[i].gnorm_inf), RP4D_ENONFINITE,
                         "non-finite cost or gradient in batch");
        }
        // 3-4. reuse test for resident preconditioners, sketch the rest
        std::vector<const rp4d_precond*> use(np, nullptr);
        if (o->sketch != RP4D_NOPREC) {
            std::vector<int> test;
            for (int i = 0; i < np; ++i)
                if (states[i]->pc && states[i]->pc_live && o->reuse_eps > 0) test.push_back(i);
            if (!test.empty()) {
                // unit test vectors from Philox, z = P v, q = (I + H) z, kappa = |q| / |v|
                std::vector<BRand> rd;
                std::vector<size_t> cnt;
                std::vector<const double*> vh, cz;
                std::vector<double*> zz, qq;
                std::vector<const rp4d_precond*> tp;
                std::vector<const rp4d_traj*> ttr;
                for (int i : test) {
                    rp4d_problem* p = b->probs[i];
                    p->ws_pcg.ensure(std::max<size_t>(p->ws_pcg.bytes, (5 * static_cast<size_t>(p->n) + 1024) * sizeof(double)));
                    double* base = p->ws_pcg.as<double>();
                    rd.push_back(BRand{base + 2 * p->n, static_cast<size_t>(p->n),
                                       o->seed ^ 0x5DEECE66DULL ^ (0xBF58476D1CE4E5B9ULL * (p->id + 1))});
                    cnt.push_back((p->n + 1) / 2);
                    vh.push_back(base + 2 * p->n);
                    zz.push_back(base);
                    qq.push_back(base + p->n);
                    tp.push_back(states[i]->pc);
                    ttr.push_back(tr[i]);
                }
                auto it = elem_items(cnt);
                auto [d_rd, d_it] = stage(b, rd, it);
                launch_bphilox(d_rd, d_it, static_cast<int>(it.size()), st);
                batch_precond_apply(b, test, tp, vh, zz);
                cz.assign(zz.begin(), zz.end());
                batch_hessian<double>(b, test, ttr, 1, cz, qq, true);
                std::vector<const double*> cq(qq.begin(), qq.end());
                batch_dot(b, test, cq, cq, SC_T0);
                batch_dot(b, test, vh, vh, SC_T1);
                std::vector<double> s2 = batch_read_scal(b);
                for (int i : test) {
                    inf[i].kappa_re = std::sqrt(s2[16 * i + SC_T0] / s2[16 * i + SC_T1]);
                    if (inf[i].kappa_re < o->reuse_eps) {
                        use[i] = states[i]->pc;
                        inf[i].reused = 1;
                        b->probs[i]->cnt.reuses += 1;
                    }
                }
            }
            std::vector<int> need;
            std::vector<const rp4d_traj*> ntr;
            for (int i = 0; i < np; ++i)
                if (!use[i]) {
                    need.push_back(i);
                    ntr.push_back(tr[i]);
                }
            if (!need.empty()) {
                std::vector<rp4d_precond*> pcs = batch_nystrom(b, need, ntr, o->ell, o->seed, o->sketch_dtype);
                for (size_t q = 0; q < need.size(); ++q) {
                    const int i = need[q];
                    if (states[i]->pc) rp4d_precond_destroy(states[i]->pc);
                    states[i]->pc = pcs[q];
                    states[i]->pc_live = true;
                    use[i] = pcs[q];
                    inf[i].sketched = 1;
                }
            }
        }
        // 5. PCG
        std::vector<const double*> rhs(bm.begin(), bm.end());
        std::vector<int> conv;
        std::vector<double> relres;
        std::vector<int> its = batch_pcg(b, sel, ctr, use, rhs, dv, o->rtol, o->maxit, conv, &relres);
        // 6. v += dv, x = x_b + Gamma^{1/2} v
        {
            std::vector<BAxpby> ad;
            for (int i = 0; i < np; ++i) ad.push_back(BAxpby{dv[i], vm[i], static_cast<size_t>(b->probs[i]->n), 1.0, nullptr, 1.0});
            batch_axpby(b, ad);
        }
        batch_bhalf<double>(b, sel, 1, v, 1, xm, 1, xb);
        bool all_conv = true;
        for (int i = 0; i < np; ++i) {
            inf[i].pcg_iters = its[i];
            inf[i].sketch_ell = use[i] ? use[i]->ell : 0;
            inf[i].pcg_converged = conv[i];
            inf[i].pcg_relres = relres[i];
            all_conv = all_conv && conv[i];
            if (infos) infos[i] = inf[i];
        }
        RP4D_HIP(hipStreamSynchronize(st));
        if (!all_conv) fail(RP4D_ENOCONV, "PCG reached maxit before the tolerance for some problem (steps applied)");
    });
}

}  // extern "C"
