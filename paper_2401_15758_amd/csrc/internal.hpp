// Internal declarations of the rp4d HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "rp4d.h"
#include "sweep_types.hpp"

namespace rp4d {

struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);

#define RP4D_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::rp4d::fail(RP4D_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define RP4D_REQUIRE(cond, code, msg)          \
    do {                                       \
        if (!(cond)) ::rp4d::fail((code), (msg)); \
    } while (0)

// Growable device buffer owned by a library handle.
// The HIP device current at construction: library objects keep it so that
// their destruction never reads the object that created them (owners and
// children may be destroyed in any order).
inline int construction_device() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

// Device bytes held through one context's objects, against the context's budget
// (0: none).  Shared by the context and every buffer allocated for it, so either
// may be destroyed first.
struct HbmAcct {
    std::atomic<long long> used{0};
    long long budget = 0;
};
// The accounting of the context whose call is running on this thread (set with
// the device at the start of a call, cleared at its end).
extern thread_local std::shared_ptr<HbmAcct> tl_acct;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    std::shared_ptr<HbmAcct> acct;  // the context the bytes are counted against
    // a view of memory the buffer does not own (the no-allocation entry point's
    // static scratch): ensure() fails instead of reallocating, release() frees nothing
    bool borrowed = false;
    void ensure(size_t b);
    void release();
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
    void swap(DevBuf& o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(borrowed, o.borrowed);
        std::swap(acct, o.acct);
    }
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
};

// ---------------------------------------------------------------------------
// Block sweeps of the Burgers model
// ---------------------------------------------------------------------------
void launch_burgers_fwd(const FwdArgs& a, const Tiling& t, hipStream_t st);
// Batched forms: `args` (device) holds one argument block per problem, `items`
// (device) one int4 (problem, tile, group, -) per workgroup.
void launch_burgers_fwd_batched(const FwdArgs* args, const int4* items, int nitems, const Tiling& t, hipStream_t st);
template <typename T>
void launch_burgers_sweep_batched(int mode, const SweepArgs<T>* args, const int4* items, int nitems, const Tiling& t,
                                  hipStream_t st);
template <typename T>
void launch_burgers_sweep(int mode, const SweepArgs<T>& a, const Tiling& t, int ngroups, hipStream_t st);
// Wall-bounded RK3-TVD sweeps (wave regions only; the tiling's exchange field
// is not consulted).  launch_burgers_fwd / launch_burgers_sweep forward here
// when the arguments' wall flag is set.
void launch_wall_fwd(const FwdArgs& a, const Tiling& t, hipStream_t st);
template <typename T>
void launch_wall_sweep(int mode, const SweepArgs<T>& a, const Tiling& t, int ngroups, hipStream_t st);

// ---------------------------------------------------------------------------
// Prior square root, layouts and tall-skinny dense kernels
// ---------------------------------------------------------------------------
// Blocked layout of k vectors of length n in groups of kc: element (j, c) at
// ((c / kc) * n + j) * kc + c % kc.  The row-major (n, k) layout is kc = k.
template <typename T>
void launch_circ_conv(const T* in, int in_kc, T* out, int out_kc, const double* gk, int D, int n, int k,
                      const T* addv, hipStream_t st);
template <typename TI, typename TO>
void launch_relayout(const TI* in, int in_kc, TO* out, int out_kc, int n, int k, hipStream_t st);
template <typename T>
void launch_fill(T* p, size_t count, T v, hipStream_t st);

// Matrix operands below use the blocked layout: element (row, col) of an
// n-row operand with layout parameter kc sits at ((col / kc) * n + row) * kc + col % kc,
// so a row-major n x w matrix is kc = w.
// C (a x b, row-major, FP64) = X^T Y; X (n x a, layout lx), Y (n x b, layout ly).
// Deterministic two-stage reduction; `work` must hold gram_work_doubles(n,a,b).
template <typename TX, typename TY>
void launch_gram(const TX* X, int lx, const TY* Y, int ly, int n, int a, int b, double* C, double* work,
                 hipStream_t st);
size_t gram_work_doubles(int n, int a, int b);
// The same Gram with both operands rounded to bfloat16 on the BF16 matrix cores
// (FP32 accumulation per chunk, chunks summed in FP64); same `work`.
template <typename TX, typename TY>
void launch_gram_bf16(const TX* X, int lx, const TY* Y, int ly, int n, int a, int b, double* C, double* work,
                      hipStream_t st);
// Out (n x b) = beta * Cin + alpha * X (n x a) * diag(dscale) * M (a x b); M row-major a x b (FP64).
// Cin may equal Out (in-place) ; dscale may be null.
template <typename TX, typename TO>
void launch_tsmm(const TX* X, int lx, const double* M, const double* dscale, int n, int a, int b, double alpha,
                 const TO* Cin, int lc, double beta, TO* Out, int lo, hipStream_t st);
// y = alpha * x + beta * y over count elements (FP64)
void launch_axpby(const double* x, double alpha, double* y, double beta, size_t count, hipStream_t st);

// ---------------------------------------------------------------------------
// Small dense FP64 linear algebra on one workgroup (l <= 128)
// ---------------------------------------------------------------------------
// In-place lower Cholesky of sym((A + A^T)/2) (lda = l); info[0] = 0 ok, j+1 if pivot j <= 0.
void launch_chol(double* A, int l, int* info, hipStream_t st);
// Linv = inverse of lower-triangular L (both l x l row-major).
void launch_trinv(const double* L, double* Linv, int l, hipStream_t st);
// The Cholesky factor of A (as launch_chol, in place) and L^{-T} into LinvT in
// one launch, for l <= 64 (bitwise the results of launch_chol, launch_trinv and
// a transpose); false (nothing launched) for larger orders.
bool launch_chol_invt(double* A, int l, int* info, double* LinvT, hipStream_t st);
// C = op(A) op(B) (l x l row-major each); ta/tb: transpose flags; alpha scaling.
void launch_small_gemm(const double* A, int ta, const double* B, int tb, double* C, int l, double alpha,
                       hipStream_t st);
// Symmetric eigendecomposition (cyclic Jacobi): A (l x l, destroyed) -> evals (desc), evecs (columns, row-major).
void launch_jacobi_eig(double* A, double* evals, double* evecs, int l, hipStream_t st);
// Whether `dyn` bytes of dynamic LDS fit beside kernel `fn`'s static LDS on this device.
bool lds_fits(const void* fn, size_t dyn);
// lambda_max of a symmetric PSD l x l matrix into out[0] (G untouched; `work`
// holds l*l doubles, used when l > 64; for l > 64 out must hold l doubles).
void launch_sym_lmax(const double* G, int l, double* out, double* work, hipStream_t st);

// ---------------------------------------------------------------------------
// Reductions, PCG helpers and RNG
// ---------------------------------------------------------------------------
// out[0] = sum x*y (deterministic); work >= dot_work_doubles(count)
void launch_dot(const double* x, const double* y, size_t count, double* out, double* work, hipStream_t st);
size_t dot_work_doubles(size_t count);
void launch_philox_normal(uint64_t seed, size_t count, double* out, hipStream_t st);
template <typename T>
void launch_philox_normal_t(uint64_t seed, size_t count, T* out, hipStream_t st);

// ---------------------------------------------------------------------------
// Batched kernels (batch_kernels.hip): descriptor arrays in device memory, one
// entry per problem; `items` = int4 work items (problem, block, block, -).
// ---------------------------------------------------------------------------
struct BGram {        // C (a x b, row-major) = X^T Y over n rows, chunks of `rows` rows
    const void* X;
    const void* Y;
    double* C;
    int n, a, b, lx, ly;
    int rows;         // rows per chunk (set by the batch driver)
    double* part;     // chunk partial sums: ceil(n/rows) * a * b doubles
};
struct BTsmm {        // Out = beta C + alpha X diag(ds) M
    const void* X;
    const double* M;
    const double* ds;
    const void* C;
    void* Out;
    int n, a, b, lx, lc, lo;
    double alpha, beta;
};
struct BSmall {       // l x l operands
    double* A;
    double* B;
    double* C;
    int* info;
};
struct BVec {         // out = x . y (or max |x|)
    const double* x;
    const double* y;
    double* out;
    int n;
};
struct BAxpby {       // y = alpha (alpha_d ? *alpha_d : 1) x + beta y (x may be null: 0)
    const double* x;
    double* y;
    size_t count;
    double alpha;
    const double* alpha_d;
    double beta;
};
struct BPcg {         // PCG vectors and scalars (sc[0] = rz, sc[1] = pq, sc[2] = rz_new)
    double *x, *r, *p, *q, *z;
    double* sc;
    int n;
};
struct BSketch {      // sketch finalisation
    const double* ev;
    double* nu;
    double* lam;
    double* D;
    double* U;
    int n;
};
struct BRand {
    double* out;
    size_t count;
    uint64_t seed;
};
struct BCopy {        // dst(j, c) = src(j, c) (or 0), layouts skc / dkc
    const void* src;
    void* dst;
    int n, k, skc, dkc, zero;
};
template <typename TX, typename TY>
void launch_bgram(const BGram* d, const int4* items, int nitems, const int4* ritems, int nritems, hipStream_t st);
template <typename TX, typename TO>
void launch_btsmm(const BTsmm* d, const int4* items, int nitems, hipStream_t st);
void launch_bchol(const BSmall* d, int np, int l, hipStream_t st);
void launch_btrinv(const BSmall* d, int np, int l, hipStream_t st);
void launch_bgemm_small(const BSmall* d, int np, int l, int ta, int tb, double alpha, hipStream_t st);
void launch_bjacobi(const BSmall* d, int np, int l, bool wantv, hipStream_t st);
void launch_bdot(const BVec* d, int np, bool absmax, hipStream_t st);
void launch_baxpby(const BAxpby* d, const int4* items, int nitems, hipStream_t st);
void launch_bpcg_xr(const BPcg* d, const int4* items, int nitems, hipStream_t st);
void launch_bpcg_p(const BPcg* d, const int4* items, int nitems, int np, hipStream_t st);
void launch_bnu(const BSketch* d, int np, double eps, hipStream_t st);
void launch_bfinalize(const BSketch* d, int np, int l, bool use_nu, hipStream_t st);
void launch_bphilox(const BRand* d, const int4* items, int nitems, hipStream_t st);
template <typename TI, typename TO>
void launch_bcopy(const BCopy* d, const int4* items, int nitems, hipStream_t st);

}  // namespace rp4d

// ---------------------------------------------------------------------------
// Opaque handle definitions
// ---------------------------------------------------------------------------
struct rp4d_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::shared_ptr<rp4d::HbmAcct> acct = std::make_shared<rp4d::HbmAcct>();
    // kernel timing: 0 off, 1 an event pair around every launch of the timed
    // classes, 2 one pair around each Burgers sweep's launch loop (SpanTimer)
    int timing = 0;
    struct Pending {
        int kind;
        hipEvent_t a, b;
        double flops;
        long long nlaunch;
    };
    // launches and flops of the open span of each class (timing mode 2)
    bool span_open[RP4D_K_COUNT] = {};
    long long span_launches[RP4D_K_COUNT] = {};
    double span_flops[RP4D_K_COUNT] = {};
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    // second stream (default priority) for work that overlaps the main stream,
    // with the two events that fork and join it
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // graph replay of the PCG iteration body (captured on a library stream)
    bool graphs = false;
    int gram_dtype = RP4D_F64;  // Grams of the sketch's eigen-estimates: RP4D_F64 or RP4D_BF16
    bool capturing = false;
    hipStream_t cap_stream = nullptr;
    long long launches[RP4D_K_COUNT] = {};
    double ms[RP4D_K_COUNT] = {};
    double flops[RP4D_K_COUNT] = {};
    ~rp4d_ctx();
};

namespace rp4d {
// Timing scope: records an event pair around the launches issued in its
// lifetime; inside an open span of its class it only counts the launch.
struct KernelTimer {
    rp4d_ctx* c;
    int kind;
    double flops;
    hipEvent_t a = nullptr;
    KernelTimer(rp4d_ctx* ctx, int k, double fl);
    ~KernelTimer();
};
// Span of one class (timing mode 2): one event pair around a loop of launches
// whose KernelTimers count launches and flops without events of their own.
struct SpanTimer {
    rp4d_ctx* c;
    int kind;
    hipEvent_t a = nullptr;
    SpanTimer(rp4d_ctx* ctx, int k);
    ~SpanTimer();
};
}  // namespace rp4d

namespace rp4d {
// Barotropic-vorticity model data: nx x ny periodic grid (fields flattened j*nx+i).
struct BveData {
    int nx = 0, ny = 0;
    double d = 0;               // grid spacing 1/nx
    DevBuf tw, tw_f;            // exp(-2 pi i m / nx), m < nx, then exp(-2 pi i m / ny): (re, im) pairs
    DevBuf dlap, dlap_f;        // (ny, nx) in FFT order: -1/|k|^2 (0 for k = 0), divided by nx ny
    DevBuf dpri, dpri_f;        // (ny, nx) in FFT order: sigma_b s_y s_x, the prior root's eigenvalues, / (nx ny)
    DevBuf ws, ws_fwd, ws_bh, ws_obs;
};
void bve_setup(rp4d_problem* p);
// Periodic spectral operators by FFT (fft2d.hip): out = F^{-1}(D .* F in) for k
// field-major fields of an nx x ny grid; D (ny x nx) in FFT order with the
// inverse's 1/(nx ny) folded in; W* twiddle tables; z scratch of
// 2 ceil(k/2) nx ny elements.  out may alias in.
bool fft_size_supported(int n);
template <typename T>
void launch_spectral_diag(const T* in, int k, int nx, int ny, const T* D, const T* Wx, const T* Wy, T* z, T* out,
                          hipStream_t st);
// The passes on their own: row spectra of the ceil(k/2) field pairs of `in`
// into z, and the column pass (forward, times D, inverse) of z in place.
template <typename T>
void launch_fft_rows_fwd(const T* in, int k, int nx, int ny, T* z, const T* Wx, hipStream_t st);
template <typename T>
void launch_fft_cols(T* z, int k, int nx, int ny, const T* D, const T* Wy, hipStream_t st);
size_t bve_traj_stage_bytes(const rp4d_problem* p);
void bve_fwd(rp4d_problem* p, const double* x0, rp4d_traj* tr, double* innov, double* obs_out);
template <typename T>
void bve_bhalf(rp4d_problem* p, int k, const T* in, int in_kc, T* out, int out_kc, const T* addv);
template <typename T>
void bve_inv_laplacian(rp4d_problem* p, int k, const T* in, T* out);
template <typename T>
void bve_tlm(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* Z);
template <typename T>
void bve_adj(rp4d_problem* p, const rp4d_traj* tr, int k, const T* W, T* U, const T* addv);
template <typename T>
void bve_hessian(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* HV, bool add_identity);
}  // namespace rp4d

// A FWD whose launches are enqueued on another stream on demand, just ahead of
// the sweeps that read its rows: the GN step runs its FWD on the side stream
// while the sketch's TLM sweep follows on the main stream, and enqueueing the two
// launch by launch lets them overlap on the device.  Every row is stored (C = 1).
struct FwdPlan {
    bool active = false;
    rp4d_traj* tr = nullptr;
    rp4d::FwdArgs a{};
    rp4d::Tiling t{};
    hipStream_t st = nullptr;       // the stream the FWD runs on
    double* in = nullptr;           // ping-pong states
    double* out = nullptr;
    int s_next = 0, s_to = 0;       // next step to enqueue, end of the window
    int enq_row = 0;                // rows 0..enq_row are enqueued
    int marked_row = 0;             // rows 0..marked_row precede the last event
    int waited_row = -1;            // rows the consumer stream has waited for
    hipStream_t waited_st = nullptr;
    int launches = 0;
    hipEvent_t span = nullptr;      // timing: start of the FWD (pooled event)
    std::vector<hipEvent_t> ev;     // one per mark; reused by the next plan
    int next_ev = 0;
    hipEvent_t last_ev = nullptr;
    FwdPlan() = default;
    FwdPlan(const FwdPlan&) = delete;
    FwdPlan& operator=(const FwdPlan&) = delete;
    ~FwdPlan() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

struct rp4d_problem {
    int device = rp4d::construction_device();
    rp4d_ctx* ctx = nullptr;
    // work to enqueue on the side stream once the next TLM sweep on the main
    // stream has been enqueued (set by a GN step; run at most once)
    std::function<void()> after_tlm;
    FwdPlan fwd_plan;
    rp4d_problem_desc d{};
    int n = 0, n_obs = 0, n_t = 0, m = 0, s_last = 0;
    double dx = 0, inv2dx = 0, nu_dx2 = 0;
    rp4d::DevBuf xb, y;
    bool has_data = false;
    rp4d::DevBuf gk;  // prior square-root kernel g_0..g_D
    int D = 0;
    // spectral form of the circulant prior square root: F (n x r) real Fourier
    // basis of the retained modes, lam (r) their eigenvalues
    bool wall = false;    // Dirichlet walls, RK3-TVD, SPDE prior (the paper's Burgers setup)
    bool spec = false;
    int r = 0;
    rp4d::DevBuf F, lamF, ws_bh;
    // workspaces
    rp4d::DevBuf ws_s0, ws_s1, ws_obs, ws_blk, ws_red, ws_scal, ws_seg, ws_pcg, ws_bg;
    rp4d::DevBuf ws_ad;  // adaptive sketch: accumulated basis Q (m x l_max), W^T (n x l_max), small blocks
    // the side lane's copies of the sweep / prior / segment workspaces (the
    // gradient's ADJ sweep runs there while the sketch runs on the main stream)
    rp4d::DevBuf side_s0, side_s1, side_obs, side_bh, side_seg, side_red;
    rp4d_counters cnt{};
    uint64_t id = 0;  // caller-chosen identity: seeds the batched random draws
    std::map<std::tuple<int, int, int>, rp4d::Tiling> tiling;  // (mode, dtype, k)
    std::unique_ptr<rp4d::BveData> bve;                          // set for the 2-D model
};

struct rp4d_traj {
    int device = rp4d::construction_device();
    rp4d_problem* p = nullptr;
    rp4d::DevBuf states;  // rows of u_s (every C-th when checkpointing)
    rp4d::DevBuf innov;   // (n_t, n_obs)
    rp4d::DevBuf stages;  // 2-D model: per step the stage values Y2..Y4 and stream functions psi1..psi4
    int C = 1;
    int rows = 0;
    bool valid = false, has_innov = false;
};


struct rp4d_precond {
    int device = rp4d::construction_device();
    rp4d_problem* p = nullptr;
    int ell = 0;
    rp4d::DevBuf V;       // (n, ell) row-major
    rp4d::DevBuf Dg;      // lam / (1 + lam); all ones in the factored form
    rp4d::DevBuf lamd;    // device: lam (ell), then nu (not formed in the factored form)
    bool fast = false;    // factored form V = W^T chol(I + W W^T)^{-T}, no eigenvalues
    // host copies of lamd, fetched on first use after a build
    mutable bool host_ok = false;
    mutable std::vector<double> lam;
    mutable double nu = 0.0;
};

struct rp4d_gn_state {
    int device = rp4d::construction_device();
    rp4d_problem* p = nullptr;
    rp4d::DevBuf v, x, dv, g, b;
    rp4d_traj* traj = nullptr;
    rp4d_precond* pc = nullptr;  // kept allocated across resets; rebuilt in place
    bool pc_live = false;        // pc holds the current resident preconditioner
};
