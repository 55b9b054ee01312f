// Barotropic vorticity model on the periodic unit square (the 2-D workload of
// Sec. 5.2 in periodic form): nonlinear RK4 sweep, discrete RK4 tangent-linear
// and adjoint sweeps over blocks of k perturbations, the separable Gaussian
// prior square root, and the spectral inverse Laplacian by fast Fourier
// transforms.
//
//   zeta_t = f(zeta) = -J_A(L zeta, zeta) + nu lap(zeta),   L = lap^{-1} (zero mean)
//   TLM:  f'(Y) w     = -J_A(L w, Y) - J_A(psi_Y, w) + nu lap(w)
//   ADJ:  f'(Y)^T mu  = -L J_A(Y, mu) + J_A(psi_Y, mu) + nu lap(mu)
//
// J_A is Arakawa's Jacobian (the average of the three second-order forms),
// lap the 5-point Laplacian, psi_Y = L Y.  The adjoint form follows from the
// antisymmetry of the trilinear form sum_p c J_A(a, b) under any exchange of
// its arguments and the symmetry of L and lap.
//
// Layout: a block of k fields is stored field-major ([v][j][i], one contiguous
// nx*ny field per vector); base fields are FP64.  The trajectory holds every
// state zeta_s and, per step, the RK4 stage values Y2..Y4 and their stream
// functions psi1..psi4, so the linearised sweeps recompute nothing.
//
// L and the prior are diagonal in the 2-D Fourier basis with even diagonals, so
// both are applied as F^{-1} (D .* F X) by the FFTs of fft2d.hip, two real fields
// per complex transform.
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace rp4d {
namespace {

#pragma clang fp contract(off)

// ---------------------------------------------------------------------------
// stencils
// ---------------------------------------------------------------------------
struct Nbr {
    int c, e, w, n, s, ne, se, nw, sw;  // offsets of (i,j), (i+-1,j), (i,j+-1), diagonals
};

__device__ __forceinline__ Nbr nbr(int p, int nx, int ny) {
    const int j = p / nx, i = p - j * nx;
    const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
    const int jp = j + 1 == ny ? 0 : j + 1, jm = j == 0 ? ny - 1 : j - 1;
    const int r = j * nx, rn = jp * nx, rs = jm * nx;
    return Nbr{r + i, r + ip, r + im, rn + i, rs + i, rn + ip, rs + ip, rn + im, rs + im};
}

// Arakawa J_A(a, b) * 12 d^2 at one point; sa, sb scale the loaded values.
template <typename T, typename TA, typename TB>
__device__ __forceinline__ T arakawa12(const TA* a, T sa, const TB* b, T sb, const Nbr& q) {
    const T ae = sa * T(a[q.e]), aw = sa * T(a[q.w]), an = sa * T(a[q.n]), as = sa * T(a[q.s]);
    const T ane = sa * T(a[q.ne]), ase = sa * T(a[q.se]), anw = sa * T(a[q.nw]), asw = sa * T(a[q.sw]);
    const T be = sb * T(b[q.e]), bw = sb * T(b[q.w]), bn = sb * T(b[q.n]), bs = sb * T(b[q.s]);
    const T bne = sb * T(b[q.ne]), bse = sb * T(b[q.se]), bnw = sb * T(b[q.nw]), bsw = sb * T(b[q.sw]);
    const T jpp = (ae - aw) * (bn - bs) - (an - as) * (be - bw);
    const T jpx = ae * (bne - bse) - aw * (bnw - bsw) - an * (bne - bnw) + as * (bse - bsw);
    const T jxp = bn * (ane - anw) - bs * (ase - asw) - be * (ane - ase) + bw * (anw - asw);
    return jpp + jpx + jxp;
}

template <typename T, typename TA>
__device__ __forceinline__ T lap5x(const TA* a, T sa, const Nbr& q) {
    // (sum of the four neighbours - 4 a) * d^2 lap
    const T c = sa * T(a[q.c]);
    return sa * T(a[q.e]) + sa * T(a[q.w]) + sa * T(a[q.n]) + sa * T(a[q.s]) - T(4) * c;
}

__constant__ double kRkB[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

// Nonlinear stage: K = -J_A(psi, Y) + nu lap(Y); acc collects the RK sum;
// stages 0-2 write the next stage input z + c K, stage 3 the new state.
__global__ void __launch_bounds__(256) bve_fwd_stage(const double* __restrict__ z, const double* __restrict__ Y,
                                                      const double* __restrict__ psi, double* __restrict__ acc,
                                                      double* __restrict__ out, int stage, double cnext, double h,
                                                      double inv12d2, double nu_d2, int nx, int ny) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nx * ny) return;
    const Nbr q = nbr(p, nx, ny);
    const double K = -(arakawa12<double>(psi, 1.0, Y, 1.0, q) * inv12d2) + nu_d2 * lap5x<double>(Y, 1.0, q);
    const double zv = z[p];
    if (stage == 0) {
        acc[p] = K * kRkB[0];
        out[p] = zv + cnext * K;
    } else if (stage < 3) {
        acc[p] = acc[p] + K * kRkB[stage];
        out[p] = zv + cnext * K;
    } else {
        out[p] = zv + h * (acc[p] + K * kRkB[3]);
    }
}

// TLM stage for k fields (grid.y = vector): kv = -J_A(phi, Y) - J_A(psi, w) + nu lap(w).
template <typename T>
__global__ void __launch_bounds__(256) bve_tlm_stage(const T* __restrict__ w, const T* __restrict__ phi,
                                                      const double* __restrict__ Y, const double* __restrict__ psi,
                                                      T* dz, T* __restrict__ acc, T* __restrict__ wnext, int stage,
                                                      T cnext, T h, T inv12d2, T nu_d2, int nx, int ny) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = nx * ny;
    if (p >= n) return;
    const long off = static_cast<long>(blockIdx.y) * n;
    const Nbr q = nbr(p, nx, ny);
    const T kv = -(arakawa12<T>(phi + off, T(1), Y, T(1), q) * inv12d2) -
                 arakawa12<T>(psi, T(1), w + off, T(1), q) * inv12d2 + nu_d2 * lap5x<T>(w + off, T(1), q);
    const T dv = dz[off + p];
    if (stage == 0) {
        acc[off + p] = kv * T(kRkB[0]);
        wnext[off + p] = dv + cnext * kv;
    } else if (stage < 3) {
        acc[off + p] = acc[off + p] + kv * T(kRkB[stage]);
        wnext[off + p] = dv + cnext * kv;
    } else {
        dz[off + p] = dv + h * (acc[off + p] + kv * T(kRkB[3]));
    }
}

// ADJ stage, first half: jq = J_A(Y, a mu) (input of L), r = J_A(psi, a mu) + nu lap(a mu).
template <typename T>
__global__ void __launch_bounds__(256) bve_adj_stencil(const T* __restrict__ mu, T a, const double* __restrict__ Y,
                                                        const double* __restrict__ psi, T* __restrict__ jq,
                                                        T* __restrict__ r, T inv12d2, T nu_d2, int nx, int ny) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = nx * ny;
    if (p >= n) return;
    const long off = static_cast<long>(blockIdx.y) * n;
    const Nbr q = nbr(p, nx, ny);
    jq[off + p] = arakawa12<T>(Y, T(1), mu + off, a, q) * inv12d2;
    r[off + p] = arakawa12<T>(psi, T(1), mu + off, a, q) * inv12d2 + nu_d2 * lap5x<T>(mu + off, a, q);
}

// ADJ stage, second half: theta = -P + r, then (stage 3) acc = lam + theta,
// (2, 1) acc += theta, with the next stage's mu = cl lam + ct theta; (0) lam = acc + theta.
template <typename T>
__global__ void __launch_bounds__(256) bve_adj_combine(const T* __restrict__ P, const T* __restrict__ r, T* lam,
                                                        T* __restrict__ acc, T* __restrict__ mu, int stage, T cl,
                                                        T ct, long count) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const T th = -P[e] + r[e];
    if (stage == 3) {
        const T l = lam[e];
        acc[e] = l + th;
        mu[e] = cl * l + ct * th;
    } else if (stage > 0) {
        acc[e] = acc[e] + th;
        mu[e] = cl * lam[e] + ct * th;
    } else {
        lam[e] = acc[e] + th;
    }
}

// Observations of k fields at one observation step: z[o][v] = x_v[idx(o)] / sigma_o.
template <typename T>
__global__ void bve_obs_gather(const T* __restrict__ x, int k, int n, int nx, int stride, int nox, int n_obs,
                               T inv_sigma, T* __restrict__ z) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_obs * k) return;
    const int o = e / k, v = e - o * k;
    const int idx = (o / nox) * stride * nx + (o % nox) * stride;
    z[e] = x[static_cast<long>(v) * n + idx] * inv_sigma;
}

// Adjoint of the above: lam_v[idx(o)] += w[o][v] / sigma_o.
template <typename T>
__global__ void bve_obs_scatter(const T* __restrict__ w, int k, int n, int nx, int stride, int nox, int n_obs,
                                T inv_sigma, T* __restrict__ lam) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_obs * k) return;
    const int o = e / k, v = e - o * k;
    const int idx = (o / nox) * stride * nx + (o % nox) * stride;
    const long a = static_cast<long>(v) * n + idx;
    lam[a] = lam[a] + w[e] * inv_sigma;
}

// Nonlinear observations and innovations of one state.
__global__ void bve_obs_fwd(const double* __restrict__ x, int nx, int stride, int nox, int n_obs,
                            const double* __restrict__ y, double inv_sigma, double* __restrict__ innov,
                            double* __restrict__ obs) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obs) return;
    const double v = x[(o / nox) * stride * nx + (o % nox) * stride];
    if (obs) obs[o] = v;
    if (innov) innov[o] = (v - y[o]) * inv_sigma;
}

// out (blocked out_kc layout) = field-major in (+ addv, same layout as out).
template <typename T>
__global__ void bve_from_fields(const T* __restrict__ in, int n, int k, T* __restrict__ out, int out_kc,
                                const T* __restrict__ addv) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<long>(n) * k) return;
    const int v = static_cast<int>(e / n), p = static_cast<int>(e - static_cast<long>(v) * n);
    const long o = (static_cast<long>(v / out_kc) * n + p) * out_kc + v % out_kc;
    T val = in[e];
    if (addv) val = val + addv[o];
    out[o] = val;
}

// field-major out = in (blocked in_kc layout).
template <typename T>
__global__ void bve_to_fields(const T* __restrict__ in, int in_kc, int n, int k, T* __restrict__ out) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<long>(n) * k) return;
    const int v = static_cast<int>(e / n), p = static_cast<int>(e - static_cast<long>(v) * n);
    out[e] = in[(static_cast<long>(v / in_kc) * n + p) * in_kc + v % in_kc];
}

template <typename T>
__global__ void bve_zero(T* x, long count) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < count) x[e] = T(0);
}

inline unsigned ublk(long count, int t = 256) { return static_cast<unsigned>((count + t - 1) / t); }

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
inline hipStream_t bst(const rp4d_problem* p) { return p->ctx->stream; }

// Twiddles exp(-2 pi i m / n) of the two axes and the two diagonals (ny x nx,
// FFT order, 1/(nx ny) folded in) in the working precision.
template <typename T>
struct Spec {
    const T *Wx, *Wy, *Dlap, *Dpri;
};

template <typename T>
Spec<T> spec_of(const rp4d_problem* p) {
    const BveData& b = *p->bve;
    const T* tw = sizeof(T) == 8 ? b.tw.as<T>() : b.tw_f.as<T>();
    Spec<T> r;
    r.Wx = tw;
    r.Wy = tw + 2 * b.nx;
    r.Dlap = sizeof(T) == 8 ? b.dlap.as<T>() : b.dlap_f.as<T>();
    r.Dpri = sizeof(T) == 8 ? b.dpri.as<T>() : b.dpri_f.as<T>();
    return r;
}

// out = F^{-1} (D .* F X) for k field-major fields X (out may alias X): the
// fields go through the FFT as ceil(k/2) complex pairs held in t1 .. t1 + 2kn,
// which must be the two consecutive k-field scratch blocks t1, t2.
template <typename T>
void spectral_apply(rp4d_problem* p, int k, const T* X, const T* D, T* out, T* t1, T* t2) {
    const BveData& b = *p->bve;
    const long n = static_cast<long>(b.nx) * b.ny;
    RP4D_REQUIRE(t2 == t1 + static_cast<long>(k) * n, RP4D_EINVAL, "spectral scratch must be two consecutive blocks");
    // FFT-equivalent flops: one complex 2-D transform pair (5 N log2 N each) per two fields
    const double fl = 5.0 * static_cast<double>(n) * std::log2(static_cast<double>(n)) * k;
    KernelTimer kt(p->ctx, RP4D_K_GEMM, fl);
    const Spec<T> sp = spec_of<T>(p);
    launch_spectral_diag<T>(X, k, b.nx, b.ny, D, sp.Wx, sp.Wy, t1, out, bst(p));
}

// Per-point flop counts of the stencil kernels (Arakawa form 34 incl. the
// scaling, 5-point Laplacian 5 + 1).
constexpr double FL_ARAKAWA = 34.0, FL_LAP = 6.0;

template <typename T>
T* ws_fields(rp4d_problem* p, int k, int count) {
    const size_t bytes = static_cast<size_t>(count) * k * p->n * sizeof(T);
    p->bve->ws.ensure(bytes);
    return p->bve->ws.as<T>();
}

inline const double* state_row(const rp4d_traj* tr, int s) {
    return tr->states.as<double>() + static_cast<size_t>(s) * tr->p->n;
}
// stage value Y_i (i = 0..3) and stream function psi_i of step s
inline const double* stage_Y(const rp4d_traj* tr, int s, int i) {
    return i == 0 ? state_row(tr, s) : tr->stages.as<double>() + (static_cast<size_t>(s) * 7 + i - 1) * tr->p->n;
}
inline const double* stage_psi(const rp4d_traj* tr, int s, int i) {
    return tr->stages.as<double>() + (static_cast<size_t>(s) * 7 + 3 + i) * tr->p->n;
}

}  // namespace

// ---------------------------------------------------------------------------
void bve_setup(rp4d_problem* p) {
    const rp4d_problem_desc& d = p->d;
    auto* b = new BveData();
    p->bve.reset(b);
    b->nx = d.nx;
    b->ny = d.ny;
    b->d = 1.0 / d.nx;
    const int nx = d.nx, ny = d.ny;
    RP4D_REQUIRE(fft_size_supported(nx) && fft_size_supported(ny), RP4D_EINVAL,
                 "2-D grid: sides must be 16 B with B in {2,3,4,5,6,8,10,12,16,20,24,32}");
    // wavenumber of FFT index c on an n-point axis (|.| is what the diagonals need)
    auto wn = [](int c, int n) { return c <= n / 2 ? c : n - c; };
    // eigenvalues of the circulant square root of the Gaussian kernel (cell units):
    // s(m) = sum_i g(min(i, n-i)) cos(2 pi m i / n), g(r) = a exp(-r^2/L^2), a^2 = 1/(L sqrt(pi/2))
    auto root_eigs = [&](int n) {
        const double L = d.L_b;
        const double a = std::sqrt(1.0 / (L * std::sqrt(M_PI / 2.0)));
        std::vector<double> s(n / 2 + 1);
        for (int m = 0; m <= n / 2; ++m) {
            double acc = 0.0;
            for (int i = 0; i < n; ++i) {
                const double r = std::min(i, n - i);
                const long q = (static_cast<long>(m) * i) % n;
                acc += a * std::exp(-(r * r) / (L * L)) * std::cos(2.0 * M_PI * static_cast<double>(q) / n);
            }
            s[m] = acc;
        }
        return s;
    };
    // twiddles exp(-2 pi i m / n), m < n, of the x axis then the y axis
    std::vector<double> tw;
    tw.reserve(2 * (nx + ny));
    for (int n : {nx, ny})
        for (int m = 0; m < n; ++m) {
            const double th = 2.0 * M_PI * static_cast<double>(m) / n;
            tw.push_back(std::cos(th));
            tw.push_back(-std::sin(th));
        }
    const std::vector<double> sx = root_eigs(nx), sy = root_eigs(ny);
    std::vector<double> dl(static_cast<size_t>(nx) * ny), dp(dl.size());
    const double tp2 = 4.0 * M_PI * M_PI, inv_n = 1.0 / (static_cast<double>(nx) * ny);
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            const int my = wn(r, ny), mx = wn(c, nx);
            const double k2 = tp2 * (static_cast<double>(my) * my + static_cast<double>(mx) * mx);
            dl[static_cast<size_t>(r) * nx + c] = (k2 > 0 ? -1.0 / k2 : 0.0) * inv_n;
            dp[static_cast<size_t>(r) * nx + c] = d.sigma_b * sy[my] * sx[mx] * inv_n;
        }
    // copies on the context stream (never the legacy stream), completed before the
    // host tables go out of scope
    auto upload = [&](DevBuf& dst, DevBuf& dstf, const std::vector<double>& h) {
        dst.ensure(h.size() * sizeof(double));
        RP4D_HIP(hipMemcpyAsync(dst.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, bst(p)));
        std::vector<float> f(h.begin(), h.end());
        dstf.ensure(f.size() * sizeof(float));
        RP4D_HIP(hipMemcpyAsync(dstf.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, bst(p)));
        RP4D_HIP(hipStreamSynchronize(bst(p)));
    };
    upload(b->tw, b->tw_f, tw);
    upload(b->dlap, b->dlap_f, dl);
    upload(b->dpri, b->dpri_f, dp);
}

size_t bve_traj_stage_bytes(const rp4d_problem* p) { return static_cast<size_t>(p->s_last) * 7 * p->n * sizeof(double); }

// Nonlinear sweep from x0 over the window.  With a trajectory, every state and
// the stage values / stream functions of every step are stored; without one
// (synthesis) only the observations are produced.
void bve_fwd(rp4d_problem* p, const double* x0, rp4d_traj* tr, double* innov, double* obs_out) {
    const int n = p->n, nx = p->bve->nx, ny = p->bve->ny;
    hipStream_t st = bst(p);
    const double h = p->d.dt, dd = p->bve->d;
    const double inv12d2 = 1.0 / (12.0 * dd * dd), nu_d2 = p->d.nu / (dd * dd);
    // scratch: 2 state rows, 7 stage fields, acc, GEMM temporaries (2)
    p->bve->ws_fwd.ensure(static_cast<size_t>(12) * n * sizeof(double));
    double* w = p->bve->ws_fwd.as<double>();
    double* rows2 = w;
    double* stg = w + 2 * n;
    double* acc = w + 9 * n;
    double* t1 = w + 10 * n;
    double* t2 = w + 11 * n;
    const int stride = p->d.obs_stride, nox = (nx + stride - 1) / stride;
    auto zrow = [&](int s) -> double* {
        return tr ? tr->states.as<double>() + static_cast<size_t>(s) * n : rows2 + static_cast<size_t>(s & 1) * n;
    };
    auto Ys = [&](int s, int i) -> double* {
        if (i == 0) return zrow(s);
        return tr ? tr->stages.as<double>() + (static_cast<size_t>(s) * 7 + i - 1) * n : stg + static_cast<size_t>(i - 1) * n;
    };
    auto Ps = [&](int s, int i) -> double* {
        return tr ? tr->stages.as<double>() + (static_cast<size_t>(s) * 7 + 3 + i) * n : stg + static_cast<size_t>(3 + i) * n;
    };
    RP4D_HIP(hipMemcpyAsync(zrow(0), x0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    const double cn[3] = {0.5 * h, 0.5 * h, h};
    const double* Dl = spec_of<double>(p).Dlap;
    for (int s = 0; s < p->s_last; ++s) {
        const double* z = zrow(s);
        for (int i = 0; i < 4; ++i) {
            const double* Y = Ys(s, i);
            double* psi = Ps(s, i);
            spectral_apply<double>(p, 1, Y, Dl, psi, t1, t2);
            double* out = i < 3 ? Ys(s, i + 1) : zrow(s + 1);
            KernelTimer kt(p->ctx, RP4D_K_STENCIL, (FL_ARAKAWA + FL_LAP + 6.0) * n);
            bve_fwd_stage<<<ublk(n), 256, 0, st>>>(z, Y, psi, acc, out, i, i < 3 ? cn[i] : 0.0, h, inv12d2, nu_d2,
                                                   nx, ny);
        }
        const int s1 = s + 1;
        if (s1 % p->d.obs_every == 0 && s1 / p->d.obs_every <= p->n_t) {
            const int it = s1 / p->d.obs_every - 1;
            const size_t o = static_cast<size_t>(it) * p->n_obs;
            bve_obs_fwd<<<ublk(p->n_obs), 256, 0, st>>>(zrow(s1), nx, stride, nox, p->n_obs,
                                                       p->has_data ? p->y.as<double>() + o : nullptr,
                                                       1.0 / p->d.sigma_o, (innov && p->has_data) ? innov + o : nullptr,
                                                       obs_out ? obs_out + o : nullptr);
        }
    }
    RP4D_HIP(hipGetLastError());
}

template <typename T>
void bve_bhalf(rp4d_problem* p, int k, const T* in, int in_kc, T* out, int out_kc, const T* addv) {
    const int n = p->n;
    hipStream_t st = bst(p);
    p->bve->ws_bh.ensure(static_cast<size_t>(3) * k * n * sizeof(T));
    T* f = p->bve->ws_bh.as<T>();
    T* t1 = f + static_cast<size_t>(k) * n;
    T* t2 = t1 + static_cast<size_t>(k) * n;
    const long cnt = static_cast<long>(k) * n;
    bve_to_fields<T><<<ublk(cnt), 256, 0, st>>>(in, in_kc, n, k, f);
    spectral_apply<T>(p, k, f, spec_of<T>(p).Dpri, f, t1, t2);
    bve_from_fields<T><<<ublk(cnt), 256, 0, st>>>(f, n, k, out, out_kc, addv);
    RP4D_HIP(hipGetLastError());
}

template <typename T>
void bve_inv_laplacian(rp4d_problem* p, int k, const T* in, T* out) {
    const int n = p->n;
    hipStream_t st = bst(p);
    p->bve->ws_bh.ensure(static_cast<size_t>(3) * k * n * sizeof(T));
    T* f = p->bve->ws_bh.as<T>();
    T* t1 = f + static_cast<size_t>(k) * n;
    T* t2 = t1 + static_cast<size_t>(k) * n;
    const long cnt = static_cast<long>(k) * n;
    bve_to_fields<T><<<ublk(cnt), 256, 0, st>>>(in, k, n, k, f);
    spectral_apply<T>(p, k, f, spec_of<T>(p).Dlap, f, t1, t2);
    bve_from_fields<T><<<ublk(cnt), 256, 0, st>>>(f, n, k, out, k, nullptr);
    RP4D_HIP(hipGetLastError());
}

namespace {

// TLM sweep of k field-major perturbations dz (overwritten); observations to Z (n_t, n_obs, k).
template <typename T>
void tlm_sweep(rp4d_problem* p, const rp4d_traj* tr, int k, T* dz, T* Z, T* ws) {
    const int n = p->n, nx = p->bve->nx, ny = p->bve->ny;
    hipStream_t st = bst(p);
    const size_t fk = static_cast<size_t>(k) * n;
    T* wA = ws;
    T* wB = ws + fk;
    T* phi = ws + 2 * fk;
    T* acc = ws + 3 * fk;
    T* t1 = ws + 4 * fk;
    T* t2 = ws + 5 * fk;
    const double h = p->d.dt, dd = p->bve->d;
    const T inv12d2 = static_cast<T>(1.0 / (12.0 * dd * dd)), nu_d2 = static_cast<T>(p->d.nu / (dd * dd));
    const int stride = p->d.obs_stride, nox = (nx + stride - 1) / stride;
    const T cn[3] = {static_cast<T>(0.5 * h), static_cast<T>(0.5 * h), static_cast<T>(h)};
    const dim3 grid(ublk(n), k);
    const T* Dl = spec_of<T>(p).Dlap;
    for (int s = 0; s < p->s_last; ++s) {
        for (int i = 0; i < 4; ++i) {
            const T* w = i == 0 ? dz : (i == 2 ? wB : wA);
            T* wn = i == 1 ? wB : wA;  // stage 0 -> A, 1 -> B, 2 -> A
            spectral_apply<T>(p, k, w, Dl, phi, t1, t2);
            KernelTimer kt(p->ctx, RP4D_K_STENCIL, (2 * FL_ARAKAWA + FL_LAP + 6.0) * static_cast<double>(fk));
            bve_tlm_stage<T><<<grid, 256, 0, st>>>(w, phi, stage_Y(tr, s, i), stage_psi(tr, s, i), dz, acc, wn, i,
                                                    i < 3 ? cn[i] : T(0), static_cast<T>(h), inv12d2, nu_d2, nx, ny);
        }
        const int s1 = s + 1;
        if (s1 % p->d.obs_every == 0 && s1 / p->d.obs_every <= p->n_t) {
            const int it = s1 / p->d.obs_every - 1;
            bve_obs_gather<T><<<ublk(static_cast<long>(p->n_obs) * k), 256, 0, st>>>(
                dz, k, n, nx, stride, nox, p->n_obs, static_cast<T>(1.0 / p->d.sigma_o),
                Z + static_cast<size_t>(it) * p->n_obs * k);
        }
    }
    RP4D_HIP(hipGetLastError());
}

// ADJ sweep with forcing W (n_t, n_obs, k); lambda_0 (field-major) left in lam.
template <typename T>
void adj_sweep(rp4d_problem* p, const rp4d_traj* tr, int k, const T* W, T* lam, T* ws) {
    const int n = p->n, nx = p->bve->nx, ny = p->bve->ny;
    hipStream_t st = bst(p);
    const size_t fk = static_cast<size_t>(k) * n;
    T* mu = ws;
    T* jq = ws + fk;
    T* r = ws + 2 * fk;
    T* P = ws + 3 * fk;
    T* acc = ws + 4 * fk;
    T* t1 = ws + 5 * fk;
    T* t2 = ws + 6 * fk;
    const double h = p->d.dt, dd = p->bve->d;
    const T inv12d2 = static_cast<T>(1.0 / (12.0 * dd * dd)), nu_d2 = static_cast<T>(p->d.nu / (dd * dd));
    const int stride = p->d.obs_stride, nox = (nx + stride - 1) / stride;
    const dim3 grid(ublk(n), k);
    const T* Dl = spec_of<T>(p).Dlap;
    // mu of the next (lower) stage: (h/3, h), (h/3, h/2), (h/6, h/2)
    const T cl[4] = {T(0), static_cast<T>(h / 6.0), static_cast<T>(h / 3.0), static_cast<T>(h / 3.0)};
    const T ct[4] = {T(0), static_cast<T>(0.5 * h), static_cast<T>(0.5 * h), static_cast<T>(h)};
    bve_zero<T><<<ublk(fk), 256, 0, st>>>(lam, static_cast<long>(fk));
    for (int s = p->s_last; s >= 1; --s) {
        if (s % p->d.obs_every == 0 && s / p->d.obs_every <= p->n_t) {
            const int it = s / p->d.obs_every - 1;
            bve_obs_scatter<T><<<ublk(static_cast<long>(p->n_obs) * k), 256, 0, st>>>(
                W + static_cast<size_t>(it) * p->n_obs * k, k, n, nx, stride, nox, p->n_obs,
                static_cast<T>(1.0 / p->d.sigma_o), lam);
        }
        for (int i = 3; i >= 0; --i) {
            {
                KernelTimer kt(p->ctx, RP4D_K_STENCIL, (2 * FL_ARAKAWA + FL_LAP + 2.0) * static_cast<double>(fk));
                bve_adj_stencil<T><<<grid, 256, 0, st>>>(i == 3 ? lam : mu, i == 3 ? static_cast<T>(h / 6.0) : T(1),
                                                          stage_Y(tr, s - 1, i), stage_psi(tr, s - 1, i), jq, r,
                                                          inv12d2, nu_d2, nx, ny);
            }
            spectral_apply<T>(p, k, jq, Dl, P, t1, t2);
            bve_adj_combine<T><<<ublk(fk), 256, 0, st>>>(P, r, lam, acc, mu, i, cl[i], ct[i], static_cast<long>(fk));
        }
    }
    RP4D_HIP(hipGetLastError());
}

}  // namespace

template <typename T>
void bve_tlm(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* Z) {
    T* ws = ws_fields<T>(p, k, 8);
    T* dz = ws + static_cast<size_t>(6) * k * p->n;
    bve_bhalf<T>(p, k, V, k, dz, 1, nullptr);  // blocked kc = 1 is field-major
    tlm_sweep<T>(p, tr, k, dz, Z, ws);
}

template <typename T>
void bve_adj(rp4d_problem* p, const rp4d_traj* tr, int k, const T* W, T* U, const T* addv) {
    T* ws = ws_fields<T>(p, k, 8);
    T* lam = ws + static_cast<size_t>(7) * k * p->n;
    adj_sweep<T>(p, tr, k, W, lam, ws);
    bve_bhalf<T>(p, k, lam, 1, U, k, addv);
}

template <typename T>
void bve_hessian(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* HV, bool add_identity) {
    T* ws = ws_fields<T>(p, k, 8);
    p->bve->ws_obs.ensure(static_cast<size_t>(p->m) * k * sizeof(T));
    T* Z = p->bve->ws_obs.as<T>();
    T* dz = ws + static_cast<size_t>(6) * k * p->n;
    T* lam = ws + static_cast<size_t>(7) * k * p->n;
    bve_bhalf<T>(p, k, V, k, dz, 1, nullptr);
    tlm_sweep<T>(p, tr, k, dz, Z, ws);
    adj_sweep<T>(p, tr, k, Z, lam, ws);
    bve_bhalf<T>(p, k, lam, 1, HV, k, add_identity ? V : nullptr);
}

template void bve_bhalf<double>(rp4d_problem*, int, const double*, int, double*, int, const double*);
template void bve_bhalf<float>(rp4d_problem*, int, const float*, int, float*, int, const float*);
template void bve_inv_laplacian<double>(rp4d_problem*, int, const double*, double*);
template void bve_inv_laplacian<float>(rp4d_problem*, int, const float*, float*);
template void bve_tlm<double>(rp4d_problem*, const rp4d_traj*, int, const double*, double*);
template void bve_tlm<float>(rp4d_problem*, const rp4d_traj*, int, const float*, float*);
template void bve_adj<double>(rp4d_problem*, const rp4d_traj*, int, const double*, double*, const double*);
template void bve_adj<float>(rp4d_problem*, const rp4d_traj*, int, const float*, float*, const float*);
template void bve_hessian<double>(rp4d_problem*, const rp4d_traj*, int, const double*, double*, bool);
template void bve_hessian<float>(rp4d_problem*, const rp4d_traj*, int, const float*, float*, bool);

}  // namespace rp4d
