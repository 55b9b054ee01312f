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

#include "fft_line.hpp"
#include "internal.hpp"

namespace rp4d {
namespace {

// A multiply-add within one expression may fuse: the 2-D kernels have one
// arithmetic per operator (no tiling choices), so results stay reproducible.
#pragma clang fp contract(on)

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

// ---------------------------------------------------------------------------
// Fused row stages of the linearised sweeps.  One launch per RK stage does the
// row-local work of the stage -- the inverse row FFTs of the column-passed
// spectra (the Poisson solve's last pass), the stencils and RK updates, and
// the forward row FFTs of the next stage's input (the next solve's first pass)
// -- so that a stage is this launch plus the column pass.  A workgroup owns
// kRowsOwn rows of one field pair and transforms one halo row on each side
// (the stencils reach one row out); 16 threads per row line, as in fft2d.hip.
// ---------------------------------------------------------------------------
constexpr int kRowsOwn = fftl::kLines - 2;

// 12 d^2 J_A(a, b) and the 5-point Laplacian times d^2 on 3 x 3 neighbourhoods
// v[dj + 1][di + 1] (the same operations, in the same order, as arakawa12 / lap5x).
template <typename T>
__device__ __forceinline__ T arakawa12_nb(const T (&a)[3][3], const T (&b)[3][3]) {
    const T ae = a[1][2], aw = a[1][0], an = a[2][1], as = a[0][1];
    const T ane = a[2][2], ase = a[0][2], anw = a[2][0], asw = a[0][0];
    const T be = b[1][2], bw = b[1][0], bn = b[2][1], bs = b[0][1];
    const T bne = b[2][2], bse = b[0][2], bnw = b[2][0], bsw = b[0][0];
    const T jpp = (ae - aw) * (bn - bs) - (an - as) * (be - bw);
    const T jpx = ae * (bne - bse) - aw * (bnw - bsw) - an * (bne - bnw) + as * (bse - bsw);
    const T jxp = bn * (ane - anw) - bs * (ase - asw) - be * (ane - ase) + bw * (anw - asw);
    return jpp + jpx + jxp;
}

template <typename T>
__device__ __forceinline__ T lap5_nb(const T (&a)[3][3]) {
    return a[1][2] + a[1][0] + a[2][1] + a[0][1] - T(4) * a[1][1];
}

// 3 x 3 neighbourhood of (j, i) of a global field (periodic).
template <typename T, typename S>
__device__ __forceinline__ void load9(const S* __restrict__ f, int nx, int ny, int j, int i, T (&o)[3][3]) {
    const int r[3] = {j == 0 ? ny - 1 : j - 1, j, j + 1 == ny ? 0 : j + 1};
    const int c[3] = {i == 0 ? nx - 1 : i - 1, i, i + 1 == nx ? 0 : i + 1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) o[a][b] = static_cast<T>(f[static_cast<size_t>(r[a]) * nx + c[b]]);
}

// 3 x 3 neighbourhood of (owned row jr, column i) from the LDS row lines
// (line 0 is the row above the block), real (f = 0) or imaginary (f = 1) part.
template <typename T, int N>
__device__ __forceinline__ void lds9(const fftl::C2<T>* lds, int jr, int i, int f, T (&o)[3][3]) {
    const int c[3] = {i == 0 ? N - 1 : i - 1, i, i + 1 == N ? 0 : i + 1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const fftl::C2<T> v = lds[(jr + a) * fftl::padded(N) + fftl::padded(c[b])];
            o[a][b] = f ? v.i : v.r;
        }
}

// 3 x 3 neighbourhood of (owned row jr, column i) from rows staged in LDS, row r
// at rows + r N.
template <typename T, int N>
__device__ __forceinline__ void st9(const T* rows, int jr, int i, T (&o)[3][3]) {
    const int c[3] = {i == 0 ? N - 1 : i - 1, i, i + 1 == N ? 0 : i + 1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) o[a][b] = rows[(jr + a) * N + c[b]];
}

// Row spectra of line l = threadIdx / 16 (row j0 - 1 + l, periodic) of pair p:
// the B values of thread q, or nothing on lines past rown + 1.
template <typename T, int B>
__device__ __forceinline__ void rows_spec_load(const T* __restrict__ z, int p, int j0, int rown, int ny,
                                               fftl::C2<T> (&v)[B]) {
    constexpr int N = 16 * B;
    const int l = threadIdx.x >> 4, q = threadIdx.x & 15;
    if (l < rown + 2) {
        int jj = j0 - 1 + l;
        jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
        const T* zr = z + (static_cast<size_t>(p) * N * ny + static_cast<size_t>(jj) * N) * 2;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int i = q + 16 * e;
            v[e] = fftl::C2<T>{zr[2 * i], zr[2 * i + 1]};
        }
    }
}

template <typename T, int B>
__device__ __forceinline__ void rows_spec_store(fftl::C2<T>* lds, int rown, const fftl::C2<T> (&v)[B]) {
    constexpr int N = 16 * B;
    const int l = threadIdx.x >> 4, q = threadIdx.x & 15;
    if (l < rown + 2) {
#pragma unroll
        for (int e = 0; e < B; ++e) lds[l * fftl::padded(N) + fftl::padded(q + 16 * e)] = v[e];
    }
}

// Inverse transform of the LDS lines 0 .. rown + 1 (after a barrier).
template <typename T, int B>
__device__ __forceinline__ void rows_inverse(fftl::C2<T>* lds, int rown, const fftl::C2<T>* wl) {
    constexpr int N = 16 * B;
    const int l = threadIdx.x >> 4, q = threadIdx.x & 15;
    fftl::line_fft<T, B>(lds + l * fftl::padded(N), q, l < rown + 2, wl, true);
}

// Forward row FFTs of `out` (owned rows, values of the pair's two fields per
// point) into the row spectra z of pair p.
template <typename T, int B, int PER>
__device__ __forceinline__ void rows_forward(fftl::C2<T>* lds, const T (&out)[2][PER], T* __restrict__ z, int p,
                                             int j0, int rown, int ny, const fftl::C2<T>* wl) {
    constexpr int N = 16 * B;
    const int tid = threadIdx.x, l = tid >> 4, q = tid & 15;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = tid + t * 16 * fftl::kLines;
        if (e < rown * N) {
            const int jr = e / N, i = e - jr * N;
            lds[jr * fftl::padded(N) + fftl::padded(i)] = fftl::C2<T>{out[0][t], out[1][t]};
        }
    }
    __syncthreads();
    fftl::C2<T>* line = lds + l * fftl::padded(N);
    const bool act = l < rown;
    fftl::line_fft<T, B>(line, q, act, wl, false);
    if (act) {
        T* zr = z + (static_cast<size_t>(p) * N * ny + static_cast<size_t>(j0 + l) * N) * 2;
#pragma unroll
        for (int e = 0; e < B; ++e) {
            const int i = q + 16 * e;
            const fftl::C2<T> v = line[fftl::padded(i)];
            zr[2 * i] = v.r;
            zr[2 * i + 1] = v.i;
        }
    }
}

template <typename T>
struct TlmRowArgs {
    const T* zc;          // column-passed row spectra of the stage input (pairs): L w after the inverse rows
    const T* w;           // stage input fields (k x n)
    const double* Y;      // base stage value and its stream function
    const double* psi;
    T* dz;                // state fields (read; the new state at stage 3)
    T* acc;               // RK accumulator fields
    T* wnext;             // next stage input (stages 0-2)
    T* znext;             // row spectra of the next stage input (pairs), or null
    const T* W;           // x twiddles
    int k, ny, stage;
    T cnext, h, inv12d2, nu_d2;
};

// TLM stage (grid: row blocks x pairs): kv = -J_A(L w, Y) - J_A(psi, w) + nu lap w
// on the owned rows of both fields of the pair, the RK update, and the row
// spectra of the next stage input.  For many pairs (few pairs take the wave
// layout below): each point loads its stencil neighbourhoods itself, which
// keeps LDS small and more workgroups per CU.
template <typename T, int B>
__global__ void __launch_bounds__(16 * fftl::kLines) bve_tlm_rows(TlmRowArgs<T> a) {
    constexpr int N = 16 * B;
    constexpr int PER = (kRowsOwn * N + 16 * fftl::kLines - 1) / (16 * fftl::kLines);
    __shared__ fftl::C2<T> lds[fftl::kLines * fftl::padded(N)];
    __shared__ fftl::C2<T> wl[N];
    const int tid = threadIdx.x;
    const int p = blockIdx.y, j0 = blockIdx.x * kRowsOwn, ny = a.ny;
    const int rown = min(kRowsOwn, ny - j0);
    const size_t n = static_cast<size_t>(N) * ny;
    const int nf = 2 * p + 1 < a.k ? 2 : 1;
    {  // every global load of the prologue in flight before the first LDS store
        fftl::C2<T> tw[fftl::twiddles_per_thread<N>()];
        fftl::load_twiddles<T, N>(a.W, tw);
        fftl::C2<T> zv[B];
        rows_spec_load<T, B>(a.zc, p, j0, rown, ny, zv);
        fftl::store_twiddles<T, N>(wl, tw);
        rows_spec_store<T, B>(lds, rown, zv);
    }
    // the points' own dz and acc, issued before the inverse row FFTs so that
    // their latency overlaps the transforms
    T dzv[2][PER], acv[2][PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = min(tid + t * 16 * fftl::kLines, rown * N - 1);
        const int jr = e / N, i = e - jr * N;
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const size_t g = static_cast<size_t>(2 * p + min(f, nf - 1)) * n + static_cast<size_t>(j0 + jr) * N + i;
            dzv[f][t] = a.dz[g];
            acv[f][t] = a.stage == 0 ? T(0) : a.acc[g];
        }
    }
    __syncthreads();
    rows_inverse<T, B>(lds, rown, wl);
    const T bst = static_cast<T>(kRkB[a.stage]);
    T out[2][PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        out[0][t] = T(0);
        out[1][t] = T(0);
        const int e = tid + t * 16 * fftl::kLines;
        if (e < rown * N) {
            const int jr = e / N, i = e - jr * N, j = j0 + jr;
            T Yn[3][3], Pn[3][3];
            load9<T, double>(a.Y, N, ny, j, i, Yn);
            load9<T, double>(a.psi, N, ny, j, i, Pn);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                if (f < nf) {
                    const size_t off = static_cast<size_t>(2 * p + f) * n;
                    T phn[3][3], wn[3][3];
                    lds9<T, N>(lds, jr, i, f, phn);
                    load9<T, T>(a.w + off, N, ny, j, i, wn);
                    const T kv = -(arakawa12_nb<T>(phn, Yn) * a.inv12d2) - arakawa12_nb<T>(Pn, wn) * a.inv12d2 +
                                 a.nu_d2 * lap5_nb<T>(wn);
                    const size_t g = off + static_cast<size_t>(j) * N + i;
                    const T dv = dzv[f][t];
                    T o;
                    if (a.stage == 0) {
                        a.acc[g] = kv * bst;
                        o = dv + a.cnext * kv;
                        a.wnext[g] = o;
                    } else if (a.stage < 3) {
                        a.acc[g] = acv[f][t] + kv * bst;
                        o = dv + a.cnext * kv;
                        a.wnext[g] = o;
                    } else {
                        o = dv + a.h * (acv[f][t] + kv * bst);
                        a.dz[g] = o;
                    }
                    out[f][t] = o;
                }
            }
        }
    }
    if (a.znext) rows_forward<T, B, PER>(lds, out, a.znext, p, j0, rown, ny, wl);
}

template <typename T>
struct AdjRowArgs {
    // combine of stage m (m = -1: none): P = L jq from the column-passed
    // spectra zc, theta = -P + r_in, then (m = 3) acc = lam + theta,
    // (m = 2, 1) acc += theta, each with mu = cl lam + ct theta, or (m = 0)
    // lam = acc + theta
    const T* zc;
    const T* r_in;
    int m;
    T cl, ct;
    T* lam;
    T* acc;
    // observation forcing added to the new lambda (m = 0), or (m = -1, the
    // sweep's first launch, lambda zero before it) lambda set to the forcing
    // alone: W[force_it][o] / sigma_o at the observed cells, 0 elsewhere;
    // force_it < 0: none.  With m = -1 the kernel writes lambda on its owned
    // rows and never reads it: a neighbour's halo would otherwise race with
    // those writes.
    const T* Wobs;
    int force_it, stride, nox, n_obs;
    T inv_sigma;
    // stencil of stage s (-1: none) on mu' = mu (s < 3) or a3 lam (s = 3):
    // jq = J_A(Y, mu'), r_out = J_A(psi, mu') + nu lap mu', row spectra of jq to znext
    int s;
    T a3;
    const double* Y;
    const double* psi;
    T* r_out;
    T* znext;
    const T* W;  // x twiddles
    int k, ny;
    T inv12d2, nu_d2;
};

// ADJ row stage (grid: row blocks x pairs): the combine of one stage and the
// stencil of the next, with the combine recomputed on the halo rows so that
// the stencil has its neighbours without another launch.
template <typename T, int B>
__global__ void __launch_bounds__(16 * fftl::kLines) bve_adj_rows(AdjRowArgs<T> a) {
    constexpr int N = 16 * B;
    constexpr int PER = (kRowsOwn * N + 16 * fftl::kLines - 1) / (16 * fftl::kLines);
    constexpr int PERH = (fftl::kLines * N + 16 * fftl::kLines - 1) / (16 * fftl::kLines);
    __shared__ fftl::C2<T> lds[fftl::kLines * fftl::padded(N)];
    __shared__ fftl::C2<T> wl[N];
    const int tid = threadIdx.x;
    const int p = blockIdx.y, j0 = blockIdx.x * kRowsOwn, ny = a.ny;
    const int rown = min(kRowsOwn, ny - j0);
    const size_t n = static_cast<size_t>(N) * ny;
    const int nf = 2 * p + 1 < a.k ? 2 : 1;
    {  // every global load of the prologue in flight before the first LDS store
        fftl::C2<T> tw[fftl::twiddles_per_thread<N>()];
        fftl::load_twiddles<T, N>(a.W, tw);
        fftl::C2<T> zv[B];
        if (a.m >= 0) rows_spec_load<T, B>(a.zc, p, j0, rown, ny, zv);
        fftl::store_twiddles<T, N>(wl, tw);
        if (a.m >= 0) rows_spec_store<T, B>(lds, rown, zv);
    }
    // mu' on the owned rows and one halo row on each side, into the LDS lines;
    // in chunks of CH points per thread, each chunk's global loads issued
    // together, the first chunk's before the inverse row FFTs so that their
    // latency overlaps the transforms
    constexpr int CH = PERH < 8 ? PERH : 8;
    const bool need_r = a.m >= 0, need_lam = a.m > 0, need_acc = a.m == 0 || a.m == 1 || a.m == 2;
    auto load_chunk = [&](int t0, T (&rv)[2][CH], T (&lv)[2][CH], T (&av)[2][CH]) {
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = min(tid + (t0 + u) * 16 * fftl::kLines, (rown + 2) * N - 1);
            const int lr = e / N, i = e - lr * N;
            int j = j0 - 1 + lr;
            j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const size_t g =
                    static_cast<size_t>(2 * p + min(f, nf - 1)) * n + static_cast<size_t>(j) * N + i;
                rv[f][u] = need_r ? a.r_in[g] : T(0);
                lv[f][u] = need_lam ? a.lam[g] : T(0);
                av[f][u] = need_acc ? a.acc[g] : T(0);
            }
        }
    };
    T rv[2][CH], lv[2][CH], av[2][CH];
    load_chunk(0, rv, lv, av);
    __syncthreads();
    if (a.m >= 0) rows_inverse<T, B>(lds, rown, wl);
#pragma unroll
    for (int t0 = 0; t0 < PERH; t0 += CH) {
        if (t0 > 0) load_chunk(t0, rv, lv, av);
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = tid + (t0 + u) * 16 * fftl::kLines;
            if (e < (rown + 2) * N) {
                const int lr = e / N, i = e - lr * N;
                int j = j0 - 1 + lr;
                j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
                const bool owned = lr >= 1 && lr <= rown;
                const bool obs = a.force_it >= 0 && (j % a.stride) == 0 && (i % a.stride) == 0;
                const int o = (j / a.stride) * a.nox + i / a.stride;
                fftl::C2<T>& slot = lds[lr * fftl::padded(N) + fftl::padded(i)];
                T mu2[2] = {T(0), T(0)};
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    if (f < nf) {
                        const int v = 2 * p + f;
                        const size_t g = static_cast<size_t>(v) * n + static_cast<size_t>(j) * N + i;
                        T mu;
                        if (a.m >= 0) {
                            const T P = f ? slot.i : slot.r;
                            const T th = -P + rv[f][u];
                            if (a.m == 3) {
                                const T l = lv[f][u];
                                if (owned) a.acc[g] = l + th;
                                mu = a.cl * l + a.ct * th;
                            } else if (a.m > 0) {
                                if (owned) a.acc[g] = av[f][u] + th;
                                mu = a.cl * lv[f][u] + a.ct * th;
                            } else {
                                T l = av[f][u] + th;
                                if (obs)
                                    l = l + a.Wobs[(static_cast<size_t>(a.force_it) * a.n_obs + o) * a.k + v] *
                                                a.inv_sigma;
                                if (owned) a.lam[g] = l;
                                mu = a.a3 * l;
                            }
                        } else {
                            T l = T(0);
                            if (obs)
                                l = l + a.Wobs[(static_cast<size_t>(a.force_it) * a.n_obs + o) * a.k + v] *
                                            a.inv_sigma;
                            if (owned) a.lam[g] = l;
                            mu = a.a3 * l;
                        }
                        mu2[f] = mu;
                    }
                }
                slot = fftl::C2<T>{mu2[0], mu2[1]};
            }
        }
    }
    if (a.s < 0) return;  // uniform across the workgroup
    __syncthreads();
    T out[2][PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        out[0][t] = T(0);
        out[1][t] = T(0);
        const int e = tid + t * 16 * fftl::kLines;
        if (e < rown * N) {
            const int jr = e / N, i = e - jr * N, j = j0 + jr;
            T Yn[3][3], Pn[3][3];
            load9<T, double>(a.Y, N, ny, j, i, Yn);
            load9<T, double>(a.psi, N, ny, j, i, Pn);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                if (f < nf) {
                    T mn[3][3];
                    lds9<T, N>(lds, jr, i, f, mn);
                    const size_t g = static_cast<size_t>(2 * p + f) * n + static_cast<size_t>(j) * N + i;
                    out[f][t] = arakawa12_nb<T>(Yn, mn) * a.inv12d2;
                    a.r_out[g] = arakawa12_nb<T>(Pn, mn) * a.inv12d2 + a.nu_d2 * lap5_nb<T>(mn);
                }
            }
        }
    }
    rows_forward<T, B, PER>(lds, out, a.znext, p, j0, rown, ny, wl);
}

// ---------------------------------------------------------------------------
// The same row stages with one wave per row line, for few field pairs
// (latency-bound launches), on every supported side.  A workgroup of L
// waves owns L - 2 rows; wave w holds line w (row j0 - 1 + w), loads it,
// transforms it, and on the owned lines runs the stencils and the update on
// its points i = lane + 64 u (ragged past N when 64 does not divide N).  The line transforms need no workgroup barrier;
// the rows the stencils read (the twiddles, Y, psi and the inputs staged in
// LDS, and the neighbours' transformed lines) need one barrier each, and a
// last one keeps the neighbours' lines until every stencil has read them.
// ---------------------------------------------------------------------------
// Lines per row workgroup: 4 (2 owned rows) spread a latency-bound stage over
// more CUs than 8 lines (6 owned) and ran 30.8 -> 26.3 ms per bve-256 k = 1
// product; 3 lines were no faster.
constexpr int kWaveLines = 4;

template <typename T, int N, int L>
__global__ void __launch_bounds__(64 * L) bve_tlm_rows_w(TlmRowArgs<T> a) {
    constexpr int P = fftl::wave_points<N>(), NT = 64 * L, OWN = L - 2, TW = (N + NT - 1) / NT, SR = L * N;
    __shared__ fftl::C2<T> lds[L * fftl::padded(N)];
    __shared__ T stg[4 * SR];
    __shared__ fftl::C2<T> wl[N];
    const int tid = threadIdx.x, w = tid >> 6, q = tid & 63;
    const int p = blockIdx.y, j0 = blockIdx.x * OWN, ny = a.ny;
    const int rown = min(OWN, ny - j0);
    const size_t n = static_cast<size_t>(N) * ny;
    const int nf = 2 * p + 1 < a.k ? 2 : 1;
    const bool live = w < rown + 2, own = w >= 1 && w <= rown;
    int jl = j0 - 1 + min(w, rown + 1);
    jl = jl < 0 ? jl + ny : (jl >= ny ? jl - ny : jl);
    fftl::C2<T>* line = lds + w * fftl::padded(N);
    T dzv[2][P], acv[2][P];
    {  // every global load first, then the LDS stores
        fftl::C2<T> tw[TW];
#pragma unroll
        for (int r = 0; r < TW; ++r) {
            const int m = min(tid + r * NT, N - 1);
            tw[r] = fftl::C2<T>{a.W[2 * m], a.W[2 * m + 1]};
        }
        fftl::C2<T> zv[P];
        double yv[P], pv[P];
        T wv[2][P];
        const T* zr = a.zc + (static_cast<size_t>(p) * n + static_cast<size_t>(jl) * N) * 2;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int i = fftl::wave_point<N>(q, u);
            const size_t r = static_cast<size_t>(jl) * N + i;
            zv[u] = fftl::C2<T>{zr[2 * i], zr[2 * i + 1]};
            yv[u] = a.Y[r];
            pv[u] = a.psi[r];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const size_t g = static_cast<size_t>(2 * p + min(f, nf - 1)) * n + r;
                wv[f][u] = a.w[g];
                dzv[f][u] = own ? a.dz[g] : T(0);
                acv[f][u] = own && a.stage > 0 ? a.acc[g] : T(0);
            }
        }
#pragma unroll
        for (int r = 0; r < TW; ++r) {
            const int m = tid + r * NT;
            if (m < N) wl[m] = tw[r];
        }
        if (live) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                if (!fftl::wave_has<N>(q, u)) continue;
                const int i = q + 64 * u;
                line[fftl::padded(i)] = zv[u];
                stg[w * N + i] = static_cast<T>(yv[u]);
                stg[SR + w * N + i] = static_cast<T>(pv[u]);
                stg[2 * SR + w * N + i] = wv[0][u];
                stg[3 * SR + w * N + i] = wv[1][u];
            }
        }
    }
    __syncthreads();
    if (live) fftl::line_fft_wave<T, N>(line, q, wl, true);
    __syncthreads();
    const T bst = static_cast<T>(kRkB[a.stage]);
    T out[2][P];
#pragma unroll
    for (int u = 0; u < P; ++u) out[0][u] = out[1][u] = T(0);
    if (own) {
        const int jr = w - 1, j = j0 + jr;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (!fftl::wave_has<N>(q, u)) continue;
            const int i = q + 64 * u;
            T Yn[3][3], Pn[3][3];
            st9<T, N>(stg, jr, i, Yn);
            st9<T, N>(stg + SR, jr, i, Pn);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                if (f < nf) {
                    T phn[3][3], wn[3][3];
                    lds9<T, N>(lds, jr, i, f, phn);
                    st9<T, N>(stg + (2 + f) * SR, jr, i, wn);
                    const T kv = -(arakawa12_nb<T>(phn, Yn) * a.inv12d2) - arakawa12_nb<T>(Pn, wn) * a.inv12d2 +
                                 a.nu_d2 * lap5_nb<T>(wn);
                    const size_t g = static_cast<size_t>(2 * p + f) * n + static_cast<size_t>(j) * N + i;
                    const T dv = dzv[f][u];
                    T o;
                    if (a.stage == 0) {
                        a.acc[g] = kv * bst;
                        o = dv + a.cnext * kv;
                        a.wnext[g] = o;
                    } else if (a.stage < 3) {
                        a.acc[g] = acv[f][u] + kv * bst;
                        o = dv + a.cnext * kv;
                        a.wnext[g] = o;
                    } else {
                        o = dv + a.h * (acv[f][u] + kv * bst);
                        a.dz[g] = o;
                    }
                    out[f][u] = o;
                }
            }
        }
    }
    if (!a.znext) return;  // uniform across the workgroup
    __syncthreads();
    if (own) {
#pragma unroll
        for (int u = 0; u < P; ++u)
            if (fftl::wave_has<N>(q, u)) line[fftl::padded(q + 64 * u)] = fftl::C2<T>{out[0][u], out[1][u]};
        fftl::wave_sync();
        fftl::line_fft_wave<T, N>(line, q, wl, false);
        T* zo = a.znext + (static_cast<size_t>(p) * n + static_cast<size_t>(j0 + w - 1) * N) * 2;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (!fftl::wave_has<N>(q, u)) continue;
            const int i = q + 64 * u;
            const fftl::C2<T> v = line[fftl::padded(i)];
            zo[2 * i] = v.r;
            zo[2 * i + 1] = v.i;
        }
    }
}

template <typename T, int N, int L>
__global__ void __launch_bounds__(64 * L) bve_adj_rows_w(AdjRowArgs<T> a) {
    constexpr int P = fftl::wave_points<N>(), NT = 64 * L, OWN = L - 2, TW = (N + NT - 1) / NT, SR = L * N;
    __shared__ fftl::C2<T> lds[L * fftl::padded(N)];
    __shared__ T stg[2 * SR];
    __shared__ fftl::C2<T> wl[N];
    const int tid = threadIdx.x, w = tid >> 6, q = tid & 63;
    const int p = blockIdx.y, j0 = blockIdx.x * OWN, ny = a.ny;
    const int rown = min(OWN, ny - j0);
    const size_t n = static_cast<size_t>(N) * ny;
    const int nf = 2 * p + 1 < a.k ? 2 : 1;
    const bool live = w < rown + 2, own = w >= 1 && w <= rown;
    int jl = j0 - 1 + min(w, rown + 1);
    jl = jl < 0 ? jl + ny : (jl >= ny ? jl - ny : jl);
    fftl::C2<T>* line = lds + w * fftl::padded(N);
    const bool need_r = a.m >= 0, need_lam = a.m > 0, need_acc = a.m == 0 || a.m == 1 || a.m == 2;
    T rv[2][P], lv[2][P], av[2][P];
    {  // every global load first, then the LDS stores
        fftl::C2<T> tw[TW];
#pragma unroll
        for (int r = 0; r < TW; ++r) {
            const int m = min(tid + r * NT, N - 1);
            tw[r] = fftl::C2<T>{a.W[2 * m], a.W[2 * m + 1]};
        }
        fftl::C2<T> zv[P];
        double yv[P], pv[P];
        const T* zr = a.zc + (static_cast<size_t>(p) * n + static_cast<size_t>(jl) * N) * 2;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int i = fftl::wave_point<N>(q, u);
            const size_t r = static_cast<size_t>(jl) * N + i;
            zv[u] = a.m >= 0 ? fftl::C2<T>{zr[2 * i], zr[2 * i + 1]} : fftl::C2<T>{T(0), T(0)};
            yv[u] = a.s >= 0 ? a.Y[r] : 0.0;
            pv[u] = a.s >= 0 ? a.psi[r] : 0.0;
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const size_t g = static_cast<size_t>(2 * p + min(f, nf - 1)) * n + r;
                rv[f][u] = need_r ? a.r_in[g] : T(0);
                lv[f][u] = need_lam ? a.lam[g] : T(0);
                av[f][u] = need_acc ? a.acc[g] : T(0);
            }
        }
#pragma unroll
        for (int r = 0; r < TW; ++r) {
            const int m = tid + r * NT;
            if (m < N) wl[m] = tw[r];
        }
        if (live) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                if (!fftl::wave_has<N>(q, u)) continue;
                const int i = q + 64 * u;
                line[fftl::padded(i)] = zv[u];
                stg[w * N + i] = static_cast<T>(yv[u]);
                stg[SR + w * N + i] = static_cast<T>(pv[u]);
            }
        }
    }
    __syncthreads();
    // the combine of stage m on the wave's own line (owned rows and the halo)
    if (live) {
        if (a.m >= 0) fftl::line_fft_wave<T, N>(line, q, wl, true);
        const int j = jl;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (!fftl::wave_has<N>(q, u)) continue;
            const int i = q + 64 * u;
            const bool obs = a.force_it >= 0 && (j % a.stride) == 0 && (i % a.stride) == 0;
            const int o = (j / a.stride) * a.nox + i / a.stride;
            fftl::C2<T>& slot = line[fftl::padded(i)];
            T mu2[2] = {T(0), T(0)};
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                if (f < nf) {
                    const int v = 2 * p + f;
                    const size_t g = static_cast<size_t>(v) * n + static_cast<size_t>(j) * N + i;
                    T mu;
                    if (a.m >= 0) {
                        const T Pv = f ? slot.i : slot.r;
                        const T th = -Pv + rv[f][u];
                        if (a.m == 3) {
                            const T l = lv[f][u];
                            if (own) a.acc[g] = l + th;
                            mu = a.cl * l + a.ct * th;
                        } else if (a.m > 0) {
                            if (own) a.acc[g] = av[f][u] + th;
                            mu = a.cl * lv[f][u] + a.ct * th;
                        } else {
                            T l = av[f][u] + th;
                            if (obs)
                                l = l + a.Wobs[(static_cast<size_t>(a.force_it) * a.n_obs + o) * a.k + v] * a.inv_sigma;
                            if (own) a.lam[g] = l;
                            mu = a.a3 * l;
                        }
                    } else {
                        T l = T(0);
                        if (obs)
                            l = l + a.Wobs[(static_cast<size_t>(a.force_it) * a.n_obs + o) * a.k + v] * a.inv_sigma;
                        if (own) a.lam[g] = l;
                        mu = a.a3 * l;
                    }
                    mu2[f] = mu;
                }
            }
            slot = fftl::C2<T>{mu2[0], mu2[1]};
        }
    }
    if (a.s < 0) return;  // uniform across the workgroup
    __syncthreads();
    T out[2][P];
#pragma unroll
    for (int u = 0; u < P; ++u) out[0][u] = out[1][u] = T(0);
    if (own) {
        const int jr = w - 1, j = j0 + jr;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (!fftl::wave_has<N>(q, u)) continue;
            const int i = q + 64 * u;
            T Yn[3][3], Pn[3][3];
            st9<T, N>(stg, jr, i, Yn);
            st9<T, N>(stg + SR, jr, i, Pn);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                if (f < nf) {
                    T mn[3][3];
                    lds9<T, N>(lds, jr, i, f, mn);
                    const size_t g = static_cast<size_t>(2 * p + f) * n + static_cast<size_t>(j) * N + i;
                    out[f][u] = arakawa12_nb<T>(Yn, mn) * a.inv12d2;
                    a.r_out[g] = arakawa12_nb<T>(Pn, mn) * a.inv12d2 + a.nu_d2 * lap5_nb<T>(mn);
                }
            }
        }
    }
    __syncthreads();
    if (own) {
#pragma unroll
        for (int u = 0; u < P; ++u)
            if (fftl::wave_has<N>(q, u)) line[fftl::padded(q + 64 * u)] = fftl::C2<T>{out[0][u], out[1][u]};
        fftl::wave_sync();
        fftl::line_fft_wave<T, N>(line, q, wl, false);
        T* zo = a.znext + (static_cast<size_t>(p) * n + static_cast<size_t>(j0 + w - 1) * N) * 2;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            if (!fftl::wave_has<N>(q, u)) continue;
            const int i = q + 64 * u;
            const fftl::C2<T> v = line[fftl::padded(i)];
            zo[2 * i] = v.r;
            zo[2 * i + 1] = v.i;
        }
    }
}

// Row stages with one wave per line while the grid has at most this many field
// pairs; sixteen threads per line beyond.
constexpr int kStagePairs = 4;


template <typename T>
void launch_tlm_rows(const TlmRowArgs<T>& a, int nx, hipStream_t st) {
    const bool stage = (a.k + 1) / 2 <= kStagePairs;
    if (stage) {
        constexpr int L = kWaveLines;
        const dim3 gw((a.ny + L - 3) / (L - 2), (a.k + 1) / 2), bw(64 * L);
        switch (nx / 16) {
#define RP4D_WAVE_ROWS(b) \
    case b: bve_tlm_rows_w<T, 16 * b, L><<<gw, bw, 0, st>>>(a); break;
            RP4D_WAVE_ROWS(2) RP4D_WAVE_ROWS(3) RP4D_WAVE_ROWS(4) RP4D_WAVE_ROWS(5) RP4D_WAVE_ROWS(6)
            RP4D_WAVE_ROWS(8) RP4D_WAVE_ROWS(10) RP4D_WAVE_ROWS(12) RP4D_WAVE_ROWS(16) RP4D_WAVE_ROWS(20)
            RP4D_WAVE_ROWS(24) RP4D_WAVE_ROWS(32)
#undef RP4D_WAVE_ROWS
            default: fail(RP4D_EINVAL, "2-D grid: unsupported nx");
        }
        RP4D_HIP(hipGetLastError());
        return;
    }
    const dim3 grid((a.ny + kRowsOwn - 1) / kRowsOwn, (a.k + 1) / 2), blk(16 * fftl::kLines);
    switch (nx / 16) {
#define RP4D_TLM_ROWS(b) \
    case b: bve_tlm_rows<T, b><<<grid, blk, 0, st>>>(a); break;
        RP4D_TLM_ROWS(2) RP4D_TLM_ROWS(3) RP4D_TLM_ROWS(4) RP4D_TLM_ROWS(5) RP4D_TLM_ROWS(6) RP4D_TLM_ROWS(8)
        RP4D_TLM_ROWS(10) RP4D_TLM_ROWS(12) RP4D_TLM_ROWS(16) RP4D_TLM_ROWS(20) RP4D_TLM_ROWS(24) RP4D_TLM_ROWS(32)
#undef RP4D_TLM_ROWS
        default: fail(RP4D_EINVAL, "2-D grid: unsupported nx");
    }
    RP4D_HIP(hipGetLastError());
}

template <typename T>
void launch_adj_rows(const AdjRowArgs<T>& a, int nx, hipStream_t st) {
    const bool stage = (a.k + 1) / 2 <= kStagePairs;
    if (stage) {
        constexpr int L = kWaveLines;
        const dim3 gw((a.ny + L - 3) / (L - 2), (a.k + 1) / 2), bw(64 * L);
        switch (nx / 16) {
#define RP4D_WAVE_ROWS(b) \
    case b: bve_adj_rows_w<T, 16 * b, L><<<gw, bw, 0, st>>>(a); break;
            RP4D_WAVE_ROWS(2) RP4D_WAVE_ROWS(3) RP4D_WAVE_ROWS(4) RP4D_WAVE_ROWS(5) RP4D_WAVE_ROWS(6)
            RP4D_WAVE_ROWS(8) RP4D_WAVE_ROWS(10) RP4D_WAVE_ROWS(12) RP4D_WAVE_ROWS(16) RP4D_WAVE_ROWS(20)
            RP4D_WAVE_ROWS(24) RP4D_WAVE_ROWS(32)
#undef RP4D_WAVE_ROWS
            default: fail(RP4D_EINVAL, "2-D grid: unsupported nx");
        }
        RP4D_HIP(hipGetLastError());
        return;
    }
    const dim3 grid((a.ny + kRowsOwn - 1) / kRowsOwn, (a.k + 1) / 2), blk(16 * fftl::kLines);
    switch (nx / 16) {
#define RP4D_ADJ_ROWS(b) \
    case b: bve_adj_rows<T, b><<<grid, blk, 0, st>>>(a); break;
        RP4D_ADJ_ROWS(2) RP4D_ADJ_ROWS(3) RP4D_ADJ_ROWS(4) RP4D_ADJ_ROWS(5) RP4D_ADJ_ROWS(6) RP4D_ADJ_ROWS(8)
        RP4D_ADJ_ROWS(10) RP4D_ADJ_ROWS(12) RP4D_ADJ_ROWS(16) RP4D_ADJ_ROWS(20) RP4D_ADJ_ROWS(24) RP4D_ADJ_ROWS(32)
#undef RP4D_ADJ_ROWS
        default: fail(RP4D_EINVAL, "2-D grid: unsupported nx");
    }
    RP4D_HIP(hipGetLastError());
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

// TLM sweep of k field-major perturbations dz (overwritten); observations to Z
// (n_t, n_obs, k).  Each RK stage is one fused row launch (bve_tlm_rows) and
// one column pass.  ws holds 8 blocks of k fields: wA, wB, acc, the two
// double-width row-spectra buffers zA (blocks 3-4) and zB (5-6); dz is block 7.
template <typename T>
void tlm_sweep(rp4d_problem* p, const rp4d_traj* tr, int k, T* dz, T* Z, T* ws) {
    const int n = p->n, nx = p->bve->nx, ny = p->bve->ny;
    hipStream_t st = bst(p);
    const size_t fk = static_cast<size_t>(k) * n;
    T* wA = ws;
    T* wB = ws + fk;
    T* acc = ws + 2 * fk;
    T* zc = ws + 3 * fk;
    T* zn = ws + 5 * fk;
    const double h = p->d.dt, dd = p->bve->d;
    const T inv12d2 = static_cast<T>(1.0 / (12.0 * dd * dd)), nu_d2 = static_cast<T>(p->d.nu / (dd * dd));
    const int stride = p->d.obs_stride, nox = (nx + stride - 1) / stride;
    const T cn[3] = {static_cast<T>(0.5 * h), static_cast<T>(0.5 * h), static_cast<T>(h)};
    const Spec<T> sp = spec_of<T>(p);
    // FFT-equivalent flops (5 N log2 N per complex 2-D transform, k/2 pairs, a
    // forward and an inverse transform per solve) split into the column passes'
    // and the row passes' halves, and the stencil work of a stage
    const double fl_col = 5.0 * static_cast<double>(n) * std::log2(static_cast<double>(ny)) * k;
    const double fl_row = 5.0 * static_cast<double>(n) * std::log2(static_cast<double>(nx)) * k;
    const double fl_sten = (2 * FL_ARAKAWA + FL_LAP + 6.0) * static_cast<double>(fk);
    {
        KernelTimer kt(p->ctx, RP4D_K_GEMM, fl_col + 0.5 * fl_row);
        launch_fft_rows_fwd<T>(dz, k, nx, ny, zc, sp.Wx, st);
        launch_fft_cols<T>(zc, k, nx, ny, sp.Dlap, sp.Wy, st);
    }
    for (int s = 0; s < p->s_last; ++s) {
        for (int i = 0; i < 4; ++i) {
            const bool last = s + 1 == p->s_last && i == 3;
            TlmRowArgs<T> a{};
            a.zc = zc;
            a.w = i == 0 ? dz : (i == 2 ? wB : wA);
            a.Y = stage_Y(tr, s, i);
            a.psi = stage_psi(tr, s, i);
            a.dz = dz;
            a.acc = acc;
            a.wnext = i == 1 ? wB : wA;  // stage 0 -> A, 1 -> B, 2 -> A
            a.znext = last ? nullptr : zn;
            a.W = sp.Wx;
            a.k = k;
            a.ny = ny;
            a.stage = i;
            a.cnext = i < 3 ? cn[i] : T(0);
            a.h = static_cast<T>(h);
            a.inv12d2 = inv12d2;
            a.nu_d2 = nu_d2;
            {
                KernelTimer kt(p->ctx, RP4D_K_STENCIL, fl_sten + (last ? 0.5 : 1.0) * fl_row);
                launch_tlm_rows<T>(a, nx, st);
            }
            if (!last) {
                KernelTimer kt(p->ctx, RP4D_K_GEMM, fl_col);
                launch_fft_cols<T>(zn, k, nx, ny, sp.Dlap, sp.Wy, st);
                std::swap(zc, zn);
            }
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
// Each RK stage is one fused row launch (bve_adj_rows: the combine of the
// stage, the observation forcing between steps, and the stencil of the next
// stage) and one column pass.  ws: r_a, r_b, acc, zA (blocks 3-4), zB (5-6).
template <typename T>
void adj_sweep(rp4d_problem* p, const rp4d_traj* tr, int k, const T* W, T* lam, T* ws) {
    const int n = p->n, nx = p->bve->nx, ny = p->bve->ny;
    hipStream_t st = bst(p);
    const size_t fk = static_cast<size_t>(k) * n;
    T* rc = ws;
    T* rn = ws + fk;
    T* acc = ws + 2 * fk;
    T* zc = ws + 3 * fk;
    T* zn = ws + 5 * fk;
    const double h = p->d.dt, dd = p->bve->d;
    const T inv12d2 = static_cast<T>(1.0 / (12.0 * dd * dd)), nu_d2 = static_cast<T>(p->d.nu / (dd * dd));
    const int stride = p->d.obs_stride, nox = (nx + stride - 1) / stride;
    const Spec<T> sp = spec_of<T>(p);
    // mu of the next (lower) stage after the combine of stage i: (h/3, h), (h/3, h/2), (h/6, h/2)
    const T cl[4] = {T(0), static_cast<T>(h / 6.0), static_cast<T>(h / 3.0), static_cast<T>(h / 3.0)};
    const T ct[4] = {T(0), static_cast<T>(0.5 * h), static_cast<T>(0.5 * h), static_cast<T>(h)};
    // FFT-equivalent flops of the column passes and of the row passes' halves
    // (as in tlm_sweep), and the stencil work of a stage
    const double fl_col = 5.0 * static_cast<double>(n) * std::log2(static_cast<double>(ny)) * k;
    const double fl_row = 5.0 * static_cast<double>(n) * std::log2(static_cast<double>(nx)) * k;
    const double fl_sten = (2 * FL_ARAKAWA + FL_LAP + 2.0) * static_cast<double>(fk);
    auto obs_it = [&](int s) {  // observation index of state s, or -1
        return (s % p->d.obs_every == 0 && s / p->d.obs_every <= p->n_t && s >= 1) ? s / p->d.obs_every - 1 : -1;
    };
    auto base = [&](AdjRowArgs<T>& a) {
        a.lam = lam;
        a.acc = acc;
        a.Wobs = W;
        a.stride = stride;
        a.nox = nox;
        a.n_obs = p->n_obs;
        a.inv_sigma = static_cast<T>(1.0 / p->d.sigma_o);
        a.a3 = static_cast<T>(h / 6.0);
        a.W = sp.Wx;
        a.k = k;
        a.ny = ny;
        a.inv12d2 = inv12d2;
        a.nu_d2 = nu_d2;
    };
    {
        // lambda set to the forcing of the last state (every point written),
        // and the stencil of stage 3 of the last step
        AdjRowArgs<T> a{};
        base(a);
        a.m = -1;
        a.force_it = obs_it(p->s_last);
        a.s = 3;
        a.Y = stage_Y(tr, p->s_last - 1, 3);
        a.psi = stage_psi(tr, p->s_last - 1, 3);
        a.r_out = rc;
        a.znext = zc;
        {
            KernelTimer kt(p->ctx, RP4D_K_STENCIL, fl_sten + 0.5 * fl_row);
            launch_adj_rows<T>(a, nx, st);
        }
        KernelTimer kt(p->ctx, RP4D_K_GEMM, fl_col);
        launch_fft_cols<T>(zc, k, nx, ny, sp.Dlap, sp.Wy, st);
    }
    for (int s = p->s_last; s >= 1; --s) {
        for (int i = 3; i >= 0; --i) {
            AdjRowArgs<T> a{};
            base(a);
            a.zc = zc;
            a.r_in = rc;
            a.m = i;
            a.cl = cl[i];
            a.ct = ct[i];
            a.force_it = -1;
            a.s = -1;
            if (i > 0) {  // stencil of the next stage of this step
                a.s = i - 1;
                a.Y = stage_Y(tr, s - 1, i - 1);
                a.psi = stage_psi(tr, s - 1, i - 1);
            } else if (s > 1) {  // forcing of state s-1, stencil of stage 3 of step s-1
                a.force_it = obs_it(s - 1);
                a.s = 3;
                a.Y = stage_Y(tr, s - 2, 3);
                a.psi = stage_psi(tr, s - 2, 3);
            }
            a.r_out = rn;
            a.znext = a.s >= 0 ? zn : nullptr;
            {
                // the combine: theta 1, accumulator 1, next mu 3 per point and field
                KernelTimer kt(p->ctx, RP4D_K_STENCIL,
                               (a.s >= 0 ? fl_sten + fl_row : 0.5 * fl_row) + 5.0 * static_cast<double>(fk));
                launch_adj_rows<T>(a, nx, st);
            }
            if (a.s >= 0) {
                KernelTimer kt(p->ctx, RP4D_K_GEMM, fl_col);
                launch_fft_cols<T>(zn, k, nx, ny, sp.Dlap, sp.Wy, st);
                std::swap(zc, zn);
                std::swap(rc, rn);
            }
        }
    }
    RP4D_HIP(hipGetLastError());
}

}  // namespace

template <typename T>
void bve_tlm(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* Z) {
    T* ws = ws_fields<T>(p, k, 8);
    T* dz = ws + static_cast<size_t>(7) * k * p->n;
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

// The TLM's state (block 7) is dead once its observations are in Z, so the
// ADJ's lambda takes the same block.
template <typename T>
void bve_hessian(rp4d_problem* p, const rp4d_traj* tr, int k, const T* V, T* HV, bool add_identity) {
    T* ws = ws_fields<T>(p, k, 8);
    p->bve->ws_obs.ensure(static_cast<size_t>(p->m) * k * sizeof(T));
    T* Z = p->bve->ws_obs.as<T>();
    T* dz = ws + static_cast<size_t>(7) * k * p->n;
    T* lam = dz;
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
