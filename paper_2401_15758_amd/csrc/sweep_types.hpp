// Argument blocks and tilings of the Burgers sweeps.  Plain C++ (no HIP
// types), shared by the device code and by host-only planning code.
#pragma once

namespace rp4d {

enum SweepMode { MODE_TLM = 1, MODE_ADJ = 2 };

// Neighbour exchange of a sweep region: the workgroup through LDS, or each
// 64-lane wave on its own through DPP lane shifts.
enum SweepExchange { XCH_LDS = 1, XCH_WAVE = 2 };

struct Tiling {
    int ppt = 0, kc = 0, threads = 0, tile = 0, steps = 0, xch = XCH_LDS;
};

template <typename T>
struct SweepArgs {
    const double* base;   // u_s stored at base[(s - base_row0) * n + g]
    int base_row0;
    int n;
    T h, inv2dx, nu_dx2;
    int s0, S;            // TLM: steps s0 .. s0+S-1 forward; ADJ: s0+S-1 .. s0 backward
    int tile, halo;
    int k;                // number of vectors
    const T* xin;         // blocked state [grp][n][KC]
    T* xout;
    int obs_stride, obs_every, n_obs, n_t;
    T inv_sigma_o;
    T* z;                 // TLM observation output (n_t, n_obs, k)
    const T* w;           // ADJ observation forcing (n_t, n_obs, k)
    int wall;             // 1: Dirichlet walls + RK3-TVD (wall-bounded sweeps)
};

struct FwdArgs {
    const double* xin;    // state at s0 (n)
    double* xout;         // state at s0+S (n)
    double* store;        // trajectory rows: u_s at store[(s/store_every - store_row0) * n + g]
    int store_every, store_row0, store_rows;
    int n;
    double h, inv2dx, nu_dx2;
    int s0, S, tile, halo;
    int obs_stride, obs_every, n_obs, n_t;
    double inv_sigma_o;
    const double* y;      // observations (n_t, n_obs) or null
    double* innov;        // innovations out (n_t, n_obs) or null
    double* obs_out;      // O x_{s_i} out (n_t, n_obs) or null
    int wall;             // 1: Dirichlet walls + RK3-TVD (wall-bounded sweeps)
};

}  // namespace rp4d
