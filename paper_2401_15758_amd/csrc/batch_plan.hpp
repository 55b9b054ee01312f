// Host-side planning of the batched Burgers sweeps: the descriptor tables that
// the fused launches read (one argument block per problem and time interval,
// one work item per region) and the placement of staged tables in the pinned
// staging ring.  Plain C++ with no HIP types: the library stages and launches
// what these functions plan, and a host-only checker replays the same plans to
// bound every index the kernels derive from them.
#pragma once

#include <algorithm>
#include <cstddef>
#include <string>
#include <vector>

#include "rp4d.h"
#include "sweep_types.hpp"

namespace rp4d {

[[noreturn]] void fail(int code, const std::string& msg);

// A work item: (argument slot within its interval, tile, vector group, unused).
// Same size and layout as HIP's int4, which the kernels read.
struct PlanItem {
    int x, y, z, w;
};

// One problem of a batch, as the planner sees it.
struct BatchProb {
    int n, s_last;                 // grid points, steps in the window
    double dt, inv2dx, nu_dx2;
    int obs_stride, obs_every, n_obs, n_t;
    double sigma_o;
    const double* traj;            // stored trajectory, every state: (s_last + 1) x n
    int traj_rows;
    const double* y;               // FWD: observations (n_t, n_obs) or null
    double* innov;                 // FWD: innovations out (n_t, n_obs) or null
    double* obs_out;               // FWD: O x_{s_i} out (n_t, n_obs)
};

// Owned points per region of an n-point problem under a batched tiling: the
// region (64 ppt points for wave regions, threads * ppt for workgroup regions)
// less a halo of 4 S + 4 points on each side, at most n.
inline int batch_tile(const Tiling& t, int n) {
    if (!(t.threads >= 64 && t.threads <= 1024 && t.threads % 64 == 0 && t.steps >= 1 && t.ppt >= 1))
        fail(RP4D_EINVAL, "batch tiling: threads must be a multiple of 64 in [64, 1024], steps and ppt >= 1");
    const int halo = 4 * t.steps + 4;
    const int room = (t.xch == XCH_WAVE ? 64 : t.threads) * t.ppt - 2 * halo;
    if (room < 1) fail(RP4D_EINVAL, "batch tiling: region too small for the halo of steps per launch");
    return std::min(room, n);
}

// Number of fused launches (time intervals) of a batched sweep.
inline int batch_intervals(const std::vector<BatchProb>& probs, const Tiling& t) {
    int nl = 0;
    for (const BatchProb& p : probs) nl = std::max(nl, (p.s_last + t.steps - 1) / t.steps);
    return nl;
}

// Tables of launches [j0, j1) of a batched sweep or FWD: argument blocks of
// interval j at args[aoff[j - j0] ..], its items at items[off[j - j0] ..];
// an item's x is the argument slot relative to aoff of its interval.
template <typename A>
struct IntervalTables {
    int j0 = 0, j1 = 0;
    std::vector<A> args;
    std::vector<PlanItem> items;
    std::vector<int> off, aoff;     // j1 - j0 + 1 entries
    std::vector<double> flops;      // algorithmic flops per launch
};

// Batched TLM (mode MODE_TLM) or ADJ sweep of k vectors, intervals [j0, j1).
// Interval j advances problem i from buffer (j even ? buf0 : buf1) into the
// other one; the TLM runs steps j S .. j S + S - 1, the ADJ the S steps below
// s_last - j S.  Problems with fewer intervals keep an inactive argument block
// (no items refer to it).  fl_vec / fl_base: flops per point-step per vector
// and shared.
template <typename T>
IntervalTables<SweepArgs<T>> plan_sweep(int mode, const std::vector<BatchProb>& probs, int k, const Tiling& t,
                                        const std::vector<T*>& buf0, const std::vector<T*>& buf1,
                                        const std::vector<T*>& z, const std::vector<const T*>& w, int j0, int j1,
                                        double fl_vec, double fl_base) {
    const int np = static_cast<int>(probs.size());
    const int groups = (k + t.kc - 1) / t.kc;
    IntervalTables<SweepArgs<T>> r;
    r.j0 = j0;
    r.j1 = j1;
    for (int j = j0; j < j1; ++j) {
        r.off.push_back(static_cast<int>(r.items.size()));
        r.aoff.push_back(static_cast<int>(r.args.size()));
        double fl = 0.0;
        for (int i = 0; i < np; ++i) {
            const BatchProb& p = probs[i];
            const int nlp = (p.s_last + t.steps - 1) / t.steps;
            SweepArgs<T> a{};
            a.n = p.n;
            if (j < nlp) {
                a.base = p.traj;
                a.base_row0 = 0;
                a.h = static_cast<T>(p.dt);
                a.inv2dx = static_cast<T>(p.inv2dx);
                a.nu_dx2 = static_cast<T>(p.nu_dx2);
                if (mode == MODE_TLM) {
                    a.s0 = j * t.steps;
                    a.S = std::min(t.steps, p.s_last - a.s0);
                } else {
                    const int s_hi = p.s_last - j * t.steps;
                    a.s0 = std::max(0, s_hi - t.steps);
                    a.S = s_hi - a.s0;
                }
                a.tile = batch_tile(t, p.n);
                a.halo = 4 * t.steps + 4;
                a.k = k;
                a.xin = (j % 2 == 0) ? buf0[i] : buf1[i];
                a.xout = (j % 2 == 0) ? buf1[i] : buf0[i];
                a.obs_stride = p.obs_stride;
                a.obs_every = p.obs_every;
                a.n_obs = p.n_obs;
                a.n_t = p.n_t;
                a.inv_sigma_o = static_cast<T>(1.0 / p.sigma_o);
                a.z = mode == MODE_TLM ? z[i] : nullptr;
                a.w = mode == MODE_ADJ ? w[i] : nullptr;
                const int slot = static_cast<int>(r.args.size()) - r.aoff.back();
                const int ntile = (p.n + a.tile - 1) / a.tile;
                for (int g = 0; g < groups; ++g)
                    for (int tl = 0; tl < ntile; ++tl) r.items.push_back(PlanItem{slot, tl, g, 0});
                fl += static_cast<double>(a.S) * p.n * (fl_vec * k + fl_base);
            }
            r.args.push_back(a);
        }
        r.flops.push_back(fl);
    }
    r.off.push_back(static_cast<int>(r.items.size()));
    r.aoff.push_back(static_cast<int>(r.args.size()));
    return r;
}

// The buffer holding each problem's state after all nl intervals of a sweep.
template <typename T>
std::vector<T*> sweep_result(const std::vector<BatchProb>& probs, const Tiling& t, const std::vector<T*>& buf0,
                             const std::vector<T*>& buf1) {
    std::vector<T*> res(probs.size());
    for (size_t i = 0; i < probs.size(); ++i) {
        const int nlp = (probs[i].s_last + t.steps - 1) / t.steps;
        res[i] = nlp == 0 ? buf0[i] : ((nlp - 1) % 2 == 0 ? buf1[i] : buf0[i]);
    }
    return res;
}

// Batched FWD, intervals [j0, j1): interval j advances from (j even ? bufA : bufB)
// into the other buffer and stores every state into the problem's trajectory.
inline IntervalTables<FwdArgs> plan_fwd(const std::vector<BatchProb>& probs, const Tiling& t,
                                        const std::vector<double*>& bufA, const std::vector<double*>& bufB, int j0,
                                        int j1, double fl_fwd) {
    const int np = static_cast<int>(probs.size());
    IntervalTables<FwdArgs> r;
    r.j0 = j0;
    r.j1 = j1;
    for (int j = j0; j < j1; ++j) {
        r.off.push_back(static_cast<int>(r.items.size()));
        r.aoff.push_back(static_cast<int>(r.args.size()));
        double fl = 0.0;
        for (int i = 0; i < np; ++i) {
            const BatchProb& p = probs[i];
            const int s0 = j * t.steps;
            FwdArgs a{};
            a.n = p.n;
            if (s0 < p.s_last) {
                a.xin = (j % 2 == 0) ? bufA[i] : bufB[i];
                a.xout = (j % 2 == 0) ? bufB[i] : bufA[i];
                a.store = const_cast<double*>(p.traj);
                a.store_every = 1;
                a.store_row0 = 0;
                a.store_rows = p.traj_rows;
                a.h = p.dt;
                a.inv2dx = p.inv2dx;
                a.nu_dx2 = p.nu_dx2;
                a.s0 = s0;
                a.S = std::min(t.steps, p.s_last - s0);
                a.tile = batch_tile(t, p.n);
                a.halo = 4 * t.steps + 4;
                a.obs_stride = p.obs_stride;
                a.obs_every = p.obs_every;
                a.n_obs = p.n_obs;
                a.n_t = p.n_t;
                a.inv_sigma_o = 1.0 / p.sigma_o;
                a.y = p.y;
                a.innov = p.innov;
                a.obs_out = p.obs_out;
                const int slot = static_cast<int>(r.args.size()) - r.aoff.back();
                const int ntile = (p.n + a.tile - 1) / a.tile;
                for (int tl = 0; tl < ntile; ++tl) r.items.push_back(PlanItem{slot, tl, 0, 0});
                fl += static_cast<double>(a.S) * p.n * fl_fwd;
            }
            r.args.push_back(a);
        }
        r.flops.push_back(fl);
    }
    r.off.push_back(static_cast<int>(r.items.size()));
    r.aoff.push_back(static_cast<int>(r.args.size()));
    return r;
}

// ---------------------------------------------------------------------------
// Staging ring.  Descriptor tables go through a pinned host ring of `cap` bytes
// and its device mirror (same offsets), used as two halves.  The tables of one
// group -- everything one set of launches reads -- are placed contiguously in
// one half.  When a group does not fit in the rest of the current half, the
// stream is drained (every launch enqueued so far, which includes every launch
// that read the other half, has completed) and the group goes to the start of
// the other half.  So a group never overwrites itself, and a half is reused
// only after everything that read it is done.  A group must fit in one half.
// ---------------------------------------------------------------------------
constexpr size_t kRingAlign = 256;
inline size_t ring_round(size_t bytes) { return (bytes + kRingAlign - 1) / kRingAlign * kRingAlign; }

struct RingPlace {
    size_t first;      // offset of the group's first table
    size_t next;       // ring offset after the group
    bool drain;        // the stream must be drained before the group is written
    bool fits;         // false: the group is larger than a half
};

inline RingPlace ring_place_group(size_t off, size_t cap, size_t group_bytes) {
    const size_t half = cap / 2;
    RingPlace r{off, off, false, group_bytes <= half};
    if (!r.fits) return r;
    const size_t base = off < half ? 0 : half;
    if (off + group_bytes > base + half) {
        r.drain = true;
        r.first = base == 0 ? half : 0;
    }
    r.next = r.first + group_bytes;
    return r;
}

// Intervals per staged chunk of a batched sweep or FWD, so that a chunk's
// argument blocks and items (one group) take at most `budget` bytes.  Returns
// the chunk boundaries [0 = c_0 < c_1 < ... = nl].
template <typename CountItems>
std::vector<int> interval_chunks(int nl, size_t arg_bytes_per_interval, CountItems items_of, size_t budget) {
    std::vector<int> cuts{0};
    size_t used = 0;
    for (int j = 0; j < nl; ++j) {
        const size_t b = arg_bytes_per_interval + static_cast<size_t>(items_of(j)) * sizeof(PlanItem);
        if (j > cuts.back() && used + b > budget) {
            cuts.push_back(j);
            used = 0;
        }
        used += b;
    }
    cuts.push_back(nl);
    return cuts;
}

}  // namespace rp4d
