// Host-only checker of the batched sweeps' descriptor tables (test
// infrastructure; built and run by tests/test_batch_plan.py).
//
// It plans the tables of a batched FWD, TLM and ADJ sweep with the library's
// own planner (batch_plan.hpp) for a list of problems and tilings, with fake
// buffer addresses of known extents, and bounds every index the sweep kernels
// derive from an item and its argument block (burgers_sweep.hip):
//   item (slot, tile, group) -> args[aoff + slot], tile < ntile, group < groups;
//   region points g = (tile*T - halo + r) mod n, r < region;
//   xin / xout at (group n + g) KC + c, c < KC;
//   trajectory rows s0 .. s0+S-1 (TLM, ADJ) and stored rows s0+1 .. s0+S (FWD);
//   observation rows (i-1) n_obs + g / stride for 1 <= i <= n_t, columns < k;
// and the invariants the kernels rely on: region >= tile + 2 halo, halo >= 4S+4,
// the owned ranges of the tiles partition [0, n), every argument block an item
// names belongs to an active problem, and each staged group fits half the ring.
//
// It also replays the ring placement of one batched FWD followed by one
// batched block Hessian's sweeps (the tables as planned before the tables were
// cut into chunks: every interval at once) under the earlier placement policy
// -- drain and restart at offset 0 when a table does not fit -- and the current
// one, and reports whether a table of a launch group is overwritten before its
// launches are enqueued.
//
// Input (stdin): nprob, then per problem "n s_last obs_stride obs_every";
// ntiling, then per tiling "xch ppt kc threads steps"; nk, then the k values.
// Output: one line per (tiling, k) and a final "violations N" line.
#include <cinttypes>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "batch_plan.hpp"

namespace rp4d {
[[noreturn]] void fail(int code, const std::string& msg) { throw std::runtime_error(std::to_string(code) + ": " + msg); }
}  // namespace rp4d

using namespace rp4d;

namespace {

// Fake buffers: buffer b starts at (b + 1) << 36 and holds extent[b] elements.
struct Buffers {
    std::vector<size_t> extent;
    std::vector<size_t> esize;
    std::vector<std::string> name;
    uintptr_t make(size_t count, size_t es, const std::string& nm) {
        extent.push_back(count);
        esize.push_back(es);
        name.push_back(nm);
        return static_cast<uintptr_t>(extent.size()) << 36;
    }
    // buffer id of a pointer and the element offset of its base within it
    bool locate(const void* p, int& id, long& off) const {
        const uintptr_t v = reinterpret_cast<uintptr_t>(p);
        const long b = static_cast<long>(v >> 36) - 1;
        if (b < 0 || b >= static_cast<long>(extent.size())) return false;
        id = static_cast<int>(b);
        const uintptr_t rel = v - (static_cast<uintptr_t>(b + 1) << 36);
        if (rel % esize[b] != 0) return false;
        off = static_cast<long>(rel / esize[b]);
        return true;
    }
};

long violations = 0;
void bad(const std::string& what) {
    if (violations < 20) std::printf("VIOLATION %s\n", what.c_str());
    ++violations;
}

// element range [lo, hi] of pointer p must lie inside its buffer, which must be `want`
void access(const Buffers& B, const void* p, long lo, long hi, int want, const char* what) {
    int id;
    long off;
    if (p == nullptr || !B.locate(p, id, off)) {
        bad(std::string(what) + ": pointer outside every buffer");
        return;
    }
    if (want >= 0 && id != want) bad(std::string(what) + ": pointer into " + B.name[id] + ", not " + B.name[want]);
    if (off + lo < 0 || off + hi >= static_cast<long>(B.extent[id]))
        bad(std::string(what) + ": elements [" + std::to_string(off + lo) + ", " + std::to_string(off + hi) +
            "] outside " + B.name[id] + " of " + std::to_string(B.extent[id]));
}

struct Prob {
    BatchProb bp;
    int traj, innov, y, fa, fb, s0, s1, z;  // buffer ids
};

struct TilingIn {
    int xch, ppt, kc, threads, steps;
};

const size_t kCap = 32u << 20;  // the library's staging ring

// Region geometry shared by the three sweeps.
void check_region(const std::string& tag, const BatchProb& p, const Tiling& t, int tile, int halo, int S) {
    const long region = static_cast<long>(t.xch == XCH_WAVE ? 64 : t.threads) * t.ppt;
    if (halo < 4 * S + 4) bad(tag + ": halo < 4 S + 4");
    if (region < tile + 2L * halo) bad(tag + ": region < tile + 2 halo");
    if (tile < 1 || tile > p.n) bad(tag + ": tile out of [1, n]");
}

template <typename A>
bool item_slot_ok(const std::string& tag, const IntervalTables<A>& tb, int q, const PlanItem& it, int np) {
    const int nslot = tb.aoff[q + 1] - tb.aoff[q];
    if (nslot != np) bad(tag + ": interval does not hold one argument block per problem");
    if (it.x < 0 || it.x >= nslot) {
        bad(tag + ": item names argument slot " + std::to_string(it.x) + " of " + std::to_string(nslot));
        return false;
    }
    return true;
}

template <typename T>
void check_sweep(const std::string& tag, int mode, const std::vector<Prob>& P, const Buffers& B, int k,
                 const Tiling& t, const IntervalTables<SweepArgs<T>>& tb) {
    const int np = static_cast<int>(P.size());
    const int groups = (k + t.kc - 1) / t.kc;
    for (int q = 0; q + tb.j0 < tb.j1; ++q) {
        const int j = tb.j0 + q;
        // how often each (tile, group) of each problem appears
        std::vector<std::vector<int>> seen(np);
        for (int i = 0; i < np; ++i) {
            const SweepArgs<T>& a = tb.args[tb.aoff[q] + i];
            if (a.S >= 1) seen[i].assign(static_cast<size_t>((P[i].bp.n + a.tile - 1) / a.tile) * groups, 0);
        }
        for (int e = tb.off[q]; e < tb.off[q + 1]; ++e) {
            const PlanItem& it = tb.items[e];
            if (!item_slot_ok(tag, tb, q, it, np)) continue;
            const int i = it.x;
            const SweepArgs<T>& a = tb.args[tb.aoff[q] + i];
            const Prob& pr = P[i];
            const BatchProb& p = pr.bp;
            if (a.S < 1 || a.n != p.n) {
                bad(tag + ": item names an inactive or foreign argument block");
                continue;
            }
            const int ntile = (p.n + a.tile - 1) / a.tile;
            if (it.y < 0 || it.y >= ntile || it.z < 0 || it.z >= groups) {
                bad(tag + ": tile or group index out of range");
                continue;
            }
            seen[i][static_cast<size_t>(it.z) * ntile + it.y] += 1;
            if (e > tb.off[q] && tb.items[e - 1].x == it.x) continue;  // the block's fields are checked once per run of items
            check_region(tag, p, t, a.tile, a.halo, a.S);
            if (a.S > t.steps || a.s0 < 0 || a.s0 + a.S > p.s_last) bad(tag + ": steps outside the window");
            // expected interval placement
            if (mode == MODE_TLM && a.s0 != j * t.steps) bad(tag + ": TLM interval starts at the wrong step");
            if (mode == MODE_ADJ && a.s0 + a.S != p.s_last - j * t.steps) bad(tag + ": ADJ interval ends at the wrong step");
            // blocked state: every group (items name group < groups), every region point, KC vectors
            const long lo = 0, hi = static_cast<long>(groups) * p.n * t.kc - 1;
            const int in_buf = (j % 2 == 0) ? pr.s0 : pr.s1, out_buf = (j % 2 == 0) ? pr.s1 : pr.s0;
            access(B, a.xin, lo, hi, in_buf, (tag + " xin").c_str());
            access(B, a.xout, lo, hi, out_buf, (tag + " xout").c_str());
            // trajectory rows s0 .. s0+S-1
            access(B, a.base, static_cast<long>(a.s0 - a.base_row0) * p.n,
                   static_cast<long>(a.s0 + a.S - 1 - a.base_row0) * p.n + p.n - 1, pr.traj, (tag + " base").c_str());
            // observations of steps s0+1 .. s0+S (rows (i-1) n_obs + g/stride, columns < k)
            long omin = -1, omax = -1;
            for (int s1 = a.s0 + 1; s1 <= a.s0 + a.S; ++s1) {
                if (s1 % a.obs_every) continue;
                const int oi = s1 / a.obs_every;
                if (oi < 1 || oi > a.n_t) continue;
                const long r0 = static_cast<long>(oi - 1) * a.n_obs, r1 = r0 + (p.n - 1) / a.obs_stride;
                if ((p.n - 1) / a.obs_stride >= a.n_obs) bad(tag + ": observation index beyond n_obs");
                omin = omin < 0 ? r0 : std::min(omin, r0);
                omax = std::max(omax, r1);
            }
            if (omin >= 0) {
                const T* obs = mode == MODE_TLM ? a.z : a.w;
                access(B, obs, omin * k, omax * k + (k - 1), pr.z, (tag + (mode == MODE_TLM ? " z" : " w")).c_str());
            }
        }
        // the tiles [t T, min((t+1) T, n)) of each active (problem, group) cover
        // [0, n): all ntile of them, each exactly once
        for (int i = 0; i < np; ++i) {
            const SweepArgs<T>& a = tb.args[tb.aoff[q] + i];
            if (a.S < 1) continue;
            for (int c : seen[i])
                if (c != 1) {
                    bad(tag + ": a (tile, group) is missing or repeated");
                    break;
                }
        }
    }
}

void check_fwd(const std::string& tag, const std::vector<Prob>& P, const Buffers& B, const Tiling& t,
               const IntervalTables<FwdArgs>& tb) {
    const int np = static_cast<int>(P.size());
    for (int q = 0; q + tb.j0 < tb.j1; ++q) {
        const int j = tb.j0 + q;
        std::vector<int> cnt(np, 0);
        for (int e = tb.off[q]; e < tb.off[q + 1]; ++e) {
            const PlanItem& it = tb.items[e];
            if (!item_slot_ok(tag, tb, q, it, np)) continue;
            const int i = it.x;
            const FwdArgs& a = tb.args[tb.aoff[q] + i];
            const Prob& pr = P[i];
            const BatchProb& p = pr.bp;
            if (a.S < 1 || a.n != p.n) {
                bad(tag + ": item names an inactive or foreign argument block");
                continue;
            }
            const int ntile = (p.n + a.tile - 1) / a.tile;
            if (it.y < 0 || it.y >= ntile) bad(tag + ": tile index out of range");
            check_region(tag, p, t, a.tile, a.halo, a.S);
            if (a.s0 != j * t.steps || a.s0 + a.S > p.s_last) bad(tag + ": steps outside the window");
            const int in_buf = (j % 2 == 0) ? pr.fa : pr.fb, out_buf = (j % 2 == 0) ? pr.fb : pr.fa;
            access(B, a.xin, 0, p.n - 1, in_buf, (tag + " xin").c_str());
            access(B, a.xout, 0, p.n - 1, out_buf, (tag + " xout").c_str());
            const long r0 = (a.s0 + 1) / a.store_every - a.store_row0, r1 = (a.s0 + a.S) / a.store_every - a.store_row0;
            if (r0 < 0 || r1 >= a.store_rows) bad(tag + ": stored rows outside the trajectory");
            access(B, a.store, r0 * p.n, r1 * p.n + p.n - 1, pr.traj, (tag + " store").c_str());
            for (int s1 = a.s0 + 1; s1 <= a.s0 + a.S; ++s1) {
                if (s1 % a.obs_every) continue;
                const int oi = s1 / a.obs_every;
                if (oi < 1 || oi > a.n_t) continue;
                const long r = static_cast<long>(oi - 1) * a.n_obs;
                const long last = r + (p.n - 1) / a.obs_stride;
                if (a.y) access(B, a.y, r, last, pr.y, (tag + " y").c_str());
                if (a.innov) access(B, a.innov, r, last, pr.innov, (tag + " innov").c_str());
                access(B, a.obs_out, r, last, pr.innov, (tag + " obs_out").c_str());
            }
            cnt[i] += 1;
        }
        for (int i = 0; i < np; ++i) {
            const FwdArgs& a = tb.args[tb.aoff[q] + i];
            if (a.S >= 1 && cnt[i] != (P[i].bp.n + a.tile - 1) / a.tile) bad(tag + ": tiles do not cover the grid once");
        }
    }
}

// Ring replay.  A group is the list of table sizes one set of launches reads.
// Returns the number of groups in which a table is overwritten by a later
// table of the same group.
long replay_old(const std::vector<std::vector<size_t>>& groups, size_t off) {
    long hits = 0;
    for (const auto& g : groups) {
        std::vector<std::pair<size_t, size_t>> placed;
        bool hit = false;
        for (size_t bytes0 : g) {
            const size_t bytes = ring_round(bytes0);
            if (bytes > kCap) return -1;  // rejected outright
            if (off + bytes > kCap) off = 0;  // drain, restart at 0
            for (auto& pl : placed)
                if (off < pl.first + pl.second && pl.first < off + bytes) hit = true;
            placed.push_back({off, bytes});
            off += bytes;
        }
        hits += hit ? 1 : 0;
    }
    return hits;
}

long replay_new(const std::vector<std::vector<size_t>>& groups, bool& fits, size_t off) {
    long hits = 0;
    fits = true;
    for (const auto& g : groups) {
        size_t total = 0;
        for (size_t b : g) total += ring_round(b);
        const RingPlace r = ring_place_group(off, kCap, total);
        if (!r.fits) {
            fits = false;
            continue;
        }
        if (r.first + total > kCap) hits += 1;
        off = r.next;
    }
    return hits;
}

}  // namespace

int main() {
    int np = 0;
    if (std::scanf("%d", &np) != 1 || np < 1) return 2;
    std::vector<Prob> P(np);
    Buffers B;
    for (int i = 0; i < np; ++i) {
        int n, sl, os, oe;
        if (std::scanf("%d %d %d %d", &n, &sl, &os, &oe) != 4) return 2;
        BatchProb& p = P[i].bp;
        p = BatchProb{};
        p.n = n;
        p.s_last = sl;
        p.dt = 1e-3;
        p.inv2dx = 0.5 * n;
        p.nu_dx2 = 0.01 * n * n;
        p.obs_stride = os;
        p.obs_every = oe;
        p.n_obs = (n + os - 1) / os;
        p.n_t = sl / oe;
        p.sigma_o = 0.01;
        p.traj_rows = sl + 1;
        const size_t m = static_cast<size_t>(p.n_obs) * p.n_t;
        P[i].traj = static_cast<int>(B.extent.size());
        p.traj = reinterpret_cast<const double*>(B.make(static_cast<size_t>(sl + 1) * n, 8, "traj" + std::to_string(i)));
        P[i].innov = static_cast<int>(B.extent.size());
        // innovations (m) and, after them, the observations O x (m): one buffer of 2m
        p.innov = reinterpret_cast<double*>(B.make(2 * m, 8, "innov" + std::to_string(i)));
        p.obs_out = p.innov + m;
        P[i].y = static_cast<int>(B.extent.size());
        p.y = reinterpret_cast<const double*>(B.make(m, 8, "y" + std::to_string(i)));
        // FWD ping-pong states: ws_red holds 2n + 512 doubles
        P[i].fa = static_cast<int>(B.extent.size());
        double* red = reinterpret_cast<double*>(B.make(static_cast<size_t>(2 * n + 512), 8, "red" + std::to_string(i)));
        P[i].fb = P[i].fa;
        (void)red;
    }
    int nt = 0;
    if (std::scanf("%d", &nt) != 1) return 2;
    std::vector<TilingIn> tilings(nt);
    for (auto& x : tilings)
        if (std::scanf("%d %d %d %d %d", &x.xch, &x.ppt, &x.kc, &x.threads, &x.steps) != 5) return 2;
    int nk = 0;
    if (std::scanf("%d", &nk) != 1) return 2;
    std::vector<int> ks(nk);
    for (int& k : ks)
        if (std::scanf("%d", &k) != 1) return 2;

    long old_hits_total = 0, new_hits_total = 0, nofit = 0, planned = 0;
    for (const TilingIn& ti : tilings) {
        Tiling t;
        t.xch = ti.xch;
        t.ppt = ti.ppt;
        t.kc = ti.kc;
        t.threads = ti.threads;
        t.steps = ti.steps;
        Tiling tf = t;
        tf.kc = 1;
        for (int k : ks) {
            Tiling tk = t;
            while (tk.kc > 1 && tk.kc > k) tk.kc /= 2;  // as the library: no padded vectors for small k
            Buffers Bk = B;
            std::vector<Prob> Pk = P;
            const int groups = (k + tk.kc - 1) / tk.kc;
            std::vector<double*> fa(np), fb(np);
            std::vector<double*> s0(np), s1(np), z(np);
            std::vector<const double*> w(np), none(np, nullptr);
            for (int i = 0; i < np; ++i) {
                const int n = Pk[i].bp.n;
                double* red = reinterpret_cast<double*>(static_cast<uintptr_t>(Pk[i].fa + 1) << 36);
                fa[i] = red;
                fb[i] = red + n;
                // block workspaces as the library sizes them: (groups + 1) kc n
                const size_t blk = static_cast<size_t>(groups + 1) * tk.kc * n;
                Pk[i].s0 = static_cast<int>(Bk.extent.size());
                s0[i] = reinterpret_cast<double*>(Bk.make(blk, 8, "s0_" + std::to_string(i)));
                Pk[i].s1 = static_cast<int>(Bk.extent.size());
                s1[i] = reinterpret_cast<double*>(Bk.make(blk, 8, "s1_" + std::to_string(i)));
                const size_t m = static_cast<size_t>(Pk[i].bp.n_obs) * Pk[i].bp.n_t;
                Pk[i].z = static_cast<int>(Bk.extent.size());
                z[i] = reinterpret_cast<double*>(Bk.make(m * k, 8, "obs_" + std::to_string(i)));
                w[i] = z[i];
            }
            std::vector<BatchProb> bp(np);
            for (int i = 0; i < np; ++i) bp[i] = Pk[i].bp;
            char tag[128];
            std::snprintf(tag, sizeof tag, "xch%d ppt%d kc%d thr%d S%d k%d", t.xch, t.ppt, tk.kc, t.threads,
                          t.steps, k);
            std::vector<std::vector<size_t>> old_groups, new_groups;
            try {
                const int nl_f = batch_intervals(bp, tf), nl = batch_intervals(bp, tk);
                std::vector<int> ntf(np), ntk(np), nlf(np), nlk(np);
                for (int i = 0; i < np; ++i) {
                    ntf[i] = (bp[i].n + batch_tile(tf, bp[i].n) - 1) / batch_tile(tf, bp[i].n);
                    ntk[i] = (bp[i].n + batch_tile(tk, bp[i].n) - 1) / batch_tile(tk, bp[i].n);
                    nlf[i] = (bp[i].s_last + tf.steps - 1) / tf.steps;
                    nlk[i] = (bp[i].s_last + tk.steps - 1) / tk.steps;
                }
                auto items_f = [&](int j) {
                    long c = 0;
                    for (int i = 0; i < np; ++i)
                        if (j < nlf[i]) c += ntf[i];
                    return c;
                };
                auto items_k = [&](int j) {
                    long c = 0;
                    for (int i = 0; i < np; ++i)
                        if (j < nlk[i]) c += static_cast<long>(ntk[i]) * groups;
                    return c;
                };
                long tot_f = 0, tot_k = 0;
                for (int j = 0; j < nl_f; ++j) tot_f += items_f(j);
                for (int j = 0; j < nl; ++j) tot_k += items_k(j);
                // the tables as first staged: every interval at once, args then items
                const size_t copy_bytes = 2 * np * 32;  // the small groups between the sweeps
                const size_t sa = sizeof(SweepArgs<double>);
                old_groups = {{copy_bytes, 4096},
                              {static_cast<size_t>(nl_f) * np * sizeof(FwdArgs), tot_f * sizeof(PlanItem)},
                              {copy_bytes, 4096},
                              {static_cast<size_t>(nl) * np * sa, tot_k * sizeof(PlanItem)},
                              {copy_bytes, 4096},
                              {static_cast<size_t>(nl) * np * sa, tot_k * sizeof(PlanItem)}};
                // the current tables, chunk by chunk (each chunk one staged group), checked as planned
                auto run_chunks = [&](int nl_x, auto items_of, size_t abytes, auto plan_check) {
                    const auto cuts = interval_chunks(nl_x, abytes * np + 2 * kRingAlign, items_of, kCap / 4);
                    for (size_t c = 0; c + 1 < cuts.size(); ++c) {
                        const auto sizes = plan_check(cuts[c], cuts[c + 1]);
                        new_groups.push_back(sizes);
                    }
                };
                new_groups.push_back({copy_bytes, 4096});
                run_chunks(nl_f, items_f, sizeof(FwdArgs), [&](int j0, int j1) {
                    const auto tb = plan_fwd(bp, tf, fa, fb, j0, j1, 48.0);
                    check_fwd(std::string(tag) + " fwd", Pk, Bk, tf, tb);
                    return std::vector<size_t>{tb.args.size() * sizeof(FwdArgs), tb.items.size() * sizeof(PlanItem)};
                });
                new_groups.push_back({copy_bytes, 4096});
                run_chunks(nl, items_k, sa, [&](int j0, int j1) {
                    const auto tb = plan_sweep<double>(MODE_TLM, bp, k, tk, s0, s1, z, none, j0, j1, 36.0, 48.0);
                    check_sweep<double>(std::string(tag) + " tlm", MODE_TLM, Pk, Bk, k, tk, tb);
                    return std::vector<size_t>{tb.args.size() * sa, tb.items.size() * sizeof(PlanItem)};
                });
                new_groups.push_back({copy_bytes, 4096});
                run_chunks(nl, items_k, sa, [&](int j0, int j1) {
                    const auto tb = plan_sweep<double>(MODE_ADJ, bp, k, tk, s0, s1, {}, w, j0, j1, 34.0, 58.0);
                    check_sweep<double>(std::string(tag) + " adj", MODE_ADJ, Pk, Bk, k, tk, tb);
                    return std::vector<size_t>{tb.args.size() * sa, tb.items.size() * sizeof(PlanItem)};
                });
            } catch (const std::exception& e) {
                std::printf("%s rejected: %s\n", tag, e.what());
                continue;
            }
            ++planned;
            // three timing repetitions, as a tiling search does, from every
            // starting offset of the ring (in steps of 1 MiB: the ring's history
            // before the first FWD) -- how many starts end with a table
            // overwritten by a later table of its own group
            std::vector<std::vector<size_t>> og, ng;
            for (int r = 0; r < 3; ++r) {
                og.insert(og.end(), old_groups.begin(), old_groups.end());
                ng.insert(ng.end(), new_groups.begin(), new_groups.end());
            }
            long oh = 0, nh = 0;
            bool fits = true;
            for (size_t start = 0; start < kCap; start += size_t(1) << 20) {
                const long o = replay_old(og, start);
                if (o < 0) {
                    oh = -1;
                    break;
                }
                oh += o > 0 ? 1 : 0;
            }
            for (size_t start = 0; start < kCap; start += size_t(1) << 20) {
                bool f = true;
                nh += replay_new(ng, f, start) > 0 ? 1 : 0;
                fits = fits && f;
            }
            size_t maxgroup = 0;
            for (auto& g : new_groups) {
                size_t tot = 0;
                for (size_t b : g) tot += ring_round(b);
                maxgroup = std::max(maxgroup, tot);
            }
            if (!fits) {
                bad(std::string(tag) + ": a chunked group exceeds half the ring");
                ++nofit;
            }
            if (nh) bad(std::string(tag) + ": the current placement overwrote a table of its own group");
            old_hits_total += oh > 0 ? oh : 0;
            new_hits_total += nh;
            std::printf("%s sweep_items %zu old_overwrites %ld new_overwrites %ld max_group_bytes %zu\n", tag,
                        old_groups[3][1] / sizeof(PlanItem), oh, nh, maxgroup);
        }
    }
    std::printf("planned %ld old_overwrites %ld new_overwrites %ld violations %ld\n", planned, old_hits_total,
                new_hits_total, violations);
    return violations == 0 ? 0 : 1;
}
