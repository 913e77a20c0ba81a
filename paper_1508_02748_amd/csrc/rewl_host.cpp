// rewl_host.cpp -- the C ABI of include/rewl.h: plan construction, buffer
// layout, launch sequencing (batched form with graph replay, plain form with
// one launch per window and a host round trip per interval), read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rewl.h"
#include "rewl_internal.h"

using namespace rewl;

namespace {

thread_local std::string g_err;

rewl_status fail(rewl_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Overlapping equal-size energy windows over e in [0, N] (Sec. 2, Fig. 1(b)):
// with overlap p/q and D = q + (n-1)(q-p), window i is
// [floor(i (q-p) N / D), min(N, ceil((i (q-p) + q) N / D))].
void window_bounds(int N, int n, int p, int q, int i, int& lo, int& hi) {
    const long long D = q + static_cast<long long>(n - 1) * (q - p);
    const long long a = static_cast<long long>(i) * (q - p) * N;
    const long long b = (static_cast<long long>(i) * (q - p) + q) * N;
    lo = static_cast<int>(a / D);
    const long long h = (b + D - 1) / D;
    hi = static_cast<int>(std::min<long long>(h, N));
}

// Realizable energy bins at magnetization bin m of the periodic L x L lattice
// (N = L^2), in closed form.  With k = min(m, N - m) minority spins:
//   * at most 2k: each unsatisfied bond has a minority spin at one end, and a
//     spin has four bonds (reached by minority spins on one sublattice);
//   * at least half the shortest closed domain wall around k sites on the
//     torus: a compact cluster has perimeter 2 ceil(2 sqrt k); once k >= L a
//     straight band around the torus needs only 2L bonds when L divides k and
//     2L + 2 otherwise.
void energy_range(int L, int m, int& emin, int& emax) {
    const int N = L * L;
    const int k = std::min(m, N - m);
    emax = 2 * k;
    if (k == 0) {
        emin = 0;
        return;
    }
    long long t = 0;  // ceil(2 sqrt k): the least t with t^2 >= 4k
    while (t * t < 4ll * k) ++t;
    long long wall = 2 * t;
    if (k >= L) wall = std::min<long long>(wall, 2ll * L + (k % L ? 2 : 0));
    emin = static_cast<int>(wall / 2);
}

// Whether some state has energy bin e and magnetization bin m: inside the
// range above every bin does, except next to m = N/2, where the bin just
// above the lowest and the two just below the highest are empty at m = N/2,
// and the one just below the highest at m = N/2 +- 1 (exhaustive enumeration
// agrees for L = 4 and 6).
bool holds_state(int L, int e, int m) {
    int emin, emax;
    energy_range(L, m, emin, emax);
    if (e < emin || e > emax) return false;
    const int N = L * L;
    if (m == N / 2) return e != emin + 1 && e != emax - 1 && e != emax - 2;
    if (m == N / 2 - 1 || m == N / 2 + 1) return e != emax - 1;
    return true;
}

bool rect_holds_state(int L, int elo, int ehi, int mlo, int mhi) {
    for (int m = mlo; m <= mhi; ++m)
        for (int e = elo; e <= ehi; ++e)
            if (holds_state(L, e, m)) return true;
    return false;
}

// The windows of one problem as rectangles of (e, m) bins, e-major, with the
// neighbouring pairs that may exchange.
struct Rect {
    int elo, ehi, mlo, mhi;
};

void problem_windows(const rewl_problem& q, std::vector<Rect>& rects, std::vector<PairDesc>& pairs, int prob) {
    const int N = q.L * q.L;
    rects.clear();
    pairs.clear();
    if (q.split != REWL_SPLIT_BOTH) {
        for (int w = 0; w < q.n_windows; ++w) {
            int lo, hi;
            window_bounds(N, q.n_windows, q.overlap_num, q.overlap_den, w, lo, hi);
            rects.push_back(q.split == REWL_SPLIT_ENERGY ? Rect{lo, hi, 0, N} : Rect{0, N, lo, hi});
            if (w > 0) pairs.push_back(PairDesc{prob, w - 1, w, 0, w - 1});
        }
        return;
    }
    const int ne = q.n_windows, nm = q.m_windows;
    std::vector<int> keep(static_cast<size_t>(ne) * nm, -1);
    for (int ie = 0; ie < ne; ++ie)
        for (int im = 0; im < nm; ++im) {
            Rect r;
            window_bounds(N, ne, q.overlap_num, q.overlap_den, ie, r.elo, r.ehi);
            window_bounds(N, nm, q.m_overlap_num, q.m_overlap_den, im, r.mlo, r.mhi);
            if (rect_holds_state(q.L, r.elo, r.ehi, r.mlo, r.mhi)) {
                keep[static_cast<size_t>(ie) * nm + im] = static_cast<int>(rects.size());
                rects.push_back(r);
            }
        }
    for (int ie = 0; ie < ne; ++ie)
        for (int im = 0; im < nm; ++im) {
            const int w = keep[static_cast<size_t>(ie) * nm + im];
            if (w < 0) continue;
            if (ie + 1 < ne && keep[static_cast<size_t>(ie + 1) * nm + im] >= 0)
                pairs.push_back(PairDesc{prob, w, keep[static_cast<size_t>(ie + 1) * nm + im], 0, ie});
            if (im + 1 < nm && keep[static_cast<size_t>(ie) * nm + im + 1] >= 0)
                pairs.push_back(PairDesc{prob, w, keep[static_cast<size_t>(ie) * nm + im + 1], 1, im});
        }
}

}  // namespace

struct rewl_plan {
    std::vector<rewl_problem> probs;
    rewl_tuning tune{};
    std::vector<PDesc> pd;
    std::vector<WDesc> wd;
    std::vector<PairDesc> pairs;
    std::vector<std::vector<Rect>> rect;   // per problem, per window
    int64_t n_walk = 0;
    uint64_t n_bins = 0;
    uint64_t n_words = 0;
    int l_max = 0;
    int64_t interval = 0;
    size_t sizes[REWL_NBUF] = {0, 0, 0};
    // STATE buffer offsets
    size_t off_wd = 0, off_pd = 0, off_pairs = 0, off_e = 0, off_m = 0, off_t = 0, off_te = 0,
           off_nseen = 0, off_flag = 0, off_scan = 0, off_aud = 0, off_stage = 0, off_wdone = 0, off_tstage = 0, off_adv = 0,
           off_lngb = 0, off_tseen = 0, off_done = 0, off_rnd = 0, off_xr = 0, off_xon = 0, off_cnt = 0;
    int32_t n_win = 0;  // windows over all problems
    int split = 0;      // the split of every problem of the plan (energy 0, magnetization 1, both 2)
    int layout = LAYOUT_DENSE;
    // binding
    bool bound = false;
    bool broken = false;
    bool initialised = false;
    void* buf[REWL_NBUF] = {nullptr, nullptr, nullptr};
    hipStream_t stream = nullptr;
    DevState S{};
    hipGraphExec_t graph = nullptr;
    int graph_g = 0;
    std::vector<hipEvent_t> ev;  // profile: [2i] before, [2i+1] after sweep i of the last run
    int ev_used = 0;
    bool profile = false;
    int n_cu = 256;
};

namespace {

rewl_status dev_fail(rewl_plan* P, hipError_t e, const char* what) {
    P->broken = true;
    return fail(REWL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(P, call, what)                        \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return dev_fail(P, e_, what); \
    } while (0)

rewl_status usable(rewl_plan* P) {
    if (!P) return fail(REWL_EINVAL, "null plan");
    if (P->broken) return fail(REWL_ESTATE, "plan is in an error state");
    if (!P->bound) return fail(REWL_ESTATE, "plan has no device buffers bound");
    return REWL_OK;
}

rewl_status validate(const rewl_problem& q, int idx) {
    auto bad = [&](const char* m) {
        return fail(REWL_EINVAL, "problem " + std::to_string(idx) + ": " + m);
    };
    if (q.L < 4 || q.L > 64 || (q.L & 1)) return bad("L must be even, 4..64");
    if (q.n_windows < 1) return bad("n_windows must be >= 1");
    if (q.overlap_den < 1 || q.overlap_num < 0 || q.overlap_num >= q.overlap_den)
        return bad("overlap must be num/den with 0 <= num < den");
    if (q.walkers_per_window < 1 || q.walkers_per_window > 256) return bad("walkers_per_window must be 1..256");
    if (q.k_final < 0 || q.k_final > 40) return bad("k_final must be 0..40");
    if (q.flat_den < 1 || q.flat_num < 0 || q.flat_num > q.flat_den) return bad("flatness must be num/den <= 1");
    if (q.interval < 1 || q.interval > (1ll << H_AUDIT_SHIFT)) return bad("interval must be 1..2^30");
    if (q.init != 0 && q.init != 1) return bad("init must be 0 or 1");
    if (q.stage_sync != REWL_SYNC_PROBLEM && q.stage_sync != REWL_SYNC_WINDOW)
        return bad("stage_sync must be REWL_SYNC_PROBLEM or REWL_SYNC_WINDOW");
    if (q.split != REWL_SPLIT_ENERGY && q.split != REWL_SPLIT_MAGNETIZATION && q.split != REWL_SPLIT_BOTH)
        return bad("split must be REWL_SPLIT_ENERGY, REWL_SPLIT_MAGNETIZATION or REWL_SPLIT_BOTH");
    if (q.reserved != 0) return bad("reserved must be 0");
    if (q.split == REWL_SPLIT_BOTH) {
        if (q.m_windows < 1 || q.m_overlap_den < 1 || q.m_overlap_num < 0 || q.m_overlap_num >= q.m_overlap_den)
            return bad("windows in both coordinates need m_windows >= 1 and an overlap num/den < 1");
        if (static_cast<long long>(q.n_windows) * q.m_windows > 4096) return bad("at most 4096 rectangles");
    } else if (q.m_windows != 0 || q.m_overlap_num != 0 || q.m_overlap_den != 0) {
        return bad("m_windows and m_overlap must be 0 unless split is REWL_SPLIT_BOTH");
    }
    const int N = q.L * q.L;
    for (int i = 0; i < q.n_windows; ++i) {
        int lo, hi;
        window_bounds(N, q.n_windows, q.overlap_num, q.overlap_den, i, lo, hi);
        if (lo > hi) return bad("too many windows for the bin range");
    }
    for (int i = 0; i < (q.split == REWL_SPLIT_BOTH ? q.m_windows : 0); ++i) {
        int lo, hi;
        window_bounds(N, q.m_windows, q.m_overlap_num, q.m_overlap_den, i, lo, hi);
        if (lo > hi) return bad("too many magnetization windows");
    }
    return REWL_OK;
}

rewl_status validate_tuning(const rewl_tuning& tn) {
    if (tn.form != REWL_FORM_BATCHED && tn.form != REWL_FORM_PLAIN) return fail(REWL_EINVAL, "unknown form");
    if (tn.walkers_per_wg != 0 && tn.walkers_per_wg != 64 && tn.walkers_per_wg != 128 && tn.walkers_per_wg != 256)
        return fail(REWL_EINVAL, "walkers_per_wg must be 0, 64, 128 or 256");
    if (tn.graph_intervals < 0 || tn.graph_intervals > 4096) return fail(REWL_EINVAL, "graph_intervals 0..4096");
    if (tn.grid_waves_per_cu < 0 || tn.grid_waves_per_cu > 64) return fail(REWL_EINVAL, "grid_waves_per_cu 0..64");
    if (tn.profile != 0 && tn.profile != 1) return fail(REWL_EINVAL, "profile must be 0 or 1");
    if (tn.walkers_per_wave < 0 || tn.walkers_per_wave > 64) return fail(REWL_EINVAL, "walkers_per_wave 0..64");
    if (tn.profile && tn.form != REWL_FORM_BATCHED) return fail(REWL_EINVAL, "profiling times the batched form");
    if (tn.table_layout < REWL_LAYOUT_DENSE || tn.table_layout > REWL_LAYOUT_BAND_PACKED)
        return fail(REWL_EINVAL, "table_layout must be one of the REWL_LAYOUT_ values");
    if (tn.audit_shift < 0 || tn.audit_shift > H_AUDIT_SHIFT) return fail(REWL_EINVAL, "audit_shift 0..30");
    return REWL_OK;
}

DevState make_state(rewl_plan* P) {
    DevState S{};
    char* st = static_cast<char*>(P->buf[REWL_BUF_STATE]);
    S.wd = reinterpret_cast<const WDesc*>(st + P->off_wd);
    S.pd = reinterpret_cast<const PDesc*>(st + P->off_pd);
    S.pairs = reinterpret_cast<const PairDesc*>(st + P->off_pairs);
    S.lng = static_cast<int64_t*>(P->buf[REWL_BUF_TABLES]);
    S.packed = (P->layout & LAYOUT_PACKED) ? 1 : 0;
    S.hb = S.packed ? nullptr : reinterpret_cast<uint32_t*>(S.lng + P->n_bins);
    S.spins = static_cast<uint32_t*>(P->buf[REWL_BUF_SPINS]);
    S.e = reinterpret_cast<int32_t*>(st + P->off_e);
    S.m = reinterpret_cast<int32_t*>(st + P->off_m);
    S.t = reinterpret_cast<int64_t*>(st + P->off_t);
    S.te = reinterpret_cast<int64_t*>(st + P->off_te);
    S.nseen = reinterpret_cast<uint32_t*>(st + P->off_nseen);
    S.flag = reinterpret_cast<uint32_t*>(st + P->off_flag);
    S.scan = reinterpret_cast<uint32_t*>(st + P->off_scan);
    S.aud = reinterpret_cast<uint32_t*>(st + P->off_aud);
    S.stage = reinterpret_cast<int32_t*>(st + P->off_stage);
    S.wdone = reinterpret_cast<int32_t*>(st + P->off_wdone);
    S.tstage = reinterpret_cast<int64_t*>(st + P->off_tstage);
    S.adv = reinterpret_cast<int32_t*>(st + P->off_adv);
    S.lngb = reinterpret_cast<int64_t*>(st + P->off_lngb);
    S.tseen = reinterpret_cast<int64_t*>(st + P->off_tseen);
    S.done = reinterpret_cast<int32_t*>(st + P->off_done);
    S.rnd = reinterpret_cast<int64_t*>(st + P->off_rnd);
    S.xr = reinterpret_cast<int64_t*>(st + P->off_xr);
    S.xon = reinterpret_cast<int32_t*>(st + P->off_xon);
    S.counters = reinterpret_cast<int32_t*>(st + P->off_cnt);
    S.n_walk = P->n_walk;
    S.n_prob = static_cast<int32_t>(P->pd.size());
    S.n_pairs = static_cast<int32_t>(P->pairs.size());
    S.n_win = P->n_win;
    S.audit_shift = P->tune.audit_shift > 0 ? P->tune.audit_shift : (S.packed ? H_AUDIT_SHIFT_PACKED : H_AUDIT_SHIFT);
    return S;
}

// Workgroup size: a tuned value, else 256 lanes once the batch fills the chip
// several times over, 64 below that (fewer, fuller waves per CU).
int wg_of(const rewl_plan* P) {
    if (P->tune.walkers_per_wg > 0) return P->tune.walkers_per_wg;
    return P->n_walk >= (1 << 17) ? 256 : 64;
}

int graph_len(const rewl_plan* P) { return P->tune.graph_intervals > 0 ? P->tune.graph_intervals : 8; }

// Persistent grid: at most grid_waves_per_cu wavefronts per CU in flight.
// Automatic choice: once the batch has at least twice that many walkers, one
// wavefront per SIMD (4 per CU) -- more walkers in flight evict each other's
// table lines from the L2 faster than they hide latency.
int max_grid_of(const rewl_plan* P) {
    int gw = P->tune.grid_waves_per_cu;
    if (gw <= 0) {
        const long long one_per_simd = 4ll * P->n_cu * 64;
        if (P->n_walk < 2 * one_per_simd) return 0;
        gw = 4;
    }
    const long long lanes = static_cast<long long>(gw) * P->n_cu * 64;
    return static_cast<int>(std::max<long long>(1, lanes / wg_of(P)));
}

// The pipelined trial pays where gathers often miss the L2: many walkers (at
// least 16,384, a quarter of the chip's lanes) whose tables are not small (2^13
// bins per walker on average, 64 KB or more packed: 16 x 16 windows and up).
// Small batches and small tables take the direct trial; the plain form's
// launches (one window) always do.
bool ahead_of(const rewl_plan* P) {
    return P->n_walk >= 16384 && P->n_bins >= (static_cast<uint64_t>(P->n_walk) << 13);
}

rewl_status enqueue_sweep(rewl_plan* P, int64_t n, int ev_slot = -1) {
    if (ev_slot >= 0) HIPCHK(P, hipEventRecord(P->ev[2 * ev_slot], P->stream), "event record");
    HIPCHK(P, launch_sweep(P->S, 0, P->n_walk, n, P->l_max, wg_of(P), max_grid_of(P), P->tune.walkers_per_wave,
                           P->split, P->layout, ahead_of(P), P->stream), "sweep launch");
    if (ev_slot >= 0) HIPCHK(P, hipEventRecord(P->ev[2 * ev_slot + 1], P->stream), "event record");
    return REWL_OK;
}

rewl_status enqueue_boundary(rewl_plan* P) {
    HIPCHK(P, launch_flat(P->S, P->stream), "flatness launch");
    HIPCHK(P, launch_stage(P->S, P->stream), "stage launch");
    HIPCHK(P, launch_average(P->S, P->stream), "average launch");
    HIPCHK(P, launch_snapshot(P->S, P->stream), "snapshot launch");
    return REWL_OK;
}

rewl_status enqueue_exchange(rewl_plan* P) {
    HIPCHK(P, launch_exchange(P->S, P->stream), "exchange launch");
    return REWL_OK;
}

rewl_status enqueue_interval_batched(rewl_plan* P, int ev_slot = -1) {
    rewl_status s = enqueue_sweep(P, P->interval, ev_slot);
    if (s != REWL_OK) return s;
    s = enqueue_boundary(P);
    if (s != REWL_OK) return s;
    return enqueue_exchange(P);
}

template <typename T>
rewl_status d2h(rewl_plan* P, std::vector<T>& v, size_t off, size_t n) {
    v.resize(n);
    if (n == 0) return REWL_OK;
    HIPCHK(P, hipMemcpyAsync(v.data(), static_cast<char*>(P->buf[REWL_BUF_STATE]) + off, n * sizeof(T),
                             hipMemcpyDeviceToHost, P->stream), "state read");
    return REWL_OK;
}

template <typename T>
rewl_status h2d(rewl_plan* P, const std::vector<T>& v, size_t off) {
    if (v.empty()) return REWL_OK;
    HIPCHK(P, hipMemcpyAsync(static_cast<char*>(P->buf[REWL_BUF_STATE]) + off, v.data(), v.size() * sizeof(T),
                             hipMemcpyHostToDevice, P->stream), "state write");
    return REWL_OK;
}

// Plain form: one sweep launch per window, then flatness on the device, and
// the stage decision and exchange arming on the host after a synchronisation
// (the same rule as the batched stage kernel), then the exchange launch.
rewl_status run_interval_plain(rewl_plan* P) {
    const int wg = wg_of(P);
    for (size_t p = 0; p < P->pd.size(); ++p) {
        const PDesc& q = P->pd[p];
        for (int w = 0; w < q.nwin; ++w) {
            HIPCHK(P, launch_sweep(P->S, q.walker_off + static_cast<int64_t>(w) * q.W, q.W, P->interval,
                                   q.L, wg, 0, P->tune.walkers_per_wave, P->split, P->layout, false, P->stream),
                   "plain sweep launch");
        }
    }
    HIPCHK(P, launch_flat(P->S, P->stream), "flatness launch");
    const size_t np = P->pd.size(), nwin = static_cast<size_t>(P->n_win);
    std::vector<int32_t> stage, wdone, adv, done, xon;
    std::vector<int64_t> tstage, lngb, tseen, rnd, xr, t;
    std::vector<uint32_t> flag;
    rewl_status s;
    if ((s = d2h(P, stage, P->off_stage, nwin)) || (s = d2h(P, wdone, P->off_wdone, nwin)) ||
        (s = d2h(P, tstage, P->off_tstage, nwin)) || (s = d2h(P, lngb, P->off_lngb, nwin)) ||
        (s = d2h(P, tseen, P->off_tseen, nwin)) || (s = d2h(P, done, P->off_done, np)) ||
        (s = d2h(P, rnd, P->off_rnd, np)) || (s = d2h(P, xr, P->off_xr, np)) || (s = d2h(P, xon, P->off_xon, np)) ||
        (s = d2h(P, t, P->off_t, P->n_walk)) || (s = d2h(P, flag, P->off_flag, P->n_walk)))
        return s;
    HIPCHK(P, hipStreamSynchronize(P->stream), "plain boundary sync");
    bool overflow = false;
    adv.assign(nwin, 0);
    for (size_t p = 0; p < np; ++p) {
        const PDesc& q = P->pd[p];
        if (done[p]) {
            xon[p] = 0;
            continue;
        }
        for (int w = 0; w < q.nwin; ++w) {
            const int wi = q.win_off + w;
            if (wdone[wi]) continue;
            const int64_t tnow = t[q.walker_off + w * q.W];
            const int64_t dt = tnow - tseen[wi];
            const int sh = q.K - stage[wi];
            const int64_t room = ((static_cast<int64_t>(1) << 62) - lngb[wi]) >> sh;
            if (dt > room) overflow = true;
            else lngb[wi] += dt << sh;
            tseen[wi] = tnow;
        }
        const int64_t r = rnd[p];
        bool ended = false;
        if (q.sync == REWL_SYNC_PROBLEM) {
            const int nw = q.nwin * q.W;
            bool all = true;
            for (int i = 0; i < nw; ++i) all = all && flag[q.walker_off + i] != 0;
            if (all) {
                const bool last = stage[q.win_off] == q.K;
                for (int w = 0; w < q.nwin; ++w) {
                    const int wi = q.win_off + w;
                    if (last) {
                        wdone[wi] = 1;
                    } else {
                        stage[wi] += 1;
                        tstage[wi] = t[q.walker_off];
                        adv[wi] = 1;
                    }
                }
                if (last) ended = true;
                else
                    for (int i = 0; i < nw; ++i) flag[q.walker_off + i] = 0;
            }
        } else {
            bool all_done = true;
            for (int w = 0; w < q.nwin; ++w) {
                const int wi = q.win_off + w;
                if (!wdone[wi]) {
                    const int g0 = q.walker_off + w * q.W;
                    bool all = true;
                    for (int a = 0; a < q.W; ++a) all = all && flag[g0 + a] != 0;
                    if (all) {
                        adv[wi] = 1;
                        if (stage[wi] == q.K) {
                            wdone[wi] = 1;
                        } else {
                            stage[wi] += 1;
                            tstage[wi] = t[g0];
                            for (int a = 0; a < q.W; ++a) flag[g0 + a] = 0;
                        }
                    }
                }
                all_done = all_done && wdone[wi] != 0;
            }
            ended = all_done;
        }
        if (ended) {
            done[p] = 1;
            xon[p] = 0;
            rnd[p] = r + 1;
            continue;
        }
        xr[p] = r;
        xon[p] = 1;
        rnd[p] = r + 1;
    }
    if ((s = h2d(P, stage, P->off_stage)) || (s = h2d(P, wdone, P->off_wdone)) ||
        (s = h2d(P, tstage, P->off_tstage)) || (s = h2d(P, adv, P->off_adv)) || (s = h2d(P, lngb, P->off_lngb)) ||
        (s = h2d(P, tseen, P->off_tseen)) || (s = h2d(P, done, P->off_done)) || (s = h2d(P, rnd, P->off_rnd)) ||
        (s = h2d(P, xr, P->off_xr)) || (s = h2d(P, xon, P->off_xon)) || (s = h2d(P, flag, P->off_flag)))
        return s;
    HIPCHK(P, launch_average(P->S, P->stream), "average launch");
    HIPCHK(P, launch_snapshot(P->S, P->stream), "snapshot launch");
    if (overflow) {
        std::vector<int32_t> cnt;
        if ((s = d2h(P, cnt, P->off_cnt, 4))) return s;
        HIPCHK(P, hipStreamSynchronize(P->stream), "plain overflow sync");
        cnt[1] |= ERR_OVERFLOW;
        if ((s = h2d(P, cnt, P->off_cnt))) return s;
    }
    HIPCHK(P, launch_exchange(P->S, P->stream), "exchange launch");
    // the host vectors above die here: keep the copies ordered before reuse
    HIPCHK(P, hipStreamSynchronize(P->stream), "plain interval sync");
    return REWL_OK;
}

rewl_status ensure_graph(rewl_plan* P, int G) {
    if (P->graph && P->graph_g == G) return REWL_OK;
    if (P->graph) {
        (void)hipGraphExecDestroy(P->graph);
        P->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    HIPCHK(P, hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal), "graph capture begin");
    rewl_status s = REWL_OK;
    for (int i = 0; i < G && s == REWL_OK; ++i) s = enqueue_interval_batched(P);
    hipError_t e = hipStreamEndCapture(P->stream, &g);
    if (s != REWL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return dev_fail(P, e, "graph capture end");
    e = hipGraphInstantiate(&P->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return dev_fail(P, e, "graph instantiate");
    P->graph_g = G;
    return REWL_OK;
}

}  // namespace

extern "C" {

const char* rewl_last_error(void) { return g_err.c_str(); }

rewl_status rewl_plan_create(const rewl_problem* problems, int32_t n_problems, const rewl_tuning* tuning,
                             rewl_plan** out) {
    if (!problems || !out || n_problems < 1) return fail(REWL_EINVAL, "problems/out must be non-null, n >= 1");
    *out = nullptr;
    for (int i = 0; i < n_problems; ++i) {
        rewl_status s = validate(problems[i], i);
        if (s != REWL_OK) return s;
    }
    rewl_tuning tn{};
    if (tuning) {
        tn = *tuning;
        rewl_status ts = validate_tuning(tn);
        if (ts != REWL_OK) return ts;
    }
    const int64_t X = problems[0].interval;
    for (int i = 1; i < n_problems; ++i)
        if (problems[i].interval != X) return fail(REWL_EINVAL, "all problems of a plan must share the interval");
    for (int i = 1; i < n_problems; ++i)
        if (problems[i].split != problems[0].split)
            return fail(REWL_EINVAL, "all problems of a plan must share the split");
    if (tn.audit_shift > 0 && X > (1ll << tn.audit_shift))
        return fail(REWL_EINVAL, "the interval exceeds 2^audit_shift trials");

    if ((tn.table_layout & REWL_LAYOUT_BAND) && problems[0].split == REWL_SPLIT_BOTH)
        return fail(REWL_EINVAL, "the band layout applies to one-coordinate splits");
    if (tn.table_layout & LAYOUT_PACKED) {
        for (int i = 0; i < n_problems; ++i)
            if (problems[i].k_final > MAX_K_PACKED) return fail(REWL_EINVAL, "packed tables need k_final <= 24");
        if (X > (1ll << H_AUDIT_SHIFT_PACKED)) return fail(REWL_EINVAL, "packed tables need an interval <= 2^24");
        if (tn.audit_shift > H_AUDIT_SHIFT_PACKED) return fail(REWL_EINVAL, "packed tables need audit_shift <= 24");
    }

    rewl_plan* P = new (std::nothrow) rewl_plan();
    if (!P) return fail(REWL_ENOMEM, "plan allocation");
    P->probs.assign(problems, problems + n_problems);
    P->tune = tn;
    P->profile = tn.profile != 0;
    P->interval = X;
    P->split = problems[0].split;
    P->layout = tn.table_layout;
    int64_t walker = 0;
    uint64_t bins = 0, words = 0;
    std::vector<Rect> rects;
    std::vector<PairDesc> pairs;
    for (int p = 0; p < n_problems; ++p) {
        const rewl_problem& q = problems[p];
        problem_windows(q, rects, pairs, p);
        if (rects.empty()) {
            delete P;
            return fail(REWL_EINVAL, "problem " + std::to_string(p) + ": no window holds a state");
        }
        PDesc d{};
        d.L = q.L;
        d.N = q.L * q.L;
        d.K = q.k_final;
        d.nwin = static_cast<int32_t>(rects.size());
        d.W = q.walkers_per_window;
        d.flat_num = q.flat_num;
        d.flat_den = q.flat_den;
        d.row_words = (q.L + 31) / 32;
        d.X = q.interval;
        d.seed = q.seed;
        d.walker_off = static_cast<int32_t>(walker);
        d.init = q.init;
        d.win_off = P->n_win;
        d.sync = static_cast<int16_t>(q.stage_sync);
        d.split = static_cast<int16_t>(q.split);
        P->pd.push_back(d);
        P->l_max = std::max(P->l_max, q.L);
        for (int w = 0; w < d.nwin; ++w) {
            const Rect& R = rects[w];
            // stored rows and tile columns of the window's tables
            int rows = R.ehi - R.elo + 1;
            uint32_t ntm = static_cast<uint32_t>((R.mhi - R.mlo + 1 + TILE_M - 1) / TILE_M);
            const bool band = (P->layout & REWL_LAYOUT_BAND) && q.split == REWL_SPLIT_ENERGY;
            if (band) {
                // widest tile row of the band (the lowest one, since the band narrows with e)
                uint32_t widest = 0;
                for (int tr = 0; 4 * tr < rows; ++tr) {
                    const int e = R.elo + 4 * tr;
                    const int c0 = band_c0(R.elo, tr), c1 = (d.N - (e + 1) / 2) / TILE_M;
                    widest = std::max<uint32_t>(widest, static_cast<uint32_t>(c1 - c0 + 1));
                }
                ntm = widest;
            } else if ((P->layout & REWL_LAYOUT_BAND) && q.split == REWL_SPLIT_MAGNETIZATION) {
                int kmax = 0;
                for (int m = R.mlo; m <= R.mhi; ++m) kmax = std::max(kmax, std::min(m, d.N - m));
                rows = std::min(d.N, 2 * kmax) + 1;
            }
            for (int a = 0; a < q.walkers_per_window; ++a) {
                WDesc wd{};
                wd.table_off = bins;
                wd.spin_off = static_cast<uint32_t>(words);
                wd.prob = p;
                wd.lo = q.split == REWL_SPLIT_MAGNETIZATION ? R.mlo : R.elo;
                wd.hi = q.split == REWL_SPLIT_MAGNETIZATION ? R.mhi : R.ehi;
                wd.mlo = R.mlo;
                wd.mhi = R.mhi;
                wd.e0 = R.elo;
                wd.m0 = R.mlo;
                wd.win = w;
                wd.gid = w * q.walkers_per_window + a;
                wd.ntm = ntm;
                wd.nrows = static_cast<uint32_t>(rows);
                wd.nbins = static_cast<uint32_t>((rows + TILE_E - 1) / TILE_E) * ntm * TILE_BINS;
                wd.band = band ? 1 : 0;
                wd.gwin = P->n_win + w;
                P->wd.push_back(wd);
                bins += wd.nbins;
                words += static_cast<uint64_t>(q.L) * d.row_words;
                ++walker;
            }
        }
        P->pairs.insert(P->pairs.end(), pairs.begin(), pairs.end());
        P->rect.push_back(rects);
        P->n_win += d.nwin;
        if (walker >= (1ll << 31) || words >= (1ull << 32)) {
            delete P;
            return fail(REWL_EINVAL, "too many walkers for one plan");
        }
    }
    P->n_walk = walker;
    P->n_bins = bins;
    P->n_words = words;
    const size_t A = 256;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, A);
        return at;
    };
    const size_t nw = static_cast<size_t>(walker), np = static_cast<size_t>(n_problems);
    P->off_wd = take(nw * sizeof(WDesc));
    P->off_pd = take(np * sizeof(PDesc));
    P->off_pairs = take(std::max<size_t>(1, P->pairs.size()) * sizeof(PairDesc));
    P->off_e = take(nw * 4);
    P->off_m = take(nw * 4);
    P->off_t = take(nw * 8);
    P->off_te = take(nw * 8);
    P->off_nseen = take(nw * 4);
    P->off_flag = take(nw * 4);
    P->off_scan = take(nw * 4);
    P->off_aud = take(nw * 4);
    const size_t nwn = static_cast<size_t>(P->n_win);
    P->off_stage = take(nwn * 4);
    P->off_wdone = take(nwn * 4);
    P->off_tstage = take(nwn * 8);
    P->off_adv = take(nwn * 4);
    P->off_lngb = take(nwn * 8);
    P->off_tseen = take(nwn * 8);
    P->off_done = take(np * 4);
    P->off_rnd = take(np * 8);
    P->off_xr = take(np * 8);
    P->off_xon = take(np * 4);
    P->off_cnt = take(16);
    // ln g and stage base: one packed word per bin, or an int64 table and a uint32 table
    const size_t per_bin = (tn.table_layout & LAYOUT_PACKED) ? sizeof(int64_t) : sizeof(int64_t) + sizeof(uint32_t);
    P->sizes[REWL_BUF_TABLES] = align_up(bins * per_bin, A);
    P->sizes[REWL_BUF_SPINS] = align_up(words * 4, A);
    P->sizes[REWL_BUF_STATE] = o;
    *out = P;
    return REWL_OK;
}

void rewl_plan_destroy(rewl_plan* P) {
    if (!P) return;
    // work enqueued on the plan's stream may still read or write the caller's
    // buffers: let it finish before the caller can release them
    if (P->bound) (void)hipStreamSynchronize(P->stream);
    if (P->graph) (void)hipGraphExecDestroy(P->graph);
    for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
    delete P;
}

rewl_status rewl_plan_buffer_sizes(const rewl_plan* P, size_t* sizes_out) {
    if (!P || !sizes_out) return fail(REWL_EINVAL, "null argument");
    for (int i = 0; i < REWL_NBUF; ++i) sizes_out[i] = P->sizes[i];
    return REWL_OK;
}

rewl_status rewl_plan_counts(const rewl_plan* P, int32_t* n_problems, int64_t* n_walkers) {
    if (!P) return fail(REWL_EINVAL, "null plan");
    if (n_problems) *n_problems = static_cast<int32_t>(P->pd.size());
    if (n_walkers) *n_walkers = P->n_walk;
    return REWL_OK;
}

rewl_status rewl_window_bounds(const rewl_plan* P, int32_t prob, int32_t w, int32_t* e_lo, int32_t* e_hi) {
    if (!P || !e_lo || !e_hi) return fail(REWL_EINVAL, "null argument");
    if (prob < 0 || prob >= static_cast<int32_t>(P->pd.size())) return fail(REWL_EINVAL, "problem out of range");
    if (w < 0 || w >= P->pd[prob].nwin) return fail(REWL_EINVAL, "window out of range");
    const Rect& R = P->rect[prob][w];
    const bool m_split = P->split == REWL_SPLIT_MAGNETIZATION;
    *e_lo = m_split ? R.mlo : R.elo;
    *e_hi = m_split ? R.mhi : R.ehi;
    return REWL_OK;
}

rewl_status rewl_window_rect(const rewl_plan* P, int32_t prob, int32_t w, int32_t* e_lo, int32_t* e_hi,
                             int32_t* m_lo, int32_t* m_hi) {
    if (!P || !e_lo || !e_hi || !m_lo || !m_hi) return fail(REWL_EINVAL, "null argument");
    if (prob < 0 || prob >= static_cast<int32_t>(P->pd.size())) return fail(REWL_EINVAL, "problem out of range");
    if (w < 0 || w >= P->pd[prob].nwin) return fail(REWL_EINVAL, "window out of range");
    const Rect& R = P->rect[prob][w];
    *e_lo = R.elo;
    *e_hi = R.ehi;
    *m_lo = R.mlo;
    *m_hi = R.mhi;
    return REWL_OK;
}

rewl_status rewl_plan_windows(const rewl_plan* P, int32_t prob, int32_t* n_windows) {
    if (!P || !n_windows) return fail(REWL_EINVAL, "null argument");
    if (prob < 0 || prob >= static_cast<int32_t>(P->pd.size())) return fail(REWL_EINVAL, "problem out of range");
    *n_windows = P->pd[prob].nwin;
    return REWL_OK;
}

rewl_status rewl_plan_bind(rewl_plan* P, void* const* dev_ptrs, void* hip_stream) {
    if (!P || !dev_ptrs) return fail(REWL_EINVAL, "null argument");
    if (P->broken) return fail(REWL_ESTATE, "plan is in an error state");
    for (int i = 0; i < REWL_NBUF; ++i) {
        if (P->sizes[i] && !dev_ptrs[i]) return fail(REWL_EINVAL, "null device buffer");
        if (reinterpret_cast<uintptr_t>(dev_ptrs[i]) % 256 != 0) return fail(REWL_EINVAL, "buffers must be 256-byte aligned");
    }
    for (int i = 0; i < REWL_NBUF; ++i) P->buf[i] = dev_ptrs[i];
    P->stream = static_cast<hipStream_t>(hip_stream);
    if (P->graph) {
        (void)hipGraphExecDestroy(P->graph);
        P->graph = nullptr;
        P->graph_g = 0;
    }
    P->S = make_state(P);
    HIPCHK(P, sweep_setup(), "kernel attributes");
    {
        int dev = 0, ncu = 0;
        HIPCHK(P, hipGetDevice(&dev), "device query");
        HIPCHK(P, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "device query");
        if (ncu > 0) P->n_cu = ncu;
    }
    char* st = static_cast<char*>(P->buf[REWL_BUF_STATE]);
    HIPCHK(P, hipMemcpyAsync(st + P->off_wd, P->wd.data(), P->wd.size() * sizeof(WDesc), hipMemcpyHostToDevice,
                             P->stream), "descriptor upload");
    HIPCHK(P, hipMemcpyAsync(st + P->off_pd, P->pd.data(), P->pd.size() * sizeof(PDesc), hipMemcpyHostToDevice,
                             P->stream), "descriptor upload");
    if (!P->pairs.empty())
        HIPCHK(P, hipMemcpyAsync(st + P->off_pairs, P->pairs.data(), P->pairs.size() * sizeof(PairDesc),
                                 hipMemcpyHostToDevice, P->stream), "descriptor upload");
    HIPCHK(P, hipStreamSynchronize(P->stream), "descriptor upload sync");
    P->bound = true;
    P->initialised = false;
    return REWL_OK;
}

rewl_status rewl_init(rewl_plan* P) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    HIPCHK(P, launch_zero(P->buf[REWL_BUF_TABLES], P->sizes[REWL_BUF_TABLES], P->stream), "table clear");
    HIPCHK(P, launch_zero(static_cast<char*>(P->buf[REWL_BUF_STATE]) + P->off_cnt, 16, P->stream), "counter clear");
    HIPCHK(P, launch_init(P->S, P->stream), "init launch");
    const int64_t cap_launch = 1 << 20;
    const int64_t cap_total = 1ll << 40;
    int64_t spent = 0;
    for (;;) {
        HIPCHK(P, launch_zero(static_cast<char*>(P->buf[REWL_BUF_STATE]) + P->off_cnt, 16, P->stream), "counter clear");
        HIPCHK(P, launch_entry(P->S, cap_launch, P->stream), "entry launch");
        int32_t cnt[4];
        HIPCHK(P, hipMemcpyAsync(cnt, static_cast<char*>(P->buf[REWL_BUF_STATE]) + P->off_cnt, 16,
                                 hipMemcpyDeviceToHost, P->stream), "entry counter read");
        HIPCHK(P, hipStreamSynchronize(P->stream), "entry sync");
        spent += cap_launch;
        if (cnt[0] == 0) break;
        if (spent >= cap_total) return fail(REWL_ESTATE, "entry walk exceeded 2^40 trials");
    }
    P->initialised = true;
    if (P->tune.form == REWL_FORM_BATCHED) {
        // capture the interval graph now, so the first rewl_run does not pay for it
        if ((s = ensure_graph(P, graph_len(P))) != REWL_OK) return s;
    }
    return REWL_OK;
}

rewl_status rewl_sweep(rewl_plan* P, int64_t n) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (!P->initialised) return fail(REWL_ESTATE, "rewl_init has not run");
    if (n < 0) return fail(REWL_EINVAL, "negative trial count");
    // pieces of at most 2^30 trials, each followed by the stage-count audit
    for (int64_t done = 0; done < n;) {
        const int64_t m = std::min<int64_t>(n - done, 1ll << P->S.audit_shift);
        if (P->tune.form == REWL_FORM_PLAIN) {
            const int wg = wg_of(P);
            for (const PDesc& q : P->pd)
                for (int w = 0; w < q.nwin; ++w)
                    HIPCHK(P, launch_sweep(P->S, q.walker_off + static_cast<int64_t>(w) * q.W, q.W, m, q.L, wg, 0,
                                           P->tune.walkers_per_wave, P->split, P->layout, false, P->stream),
                           "plain sweep launch");
        } else if ((s = enqueue_sweep(P, m)) != REWL_OK) {
            return s;
        }
        HIPCHK(P, launch_flat(P->S, P->stream, 1), "audit launch");
        done += m;
    }
    return REWL_OK;
}

rewl_status rewl_reduce_lnf(rewl_plan* P) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (!P->initialised) return fail(REWL_ESTATE, "rewl_init has not run");
    return enqueue_boundary(P);
}

rewl_status rewl_exchange(rewl_plan* P) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (!P->initialised) return fail(REWL_ESTATE, "rewl_init has not run");
    return enqueue_exchange(P);
}

rewl_status rewl_run(rewl_plan* P, int64_t n) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (!P->initialised) return fail(REWL_ESTATE, "rewl_init has not run");
    if (n < 0) return fail(REWL_EINVAL, "negative interval count");
    if (P->tune.form == REWL_FORM_PLAIN) {
        for (int64_t i = 0; i < n; ++i)
            if ((s = run_interval_plain(P)) != REWL_OK) return s;
        return REWL_OK;
    }
    if (P->profile) {
        // eager launches with an event pair around every sweep kernel
        while (P->ev.size() < 2 * static_cast<size_t>(n)) {
            hipEvent_t e;
            HIPCHK(P, hipEventCreate(&e), "event create");
            P->ev.push_back(e);
        }
        P->ev_used = 0;
        for (int64_t i = 0; i < n; ++i) {
            if ((s = enqueue_interval_batched(P, static_cast<int>(i))) != REWL_OK) return s;
            P->ev_used = static_cast<int>(i + 1);
        }
        return REWL_OK;
    }
    const int G = graph_len(P);
    int64_t i = 0;
    if (n >= G) {
        if ((s = ensure_graph(P, G)) != REWL_OK) return s;
        for (; i + G <= n; i += G) HIPCHK(P, hipGraphLaunch(P->graph, P->stream), "graph launch");
    }
    for (; i < n; ++i)
        if ((s = enqueue_interval_batched(P)) != REWL_OK) return s;
    return REWL_OK;
}

rewl_status rewl_query(rewl_plan* P, int32_t* stage_out, int32_t* done_out, int64_t* trials_out) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    const size_t np = P->pd.size();
    std::vector<int32_t> stage, done, cnt;
    std::vector<int64_t> t;
    if ((s = d2h(P, stage, P->off_stage, static_cast<size_t>(P->n_win))) || (s = d2h(P, done, P->off_done, np)) ||
        (s = d2h(P, t, P->off_t, P->n_walk)) || (s = d2h(P, cnt, P->off_cnt, 4)))
        return s;
    HIPCHK(P, hipStreamSynchronize(P->stream), "query sync");
    for (size_t p = 0; p < np; ++p) {
        const PDesc& q = P->pd[p];
        int lowest = stage[q.win_off];
        for (int w = 1; w < q.nwin; ++w) lowest = std::min(lowest, stage[q.win_off + w]);
        if (stage_out) stage_out[p] = lowest;
        if (done_out) done_out[p] = done[p];
        if (trials_out) trials_out[p] = t[P->pd[p].walker_off];
    }
    if (cnt[1] & ERR_OVERFLOW) return fail(REWL_EOVERFLOW, "ln g would exceed 2^62 units");
    if (cnt[1] & ERR_HWRAP)
        return fail(REWL_EOVERFLOW, "a bin reached the audit limit of visits in one stage: its stage count could wrap");
    if (cnt[1] & ERR_PACK)
        return fail(REWL_EOVERFLOW, "ln g reached 2^37 units, more than a packed table word holds");
    if (cnt[1] & ERR_LAYOUT) return fail(REWL_ESTATE, "an exchanged state lies outside a stored table band");
    return REWL_OK;
}

rewl_status rewl_query_windows(rewl_plan* P, int32_t prob, int32_t* stage_out, int32_t* done_out,
                               int64_t* trials_out) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (prob < 0 || prob >= static_cast<int32_t>(P->pd.size())) return fail(REWL_EINVAL, "problem out of range");
    const PDesc& q = P->pd[prob];
    std::vector<int32_t> stage, wdone;
    std::vector<int64_t> t;
    const size_t nwn = static_cast<size_t>(P->n_win);
    if ((s = d2h(P, stage, P->off_stage, nwn)) || (s = d2h(P, wdone, P->off_wdone, nwn)) ||
        (s = d2h(P, t, P->off_t, P->n_walk)))
        return s;
    HIPCHK(P, hipStreamSynchronize(P->stream), "query sync");
    for (int w = 0; w < q.nwin; ++w) {
        if (stage_out) stage_out[w] = stage[q.win_off + w];
        if (done_out) done_out[w] = wdone[q.win_off + w];
        if (trials_out) trials_out[w] = t[q.walker_off + w * q.W];
    }
    return REWL_OK;
}

rewl_status rewl_read_walker(rewl_plan* P, int32_t prob, int32_t w, int32_t a, int64_t* lng, uint64_t* H,
                             size_t cap_bins, int8_t* spins, int32_t* e, int32_t* m, int64_t* t) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (prob < 0 || prob >= static_cast<int32_t>(P->pd.size())) return fail(REWL_EINVAL, "problem out of range");
    const PDesc& q = P->pd[prob];
    if (w < 0 || w >= q.nwin || a < 0 || a >= q.W) return fail(REWL_EINVAL, "walker out of range");
    const int64_t g = q.walker_off + static_cast<int64_t>(w) * q.W + a;
    const WDesc& d = P->wd[g];
    const Rect& R = P->rect[prob][w];
    const int nE = R.ehi - R.elo + 1;  // rows of the dense output
    const int nM = R.mhi - R.mlo + 1;  // columns
    const size_t nb = static_cast<size_t>(nE) * nM;
    if ((lng || H) && cap_bins < nb) return fail(REWL_EINVAL, "cap_bins too small");
    std::vector<int64_t> tl;
    std::vector<uint32_t> ts;
    const bool packed = P->S.packed != 0;
    std::vector<uint32_t> words;
    std::vector<int32_t> ev, mv, stage;
    std::vector<int64_t> tv;
    if (lng || H) {
        tl.resize(d.nbins);
        HIPCHK(P, hipMemcpyAsync(tl.data(), P->S.lng + d.table_off, d.nbins * sizeof(int64_t),
                                 hipMemcpyDeviceToHost, P->stream), "table read");
        if (!packed) {
            ts.resize(d.nbins);
            HIPCHK(P, hipMemcpyAsync(ts.data(), P->S.hb + d.table_off, d.nbins * sizeof(uint32_t),
                                     hipMemcpyDeviceToHost, P->stream), "table read");
        }
    }
    const size_t nwords = static_cast<size_t>(q.L) * q.row_words;
    if (spins) {
        words.resize(nwords);
        HIPCHK(P, hipMemcpyAsync(words.data(), static_cast<uint32_t*>(P->buf[REWL_BUF_SPINS]) + d.spin_off,
                                 nwords * 4, hipMemcpyDeviceToHost, P->stream), "spin read");
    }
    if ((s = d2h(P, ev, P->off_e, P->n_walk)) || (s = d2h(P, mv, P->off_m, P->n_walk)) ||
        (s = d2h(P, tv, P->off_t, P->n_walk)) || (s = d2h(P, stage, P->off_stage, static_cast<size_t>(P->n_win))))
        return s;
    HIPCHK(P, hipStreamSynchronize(P->stream), "walker read sync");
    const int sh = q.K - stage[d.gwin];
    if (lng || H)
        for (int er = 0; er < nE; ++er)
            for (int mm = 0; mm < nM; ++mm) {
                const int64_t ti = table_index_or_none(d, R.elo + er, R.mlo + mm);
                const size_t oi = static_cast<size_t>(er) * nM + mm;
                if (lng) lng[oi] = ti < 0 ? 0 : packed ? packed_lng(tl[ti]) : tl[ti];
                if (H)
                    H[oi] = ti < 0     ? 0
                            : packed ? packed_visits(tl[ti], sh)
                                     : static_cast<uint32_t>(static_cast<uint32_t>(static_cast<uint64_t>(tl[ti]) >> sh) - ts[ti]);
            }
    if (spins)
        for (int r = 0; r < q.L; ++r)
            for (int c = 0; c < q.L; ++c)
                spins[r * q.L + c] = ((words[r * q.row_words + (c >> 5)] >> (c & 31)) & 1u) ? 1 : -1;
    if (e) *e = ev[g];
    if (m) *m = mv[g];
    if (t) *t = tv[g];
    return REWL_OK;
}

}  // extern "C"

extern "C" {

rewl_status rewl_lnz_forward(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                             const double* beta, const double* h, int64_t G, double* lnz, void* hip_stream) {
    if (!lng || !beta || !h || !lnz) return fail(REWL_EINVAL, "null pointer");
    if (N < 1 || nE < 1 || nM < 1 || e0 < 0 || m0 < 0 || e0 + nE > N + 1 || m0 + nM > N + 1 || G < 0)
        return fail(REWL_EINVAL, "bad reweighting geometry");
    hipError_t e = launch_lnz_forward(lng, N, e0, nE, m0, nM, beta, h, G, lnz, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("lnz forward: ") + hipGetErrorString(e));
    return REWL_OK;
}

rewl_status rewl_lnz_backward(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                              const double* beta, const double* h, int64_t G, const double* lnz,
                              const double* grad_out, double* grad_beta, double* grad_h, double* grad_lng,
                              double* mom, int32_t order, void* hip_stream) {
    if (!lng || !beta || !h || !lnz) return fail(REWL_EINVAL, "null pointer");
    if (N < 1 || nE < 1 || nM < 1 || e0 < 0 || m0 < 0 || e0 + nE > N + 1 || m0 + nM > N + 1 || G < 0)
        return fail(REWL_EINVAL, "bad reweighting geometry");
    if (order != 1 && order != 2) return fail(REWL_EINVAL, "order must be 1 or 2");
    if (order == 2 && !mom) return fail(REWL_EINVAL, "order 2 needs mom");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipError_t e;
    if (order == 1) {
        e = launch_lnz_moments(lng, N, e0, nE, m0, nM, beta, h, G, lnz, grad_out, mom, grad_beta, grad_h, st);
        if (e == hipSuccess && grad_lng)
            e = launch_lnz_grad_lng(lng, N, e0, nE, m0, nM, beta, h, G, lnz, grad_out, grad_lng, st);
    } else {
        e = launch_lnz_moments(lng, N, e0, nE, m0, nM, beta, h, G, lnz, nullptr, mom, nullptr, nullptr, st);
    }
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("lnz backward: ") + hipGetErrorString(e));
    return REWL_OK;
}

rewl_status rewl_lnz_backward2(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                               const double* beta, const double* h, int64_t G, const double* lnz,
                               const double* grad_out, const double* up_beta, const double* up_h, double* d_grad_out,
                               double* d_beta, double* d_h, void* hip_stream) {
    if (!lng || !beta || !h || !lnz || !d_grad_out || !d_beta || !d_h) return fail(REWL_EINVAL, "null pointer");
    if (N < 1 || nE < 1 || nM < 1 || e0 < 0 || m0 < 0 || e0 + nE > N + 1 || m0 + nM > N + 1 || G < 0)
        return fail(REWL_EINVAL, "bad reweighting geometry");
    hipError_t e = launch_lnz_second(lng, N, e0, nE, m0, nM, beta, h, G, lnz, grad_out, up_beta, up_h, d_grad_out,
                                     d_beta, d_h, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("lnz second-order backward: ") + hipGetErrorString(e));
    return REWL_OK;
}

}  // extern "C"

// Tensor-product grids beta_i x h_j (factorised through the M columns).
rewl_status rewl::lnz_grid_check(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                                 const double* beta, int64_t nB, const double* h, int64_t nH) {
    if (!lng || !beta || !h) return fail(REWL_EINVAL, "null pointer");
    if (N < 1 || nE < 1 || nM < 1 || e0 < 0 || m0 < 0 || e0 + nE > N + 1 || m0 + nM > N + 1)
        return fail(REWL_EINVAL, "bad reweighting geometry");
    if (nB < 0 || nH < 0 || nB > 65535 || nH > 256LL * 65535) return fail(REWL_EINVAL, "bad grid size");
    return REWL_OK;
}

rewl_status rewl::set_error(rewl_status st, const char* msg) { return fail(st, msg); }

extern "C" {

static rewl_status grid_check(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                              const double* beta, int64_t nB, const double* h, int64_t nH) {
    return lnz_grid_check(lng, N, e0, nE, m0, nM, beta, nB, h, nH);
}

static size_t grid_ws_bytes(int32_t nM, int64_t nB, int64_t nH) {
    return (4 * static_cast<size_t>(nB) * static_cast<size_t>(nM) + 2 * static_cast<size_t>(nB) * nH) *
           sizeof(double);
}

rewl_status rewl_lnz_grid_workspace_size(int32_t nM, int64_t nB, int64_t nH, size_t* bytes) {
    if (!bytes || nM < 1 || nB < 0 || nH < 0) return fail(REWL_EINVAL, "bad arguments");
    *bytes = grid_ws_bytes(nM, nB, nH);
    return REWL_OK;
}

rewl_status rewl_lnz_grid_forward(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                                  const double* beta, int64_t nB, const double* h, int64_t nH, void* workspace,
                                  size_t workspace_bytes, double* lnz, void* hip_stream) {
    rewl_status s = grid_check(lng, N, e0, nE, m0, nM, beta, nB, h, nH);
    if (s != REWL_OK) return s;
    if (!lnz || (!workspace && nB * nH > 0)) return fail(REWL_EINVAL, "null pointer");
    if (workspace_bytes < grid_ws_bytes(nM, nB, nH)) return fail(REWL_EINVAL, "workspace too small");
    hipError_t e = launch_lnz_grid_forward(lng, N, e0, nE, m0, nM, beta, nB, h, nH, static_cast<double*>(workspace),
                                           lnz, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("lnz grid forward: ") + hipGetErrorString(e));
    return REWL_OK;
}

rewl_status rewl_lnz_grid_backward(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                                   const double* beta, int64_t nB, const double* h, int64_t nH, const double* lnz,
                                   const double* grad_out, void* workspace, size_t workspace_bytes,
                                   double* grad_beta, double* grad_h, double* grad_lng, double* mom,
                                   void* hip_stream) {
    rewl_status s = grid_check(lng, N, e0, nE, m0, nM, beta, nB, h, nH);
    if (s != REWL_OK) return s;
    if (!lnz || (!workspace && nB * nH > 0)) return fail(REWL_EINVAL, "null pointer");
    if ((grad_beta == nullptr) != (grad_h == nullptr)) return fail(REWL_EINVAL, "grad_beta and grad_h go together");
    if (!grad_beta && !grad_lng && !mom) return fail(REWL_EINVAL, "nothing to compute");
    if (workspace_bytes < grid_ws_bytes(nM, nB, nH)) return fail(REWL_EINVAL, "workspace too small");
    const size_t cm = static_cast<size_t>(nB) * nM, ch = static_cast<size_t>(nB) * nH;
    double* w = static_cast<double*>(workspace);
    double *A = w, *u1 = w + cm, *u2 = w + 2 * cm, *cw = w + 3 * cm, *tb = w + 4 * cm, *th = tb + ch;
    hipError_t e = launch_lnz_grid_backward(lng, N, e0, nE, m0, nM, beta, nB, h, nH, lnz, grad_out, A, u1, u2, cw,
                                            grad_beta ? tb : nullptr, grad_beta ? th : nullptr, grad_beta, grad_h,
                                            grad_lng, mom, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("lnz grid backward: ") + hipGetErrorString(e));
    return REWL_OK;
}

rewl_status rewl_lnz_grid_backward2(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                                    const double* beta, int64_t nB, const double* h, int64_t nH, const double* lnz,
                                    const double* grad_out, const double* up_beta, const double* up_h,
                                    void* workspace, size_t workspace_bytes, double* d_grad_out, double* d_beta,
                                    double* d_h, void* hip_stream) {
    rewl_status s = grid_check(lng, N, e0, nE, m0, nM, beta, nB, h, nH);
    if (s != REWL_OK) return s;
    if (!lnz || !d_grad_out || !d_beta || !d_h || (!workspace && nB * nH > 0)) return fail(REWL_EINVAL, "null pointer");
    if (workspace_bytes < grid_ws_bytes(nM, nB, nH)) return fail(REWL_EINVAL, "workspace too small");
    const size_t cm = static_cast<size_t>(nB) * nM, ch = static_cast<size_t>(nB) * nH;
    double* w = static_cast<double*>(workspace);
    double *A = w, *u1 = w + cm, *u2 = w + 2 * cm, *tb = w + 4 * cm, *th = tb + ch;
    hipError_t e = launch_lnz_grid_second(lng, N, e0, nE, m0, nM, beta, nB, h, nH, lnz, grad_out, up_beta, up_h, A,
                                          u1, u2, tb, th, d_grad_out, d_beta, d_h,
                                          static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess)
        return fail(REWL_EDEVICE, std::string("lnz grid second-order backward: ") + hipGetErrorString(e));
    return REWL_OK;
}

}  // extern "C"

extern "C" rewl_status rewl_set_profile(rewl_plan* P, int32_t on) {
    if (!P) return fail(REWL_EINVAL, "null plan");
    if (on != 0 && on != 1) return fail(REWL_EINVAL, "on must be 0 or 1");
    if (on && P->tune.form != REWL_FORM_BATCHED) return fail(REWL_EINVAL, "profiling times the batched form");
    P->profile = on != 0;
    return REWL_OK;
}

extern "C" rewl_status rewl_sweep_times(rewl_plan* P, float* ms, int32_t cap, int32_t* count) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (!ms || !count || cap < 0) return fail(REWL_EINVAL, "null argument");
    if (!P->profile || P->ev_used == 0) return fail(REWL_ESTATE, "no profiled rewl_run yet");
    HIPCHK(P, hipStreamSynchronize(P->stream), "timing sync");
    for (int i = 0; i < P->ev_used && i < cap; ++i)
        HIPCHK(P, hipEventElapsedTime(&ms[i], P->ev[2 * i], P->ev[2 * i + 1]), "event time");
    *count = P->ev_used;
    return REWL_OK;
}

// Self-check of the sweep's acceptance filter (not declared in the public
// header): runs k_accept_check synchronously on the current device and
// returns the disagreement, exact-path and acceptance counts, plus the first
// n_samp pairs and decisions (host arrays, nullable when n_samp = 0).
// packed = 1 checks the form the sweep uses for packed table words (delta in
// units of 2^-(K + 26), K <= 24).
extern "C" rewl_status rewl_selfcheck_accept(int32_t K, uint64_t seed, int64_t n, double rel, int64_t* counts_out,
                                             int64_t* samp_delta, uint32_t* samp_u, int32_t* samp_dec,
                                             int32_t n_samp, int32_t packed) {
    if (K < 6 || K > (packed ? MAX_K_PACKED : 40) || n < 0 || n_samp < 0 || n_samp > n || !counts_out ||
        !(rel >= 0.0) || (packed != 0 && packed != 1))
        return fail(REWL_EINVAL, "bad self-check arguments");
    if (n_samp > 0 && (!samp_delta || !samp_u || !samp_dec)) return fail(REWL_EINVAL, "null sample arrays");
    void* d = nullptr;
    const size_t ns = static_cast<size_t>(n_samp);
    const size_t bytes = 32 + ns * (8 + 4 + 4);
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("self-check alloc: ") + hipGetErrorString(e));
    char* base = static_cast<char*>(d);
    auto* cnt = reinterpret_cast<unsigned long long*>(base);
    auto* sd = reinterpret_cast<int64_t*>(base + 32);
    auto* su = reinterpret_cast<uint32_t*>(base + 32 + ns * 8);
    auto* sdec = reinterpret_cast<int32_t*>(base + 32 + ns * 12);
    unsigned long long h[4] = {0, 0, 0, 0};
    e = hipMemcpy(cnt, h, 32, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_accept_check(K, seed, n, rel, cnt, sd, su, sdec, n_samp, packed, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(h, cnt, 32, hipMemcpyDeviceToHost);
    if (e == hipSuccess && ns) e = hipMemcpy(samp_delta, sd, ns * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && ns) e = hipMemcpy(samp_u, su, ns * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && ns) e = hipMemcpy(samp_dec, sdec, ns * 4, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("self-check: ") + hipGetErrorString(e));
    for (int i = 0; i < 3; ++i) counts_out[i] = static_cast<int64_t>(h[i]);
    return REWL_OK;
}

namespace {

// Geometry of the merge of one problem: the windows grouped into magnetization
// columns (see MergeGeo), and the workspace layout.
struct MergeLayout {
    size_t bytes = 0;
    MergeGeo G{};
    int max_nE = 0;
    int n_points = 0;
    std::vector<int32_t> ints;    // the int region (flags cleared on the device)
    std::vector<int64_t> avg_off;
    size_t ints_at = 0, offs_at = 0;  // byte offsets of the two regions
};

rewl_status merge_layout(const rewl_plan* P, int32_t prob, MergeLayout& out) {
    if (prob < 0 || prob >= static_cast<int32_t>(P->pd.size())) return fail(REWL_EINVAL, "problem out of range");
    const PDesc& q = P->pd[prob];
    const std::vector<Rect>& R = P->rect[prob];
    const int nwin = q.nwin, N = q.N;
    // columns: windows sharing one magnetization range, by m_lo, each by energy
    std::vector<int> order(nwin);
    for (int w = 0; w < nwin; ++w) order[w] = w;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (R[a].mlo != R[b].mlo) return R[a].mlo < R[b].mlo;
        if (R[a].mhi != R[b].mhi) return R[a].mhi < R[b].mhi;
        return R[a].elo < R[b].elo;
    });
    std::vector<int> col(nwin), first, count, cmlo, cmhi;
    for (int k = 0; k < nwin; ++k) {
        const Rect& r = R[order[k]];
        if (k == 0 || r.mlo != cmlo.back() || r.mhi != cmhi.back()) {
            first.push_back(k);
            count.push_back(0);
            cmlo.push_back(r.mlo);
            cmhi.push_back(r.mhi);
        }
        count.back() += 1;
        col[order[k]] = static_cast<int>(first.size()) - 1;
    }
    const int ncol = static_cast<int>(first.size());
    MergeGeo G{};
    G.prob = prob;
    G.nwin = nwin;
    G.ncol = ncol;
    G.W = q.W;
    G.N = N;
    G.K = q.K;
    int64_t o = 0;
    auto take = [&](int64_t n) {
        const int64_t at = o;
        o += n;
        return at;
    };
    G.off_shift = take(static_cast<int64_t>(nwin) * q.W);
    out.avg_off.assign(nwin, 0);
    int max_nE = 0;
    for (int w = 0; w < nwin; ++w) {
        const int64_t nE = R[w].ehi - R[w].elo + 1, nM = R[w].mhi - R[w].mlo + 1;
        max_nE = std::max<int>(max_nE, static_cast<int>(nE));
        out.avg_off[w] = take(2 * nE * nM);  // averages, then their standard errors
    }
    G.off_margA = take(static_cast<int64_t>(nwin) * (N + 1));
    G.off_runA = take(static_cast<int64_t>(ncol) * (N + 1));
    G.off_shiftA = take(nwin);
    G.off_stageA = take(nwin);
    G.off_margB = take(static_cast<int64_t>(ncol) * (N + 1));
    G.off_runB = take(N + 1);
    G.off_shiftB = take(ncol);
    G.off_cst = take(1);
    const size_t dbl_bytes = align_up(static_cast<size_t>(o) * sizeof(double), 256);
    const size_t off_bytes = align_up(static_cast<size_t>(nwin) * sizeof(int64_t), 256);
    int32_t io = 4;  // flags
    auto itake = [&](int32_t n) {
        const int32_t at = io;
        io += n;
        return at;
    };
    G.off_col = itake(nwin);
    G.off_ematA = itake(nwin);
    G.off_first = itake(ncol);
    G.off_count = itake(ncol);
    G.off_cmlo = itake(ncol);
    G.off_cmhi = itake(ncol);
    G.off_mmat = itake(ncol);
    G.off_members = itake(nwin);
    G.off_stage = itake(nwin);
    G.off_rect = itake(4 * nwin);
    out.ints.assign(io, 0);
    for (int w = 0; w < nwin; ++w) {
        out.ints[G.off_col + w] = col[w];
        out.ints[G.off_members + w] = order[w];
        out.ints[G.off_rect + 4 * w] = R[w].elo;
        out.ints[G.off_rect + 4 * w + 1] = R[w].ehi;
        out.ints[G.off_rect + 4 * w + 2] = R[w].mlo;
        out.ints[G.off_rect + 4 * w + 3] = R[w].mhi;
    }
    for (int c = 0; c < ncol; ++c) {
        out.ints[G.off_first + c] = first[c];
        out.ints[G.off_count + c] = count[c];
        out.ints[G.off_cmlo + c] = cmlo[c];
        out.ints[G.off_cmhi + c] = cmhi[c];
    }
    out.offs_at = dbl_bytes;
    out.ints_at = dbl_bytes + off_bytes;
    out.bytes = out.ints_at + align_up(static_cast<size_t>(io) * sizeof(int32_t), 256);
    out.G = G;
    out.max_nE = max_nE;
    out.n_points = P->split == REWL_SPLIT_BOTH ? nwin + ncol - 1 : nwin - 1;
    return REWL_OK;
}

}  // namespace

extern "C" rewl_status rewl_merge_workspace_size(const rewl_plan* P, int32_t prob, size_t* bytes) {
    if (!P || !bytes) return fail(REWL_EINVAL, "null argument");
    MergeLayout ml;
    rewl_status s = merge_layout(P, prob, ml);
    if (s != REWL_OK) return s;
    *bytes = ml.bytes;
    return REWL_OK;
}

extern "C" rewl_status rewl_merge_points(const rewl_plan* P, int32_t prob, int32_t* n_points) {
    if (!P || !n_points) return fail(REWL_EINVAL, "null argument");
    MergeLayout ml;
    rewl_status s = merge_layout(P, prob, ml);
    if (s != REWL_OK) return s;
    *n_points = ml.n_points;
    return REWL_OK;
}

extern "C" rewl_status rewl_merge_lng(rewl_plan* P, int32_t prob, int32_t norm, void* workspace, size_t ws_bytes,
                                      double* lng_out, double* lnge_out, int32_t* e_mat_out, double* lng_err_out) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (!P->initialised) return fail(REWL_ESTATE, "rewl_init has not run");
    if (norm != 0 && norm != 1) return fail(REWL_EINVAL, "norm must be 0 (ground state) or 1 (sum)");
    if (!workspace || !lng_out || !lnge_out) return fail(REWL_EINVAL, "null device pointer");
    MergeLayout ml;
    if ((s = merge_layout(P, prob, ml)) != REWL_OK) return s;
    if (ws_bytes < ml.bytes) return fail(REWL_EINVAL, "workspace too small");
    char* base = static_cast<char*>(workspace);
    ml.G.ws = reinterpret_cast<double*>(base);
    ml.G.avg_off = reinterpret_cast<int64_t*>(base + ml.offs_at);
    ml.G.iws = reinterpret_cast<int32_t*>(base + ml.ints_at);
    HIPCHK(P, hipMemcpyAsync(ml.G.avg_off, ml.avg_off.data(), ml.avg_off.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, P->stream), "merge geometry upload");
    HIPCHK(P, hipMemcpyAsync(ml.G.iws, ml.ints.data(), ml.ints.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                             P->stream), "merge geometry upload");
    HIPCHK(P, launch_merge(P->S, ml.G, ml.max_nE, norm, lng_out, lnge_out, lng_err_out, P->stream), "merge launch");
    if (e_mat_out && ml.n_points > 0)
        HIPCHK(P, launch_merge_points(ml.G, P->split, e_mat_out, P->stream), "merge points launch");
    int32_t flags[4];
    HIPCHK(P, hipMemcpyAsync(flags, ml.G.iws, 16, hipMemcpyDeviceToHost, P->stream), "merge flag read");
    HIPCHK(P, hipStreamSynchronize(P->stream), "merge sync");
    if (flags[0] == 1) return fail(REWL_ESTATE, "the walkers of a window share no visited bin");
    if (flags[0] == 2) return fail(REWL_ESTATE, "no matching point in the overlap of two windows");
    return REWL_OK;
}

extern "C" rewl_status rewl_set_tuning(rewl_plan* P, const rewl_tuning* tuning) {
    if (!P || !tuning) return fail(REWL_EINVAL, "null argument");
    if (P->broken) return fail(REWL_ESTATE, "plan is in an error state");
    rewl_status s = validate_tuning(*tuning);
    if (s != REWL_OK) return s;
    if (tuning->form != P->tune.form) return fail(REWL_EINVAL, "the form of a plan cannot change");
    if (tuning->table_layout != P->tune.table_layout) return fail(REWL_EINVAL, "the table layout of a plan cannot change");
    if (tuning->audit_shift != P->tune.audit_shift) return fail(REWL_EINVAL, "the audit shift of a plan cannot change");
    P->tune = *tuning;
    P->profile = tuning->profile != 0;
    if (P->graph) {
        (void)hipGraphExecDestroy(P->graph);
        P->graph = nullptr;
        P->graph_g = 0;
    }
    return REWL_OK;
}

namespace {
constexpr uint64_t SAVE_MAGIC = 0x3430574C57455232ull;  // "2REWLW04": 32-bit stage base, audit epochs
struct SaveHeader {
    uint64_t magic;
    uint64_t n_problems;
    uint64_t sizes[REWL_NBUF];
};
}  // namespace

extern "C" rewl_status rewl_save_size(const rewl_plan* P, size_t* bytes) {
    if (!P || !bytes) return fail(REWL_EINVAL, "null argument");
    size_t n = sizeof(SaveHeader) + P->probs.size() * sizeof(rewl_problem);
    for (int i = 0; i < REWL_NBUF; ++i) n += P->sizes[i];
    *bytes = n;
    return REWL_OK;
}

extern "C" rewl_status rewl_save(rewl_plan* P, void* blob, size_t cap, size_t* used) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (!P->initialised) return fail(REWL_ESTATE, "rewl_init has not run");
    size_t need = 0;
    rewl_save_size(P, &need);
    if (!blob || cap < need) return fail(REWL_EINVAL, "blob too small (see rewl_save_size)");
    char* out = static_cast<char*>(blob);
    SaveHeader h{SAVE_MAGIC, P->probs.size(), {P->sizes[0], P->sizes[1], P->sizes[2]}};
    std::memcpy(out, &h, sizeof h);
    size_t o = sizeof h;
    std::memcpy(out + o, P->probs.data(), P->probs.size() * sizeof(rewl_problem));
    o += P->probs.size() * sizeof(rewl_problem);
    for (int i = 0; i < REWL_NBUF; ++i) {
        HIPCHK(P, hipMemcpyAsync(out + o, P->buf[i], P->sizes[i], hipMemcpyDeviceToHost, P->stream), "save copy");
        o += P->sizes[i];
    }
    HIPCHK(P, hipStreamSynchronize(P->stream), "save sync");
    if (used) *used = o;
    return REWL_OK;
}

extern "C" rewl_status rewl_load(rewl_plan* P, const void* blob, size_t size) {
    rewl_status s = usable(P);
    if (s != REWL_OK) return s;
    if (!blob || size < sizeof(SaveHeader)) return fail(REWL_EINVAL, "blob truncated");
    const char* in = static_cast<const char*>(blob);
    SaveHeader h;
    std::memcpy(&h, in, sizeof h);
    if (h.magic != SAVE_MAGIC) return fail(REWL_EINVAL, "not a saved plan (magic)");
    if (h.n_problems != P->probs.size()) return fail(REWL_EINVAL, "saved plan has other problems");
    size_t need = 0;
    rewl_save_size(P, &need);
    if (size < need) return fail(REWL_EINVAL, "blob truncated");
    for (int i = 0; i < REWL_NBUF; ++i)
        if (h.sizes[i] != P->sizes[i]) return fail(REWL_EINVAL, "saved plan has other buffer sizes");
    if (std::memcmp(in + sizeof h, P->probs.data(), P->probs.size() * sizeof(rewl_problem)) != 0)
        return fail(REWL_EINVAL, "saved plan has other problems");
    size_t o = sizeof h + P->probs.size() * sizeof(rewl_problem);
    for (int i = 0; i < REWL_NBUF; ++i) {
        HIPCHK(P, hipMemcpyAsync(P->buf[i], in + o, P->sizes[i], hipMemcpyHostToDevice, P->stream), "load copy");
        o += P->sizes[i];
    }
    HIPCHK(P, hipStreamSynchronize(P->stream), "load sync");
    P->initialised = true;
    if (P->tune.form == REWL_FORM_BATCHED) {
        if ((s = ensure_graph(P, graph_len(P))) != REWL_OK) return s;
    }
    return REWL_OK;
}
