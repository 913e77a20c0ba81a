// rewl_internal.h -- device data layout shared by the host plan (rewl_host.cpp)
// and the kernels (rewl_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl {

// Window tables.  Each walker owns two tables over its window's rectangle of
// (e, m) bins: rows e in [lo, hi] and all m in [0, N] when the windows split
// the energy, all rows e and columns m in [lo, hi] when they split the
// magnetization, both ranges for windows in both coordinates.  The table row is
// e - e0, the column m - m0 (e0, m0 the rectangle's corner).  The first holds
// ln g as int64 in units of 2^-K (> 0 marks a bin the walker has visited; ln g
// only grows).  The second, the stage base, holds uint32 (ln g >> (K - s))
// modulo 2^32 as it was when the current stage s began.  Every visit in stage
// s adds 2^(K-s), and ln g keeps its residue modulo 2^(K-s) through the stage,
// so the stage's visit count is H = (ln g >> (K - s)) - base, exact modulo
// 2^32: a trial touches only ln g, and resetting H at a stage change is one
// pass over the table.  H < 2^32 is guarded by an audit (k_flat): at the first
// check after a walker's stage trial count passes a multiple of 2^a (a =
// audit_shift <= 30) every bin must show H < 2^(a+1), else the run stops with
// an overflow error.  Checks come at least every 2^a trials (the interval X <=
// 2^a, and rewl_sweep pieces), so two audits lie less than 2^(a+1) trials
// apart, no bin exceeds 2^(a+1) + 2^(a+1) <= 2^32 visits between them, and no
// count can wrap unnoticed.
//
// Packed layouts keep both in one 64-bit word per bin: ln g in bits 63..26
// (PACK_SHIFT) and a 26-bit stage base, (ln g >> (K - s)) mod 2^26, in bits
// 25..0; 8 bytes per bin instead of 12.  Increments of ln g are multiples of
// 2^26 in the word and leave the base alone.  The word stays a non-negative
// int64 while ln g < 2^37 units; the sweep checks that after every increment
// and stops the run otherwise, so differences of words never overflow.  The
// audit period is at most 2^24 trials there (limit 2^25 visits, and counts
// below 2^26 between audits), and K is at most 24, so 2^37 units are at least
// 8192 in ln g.
//
// Both tables are stored in tiles of 4 energy rows x 4 magnetization columns
// (16 bins; 128 bytes of ln g, one cache line), tiles row-major: a walker's
// trial bins (e-2..e+2, m-1 / m+1) fall into about two lines instead of five.
//
// Band layout (energy windows): a state in energy bin e has at least e/2
// minority spins (each unsatisfied bond touches a minority spin, which has four
// bonds), so its magnetization bin lies in [ceil(e/2), N - ceil(e/2)].  Tile row
// tr (energies e0 + 4 tr .. e0 + 4 tr + 3) keeps only the tile columns from
// band_c0 = ceil((e0 + 4 tr)/2) / 4 on, ntm of them, ntm being the widest row
// of the window.  With windows in magnetization the band layout keeps the
// energy rows 0 .. 2 k_max only (k_max the largest minority count of the
// window's m), which needs no change of addressing.
constexpr int TILE_E = 4, TILE_M = 4, TILE_BINS = TILE_E * TILE_M;
enum : int32_t { LAYOUT_DENSE = 0, LAYOUT_BAND = 1, LAYOUT_PACKED = 2 };  // band and packed are bits

constexpr int PACK_SHIFT = 26;
constexpr int64_t PACK_MASK = (static_cast<int64_t>(1) << PACK_SHIFT) - 1;
constexpr int MAX_K_PACKED = 24;

// ln g of a packed word (units 2^-K).
__host__ __device__ inline int64_t packed_lng(int64_t w) {
    return static_cast<int64_t>(static_cast<uint64_t>(w) >> PACK_SHIFT);
}

// Visits in the current stage of a packed word, with sh = K - s.
__host__ __device__ inline uint32_t packed_visits(int64_t w, int sh) {
    return static_cast<uint32_t>((static_cast<uint64_t>(w) >> (PACK_SHIFT + sh)) - static_cast<uint64_t>(w)) &
           static_cast<uint32_t>(PACK_MASK);
}

__host__ __device__ inline uint32_t tile_index(int er, int m, uint32_t ntm) {
    return ((static_cast<uint32_t>(er >> 2) * ntm + static_cast<uint32_t>(m >> 2)) << 4) |
           (static_cast<uint32_t>(er & 3) << 2) | static_cast<uint32_t>(m & 3);
}

// First stored tile column of tile row tr of a band-layout energy window whose
// table starts at energy bin e0.
__host__ __device__ inline int band_c0(int e0, int tr) { return ((e0 + 4 * tr + 1) >> 1) >> 2; }

// Static description of one walker.
struct WDesc {
    uint64_t table_off;  // first bin of its tiled table (ln g; the stage base sits at the same
                         // offset of the stage-base table)
    uint32_t spin_off;   // first word of its L x row_words packed spins
    int32_t prob;        // problem index
    int32_t lo, hi;      // window in the split coordinate (e, or m for the magnetization
                         // split); the energy range for windows in both coordinates
    int32_t mlo, mhi;    // magnetization range of the window
    int32_t e0, m0;      // table origin: row e - e0, column m - m0
    int32_t win;         // window index within the problem
    int32_t gid;         // walker id within the problem: win * W + a
    uint32_t ntm;        // tiles per stored table row
    uint32_t nbins;      // bins of its tiled table = ceil(nrows / 4) * ntm * 16
    uint32_t nrows;      // energy rows stored (e - e0 < nrows)
    int32_t band;        // 1: band addressing of energy windows (band_c0)
    int32_t gwin;        // window index over all problems of the plan
    int32_t pad_;
};

// a * b for a, b < 2^24 (tile rows and columns never exceed 1025): one
// full-rate 24-bit multiply on the device.
__host__ __device__ inline uint32_t mul24(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return static_cast<uint32_t>(__umul24(a, b));
#else
    return a * b;
#endif
}

// Index of bin (e, m) in a walker's table, for a bin the table stores (any
// state of the window): BAND = 1 for the band addressing of energy windows.
template <int BAND>
__host__ __device__ inline uint32_t table_index(const WDesc& d, int e, int m) {
    const int er = e - d.e0, mc = m - d.m0;
    if (BAND) {
        const int tr = er >> 2;
        return ((mul24(static_cast<uint32_t>(tr), d.ntm) + static_cast<uint32_t>((mc >> 2) - band_c0(d.e0, tr)))
                << 4) |
               (static_cast<uint32_t>(er & 3) << 2) | static_cast<uint32_t>(mc & 3);
    }
    return tile_index(er, mc, d.ntm);
}

// Index of any bin (e, m) of the walker's rectangle, or -1 when the table does
// not store it (no state can be there, so its ln g is 0).
__host__ __device__ inline int64_t table_index_or_none(const WDesc& d, int e, int m) {
    const int er = e - d.e0, mc = m - d.m0;
    if (er < 0 || mc < 0 || er >= static_cast<int>(d.nrows)) return -1;
    const int tc = (mc >> 2) - (d.band ? band_c0(d.e0, er >> 2) : 0);
    if (tc < 0 || tc >= static_cast<int>(d.ntm)) return -1;
    return d.band ? static_cast<int64_t>(table_index<1>(d, e, m)) : static_cast<int64_t>(table_index<0>(d, e, m));
}

// Static description of one problem.
struct PDesc {
    int32_t L, N, K, nwin, W, flat_num, flat_den, row_words;
    int64_t X;
    uint64_t seed;
    int32_t walker_off;  // first global walker index
    int32_t init;
    int32_t win_off;     // first global window index
    int16_t sync;        // 0: all windows change stage together; 1: each window alone
    int16_t split;       // 0: energy windows; 1: magnetization windows; 2: both
};

// A pair of neighbouring windows (wa below wb along direction dir) of one
// problem that may exchange configurations.  along = index of wa along dir (the
// window index for one-coordinate splits, its grid row or column otherwise).
struct PairDesc {
    int32_t prob, wa, wb, dir, along;
};

// Device pointers into the three caller buffers.
struct DevState {
    const WDesc* wd;
    const PDesc* pd;
    const PairDesc* pairs;
    int64_t* lng;     // ln g tables
    uint32_t* hb;     // stage base: (ln g >> (K - s)) mod 2^32 at the start of stage s
    uint32_t* spins;
    // per walker
    int32_t* e;
    int32_t* m;
    int64_t* t;       // WL trials made
    int64_t* te;      // entry trials made
    uint32_t* nseen;  // bins with ln g > 0
    uint32_t* flag;   // flat in the current stage (latched)
    uint32_t* scan;   // chunk where the last flatness scan failed (a hint)
    uint32_t* aud;    // (stage trials) >> audit_shift when its table was last audited
    // per window (index gwin)
    int32_t* stage;   // ln f = 2^-stage
    int32_t* wdone;   // the window has finished its last stage; its walkers stop
    int64_t* tstage;  // trial count of its walkers at the start of the stage
    int32_t* adv;     // the window ended a stage at the boundary just closed
    int64_t* lngb;    // upper bound of any ln g entry (units), for the int64 headroom guard
    int64_t* tseen;   // trial count at the last boundary
    // per problem
    int32_t* done;    // every window has finished
    int64_t* rnd;     // boundaries passed
    int64_t* xr;      // exchange round of the boundary just closed
    int32_t* xon;     // that boundary exchanges
    // misc
    int32_t* counters;  // [0] walkers outside their window (entry), [1] error bits
    int64_t n_walk;
    int32_t n_prob;
    int32_t n_pairs;
    int32_t n_win;      // windows over all problems
    int32_t audit_shift;  // stage-count audit period 2^audit_shift trials (<= H_AUDIT_SHIFT)
    int32_t packed;       // tables hold packed words (ln g and stage base in one int64)
};

// ln g (units 2^-K) of table entry i, in either table format.
__host__ __device__ inline int64_t lng_at(const DevState& S, uint64_t i) {
    return S.packed ? packed_lng(S.lng[i]) : S.lng[i];
}

enum : int32_t { ERR_OVERFLOW = 1, ERR_LAYOUT = 2, ERR_HWRAP = 4, ERR_PACK = 8 };

// Longest audit period of the stage visit counts, log2 of trials (see the
// table notes): 2^30 for the 32-bit stage base, 2^24 for the packed 26-bit
// one; a plan may audit more often (DevState::audit_shift).
constexpr int H_AUDIT_SHIFT = 30;
constexpr int H_AUDIT_SHIFT_PACKED = 24;

// Workspace of the merge of one problem.  The windows are joined in two
// steps: first along E within each magnetization column (the windows sharing
// one magnetization range, ordered by energy), then the columns along M.  An
// energy split has one column holding every window; a magnetization split one
// window per column.  Double offsets are from ws, int offsets from iws.
struct MergeGeo {
    int32_t prob, nwin, ncol, W, N, K;
    double* ws;
    int32_t* iws;
    int64_t* avg_off;     // per window: offset (doubles) of its averaged table (rows e - e_lo,
                          // columns m - m_lo), followed by the table's standard errors
    int64_t off_shift;    // nwin * W walker alignment constants
    int64_t off_margA;    // nwin * (N + 1): each window's marginal over M, as a function of e
    int64_t off_runA;     // ncol * (N + 1): running marginal of each column's join
    int64_t off_shiftA;   // nwin: additive constant of each window in its column
    int64_t off_stageA;   // nwin: the same constants in column-member order (join scratch)
    int64_t off_margB;    // ncol * (N + 1): each joined column's marginal over E, a function of m
    int64_t off_runB;     // N + 1: running marginal of the join along M
    int64_t off_shiftB;   // ncol: additive constant of each column
    int64_t off_cst;      // normalisation constant
    // int region: [0, 4) flags ([0] != 0: no common bin (1) or no matching point (2));
    // then per window: column, E_mat where it starts within its column (its e_lo for
    // the first); per column: first member (index into members), member count, m_lo,
    // m_hi, M_mat where it starts (its m_lo for the first); members: windows by column
    // then energy; join scratch (nwin); rectangles e_lo, e_hi, m_lo, m_hi per window
    int32_t off_col, off_ematA, off_first, off_count, off_cmlo, off_cmhi, off_mmat, off_members, off_stage,
        off_rect;
};

}  // namespace rewl

#include "rewl.h"

namespace rewl {

// Host helpers shared by the C-ABI sources (rewl_host.cpp): argument checks of
// the tensor-product reweighting, and recording an error message.
rewl_status lnz_grid_check(const double* lng, int32_t N, int32_t e0, int32_t nE, int32_t m0, int32_t nM,
                           const double* beta, int64_t nB, const double* h, int64_t nH);
rewl_status set_error(rewl_status st, const char* msg);

// Launchers (rewl_kernels.hip).  All enqueue on `st` and return the launch status.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_init(const DevState& S, hipStream_t st);
hipError_t launch_entry(const DevState& S, int64_t cap, hipStream_t st);
// ahead: the pipelined trial (the next trial's proposal and targets made under
// the current gather), for launches whose gathers often miss the L2.
hipError_t launch_sweep(const DevState& S, int64_t g_begin, int64_t g_count, int64_t n_trials,
                        int l_max, int wg, int max_grid, int wpw, int split, int layout, bool ahead, hipStream_t st);
hipError_t sweep_setup();
hipError_t launch_flat(const DevState& S, hipStream_t st, int audit_only = 0);
hipError_t launch_stage(const DevState& S, hipStream_t st);
hipError_t launch_average(const DevState& S, hipStream_t st);
hipError_t launch_snapshot(const DevState& S, hipStream_t st);
hipError_t launch_exchange(const DevState& S, hipStream_t st);
hipError_t launch_accept_check(int K, uint64_t seed, int64_t n, double rel, unsigned long long* counts, int64_t* sd,
                               uint32_t* su, int32_t* sdec, int n_samp, int packed, hipStream_t st);

hipError_t launch_merge(const DevState& S, const MergeGeo& G, int max_nE, int norm, double* lng_out,
                        double* lnge_out, double* err_out, hipStream_t st);
hipError_t launch_merge_points(const MergeGeo& G, int split, int32_t* out, hipStream_t st);

// Reweighting.
hipError_t launch_lnz_forward(const double* lng, int N, int e0, int nE, int m0, int nM,
                              const double* beta, const double* h, int64_t G, double* lnz,
                              hipStream_t st);
hipError_t launch_lnz_moments(const double* lng, int N, int e0, int nE, int m0, int nM,
                              const double* beta, const double* h, int64_t G, const double* lnz,
                              const double* gout, double* mom, double* gbeta, double* gh,
                              hipStream_t st);
hipError_t launch_lnz_second(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                             const double* h, int64_t G, const double* lnz, const double* gout, const double* up_b,
                             const double* up_h, double* d_go, double* d_b, double* d_h, hipStream_t st);
hipError_t launch_lnz_grid_second(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                                  int64_t nB, const double* h, int64_t nH, const double* lnz, const double* gout,
                                  const double* up_b, const double* up_h, double* A, double* u1, double* u2,
                                  double* tb, double* th, double* d_go, double* d_b, double* d_h, hipStream_t st);
hipError_t launch_lnz_grad_lng(const double* lng, int N, int e0, int nE, int m0, int nM,
                               const double* beta, const double* h, int64_t G, const double* lnz,
                               const double* grad_out, double* grad_lng, hipStream_t st);
hipError_t launch_lnz_grid_forward(const double* lng, int N, int e0, int nE, int m0, int nM,
                                   const double* beta, int64_t nB, const double* h, int64_t nH, double* A,
                                   double* lnz, hipStream_t st);
hipError_t launch_lnz_grid_backward(const double* lng, int N, int e0, int nE, int m0, int nM,
                                    const double* beta, int64_t nB, const double* h, int64_t nH,
                                    const double* lnz, const double* gout, double* A, double* u1, double* u2,
                                    double* cw, double* tb, double* th, double* gbeta, double* gh,
                                    double* glng, double* mom, hipStream_t st);

}  // namespace rewl
