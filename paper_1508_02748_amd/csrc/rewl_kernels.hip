// rewl_kernels.hip -- gfx950 kernels of two-dimensional replica-exchange
// Wang-Landau sampling of the periodic L x L Ising model (Valentim et al.,
// arXiv:1508.02748, Sec. 2).
//
// Layout (one lane = one walker; no checkerboard: each walker's chain of
// trials is sequential, and the wavefront's 64 lanes run 64 independent
// walkers):
//   * spins: L rows of L bits, bit-packed, one 32- or 64-bit word per row.
//     During a sweep they live in LDS as lds[row * WG + lane] so that any mix
//     of rows read by the 64 lanes hits 64 distinct consecutive words (no bank
//     conflicts); in HBM they are packed per walker (row_words words per row).
//   * ln g: one int64 table per walker (single owner, no atomics) over the
//     window rows e in [lo, hi] and all m in [0, N], in 4 x 4 tiles of
//     (e, m) bins, one 128-byte line per tile, so the bins a walker can reach
//     in the next few trials share a few lines.  H is not stored: a 32-bit
//     stage base, (ln g >> (K - s)) taken when the stage began, gives
//     H = (ln g >> (K - s)) - base.
//     The walker keeps the bin it occupies in registers and writes it back only
//     when it leaves, so a trial costs one 8-byte gather of the proposed bin
//     plus, on acceptance, one 8-byte store.
//   * random numbers: Philox4x32-10 addressed by (seed; trial block, walker,
//     stream tag); one block serves two consecutive trials, and the next
//     block's rounds run while each trial waits for its gather.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rewl_internal.h"

namespace rewl {
namespace {

constexpr uint32_t TAG_WL = 0, TAG_INIT = 1, TAG_ENTRY = 2, TAG_XPERM = 3, TAG_XACC = 4;

struct Words4 {
    uint32_t x, y, z, w;
};

// Three-input xor in one gfx950 instruction (v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64 multiplies mixing the counter with a Weyl-incremented key.
__device__ __forceinline__ Words4 philox4x32_10(uint64_t key, uint32_t c0, uint32_t c1,
                                                uint32_t c2, uint32_t c3) {
    uint32_t k0 = static_cast<uint32_t>(key);
    uint32_t k1 = static_cast<uint32_t>(key >> 32);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t a_lo = 0xD2511F53u * c0;
        const uint32_t a_hi = __umulhi(0xD2511F53u, c0);
        const uint32_t b_lo = 0xCD9E8D57u * c2;
        const uint32_t b_hi = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = xor3(b_hi, c1, k0);
        const uint32_t n2 = xor3(a_hi, c3, k1);
        c0 = n0;
        c1 = b_lo;
        c2 = n2;
        c3 = a_lo;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// exp(x) for -23 < x <= 0, as a fixed sequence of correctly rounded IEEE
// operations: x = k ln2 + r (k nearest to x / ln2, ln2 split into a 32-bit
// head and a tail so k * head is exact), exp(r) by its degree-13 Taylor
// polynomial in Horner form with fused multiply-adds, then scaling by 2^k.
__device__ __forceinline__ double exp_neg(double x) {
    const double log2e = 1.4426950408889634;                  // RN(1 / ln 2)
    const double ln2_head = 2977044471.0 / 4294967296.0;      // floor(ln 2 * 2^32) / 2^32
    const double ln2_tail = 1.9082149292705877e-10;           // RN(ln 2 - head)
    const double k = floor(__dadd_rn(__dmul_rn(x, log2e), 0.5));
    double r = __fma_rn(-k, ln2_head, x);
    r = __fma_rn(-k, ln2_tail, r);
    double p = 1.0 / 6227020800.0;                            // 1/13!
    p = __fma_rn(p, r, 1.0 / 479001600.0);
    p = __fma_rn(p, r, 1.0 / 39916800.0);
    p = __fma_rn(p, r, 1.0 / 3628800.0);
    p = __fma_rn(p, r, 1.0 / 362880.0);
    p = __fma_rn(p, r, 1.0 / 40320.0);
    p = __fma_rn(p, r, 1.0 / 5040.0);
    p = __fma_rn(p, r, 1.0 / 720.0);
    p = __fma_rn(p, r, 1.0 / 120.0);
    p = __fma_rn(p, r, 1.0 / 24.0);
    p = __fma_rn(p, r, 1.0 / 6.0);
    p = __fma_rn(p, r, 0.5);
    p = __fma_rn(p, r, 1.0);
    p = __fma_rn(p, r, 1.0);
    return ldexp(p, static_cast<int>(k));
}

// Acceptance with probability min[1, exp(delta 2^-K)] (Eq. 1 and Eq. 2 with
// ln g in fixed point): u = (w + 1/2) 2^-32 >= 2^-33 > e^-23, so a ratio
// below e^-23 is always a rejection.
__device__ __forceinline__ bool accept_move(int64_t delta, uint32_t u_word, int K) {
    if (delta >= 0) return true;
    if (delta <= -(static_cast<int64_t>(23) << K)) return false;
    const double x = ldexp(static_cast<double>(delta), -K);
    const double u = __dmul_rn(__dadd_rn(static_cast<double>(u_word), 0.5), 1.0 / 4294967296.0);
    return u < exp_neg(x);
}

__device__ __forceinline__ uint32_t gbit(const uint32_t* sp, int rw, int r, int c) {
    return (sp[r * rw + (c >> 5)] >> (c & 31)) & 1u;
}

__device__ __forceinline__ void gflip(uint32_t* sp, int rw, int r, int c) {
    sp[r * rw + (c >> 5)] ^= 1u << (c & 31);
}

// (row, column) of the site floor(w N / 2^32), N = L*L, without a division:
// w L = r 2^32 + q  gives  w N / 2^32 = r L + q L / 2^32.
__device__ __forceinline__ void site_rc(uint32_t w, int L, int& r, int& c) {
    const uint64_t x = static_cast<uint64_t>(w) * static_cast<uint32_t>(L);
    r = static_cast<int>(x >> 32);
    c = static_cast<int>((static_cast<uint64_t>(static_cast<uint32_t>(x)) * static_cast<uint32_t>(L)) >> 32);
}

// ------------------------------------------------------------------ zero fill
__global__ void k_zero(uint4* p, size_t n16) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

// ------------------------------------------------------------------ init
// Initial configuration: site 128q + 32j + k takes bit k of word j of the
// INIT block q of the walker (1 = up), or all up; then E, M and a clean state.
__global__ void k_init(DevState S) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= S.n_walk) return;
    const WDesc d = S.wd[g];
    const PDesc P = S.pd[d.prob];
    const int L = P.L, N = P.N, rw = P.row_words;
    uint32_t* sp = S.spins + d.spin_off;
    for (int i = 0; i < L * rw; ++i) sp[i] = 0;
    if (P.init == 1) {
        for (int r = 0; r < L; ++r)
            for (int c = 0; c < L; ++c) sp[r * rw + (c >> 5)] |= 1u << (c & 31);
    } else {
        for (int q = 0; 128 * q < N; ++q) {
            const Words4 b = philox4x32_10(P.seed, static_cast<uint32_t>(q), 0u,
                                           static_cast<uint32_t>(d.gid), TAG_INIT << 24);
            const uint32_t ws[4] = {b.x, b.y, b.z, b.w};
            for (int j = 0; j < 4; ++j)
                for (int k = 0; k < 32; ++k) {
                    const int site = 128 * q + 32 * j + k;
                    if (site < N && ((ws[j] >> k) & 1u)) {
                        const int r = site / L, c = site % L;
                        sp[r * rw + (c >> 5)] |= 1u << (c & 31);
                    }
                }
        }
    }
    int E = 0, M = 0;
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) {
            const int s0 = 2 * static_cast<int>(gbit(sp, rw, r, c)) - 1;
            const int sr = 2 * static_cast<int>(gbit(sp, rw, r, c + 1 == L ? 0 : c + 1)) - 1;
            const int sd = 2 * static_cast<int>(gbit(sp, rw, r + 1 == L ? 0 : r + 1, c)) - 1;
            E -= s0 * (sr + sd);
            M += s0;
        }
    S.e[g] = (E + 2 * N) / 4;
    S.m[g] = (M + N) / 2;
    S.t[g] = 0;
    S.te[g] = 0;
    S.nseen[g] = 0;
    S.flag[g] = 0;
    S.scan[g] = 0;
    S.aud[g] = 0;
    if (d.gid % P.W == 0) {  // first walker of its window
        const int wi = d.gwin;
        S.stage[wi] = 0;
        S.wdone[wi] = 0;
        S.tstage[wi] = 0;
        S.adv[wi] = 0;
        S.lngb[wi] = 0;
        S.tseen[wi] = 0;
    }
    if (d.gid == 0) {
        const int p = d.prob;
        S.done[p] = 0;
        S.rnd[p] = 0;
        S.xr[p] = 0;
        S.xon[p] = 0;
    }
}

// ------------------------------------------------------------------ entry
// Walk each walker into its energy window: Metropolis at unit temperature on
// the distance d (bins) to the window; a flip that does not increase d is
// taken, one that increases it by k bins with probability exp(-4k).
__device__ __forceinline__ int win_dist(int e, int lo, int hi) {
    return e < lo ? lo - e : (e > hi ? e - hi : 0);
}

// Distance in bins from (e, m) to the window: in the split coordinate, or the
// sum of both coordinates' distances for windows in both.
__device__ __forceinline__ int window_distance(int split, const WDesc& d, int e, int m) {
    if (split == 0) return win_dist(e, d.lo, d.hi);
    if (split == 1) return win_dist(m, d.lo, d.hi);
    return win_dist(e, d.lo, d.hi) + win_dist(m, d.mlo, d.mhi);
}

__device__ __forceinline__ bool in_window(int split, const WDesc& d, int e, int m) {
    return window_distance(split, d, e, m) == 0;
}

__global__ void k_entry(DevState S, int64_t cap) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= S.n_walk) return;
    const WDesc d = S.wd[g];
    const PDesc P = S.pd[d.prob];
    int e = S.e[g], m = S.m[g];
    int dist = window_distance(P.split, d, e, m);
    if (dist == 0) return;
    const int L = P.L, rw = P.row_words, K = P.K;
    uint32_t* sp = S.spins + d.spin_off;
    int64_t te = S.te[g];
    for (int64_t i = 0; i < cap && dist > 0; ++i) {
        const uint64_t blk = static_cast<uint64_t>(te) >> 1;
        const Words4 b = philox4x32_10(P.seed, static_cast<uint32_t>(blk), static_cast<uint32_t>(blk >> 32),
                                       static_cast<uint32_t>(d.gid), TAG_ENTRY << 24);
        const uint32_t sw = (te & 1) ? b.z : b.x;
        const uint32_t uw = (te & 1) ? b.w : b.y;
        int r, c;
        site_rc(sw, L, r, c);
        const uint32_t bc = gbit(sp, rw, r, c);
        const uint32_t k = (gbit(sp, rw, r, c == 0 ? L - 1 : c - 1) ^ bc) +
                           (gbit(sp, rw, r, c == L - 1 ? 0 : c + 1) ^ bc) +
                           (gbit(sp, rw, r == 0 ? L - 1 : r - 1, c) ^ bc) +
                           (gbit(sp, rw, r == L - 1 ? 0 : r + 1, c) ^ bc);
        const int e2 = e + 2 - static_cast<int>(k);
        const int m2 = m + 1 - 2 * static_cast<int>(bc);
        const int dist2 = window_distance(P.split, d, e2, m2);
        const bool acc = dist2 <= dist ||
                         accept_move(-static_cast<int64_t>(4 * (dist2 - dist)) * (static_cast<int64_t>(1) << K),
                                     uw, K);
        if (acc) {
            gflip(sp, rw, r, c);
            e = e2;
            m = m2;
            dist = dist2;
        }
        ++te;
    }
    S.e[g] = e;
    S.m[g] = m;
    S.te[g] = te;
    if (dist > 0) atomicAdd(&S.counters[0], 1);
}

// ------------------------------------------------------------------ sweep
// Acceptance decision identical to accept_move, reached faster: a single
// precision estimate a of exp(x) (hardware exp2, relative error below 1e-5
// for -23 < x < 0 including the roundings of x to float and of the uniform
// below) decides unless u lies within about 1e-4 relative of a;
// only then is the double-precision exp_neg evaluated, with u = (w + 1/2)
// 2^-32 formed exactly in double.  Every path gives u < exp_neg(x) exactly.
// The float uniform uf = fl(fl(w) 2^-32 + 2^-33) (relative error below
// 2^-23) and its two scaled copies, uf / 0.9999 and uf / 1.0001 (one more
// rounding each), are formed before the gathered ln g arrives, so that only
// the exponential and two compares follow it; the filter has no branches:
// only the rare near-tie branches.
struct Uniform {
    float acc_below;  // accept when a exceeds it: uf / 0.9999
    float rej_above;  // reject when a is below it: uf / 1.0001
};

__device__ __forceinline__ Uniform uniform_f(uint32_t w) {
    const float uf = __fmaf_rn(static_cast<float>(w), 0x1p-32f, 0x1p-33f);
    return {uf * 1.00010001f, uf * 0.99990001f};
}

//
// LOW0: delta has its low 26 bits clear (packed table words, K >= 26).  Its
// float value then comes from its two 32-bit halves with no double-precision
// step: the low half has at most six significant bits and converts exactly,
// the high half and the fused multiply-add round once each; the exact double
// x is formed only on the near-tie path.
//
// No range test: for x <= -23 the roundings of x move the estimate by less
// than 1e-4 relative (x log2(e) > -150 before it flushes to zero), so it
// stays below 1.03e-10, under the smallest rej_above, 0.9999 * 2^-33 =
// 1.16e-10, and the trial is rejected; the exact path is reached only with
// a >= rej_above, that is x > -22.9, inside the range of exp_neg.
template <bool LOW0 = false>
__device__ __forceinline__ bool accept_pre(int64_t delta, uint32_t w, Uniform uf, int K, bool& exact_path) {
    float x2;  // x log2(e)
    if constexpr (LOW0) {
        const float dh = static_cast<float>(static_cast<int32_t>(delta >> 32));
        const float dl = static_cast<float>(static_cast<uint32_t>(delta));
        x2 = __fmaf_rn(dh, 0x1p32f, dl) * ldexpf(1.44269504f, -K);
    } else {
        x2 = static_cast<float>(ldexp(static_cast<double>(delta), -K)) * 1.44269504f;
    }
    const float a = __builtin_amdgcn_exp2f(x2);
    bool acc = delta >= 0 || uf.acc_below < a;
    const bool rej = uf.rej_above > a;
    exact_path = !acc && !rej;
    if (exact_path) {
        const double x = ldexp(static_cast<double>(delta), -K);
        const double u = __dmul_rn(__dadd_rn(static_cast<double>(w), 0.5), 1.0 / 4294967296.0);
        acc = u < exp_neg(x);
    }
    return acc;
}

template <bool LOW0 = false>
__device__ __forceinline__ bool accept_pre(int64_t delta, uint32_t w, Uniform uf, int K) {
    bool unused;
    return accept_pre<LOW0>(delta, w, uf, K, unused);
}

// First and second halves of a Philox4x32-10 evaluation, so that the next
// block's rounds can run while the current trials wait for their gathers.
struct PhiloxRun {
    uint32_t c0, c1, c2, c3, k0, k1;
};

__device__ __forceinline__ PhiloxRun philox_start(uint64_t key, uint64_t block, uint32_t walker) {
    return {static_cast<uint32_t>(block), static_cast<uint32_t>(block >> 32), walker, TAG_WL << 24,
            static_cast<uint32_t>(key), static_cast<uint32_t>(key >> 32)};
}

template <int NR>
__device__ __forceinline__ void philox_rounds(PhiloxRun& q) {
#pragma unroll
    for (int round = 0; round < NR; ++round) {
        // one 32x32 -> 64 multiply per product (low and high words together)
        const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * q.c0;
        const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * q.c2;
        const uint32_t n0 = xor3(static_cast<uint32_t>(pb >> 32), q.c1, q.k0);
        const uint32_t n2 = xor3(static_cast<uint32_t>(pa >> 32), q.c3, q.k1);
        q.c0 = n0;
        q.c1 = static_cast<uint32_t>(pb);
        q.c2 = n2;
        q.c3 = static_cast<uint32_t>(pa);
        q.k0 += 0x9E3779B9u;
        q.k1 += 0xBB67AE85u;
    }
}

struct NoRounds {};

// Pins the Philox state and the gathered ln g in registers at this point of
// the trial: the rounds computed before it overlap the table gather issued
// before them (instead of being moved after the acceptance branch), and the
// gather is waited for here on every path, not only inside the branch.
__device__ __forceinline__ void pin(PhiloxRun& q, int64_t& v, Uniform& f) {
    asm volatile("" : "+v"(q.c0), "+v"(q.c1), "+v"(q.c2), "+v"(q.c3), "+v"(v), "+v"(f.acc_below), "+v"(f.rej_above)
                 : : "memory");
}

__device__ __forceinline__ void pin(NoRounds&, int64_t& v, Uniform& f) {
    asm volatile("" : "+v"(v), "+v"(f.acc_below), "+v"(f.rej_above) : : "memory");
}

// Pins the next trial's targets (both table indices, and the accepted
// outcome's corrected spin and neighbour count) at the same point, so that
// its proposal (LDS reads, neighbour count) and both targets are made while
// the gather is in flight.
__device__ __forceinline__ void pin_next(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) {
    asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
}

// lo <= v <= hi (lo <= hi) as one unsigned compare.
__device__ __forceinline__ bool in_range(int v, int lo, int hi) {
    return static_cast<uint32_t>(v - lo) <= static_cast<uint32_t>(hi - lo);
}

// n_trials Wang-Landau trials (Eq. 1) for walker g (lane `lane` of a
// workgroup of WG lanes).  Its spins sit in LDS column `lane`; no lane touches
// another's data, so there are no barriers.  The bin the walker occupies is
// held in registers and written back when the walker leaves it.  SPLIT: the
// window coordinate (0 energy, 1 magnetization, 2 both); LAYOUT bit 0: band
// addressing of energy-window tables, bit 1: packed words (ln g in the high 38
// bits; ln g differences then come from the words with their base bits
// cleared, in units of 2^-(K + PACK_SHIFT)).  AHEAD: each trial makes the next
// trial's proposal and targets while its own gather is in flight (large
// batches, where gathers often miss the L2); otherwise each trial makes its
// own proposal first (small batches, whose gathers hit and leave nothing to
// hide that work behind).  Both give the same trials.
template <typename RowT, int SPLIT, int LAYOUT, bool AHEAD>
__device__ __forceinline__ void sweep_walker(const DevState& S, RowT* lds, int lane, int WG, int64_t g,
                                             int64_t n_trials) {
    constexpr int BAND = LAYOUT & 1;
    constexpr bool PACKED = (LAYOUT & 2) != 0;
    constexpr int PS = PACKED ? PACK_SHIFT : 0;
    constexpr int64_t HI = PACKED ? ~PACK_MASK : ~static_cast<int64_t>(0);
    const WDesc d = S.wd[g];
    const int p = d.prob;
    if (S.wdone[d.gwin]) return;  // the window (or the whole problem) has finished
    const PDesc P = S.pd[p];
    const int L = P.L, K = P.K, rw = P.row_words;
    const int s = S.stage[d.gwin];
    const int64_t inc = static_cast<int64_t>(1) << (K - s + PS);
    const int lo = d.lo, hi = d.hi, mlo = d.mlo, mhi = d.mhi;
    const uint64_t seed = P.seed;
    const uint32_t gid = static_cast<uint32_t>(d.gid);
    int64_t* tab = S.lng + d.table_off;
    const int wsh = __builtin_ctz(static_cast<unsigned>(WG));  // WG is 64, 128 or 256

    const uint32_t* gsp = S.spins + d.spin_off;
    for (int r = 0; r < L; ++r) {
        RowT v = static_cast<RowT>(gsp[r * rw]);
        if constexpr (sizeof(RowT) == 8) {
            if (rw == 2) v |= static_cast<RowT>(gsp[2 * r + 1]) << 32;
        }
        lds[r * WG + lane] = v;
    }

    int e = S.e[g], m = S.m[g];
    int64_t t = S.t[g];
    uint32_t nseen = S.nseen[g];
    uint32_t cur = table_index<BAND>(d, e, m);
    int64_t lng_cur = tab[cur];
    bool ovf = false;       // packed words: ln g reached 2^37 units
    uint32_t ovf_hi = 0;    // the same, as the OR of the words' high halves (sign bit)

    if constexpr (!AHEAD) {
    // One trial with the words (sw, uw) of its Philox block; `q` (a PhiloxRun)
    // advances the next block by five rounds while the gather is in flight.
    auto trial = [&](uint32_t sw, uint32_t uw, auto& q) {
        int r, c;
        site_rc(sw, L, r, c);
        const int ru = r == 0 ? L - 1 : r - 1;
        const int rd = r == L - 1 ? 0 : r + 1;
        const int cl = c == 0 ? L - 1 : c - 1;
        const int cr = c == L - 1 ? 0 : c + 1;
        const RowT row = lds[(r << wsh) + lane];
        const RowT rowu = lds[(ru << wsh) + lane];
        const RowT rowd = lds[(rd << wsh) + lane];
        const uint32_t bc = static_cast<uint32_t>(row >> c) & 1u;
        // number of the four neighbours anti-aligned with the site
        const uint32_t k = ((static_cast<uint32_t>(row >> cl) & 1u) ^ bc) +
                           ((static_cast<uint32_t>(row >> cr) & 1u) ^ bc) +
                           ((static_cast<uint32_t>(rowu >> c) & 1u) ^ bc) +
                           ((static_cast<uint32_t>(rowd >> c) & 1u) ^ bc);
        const int e2 = e + 2 - static_cast<int>(k);       // dE = 8 - 4k
        const int m2 = m + 1 - 2 * static_cast<int>(bc);  // dM = -2 s
        bool in;
        if constexpr (SPLIT == 0) in = e2 >= lo && e2 <= hi;
        else if constexpr (SPLIT == 1) in = m2 >= lo && m2 <= hi;
        else in = e2 >= lo && e2 <= hi && m2 >= mlo && m2 <= mhi;
        // gather unconditionally (the current bin when the proposal leaves the window)
        const uint32_t idx2 = in ? table_index<BAND>(d, e2, m2) : cur;
        int64_t lng2 = tab[idx2];
        Uniform uf = uniform_f(uw);
        const int64_t cur_hi = lng_cur & HI;
        if constexpr (!std::is_same_v<std::decay_t<decltype(q)>, NoRounds>) philox_rounds<5>(q);
        pin(q, lng2, uf);
        if (in && accept_pre<PACKED>(cur_hi - (lng2 & HI), uw, uf, K + PS)) {
            tab[cur] = lng_cur;
            lds[(r << wsh) + lane] = row ^ (static_cast<RowT>(1) << c);
            e = e2;
            m = m2;
            cur = idx2;
            lng_cur = lng2;
        }
        nseen += (lng_cur == 0) ? 1u : 0u;
        lng_cur += inc;
        if constexpr (PACKED) ovf = ovf || lng_cur < 0;
        ++t;
    };

    int64_t i = 0;
    Words4 blk = {0, 0, 0, 0};
    NoRounds none;
    if (n_trials > 0 && (t & 1)) {  // odd start: second half of the current block
        const uint64_t b = static_cast<uint64_t>(t) >> 1;
        blk = philox4x32_10(seed, static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), gid, TAG_WL << 24);
        trial(blk.z, blk.w, none);
        ++i;
    }
    if (i + 2 <= n_trials) {
        const uint64_t b = static_cast<uint64_t>(t) >> 1;
        blk = philox4x32_10(seed, static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), gid, TAG_WL << 24);
    }
    for (; i + 2 <= n_trials; i += 2) {
        // t is even here; blk is block t/2; the next block is computed in two
        // halves, each under the table gather of one of this pair of trials
        PhiloxRun q = philox_start(seed, (static_cast<uint64_t>(t) >> 1) + 1, gid);
        trial(blk.x, blk.y, q);
        trial(blk.z, blk.w, q);
        blk = {q.c0, q.c1, q.c2, q.c3};
    }
    if (i < n_trials) {  // one trial left, t even: first half of block t/2
        const uint64_t b = static_cast<uint64_t>(t) >> 1;
        blk = philox4x32_10(seed, static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), gid, TAG_WL << 24);
        trial(blk.x, blk.y, none);
    }
    } else {
    // The proposal of a trial: its site, the site's spin and the number of its
    // four neighbours anti-aligned with it, and the linear indices of the five
    // sites it reads (for the check after a flip).
    struct Prop {
        int r, c;
        uint32_t bc, k;
        int s0, s1, s2, s3, s4;
    };
    auto propose = [&](uint32_t sw) {
        Prop pr;
        site_rc(sw, L, pr.r, pr.c);
        const int r = pr.r, c = pr.c;
        const int ru = r == 0 ? L - 1 : r - 1;
        const int rd = r == L - 1 ? 0 : r + 1;
        const int cl = c == 0 ? L - 1 : c - 1;
        const int cr = c == L - 1 ? 0 : c + 1;
        const RowT row = lds[(r << wsh) + lane];
        const RowT rowu = lds[(ru << wsh) + lane];
        const RowT rowd = lds[(rd << wsh) + lane];
        pr.bc = static_cast<uint32_t>(row >> c) & 1u;
        pr.k = ((static_cast<uint32_t>(row >> cl) & 1u) ^ pr.bc) + ((static_cast<uint32_t>(row >> cr) & 1u) ^ pr.bc) +
               ((static_cast<uint32_t>(rowu >> c) & 1u) ^ pr.bc) + ((static_cast<uint32_t>(rowd >> c) & 1u) ^ pr.bc);
        pr.s0 = r * L + c;
        pr.s1 = r * L + cl;
        pr.s2 = r * L + cr;
        pr.s3 = ru * L + c;
        pr.s4 = rd * L + c;
        return pr;
    };

    // Where a proposal leads from the state (ee, mm) with table entry ci: the
    // trial bin, whether it lies in the window, and the table entry to gather
    // (the current one when the proposal leaves the window).
    struct Tgt {
        int e2, m2;
        uint32_t in;  // 0 or 1 (a word, not a lane mask, so that selecting it is one instruction)
        uint32_t idx;
    };
    auto target = [&](const Prop& pr, int ee, int mm, uint32_t ci) {
        Tgt tg;
        tg.e2 = ee + 2 - static_cast<int>(pr.k);       // dE = 8 - 4k
        tg.m2 = mm + 1 - 2 * static_cast<int>(pr.bc);  // dM = -2 s
        bool in;
        if constexpr (SPLIT == 0) in = in_range(tg.e2, lo, hi);
        else if constexpr (SPLIT == 1) in = in_range(tg.m2, lo, hi);
        else in = in_range(tg.e2, lo, hi) & in_range(tg.m2, mlo, mhi);
        tg.in = in ? 1u : 0u;
        // the index is formed for every lane and then selected (an arithmetic
        // result for a bin outside the window, never used as an address)
        const uint32_t ti = table_index<BAND>(d, tg.e2, tg.m2);
        tg.idx = in ? ti : ci;
        return tg;
    };

    // One trial with the proposal `pr` and its target `tg` (both made before
    // this trial began, and the target's gather issued) and the uniform word
    // uw.  While the gather is in flight, `q` (a PhiloxRun) advances the next
    // block by five rounds, and the next trial's proposal is made from the
    // spins as they are now (site word swn, or q.c0 after the rounds when
    // from_q), with its target for either outcome of this trial.  Right after
    // the decision the next target's gather is issued (when `more`).  When this
    // trial's flip is at one of the five sites that proposal read, the
    // proposal for the accepted outcome is corrected arithmetically (the
    // flipped spin is pr.bc before and 1 - pr.bc after): at its own site the
    // spin and all four anti-alignments invert, at a neighbour that one
    // anti-alignment does (the five sites are distinct for L >= 4).  Flips are
    // xors in LDS, so a row read before an earlier flip is never written back.
    int64_t lng_nx = 0;  // the gather of the next trial's target, issued by the trial before
    auto trial = [&](Prop& pr, Tgt& tg, uint32_t uw, uint32_t swn, bool more, bool from_q, auto& q) {
        int64_t lng2 = lng_nx;
        const int64_t cur_hi = lng_cur & HI;
        // the 32-bit LDS word holding the proposed site's spin (its byte offset), and its bit
        uint32_t xoff = static_cast<uint32_t>(((pr.r << wsh) + lane) * sizeof(RowT)) + ((pr.c >> 5) << 2);
        const uint32_t xb = 1u << (pr.c & 31);
        Uniform uf = uniform_f(uw);
        if constexpr (!std::is_same_v<std::decay_t<decltype(q)>, NoRounds>) {
            philox_rounds<5>(q);
            if (from_q) swn = q.c0;
        }
        Prop nx{};
        Tgt ta{}, tr{};
        uint32_t bca = 0, ka = 0;  // nx's spin and neighbour count after this trial's flip
        if (more) {
            nx = propose(swn);
            tr = target(nx, e, m, cur);
            const int f = pr.s0;
            const uint32_t same = f == nx.s0 ? 1u : 0u;
            const uint32_t nbr = ((f == nx.s1) | (f == nx.s2) | (f == nx.s3) | (f == nx.s4)) ? 1u : 0u;
            bca = nx.bc ^ same;
            // k + same (4 - 2k) + nbr (1 - 2 (pr.bc ^ nx.bc)), same and nbr exclusive
            ka = nx.k + (same ? 4u - 2u * nx.k : 0u) + (nbr ? 1u - 2u * (pr.bc ^ nx.bc) : 0u);
            Prop nxa = nx;
            nxa.bc = bca;
            nxa.k = ka;
            ta = target(nxa, tg.e2, tg.m2, tg.idx);
        }
        pin_next(tr.idx, ta.idx, bca, ka);
        // where the bin is written back on a move, and the next gather's
        // address for either outcome (global pointers, so that the accesses stay
        // global ones after the asm below)
        using gptr = __attribute__((address_space(1))) int64_t*;
        gptr cur_p = (gptr)(tab + cur);
        gptr ta_p = (gptr)(tab + ta.idx);
        gptr tr_p = (gptr)(tab + tr.idx);
        uint32_t xbw = xb;
        asm volatile("" : "+v"(cur_p), "+v"(ta_p), "+v"(tr_p), "+v"(xbw), "+v"(xoff));
        pin(q, lng2, uf);
        // Every lane runs the filter (no branch on `in`): a lane whose proposal
        // leaves the window gathered its own bin, whose stored ln g is at most
        // the one it holds, so the filter accepts there at once and `in` rejects.
        // Only the write-back of the bin left is branched on: the flip is an xor
        // with a zero mask on a rejection, and the new state is selected.
        const bool acc = accept_pre<PACKED>(cur_hi - (lng2 & HI), uw, uf, K + PS) & (tg.in != 0);
        const Tgt tg_old = tg;
        // the bin left behind is written back before the next gather, which may read it
        if (acc) *cur_p = lng_cur;
        if (more) lng_nx = *(acc ? ta_p : tr_p);
        // the rest of the new state is selected after that gather is issued (the
        // decision and the flip's LDS offset pass through an empty asm, after the
        // gather in program order, so that this work is not moved ahead of it)
        uint32_t accw = acc ? 1u : 0u;
        uint32_t xo = xoff;
        asm volatile("" : "+v"(accw), "+v"(xo) : : "memory");
        const bool acc2 = accw != 0;
        tg = acc2 ? ta : tr;
        atomicXor(reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(lds) + xo), acc2 ? xbw : 0u);
        e = acc2 ? tg_old.e2 : e;
        m = acc2 ? tg_old.m2 : m;
        cur = acc2 ? tg_old.idx : cur;
        lng_cur = acc2 ? lng2 : lng_cur;
        nx.bc = acc2 ? bca : nx.bc;
        nx.k = acc2 ? ka : nx.k;
        nseen += (lng_cur == 0) ? 1u : 0u;
        lng_cur += inc;
        if constexpr (PACKED) ovf_hi |= static_cast<uint32_t>(static_cast<uint64_t>(lng_cur) >> 32);
        ++t;
        pr = nx;
    };

    // trial t uses words (x, y) of Philox block t/2 when t is even, (z, w) when odd
    NoRounds none;
    Words4 blk = {0, 0, 0, 0};
    Prop pr{};
    Tgt tg{};
    const bool odd = n_trials > 0 && (t & 1);
    if (n_trials > 0) {
        const uint64_t b = static_cast<uint64_t>(t) >> 1;
        blk = philox4x32_10(seed, static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), gid, TAG_WL << 24);
        pr = propose((t & 1) ? blk.z : blk.x);
        tg = target(pr, e, m, cur);
        lng_nx = tab[tg.idx];
    }
    // The load of the first bin's ln g completes here, so that the trial loop
    // never waits on it (it would otherwise wait on every gather in flight).
    asm volatile("" : "+v"(lng_cur));
    if (odd) {  // odd start: second half of the current block
        const bool more = n_trials > 1;
        const uint64_t b = (static_cast<uint64_t>(t) >> 1) + 1;
        const Words4 nb = more ? philox4x32_10(seed, static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), gid,
                                               TAG_WL << 24)
                               : Words4{0, 0, 0, 0};
        trial(pr, tg, blk.w, nb.x, more, false, none);
        blk = nb;
    }
    // t is even here and blk is block t/2.  A pair of trials computes the next
    // block in two halves, one under each trial's gather.  The pairs run
    // (n_trials - 1) / 2 times on every lane, whatever its parity, so that the
    // loop is uniform across the wavefront; their second trial makes the next
    // proposal even when no trial follows (it is then not used).  One pair or
    // one trial is left.
    auto pair = [&](bool more) {
        PhiloxRun q = philox_start(seed, (static_cast<uint64_t>(t) >> 1) + 1, gid);
        trial(pr, tg, blk.y, blk.z, true, false, q);
        trial(pr, tg, blk.w, 0u, more, true, q);
        blk = {q.c0, q.c1, q.c2, q.c3};
    };
    const int64_t npairs = n_trials > 0 ? (n_trials - 1) >> 1 : 0;  // below 2^30 (at most 2^31 trials a launch)
    for (int32_t j = 0; j < static_cast<int32_t>(npairs); ++j) pair(true);
    const int64_t rem = n_trials - (odd ? 1 : 0) - 2 * npairs;  // 0, 1 or 2
    if (rem == 2) pair(false);
    else if (rem == 1) trial(pr, tg, blk.y, 0u, false, false, none);  // first half of block t/2
    }
    tab[cur] = lng_cur;
    if (PACKED && (ovf || (ovf_hi >> 31) != 0)) atomicOr(&S.counters[1], ERR_PACK);
    S.e[g] = e;
    S.m[g] = m;
    S.t[g] = t;
    S.nseen[g] = nseen;
    uint32_t* osp = S.spins + d.spin_off;
    for (int r = 0; r < L; ++r) {
        const RowT v = lds[r * WG + lane];
        osp[r * rw] = static_cast<uint32_t>(v);
        if constexpr (sizeof(RowT) == 8) {
            if (rw == 2) osp[2 * r + 1] = static_cast<uint32_t>(v >> 32);
        }
    }
}

// The sweep kernel: walkers [g_begin, g_begin + g_count) in tiles of WG
// lanes.  With a grid smaller than the tile count each workgroup runs its
// tiles one after another (persistent form), which bounds the number of
// walkers in flight and so the set of table lines competing for the L2; the
// tile-to-workgroup map is the same at every launch, so a walker stays on the
// same XCD.
template <typename RowT, int SPLIT, int LAYOUT, bool AHEAD>
__global__ void __launch_bounds__(256) k_sweep(DevState S, int64_t g_begin, int64_t g_count,
                                               int64_t n_trials, int wpw) {
    extern __shared__ unsigned char lds_raw[];
    RowT* lds = reinterpret_cast<RowT*>(lds_raw);
    const int lane = threadIdx.x;
    const int WG = blockDim.x;
    // the first wpw lanes of each wavefront carry a walker (fewer than 64 spread
    // a small batch over more CUs, so each walker has more of an L1 to itself)
    const int wave = lane >> 6, wl = lane & 63;
    const int per = (WG >> 6) * wpw;
    const int64_t n_tiles = (g_count + per - 1) / per;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t gi = tile * per + wave * wpw + wl;
        if (wl < wpw && gi < g_count)
            sweep_walker<RowT, SPLIT, LAYOUT, AHEAD>(S, lds, lane, WG, g_begin + gi, n_trials);
    }
}

// ------------------------------------------------------------------ flatness
// One wavefront per walker scans its table in chunks of 64 bins, four chunks
// (eight loads per lane) in flight at a time, starting where the previous
// scan failed: the walker is flat iff every visited bin (ln g > 0) has
// flat_den * H * n_seen >= flat_num * sum H, with H = (ln g >> (K - s)) -
// base (mod 2^32) and sum H = trials made in this stage.  The first failing
// chunk in scan order ends the scan and is where the next one starts; the
// latch is set only after a full pass, so the result does not depend on the
// order.
//
// Before that, once per 2^a stage trials (a = audit_shift), the whole table is
// audited: every bin must have H < 2^(a+1) (see the table notes in
// rewl_internal.h); flat and
// unflat walkers alike, since a latched walker keeps walking.  audit_only
// stops after the audit (after trials made outside an interval).
constexpr int FLAT_GROUP = 4;

__device__ __forceinline__ uint32_t stage_visits(int64_t lng, uint32_t base, int sh) {
    return static_cast<uint32_t>(static_cast<uint64_t>(lng) >> sh) - base;
}

__global__ void __launch_bounds__(256) k_flat(DevState S, int audit_only) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * 4 + wave;
    if (g >= S.n_walk) return;
    const WDesc d = S.wd[g];
    const int p = d.prob;
    if (S.wdone[d.gwin]) return;
    const PDesc P = S.pd[p];
    const int sh = P.K - S.stage[d.gwin];
    const uint64_t sum = static_cast<uint64_t>(S.t[g] - S.tstage[d.gwin]);
    const int64_t* tab = S.lng + d.table_off;
    const uint32_t* hb = S.packed ? nullptr : S.hb + d.table_off;
    const int64_t nb = d.nbins;
    const uint32_t epoch = static_cast<uint32_t>(sum >> S.audit_shift);
    if (epoch != S.aud[g]) {
        const uint32_t lim = 1u << (S.audit_shift + 1);
        bool wrap = false;
        for (int64_t i = lane; i < nb; i += 64)
            wrap = wrap || (hb ? stage_visits(tab[i], hb[i], sh) : packed_visits(tab[i], sh)) >= lim;
        if (__any(wrap) && lane == 0) atomicOr(&S.counters[1], ERR_HWRAP);
        if (lane == 0) S.aud[g] = epoch;
    }
    if (audit_only || S.flag[g]) return;
    const uint64_t n = S.nseen[g];
    if (n == 0) return;
    const int64_t nch = (nb + 63) / 64;
    int64_t c0 = S.scan[g];
    if (c0 >= nch) c0 = 0;
    const unsigned __int128 rhs = static_cast<unsigned __int128>(static_cast<uint64_t>(P.flat_num)) * sum;
    for (int64_t k = 0; k < nch; k += FLAT_GROUP) {
        int64_t c[FLAT_GROUP], l[FLAT_GROUP];
        uint32_t b[FLAT_GROUP];
        bool on[FLAT_GROUP];
#pragma unroll
        for (int j = 0; j < FLAT_GROUP; ++j) {
            int64_t cj = c0 + k + j;
            if (cj >= nch) cj -= nch;
            c[j] = cj;
            const int64_t i = cj * 64 + lane;
            on[j] = k + j < nch && i < nb;
            l[j] = on[j] ? tab[i] : 0;
            b[j] = on[j] && hb ? hb[i] : 0;
        }
#pragma unroll
        for (int j = 0; j < FLAT_GROUP; ++j) {
            int fail = 0;
            if (l[j] != 0) {
                const uint64_t H = hb ? stage_visits(l[j], b[j], sh) : packed_visits(l[j], sh);
                fail = static_cast<unsigned __int128>(static_cast<uint64_t>(P.flat_den)) * H * n < rhs;
            }
            if (__any(fail)) {
                if (lane == 0) S.scan[g] = static_cast<uint32_t>(c[j]);
                return;
            }
        }
    }
    if (lane == 0) S.flag[g] = 1;
}

// ------------------------------------------------------------------ stage
// Per problem, at an interval boundary.  sync 0 (the paper, Sec. 2): when
// every walker is flat all windows move to the next stage together (ln f
// halves; H restarts from zero through a new stage base); flatness at
// the last stage ends the problem.  sync 1: each window whose walkers are all
// flat averages their ln g (k_average) and moves on alone; its last stage
// ends it and its walkers stop; the problem ends with its last window.
// Unless the problem has ended, the boundary's exchange round is armed.
// Also guards the int64 headroom of ln g per window.
__global__ void k_stage(DevState S) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= S.n_prob) return;
    const PDesc P = S.pd[p];
    for (int w = 0; w < P.nwin; ++w) S.adv[P.win_off + w] = 0;
    if (S.done[p]) {
        S.xon[p] = 0;
        return;
    }
    // every ln g entry is at most the sum of all increments made so far
    for (int w = 0; w < P.nwin; ++w) {
        const int wi = P.win_off + w;
        if (S.wdone[wi]) continue;
        const int64_t tnow = S.t[P.walker_off + w * P.W];
        const int64_t dt = tnow - S.tseen[wi];
        const int sh = P.K - S.stage[wi];
        const int64_t room = ((static_cast<int64_t>(1) << 62) - S.lngb[wi]) >> sh;
        if (dt > room) atomicOr(&S.counters[1], ERR_OVERFLOW);
        else S.lngb[wi] += dt << sh;
        S.tseen[wi] = tnow;
    }
    const int64_t r = S.rnd[p];
    bool ended = false;
    if (P.sync == 0) {
        const int nw = P.nwin * P.W;
        bool all = true;
        for (int i = 0; i < nw; ++i) all = all && (S.flag[P.walker_off + i] != 0);
        if (all) {
            const int64_t tnow = S.t[P.walker_off];
            const bool last = S.stage[P.win_off] == P.K;
            for (int w = 0; w < P.nwin; ++w) {
                const int wi = P.win_off + w;
                if (last) {
                    S.wdone[wi] = 1;
                } else {
                    S.stage[wi] += 1;
                    S.tstage[wi] = tnow;
                    S.adv[wi] = 1;
                }
            }
            if (last) ended = true;
            else
                for (int i = 0; i < nw; ++i) S.flag[P.walker_off + i] = 0;
        }
    } else {
        bool all_done = true;
        for (int w = 0; w < P.nwin; ++w) {
            const int wi = P.win_off + w;
            if (!S.wdone[wi]) {
                const int g0 = P.walker_off + w * P.W;
                bool all = true;
                for (int a = 0; a < P.W; ++a) all = all && (S.flag[g0 + a] != 0);
                if (all) {
                    S.adv[wi] = 1;  // average (and, if it goes on, take a new stage base)
                    if (S.stage[wi] == P.K) {
                        S.wdone[wi] = 1;
                    } else {
                        S.stage[wi] += 1;
                        S.tstage[wi] = S.t[g0];
                        for (int a = 0; a < P.W; ++a) S.flag[g0 + a] = 0;
                    }
                }
            }
            all_done = all_done && S.wdone[wi] != 0;
        }
        ended = all_done;
    }
    if (ended) {
        S.done[p] = 1;
        S.xon[p] = 0;
        S.rnd[p] = r + 1;
        return;
    }
    S.xr[p] = r;
    S.xon[p] = 1;
    S.rnd[p] = r + 1;
}

// Per-window averaging (sync 1) of a window that has just ended a stage: in
// every bin some walker of the window has visited (ln g > 0) all its walkers
// take floor(mean over those walkers); the other bins stay 0.  The number of
// visited bins becomes every walker's n_seen.  One workgroup per window; the
// walkers of a window share one tiled geometry.
__global__ void __launch_bounds__(256) k_average(DevState S) {
    const int wi = blockIdx.x;
    if (wi >= S.n_win || !S.adv[wi]) return;
    __shared__ int32_t g0s;
    __shared__ uint32_t cnt[256];
    if (threadIdx.x == 0) {
        // first walker of window wi: the walkers are laid out window by window
        int lo = 0, hi = S.n_prob - 1;
        while (lo < hi) {  // last problem with win_off <= wi
            const int mid = (lo + hi + 1) / 2;
            if (S.pd[mid].win_off <= wi) lo = mid;
            else hi = mid - 1;
        }
        const PDesc P = S.pd[lo];
        g0s = P.sync == 1 ? P.walker_off + (wi - P.win_off) * P.W : -1;
    }
    __syncthreads();
    const int g0 = g0s;
    if (g0 < 0) return;
    const WDesc d0 = S.wd[g0];
    const int W = S.pd[d0.prob].W;
    uint32_t seen = 0;
    for (uint32_t i = threadIdx.x; i < d0.nbins; i += blockDim.x) {
        unsigned __int128 sum = 0;
        uint32_t n = 0;
        for (int a = 0; a < W; ++a) {
            const int64_t v = lng_at(S, S.wd[g0 + a].table_off + i);
            if (v > 0) {
                sum += static_cast<uint64_t>(v);
                ++n;
            }
        }
        if (n == 0) continue;
        const int64_t avg = static_cast<int64_t>(sum / n);
        // packed: the base bits are rewritten by k_snapshot right after
        const int64_t word = S.packed ? static_cast<int64_t>(static_cast<uint64_t>(avg) << PACK_SHIFT) : avg;
        for (int a = 0; a < W; ++a) S.lng[S.wd[g0 + a].table_off + i] = word;
        ++seen;
    }
    cnt[threadIdx.x] = seen;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
        __syncthreads();
    }
    if (static_cast<int>(threadIdx.x) < W) S.nseen[g0 + threadIdx.x] = cnt[0];
}

// New stage base for the walkers of windows that just ended a stage (stage s
// now holds the new one): one workgroup per walker, a coalesced pass over its
// table, and its audit epoch restarts with the stage.
__global__ void __launch_bounds__(256) k_snapshot(DevState S) {
    const int64_t g = blockIdx.x;
    const WDesc d = S.wd[g];
    if (!S.adv[d.gwin]) return;
    const int sh = S.pd[d.prob].K - S.stage[d.gwin];
    int64_t* src = S.lng + d.table_off;
    if (S.packed) {
        for (uint32_t i = threadIdx.x; i < d.nbins; i += blockDim.x) {
            const int64_t w = src[i];
            src[i] = (w & ~PACK_MASK) | static_cast<int64_t>((static_cast<uint64_t>(w) >> (PACK_SHIFT + sh)) &
                                                             static_cast<uint64_t>(PACK_MASK));
        }
    } else {
        uint32_t* dst = S.hb + d.table_off;
        for (uint32_t i = threadIdx.x; i < d.nbins; i += blockDim.x)
            dst[i] = static_cast<uint32_t>(static_cast<uint64_t>(src[i]) >> sh);
    }
    if (threadIdx.x == 0) S.aud[g] = 0;
}

// ------------------------------------------------------------------ exchange
// One workgroup per neighbouring window pair (w, v) of a problem; pairs whose
// lower window w has index = r (mod 2) along their direction act in round r
// (Sec. 2, Eq. 2).  Lane 0 draws the random
// matching (Fisher-Yates from the XPERM stream), tests that both
// configurations lie in the overlap, and accepts with
// min[1, g_A(X) g_B(Y) / (g_A(Y) g_B(X))]; then the workgroup swaps the
// accepted configurations.  ln g and H do not change.
__global__ void __launch_bounds__(64) k_exchange(DevState S) {
    __shared__ int perm[256];
    __shared__ int32_t acc_a[256], acc_b[256];
    __shared__ int n_acc;
    const PairDesc pr = S.pairs[blockIdx.x];
    const int p = pr.prob, w = pr.wa, v = pr.wb;
    if (!S.xon[p]) return;
    const int64_t r = S.xr[p];
    // round r: pairs whose lower window has index along its direction = r (mod 2);
    // with windows in both coordinates, pairs along E on rounds with bit 1 of r
    // clear and along M on the others
    if ((pr.along & 1) != static_cast<int>(r & 1)) return;
    if (pr.dir != static_cast<int>((r >> 1) & 1) && S.pd[p].split == 2) return;
    const PDesc P = S.pd[p];
    if (S.wdone[P.win_off + w] || S.wdone[P.win_off + v]) return;  // a finished window does not exchange
    const int W = P.W;
    if (threadIdx.x == 0) {
        const uint32_t r_lo = static_cast<uint32_t>(r), r_hi = static_cast<uint32_t>(static_cast<uint64_t>(r) >> 32);
        for (int a = 0; a < W; ++a) perm[a] = a;
        for (int i = W - 1; i >= 1; --i) {
            const Words4 b = philox4x32_10(P.seed, r_lo, r_hi, static_cast<uint32_t>(w),
                                           (TAG_XPERM << 24) | static_cast<uint32_t>(i));
            const int j = static_cast<int>((static_cast<uint64_t>(b.x) * static_cast<uint64_t>(i + 1)) >> 32);
            const int tmp = perm[i];
            perm[i] = perm[j];
            perm[j] = tmp;
        }
        int n = 0;
        for (int a = 0; a < W; ++a) {
            const int A = P.walker_off + w * W + a;
            const int B = P.walker_off + v * W + perm[a];
            const WDesc dA = S.wd[A], dB = S.wd[B];
            const int eA = S.e[A], mA = S.m[A], eB = S.e[B], mB = S.m[B];
            if (!in_window(P.split, dB, eA, mA) || !in_window(P.split, dA, eB, mB)) continue;
            const uint64_t tA = dA.table_off, tB = dB.table_off;
            // both configurations are states of both windows, so every bin below is stored;
            // a bin that is not would be a layout error, reported instead of read
            const int64_t iAX = table_index_or_none(dA, eA, mA), iAY = table_index_or_none(dA, eB, mB);
            const int64_t iBY = table_index_or_none(dB, eB, mB), iBX = table_index_or_none(dB, eA, mA);
            if (iAX < 0 || iAY < 0 || iBY < 0 || iBX < 0) {
                atomicOr(&S.counters[1], ERR_LAYOUT);
                continue;
            }
            const int64_t delta = lng_at(S, tA + iAX) - lng_at(S, tA + iAY) + lng_at(S, tB + iBY) -
                                  lng_at(S, tB + iBX);
            const Words4 b = philox4x32_10(P.seed, r_lo, r_hi, static_cast<uint32_t>(w),
                                           (TAG_XACC << 24) | static_cast<uint32_t>(a));
            if (accept_move(delta, b.x, P.K)) {
                S.e[A] = eB;
                S.m[A] = mB;
                S.e[B] = eA;
                S.m[B] = mA;
                acc_a[n] = A;
                acc_b[n] = B;
                ++n;
            }
        }
        n_acc = n;
    }
    __syncthreads();
    const int words = P.L * P.row_words;
    for (int k = 0; k < n_acc; ++k) {
        uint32_t* sa = S.spins + S.wd[acc_a[k]].spin_off;
        uint32_t* sb = S.spins + S.wd[acc_b[k]].spin_off;
        for (int i = threadIdx.x; i < words; i += blockDim.x) {
            const uint32_t tmp = sa[i];
            sa[i] = sb[i];
            sb[i] = tmp;
        }
    }
}

// ------------------------------------------------------------------ self-check
// Not part of the sampling path: the sweep's acceptance (accept_pre, float
// filter plus exact fallback) against the specified comparison (accept_move)
// on n trial pairs (delta, u word) placed near the decision boundary.  Pair i
// draws delta uniformly from [-23 2^K, -1] and a relative offset r in
// [-rel, rel] from Philox block (i, 0, 0, 5 << 24) of `seed`, and takes the
// word w nearest to exp(delta 2^-K) (1 + r) 2^32 - 1/2; every eighth pair
// takes instead the word next to the boundary itself (offset -2 .. 2 words),
// where the exact path must decide.  counts[0] += disagreements, counts[1] +=
// pairs decided by the exact path, counts[2] += acceptances; the first n_samp
// pairs and decisions are written out for a check against the CPU.
__global__ void k_accept_check(int K, uint64_t seed, int64_t n, double rel, unsigned long long* counts,
                               int64_t* sd, uint32_t* su, int32_t* sdec, int n_samp, int packed) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Words4 b = philox4x32_10(seed, static_cast<uint32_t>(i), static_cast<uint32_t>(static_cast<uint64_t>(i) >> 32),
                                   0u, 5u << 24);
    const uint64_t span = static_cast<uint64_t>(23) << K;
    const uint64_t r64 = (static_cast<uint64_t>(b.x) << 32) | b.y;
    int64_t delta = -static_cast<int64_t>(r64 % span) - 1;
    if ((i & 15) == 14) {
        // far below the boundary (x <= -23, down to the largest ln g the layout holds: 2^37 units
        // for packed words, 2^62 otherwise), where the filter decides with no range test
        const uint64_t lim = static_cast<uint64_t>(1) << (packed ? 37 : 62);
        delta = -static_cast<int64_t>(span + r64 % (lim - span));
    }
    const double x = ldexp(static_cast<double>(delta), -K);
    const double ex = exp_neg(x) * 4294967296.0;
    double target;
    if ((i & 7) == 7) {
        target = floor(ex - 0.5) + static_cast<double>(static_cast<int>(b.z % 5u) - 2);
    } else {
        const double off = (static_cast<double>(b.z) / 4294967296.0 * 2.0 - 1.0) * rel;
        target = floor(ex * (1.0 + off) - 0.5);
    }
    target = fmin(fmax(target, 0.0), 4294967295.0);
    const uint32_t w = static_cast<uint32_t>(target);
    bool exact_path = false;
    // packed: the sweep's form for packed table words, delta in units of 2^-(K + 26)
    const bool fast = packed ? accept_pre<true>(delta * (static_cast<int64_t>(1) << PACK_SHIFT), w, uniform_f(w),
                                                K + PACK_SHIFT, exact_path)
                             : accept_pre(delta, w, uniform_f(w), K, exact_path);
    const bool spec = accept_move(delta, w, K);
    if (fast != spec) atomicAdd(&counts[0], 1ull);
    if (exact_path) atomicAdd(&counts[1], 1ull);
    if (spec) atomicAdd(&counts[2], 1ull);
    if (i < n_samp) {
        sd[i] = delta;
        su[i] = w;
        sdec[i] = fast ? 1 : 0;
    }
}

int blocks_for(int64_t n, int per) { return static_cast<int>((n + per - 1) / per); }

}  // namespace

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    int grid = static_cast<int>((n16 + 255) / 256);
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, st, static_cast<uint4*>(p), n16);
    return hipGetLastError();
}

hipError_t launch_init(const DevState& S, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3(blocks_for(S.n_walk, 64)), dim3(64), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_entry(const DevState& S, int64_t cap, hipStream_t st) {
    hipLaunchKernelGGL(k_entry, dim3(blocks_for(S.n_walk, 64)), dim3(64), 0, st, S, cap);
    return hipGetLastError();
}

// Instantiations: every split with dense addressing, energy windows also with
// band addressing, each with unpacked and packed tables, each in the direct
// and the pipelined (AHEAD) form.
#define REWL_SWEEP_KERNELS_A(RowT, A)                                                                     \
    &k_sweep<RowT, 0, 0, A>, &k_sweep<RowT, 0, 1, A>, &k_sweep<RowT, 1, 0, A>, &k_sweep<RowT, 2, 0, A>, \
        &k_sweep<RowT, 0, 2, A>, &k_sweep<RowT, 0, 3, A>, &k_sweep<RowT, 1, 2, A>, &k_sweep<RowT, 2, 2, A>
#define REWL_SWEEP_KERNELS(RowT) REWL_SWEEP_KERNELS_A(RowT, false), REWL_SWEEP_KERNELS_A(RowT, true)

template <typename RowT>
hipError_t launch_sweep_t(int split, int layout, bool ahead, dim3 grid, dim3 wg, size_t lds, hipStream_t st,
                          const DevState& S, int64_t g_begin, int64_t g_count, int64_t n_trials, int wpw) {
    using Kern = void (*)(DevState, int64_t, int64_t, int64_t, int);
    static const Kern kerns[16] = {REWL_SWEEP_KERNELS(RowT)};
    const int band = split == 0 && (layout & LAYOUT_BAND);
    const int base = split == 0 ? band : split + 1;  // 0..3: (0, dense) (0, band) (1) (2)
    const Kern k = kerns[base + ((layout & LAYOUT_PACKED) ? 4 : 0) + (ahead ? 8 : 0)];
    DevState s_arg = S;
    void* args[] = {&s_arg, &g_begin, &g_count, &n_trials, &wpw};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), grid, wg, args, lds, st);
}

hipError_t launch_sweep(const DevState& S, int64_t g_begin, int64_t g_count, int64_t n_trials,
                        int l_max, int wg, int max_grid, int wpw, int split, int layout, bool ahead, hipStream_t st) {
    if (g_count <= 0 || n_trials <= 0) return hipSuccess;
    if (n_trials > (static_cast<int64_t>(1) << 31)) return hipErrorInvalidValue;  // the pair loop counts in 32 bits
    if (wpw <= 0 || wpw > 64) wpw = 64;
    int grid = blocks_for(g_count, (wg / 64) * wpw);
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    const size_t lds = static_cast<size_t>(l_max) * wg * (l_max <= 32 ? sizeof(uint32_t) : sizeof(uint64_t));
    // band addressing applies to energy windows only (magnetization windows keep dense addressing)
    const hipError_t e =
        l_max <= 32
            ? launch_sweep_t<uint32_t>(split, layout, ahead, dim3(grid), dim3(wg), lds, st, S, g_begin, g_count,
                                       n_trials, wpw)
            : launch_sweep_t<uint64_t>(split, layout, ahead, dim3(grid), dim3(wg), lds, st, S, g_begin, g_count,
                                       n_trials, wpw);
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t sweep_setup() {
    using Kern = void (*)(DevState, int64_t, int64_t, int64_t, int);
    const Kern fns[32] = {REWL_SWEEP_KERNELS(uint32_t), REWL_SWEEP_KERNELS(uint64_t)};
    for (Kern f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_flat(const DevState& S, hipStream_t st, int audit_only) {
    hipLaunchKernelGGL(k_flat, dim3(blocks_for(S.n_walk, 4)), dim3(256), 0, st, S, audit_only);
    return hipGetLastError();
}

hipError_t launch_stage(const DevState& S, hipStream_t st) {
    hipLaunchKernelGGL(k_stage, dim3(blocks_for(S.n_prob, 64)), dim3(64), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_average(const DevState& S, hipStream_t st) {
    if (S.n_win <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_average, dim3(S.n_win), dim3(256), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_snapshot(const DevState& S, hipStream_t st) {
    if (S.n_walk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_snapshot, dim3(static_cast<unsigned>(S.n_walk)), dim3(256), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_accept_check(int K, uint64_t seed, int64_t n, double rel, unsigned long long* counts, int64_t* sd,
                               uint32_t* su, int32_t* sdec, int n_samp, int packed, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_accept_check, dim3(blocks_for(n, 256)), dim3(256), 0, st, K, seed, n, rel, counts, sd, su,
                       sdec, n_samp, packed);
    return hipGetLastError();
}

hipError_t launch_exchange(const DevState& S, hipStream_t st) {
    if (S.n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_exchange, dim3(S.n_pairs), dim3(64), 0, st, S);
    return hipGetLastError();
}

}  // namespace rewl
