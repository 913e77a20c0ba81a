/*
 * rewl_oracle.c -- plain CPU oracle for two-dimensional replica-exchange
 * Wang-Landau (2D-REWL) sampling of the periodic L x L Ising model
 * (Valentim et al., "Exploring Replica-Exchange Wang-Landau sampling in
 * higher-dimensional parameter space", arXiv:1508.02748).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant generator with the HIP path; it exists to say what
 * the HIP path must compute, bit for bit, under the same Philox stream.
 *
 * Everything is written for clarity, not speed: spins are one signed byte per
 * site, ln g and H are plain arrays over the walker's whole energy window times
 * the full magnetization range, flatness is a full scan, and every random
 * number is drawn by calling Philox once per use.
 *
 * What the paper fixes, and where:
 *   - joint density of states g(E,M) and histogram H(E,M) per walker (Sec. 2);
 *   - acceptance min[1, g(E',M')/g(E'',M'')] of a trial configuration (Eq. 1);
 *   - on accept update g, H at the trial state, else at the current one (Sec. 2);
 *   - iterate until H is flat, then reset H and refine f -> sqrt(f) (Sec. 2);
 *   - 80 % flatness: every entry >= 0.8 * mean (Sec. 3);
 *   - overlapping equal-size energy windows, unrestricted M (Sec. 2, Sec. 3),
 *     or, as the alternatives Sec. 2 names, magnetization windows with
 *     unrestricted E (or_set_split) or rectangles in both (or_create_2d);
 *   - several independent walkers per window with their own g, H (Sec. 2);
 *   - configuration exchange between random walker pairs of adjacent windows,
 *     attempted only when both lie in the overlap, accepted with Eq. 2;
 *   - all walkers advance to the next iteration together (Sec. 2).
 * What the paper leaves open is fixed by the determinism readings below
 * (D-1 ... D-10); each is listed, with its reason, in the design notes.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math
 *        -fopenmp rewl_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* D-2  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: */
/* as easy as 1, 2, 3", SC'11).  Ten rounds; each round multiplies counter   */
/* words 0 and 2 by the two Philox multipliers, and mixes the high halves    */
/* with words 1 and 3 and the round key; the key is bumped by the two Weyl   */
/* constants between rounds.                                                 */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4],
                         uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream tags (counter word 3, bits 24..31). */
enum { TAG_WL = 0, TAG_INIT = 1, TAG_ENTRY = 2, TAG_XPERM = 3, TAG_XACC = 4 };

/* Draw the two words used by sequential attempt number `a` of a walker's
 * stream `tag` (WL or ENTRY): block a>>1, words (2j, 2j+1) with j = a & 1. */
static void draw_pair(uint64_t seed, uint64_t a, uint32_t walker, uint32_t tag,
                      uint32_t *site_word, uint32_t *u_word) {
    uint64_t b = a >> 1;
    uint32_t ctr[4] = {(uint32_t)b, (uint32_t)(b >> 32), walker, tag << 24};
    uint32_t w[4];
    or_philox((uint32_t)seed, (uint32_t)(seed >> 32), ctr, w);
    int j = (int)(a & 1);
    *site_word = w[2 * j];
    *u_word = w[2 * j + 1];
}

/* ------------------------------------------------------------------------ */
/* D-5  Acceptance of Eq. (1) and Eq. (2) in exact fixed point.              */
/* ln g is an int64 in units of 2^-K.  For delta = ln g(current) -           */
/* ln g(trial) the move is accepted with probability min[1, exp(delta)]:     */
/* accept iff delta >= 0 or u < exp(delta * 2^-K), with u drawn uniformly    */
/* as (w + 1/2) 2^-32 from one 32-bit word.  Because u >= 2^-33 > e^-23, any */
/* delta <= -23 * 2^K is a rejection without evaluating the exponential.     */
/* ------------------------------------------------------------------------ */

/* exp(x) for x in (-23, 0): x = k ln2 + r with k = nearest integer to
 * x/ln2 and a two-part ln2 (high part with 32 significant bits, so k*hi is
 * exact), then exp(r) by its Taylor series to degree 13 (|r| <= 0.35, the
 * truncation is below 4e-18), evaluated by Horner with fused multiply-adds,
 * finally scaled by 2^k.  Every operation is a single correctly rounded IEEE
 * operation, so any conforming implementation of the same sequence returns the
 * same bits. */
OR_EXPORT double or_exp_spec(double x) {
    static const double inv_fact[14] = {
        0x1.0000000000000p+0,  0x1.0000000000000p+0,  0x1.0000000000000p-1,
        0x1.5555555555555p-3,  0x1.5555555555555p-5,  0x1.1111111111111p-7,
        0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16,
        0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26,
        0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
    const double log2e = 0x1.71547652b82fep+0;   /* RN(1/ln 2) */
    const double ln2_hi = 0x1.62e42fee00000p-1;  /* floor(ln2 * 2^32) / 2^32 */
    const double ln2_lo = 0x1.a39ef35793c76p-33; /* RN(ln2 - ln2_hi) */
    double k = floor(x * log2e + 0.5);
    double r = fma(-k, ln2_hi, x);
    r = fma(-k, ln2_lo, r);
    double p = inv_fact[13];
    for (int j = 12; j >= 0; --j) p = fma(p, r, inv_fact[j]);
    return ldexp(p, (int)k);
}

OR_EXPORT double or_uniform(uint32_t w) {
    return ((double)w + 0.5) * 0x1p-32;
}

OR_EXPORT int or_accept(int64_t delta, uint32_t u_word, int K) {
    if (delta >= 0) return 1;
    if (delta <= -((int64_t)23 << K)) return 0;
    double x = ldexp((double)delta, -K);
    return or_uniform(u_word) < or_exp_spec(x);
}

/* ------------------------------------------------------------------------ */
/* D-6  Overlapping, equal-size energy windows (Sec. 2, Fig. 1(b); Sec. 3).   */
/* The energy-bin range [0, S] (S = N) is split into n windows whose         */
/* neighbours overlap by the fraction p/q: with D = q + (n-1)(q-p), window i */
/* is [floor(i(q-p)S/D), min(S, ceil((i(q-p)+q)S/D))].                       */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_window(int N, int n, int p, int q, int i, int *lo, int *hi) {
    int64_t D = (int64_t)q + (int64_t)(n - 1) * (q - p);
    int64_t a = (int64_t)i * (q - p) * N;
    int64_t b = ((int64_t)i * (q - p) + q) * (int64_t)N;
    int64_t h = (b + D - 1) / D;
    *lo = (int)(a / D);
    *hi = (int)(h > N ? N : h);
}

/* D-1  Energy E = -sum over nearest-neighbour bonds s_i s_j (periodic), and
 * magnetization M = sum s_i, of a configuration of +-1 bytes. */
OR_EXPORT void or_energy(const int8_t *s, int L, int *E, int *M) {
    int e = 0, m = 0;
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) {
            int si = s[r * L + c];
            e -= si * s[r * L + (c + 1) % L];
            e -= si * s[((r + 1) % L) * L + c];
            m += si;
        }
    *E = e;
    *M = m;
}

/* ------------------------------------------------------------------------ */
/* One REWL simulation.                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int L, N, n_win, W, K, flat_num, flat_den, ovl_num, ovl_den, init;
    int64_t X;
    uint64_t seed;
    int nwalk;
    int split;         /* 0: windows split the energy bins e = (E + 2N)/4 (the
                          paper's runs); 1: they split the magnetization bins
                          m = (M + N)/2, every window keeping all energies;
                          2: rectangles of both (or_create_2d) */
    int *lo, *hi;      /* window bounds in the split coordinate (splits 0, 1) */
    int *elo, *ehi, *mlo, *mhi;  /* every window as a rectangle of (e, m) bins */
    int n_pairs;       /* neighbouring window pairs that may exchange */
    int *pa, *pb;      /* lower and upper window of each pair */
    int *pdir;         /* 0: neighbours in e, 1: neighbours in m (split 2) */
    int *palong;       /* grid index of the lower window along pdir (split 2) */
    int8_t *spin;      /* [nwalk][N] */
    int *e, *m;        /* current bins; m = (M + N)/2 */
    int64_t *t;        /* WL attempts made */
    int64_t *te;       /* entry attempts made */
    int64_t **lng;     /* [nwalk][(ehi-elo+1)(mhi-mlo+1)]  ln g in units 2^-K,
                          rows e - elo, columns m - mlo */
    uint64_t **H;      /* same shape */
    uint8_t *flag;     /* flat in the current stage (latched) */
    int s;             /* stage: ln f = 2^-s (the lowest window stage) */
    int done;
    int64_t r;         /* interval boundaries passed */
    int sync;          /* 0: all windows refine together; 1: each window alone */
    int *sw;           /* stage of each window */
    uint8_t *wdone;    /* window has finished its last stage */
} or_rewl;

static int win_of(const or_rewl *P, int g) { return g / P->W; }
static int64_t bins_of(const or_rewl *P, int w) {
    return (int64_t)(P->ehi[w] - P->elo[w] + 1) * (P->mhi[w] - P->mlo[w] + 1);
}
static int64_t bin_index(const or_rewl *P, int w, int e, int m) {
    return (int64_t)(e - P->elo[w]) * (P->mhi[w] - P->mlo[w] + 1) + (m - P->mlo[w]);
}
static int in_window(const or_rewl *P, int w, int e, int m) {
    return e >= P->elo[w] && e <= P->ehi[w] && m >= P->mlo[w] && m <= P->mhi[w];
}
/* Rectangles of the one-coordinate splits: [lo, hi] in the split coordinate,
 * everything in the other. */
static void rects_from_split(or_rewl *P) {
    for (int w = 0; w < P->n_win; ++w) {
        int e_split = P->split == 0;
        P->elo[w] = e_split ? P->lo[w] : 0;
        P->ehi[w] = e_split ? P->hi[w] : P->N;
        P->mlo[w] = e_split ? 0 : P->lo[w];
        P->mhi[w] = e_split ? P->N : P->hi[w];
    }
}

OR_EXPORT void or_destroy(or_rewl *P) {
    if (!P) return;
    if (P->lng)
        for (int g = 0; g < P->nwalk; ++g) free(P->lng[g]);
    if (P->H)
        for (int g = 0; g < P->nwalk; ++g) free(P->H[g]);
    free(P->lng); free(P->H); free(P->lo); free(P->hi); free(P->spin);
    free(P->elo); free(P->ehi); free(P->mlo); free(P->mhi);
    free(P->pa); free(P->pb); free(P->pdir); free(P->palong);
    free(P->e); free(P->m); free(P->t); free(P->te); free(P->flag);
    free(P->sw); free(P->wdone);
    free(P);
}

static int alloc_tables(or_rewl *P);

OR_EXPORT or_rewl *or_create(int L, int n_win, int ovl_num, int ovl_den, int W,
                             int K, int flat_num, int flat_den, int64_t X,
                             uint64_t seed, int init) {
    if (L < 2 || (L & 1) || n_win < 1 || W < 1 || K < 0 || K > 40 || X < 1 ||
        ovl_den < 1 || ovl_num < 0 || ovl_num >= ovl_den || flat_den < 1 ||
        flat_num < 0 || flat_num > flat_den)
        return NULL;
    or_rewl *P = (or_rewl *)calloc(1, sizeof(or_rewl));
    if (!P) return NULL;
    P->L = L; P->N = L * L; P->n_win = n_win; P->W = W; P->K = K;
    P->flat_num = flat_num; P->flat_den = flat_den;
    P->ovl_num = ovl_num; P->ovl_den = ovl_den;
    P->init = init; P->X = X; P->seed = seed;
    P->nwalk = n_win * W;
    P->lo = calloc(n_win, sizeof(int));
    P->hi = calloc(n_win, sizeof(int));
    P->elo = calloc(n_win, sizeof(int));
    P->ehi = calloc(n_win, sizeof(int));
    P->mlo = calloc(n_win, sizeof(int));
    P->mhi = calloc(n_win, sizeof(int));
    P->pa = calloc(2 * (size_t)n_win + 1, sizeof(int));
    P->pb = calloc(2 * (size_t)n_win + 1, sizeof(int));
    P->pdir = calloc(2 * (size_t)n_win + 1, sizeof(int));
    P->palong = calloc(2 * (size_t)n_win + 1, sizeof(int));
    P->spin = calloc((size_t)P->nwalk * P->N, 1);
    P->e = calloc(P->nwalk, sizeof(int));
    P->m = calloc(P->nwalk, sizeof(int));
    P->t = calloc(P->nwalk, sizeof(int64_t));
    P->te = calloc(P->nwalk, sizeof(int64_t));
    P->flag = calloc(P->nwalk, 1);
    P->lng = calloc(P->nwalk, sizeof(int64_t *));
    P->H = calloc(P->nwalk, sizeof(uint64_t *));
    P->sw = calloc(n_win, sizeof(int));
    P->wdone = calloc(n_win, 1);
    if (!P->lo || !P->hi || !P->elo || !P->ehi || !P->mlo || !P->mhi || !P->pa ||
        !P->pb || !P->pdir || !P->palong || !P->spin || !P->e || !P->m || !P->t ||
        !P->te || !P->flag || !P->lng || !P->H || !P->sw || !P->wdone) {
        or_destroy(P);
        return NULL;
    }
    for (int w = 0; w < n_win; ++w)
        or_window(P->N, n_win, ovl_num, ovl_den, w, &P->lo[w], &P->hi[w]);
    rects_from_split(P);
    /* neighbours along the split coordinate: (w, w+1) */
    for (int w = 0; w + 1 < n_win; ++w) {
        P->pa[P->n_pairs] = w;
        P->pb[P->n_pairs] = w + 1;
        P->pdir[P->n_pairs] = 0;
        P->palong[P->n_pairs] = w;
        P->n_pairs += 1;
    }
    if (alloc_tables(P) != 0) {
        or_destroy(P);
        return NULL;
    }
    return P;
}

static int alloc_tables(or_rewl *P) {
    for (int g = 0; g < P->nwalk; ++g) {
        int64_t nb = bins_of(P, win_of(P, g));
        free(P->lng[g]);
        free(P->H[g]);
        P->lng[g] = calloc((size_t)nb, sizeof(int64_t));
        P->H[g] = calloc((size_t)nb, sizeof(uint64_t));
        if (!P->lng[g] || !P->H[g]) return -1;
    }
    return 0;
}

/* Neighbour-sum bookkeeping of a single spin flip at `site` (D-1): returns the
 * new energy bin and magnetization bin the flip would produce. */
static void flip_target(const or_rewl *P, const int8_t *s, int site, int e,
                        int m, int *e2, int *m2) {
    int L = P->L;
    int r = site / L, c = site % L;
    int si = s[site];
    int nb = s[((r + L - 1) % L) * L + c] + s[((r + 1) % L) * L + c] +
             s[r * L + (c + L - 1) % L] + s[r * L + (c + 1) % L];
    int dE = 2 * si * nb; /* energy change of the flip */
    int dM = -2 * si;     /* magnetization change */
    *e2 = e + dE / 4;
    *m2 = m + dM / 2;
}

/* D-3  site = floor(word * N / 2^32). */
static int site_of(uint32_t word, int N) {
    return (int)(((uint64_t)word * (uint64_t)N) >> 32);
}

/* ------------------------------------------------------------------------ */
/* D-10  Initial configuration and entry into the walker's window.           */
/* Spins: site 128q + 32j + k takes bit k of word j of INIT block q          */
/* (1 -> +1), or all +1 when init = 1.  Entry: Metropolis at unit            */
/* temperature on the distance d (in bins of the split coordinate) from the */
/* window: a flip that does not increase d is accepted, one that increases   */
/* it by k bins is accepted with exp(-4k); the walk stops once d = 0.        */
/* ------------------------------------------------------------------------ */
static int dist1(int x, int lo, int hi) {
    if (x < lo) return lo - x;
    if (x > hi) return x - hi;
    return 0;
}
/* bins from (e, m) to the window's rectangle: the sum of the two coordinates' */
/* distances (one of them is always 0 for a one-coordinate split)            */
static int dist_to(const or_rewl *P, int w, int e, int m) {
    return dist1(e, P->elo[w], P->ehi[w]) + dist1(m, P->mlo[w], P->mhi[w]);
}

OR_EXPORT int or_init(or_rewl *P, int64_t entry_cap) {
    int N = P->N;
    int bad = 0;
    /* walkers are independent until the first boundary */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int g = 0; g < P->nwalk; ++g) {
        int8_t *s = P->spin + (size_t)g * N;
        if (P->init == 1) {
            for (int i = 0; i < N; ++i) s[i] = 1;
        } else {
            for (int q = 0; 128 * q < N; ++q) {
                uint32_t ctr[4] = {(uint32_t)q, 0u, (uint32_t)g,
                                   (uint32_t)TAG_INIT << 24};
                uint32_t w[4];
                or_philox((uint32_t)P->seed, (uint32_t)(P->seed >> 32), ctr, w);
                for (int j = 0; j < 4; ++j)
                    for (int k = 0; k < 32; ++k) {
                        int site = 128 * q + 32 * j + k;
                        if (site < N) s[site] = ((w[j] >> k) & 1u) ? 1 : -1;
                    }
            }
        }
        int E, M;
        or_energy(s, P->L, &E, &M);
        P->e[g] = (E + 2 * N) / 4;
        P->m[g] = (M + N) / 2;
        P->t[g] = 0;
        P->te[g] = 0;
        int w = win_of(P, g);
        int d = dist_to(P, w, P->e[g], P->m[g]);
        while (d > 0) {
            if (P->te[g] >= entry_cap) { bad |= 1; break; }
            uint32_t sw, uw;
            draw_pair(P->seed, (uint64_t)P->te[g], (uint32_t)g, TAG_ENTRY, &sw, &uw);
            int site = site_of(sw, N);
            int e2, m2;
            flip_target(P, s, site, P->e[g], P->m[g], &e2, &m2);
            int d2 = dist_to(P, w, e2, m2);
            int acc = d2 <= d ||
                      or_accept(-((int64_t)4 * (d2 - d)) * ((int64_t)1 << P->K),
                                uw, P->K);
            if (acc) {
                s[site] = (int8_t)-s[site];
                P->e[g] = e2;
                P->m[g] = m2;
                d = d2;
            }
            P->te[g] += 1;
        }
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* D-8  One Wang-Landau trial (Sec. 2, Eq. 1): propose flipping a uniformly   */
/* chosen site, reject a proposal that leaves the walker's window (in e, or  */
/* in m for split = 1), otherwise accept with min[1, g(current)/g(trial)];   */
/* then multiply g by f (add ln f = 2^(K-s) units) and add one to H at the  */
/* state the walker is in after the decision.                                */
/* ------------------------------------------------------------------------ */
static void wl_attempt(or_rewl *P, int g) {
    int N = P->N;
    int w = win_of(P, g);
    int8_t *s = P->spin + (size_t)g * N;
    uint32_t sw, uw;
    draw_pair(P->seed, (uint64_t)P->t[g], (uint32_t)g, TAG_WL, &sw, &uw);
    int site = site_of(sw, N);
    int e = P->e[g], m = P->m[g];
    int e2, m2;
    flip_target(P, s, site, e, m, &e2, &m2);
    int acc = 0;
    if (in_window(P, w, e2, m2)) {
        int64_t delta = P->lng[g][bin_index(P, w, e, m)] -
                        P->lng[g][bin_index(P, w, e2, m2)];
        acc = or_accept(delta, uw, P->K);
    }
    if (acc) {
        s[site] = (int8_t)-s[site];
        P->e[g] = e = e2;
        P->m[g] = m = m2;
    }
    int64_t bi = bin_index(P, w, e, m);
    P->lng[g][bi] += (int64_t)1 << (P->K - P->sw[w]);
    P->H[g][bi] += 1;
    P->t[g] += 1;
}

/* Run `n` trials for every walker.  Walkers are independent between
 * boundaries, so the loop over them may be split across threads. */
OR_EXPORT void or_sweep(or_rewl *P, int64_t n) {
    if (P->done) return;
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < P->nwalk; ++g) {
        if (P->wdone[win_of(P, g)]) continue;  /* a finished window stops */
        for (int64_t i = 0; i < n; ++i) wl_attempt(P, g);
    }
}

/* ------------------------------------------------------------------------ */
/* D-9.1  Flatness (Sec. 2; 80 % criterion of Sec. 3) over the bins the      */
/* walker has ever visited (ln g > 0): flat iff                              */
/*   flat_den * min H * n_seen >= flat_num * sum H.                          */
/* ------------------------------------------------------------------------ */
OR_EXPORT int or_is_flat(const or_rewl *P, int g) {
    int64_t nb = bins_of(P, win_of(P, g));
    uint64_t n_seen = 0, sum = 0, mn = UINT64_MAX;
    for (int64_t i = 0; i < nb; ++i) {
        if (P->lng[g][i] > 0) {
            n_seen += 1;
            sum += P->H[g][i];
            if (P->H[g][i] < mn) mn = P->H[g][i];
        }
    }
    if (n_seen == 0) return 0;
    unsigned __int128 lhs = (unsigned __int128)P->flat_den * mn * n_seen;
    unsigned __int128 rhs = (unsigned __int128)P->flat_num * sum;
    return lhs >= rhs;
}

/* ------------------------------------------------------------------------ */
/* D-9.3  Replica exchange between adjacent windows (Sec. 2, Eq. 2).         */
/* Round r pairs windows (w, w+1) with w = r (mod 2).  The walkers of w+1    */
/* are matched to those of w by a Fisher-Yates permutation drawn from the    */
/* XPERM stream; pair (A = (w,a), B = (w+1,pi[a])) is attempted only if A's  */
/* state lies in window w+1 and B's in window w (rectangles), accepted with */
/* min[1, g_A(X) g_B(Y) / (g_A(Y) g_B(X))], X and Y being the configurations */
/* A and B hold.  On accept the two configurations are swapped; neither      */
/* ln g nor H changes.                                                        */
/* ------------------------------------------------------------------------ */
static void swap_config(or_rewl *P, int A, int B) {
    int N = P->N;
    int8_t *a = P->spin + (size_t)A * N, *b = P->spin + (size_t)B * N;
    for (int i = 0; i < N; ++i) {
        int8_t tmp = a[i]; a[i] = b[i]; b[i] = tmp;
    }
    int te = P->e[A]; P->e[A] = P->e[B]; P->e[B] = te;
    int tm = P->m[A]; P->m[A] = P->m[B]; P->m[B] = tm;
}

/* Pairs taking part in round r: for a one-coordinate split, (w, w+1) with   */
/* w = r (mod 2); for rectangles, neighbours in e on rounds with bit 1 of r   */
/* clear and in m on the others, the lower one's grid index along that       */
/* direction = r (mod 2).                                                     */
static int pair_active(const or_rewl *P, int k, int64_t r) {
    if (P->split != 2) return (P->palong[k] & 1) == (int)(r & 1);
    return P->pdir[k] == (int)((r >> 1) & 1) && (P->palong[k] & 1) == (int)(r & 1);
}

/* The random matching of round r for the pair whose lower window is w: a    */
/* Fisher-Yates shuffle of (0 .. W-1), position i (from W-1 down to 1)       */
/* exchanged with position j = floor(word * (i + 1) / 2^32), the word taken  */
/* from the XPERM stream at (r, w, i).  Walker a of the lower window meets   */
/* walker pi[a] of the upper one.                                             */
OR_EXPORT void or_draw_matching(uint64_t seed, int64_t r, int w, int W, int *pi) {
    for (int a = 0; a < W; ++a) pi[a] = a;
    for (int i = W - 1; i >= 1; --i) {
        uint32_t ctr[4] = {(uint32_t)r, (uint32_t)((uint64_t)r >> 32),
                           (uint32_t)w, ((uint32_t)TAG_XPERM << 24) | (uint32_t)i};
        uint32_t out[4];
        or_philox((uint32_t)seed, (uint32_t)(seed >> 32), ctr, out);
        int j = (int)(((uint64_t)out[0] * (uint64_t)(i + 1)) >> 32);
        int tmp = pi[i]; pi[i] = pi[j]; pi[j] = tmp;
    }
}

OR_EXPORT int64_t or_exchange(or_rewl *P, int64_t r) {
    int W = P->W;
    int64_t n_acc = 0;
    int *pi = (int *)malloc(sizeof(int) * (size_t)W);
    for (int k = 0; k < P->n_pairs; ++k) {
        if (!pair_active(P, k, r)) continue;
        int w = P->pa[k], v = P->pb[k];
        or_draw_matching(P->seed, r, w, W, pi);
        for (int a = 0; a < W; ++a) {
            int A = w * W + a, B = v * W + pi[a];
            int eA = P->e[A], mA = P->m[A], eB = P->e[B], mB = P->m[B];
            if (P->wdone[w] || P->wdone[v]) continue;
            if (!in_window(P, v, eA, mA) || !in_window(P, w, eB, mB)) continue;
            int64_t delta = P->lng[A][bin_index(P, w, eA, mA)] -
                            P->lng[A][bin_index(P, w, eB, mB)] +
                            P->lng[B][bin_index(P, v, eB, mB)] -
                            P->lng[B][bin_index(P, v, eA, mA)];
            uint32_t ctr[4] = {(uint32_t)r, (uint32_t)((uint64_t)r >> 32),
                               (uint32_t)w, ((uint32_t)TAG_XACC << 24) | (uint32_t)a};
            uint32_t out[4];
            or_philox((uint32_t)P->seed, (uint32_t)(P->seed >> 32), ctr, out);
            if (or_accept(delta, out[0], P->K)) {
                swap_config(P, A, B);
                n_acc += 1;
            }
        }
    }
    free(pi);
    return n_acc;
}

/* ------------------------------------------------------------------------ */
/* Averaging of one window's walkers (the per-window variant): in every bin  */
/* some walker of the window has visited (ln g > 0), all walkers of the      */
/* window take floor(mean over those walkers of ln g); other bins stay 0.   */
/* ------------------------------------------------------------------------ */
static void average_window(or_rewl *P, int w) {
    int64_t nb = bins_of(P, w);
    for (int64_t i = 0; i < nb; ++i) {
        __int128 sum = 0;
        int n = 0;
        for (int a = 0; a < P->W; ++a) {
            int64_t v = P->lng[w * P->W + a][i];
            if (v > 0) {
                sum += v;
                n += 1;
            }
        }
        if (n == 0) continue;
        int64_t avg = (int64_t)(sum / n);
        for (int a = 0; a < P->W; ++a) P->lng[w * P->W + a][i] = avg;
    }
}

/* ------------------------------------------------------------------------ */
/* D-9  Interval boundary: latch per-walker flatness; when every walker of   */
/* the simulation is flat, all move to the next stage together (Sec. 2):     */
/* ln f halves (f -> sqrt f), H is reset to zero, g is kept.  Flatness at the */
/* last stage K ends the run.  Otherwise an exchange round follows.          */
/* Per-window variant (sync = 1): a window whose walkers are all flat       */
/* averages their ln g, clears their H and moves to its next stage alone    */
/* (its last stage ends it; its walkers then stop); the run ends when every */
/* window has ended; pairs with an ended window do not exchange.            */
/* ------------------------------------------------------------------------ */
static void reset_window(or_rewl *P, int w) {
    for (int a = 0; a < P->W; ++a) {
        int g = w * P->W + a;
        memset(P->H[g], 0, sizeof(uint64_t) * (size_t)bins_of(P, w));
        P->flag[g] = 0;
    }
}

OR_EXPORT void or_boundary(or_rewl *P) {
    if (P->done) return;
    if (P->sync == 0) {
        int all = 1;
        for (int g = 0; g < P->nwalk; ++g) {
            if (!P->flag[g]) P->flag[g] = (uint8_t)or_is_flat(P, g);
            all &= P->flag[g];
        }
        if (all) {
            if (P->s == P->K) {
                P->done = 1;
                for (int w = 0; w < P->n_win; ++w) P->wdone[w] = 1;
                P->r += 1;
                return;
            }
            P->s += 1;
            for (int w = 0; w < P->n_win; ++w) {
                P->sw[w] = P->s;
                reset_window(P, w);
            }
        }
    } else {
        for (int g = 0; g < P->nwalk; ++g)
            if (!P->wdone[win_of(P, g)] && !P->flag[g]) P->flag[g] = (uint8_t)or_is_flat(P, g);
        int all_done = 1, lowest = P->K;
        for (int w = 0; w < P->n_win; ++w) {
            if (!P->wdone[w]) {
                int all = 1;
                for (int a = 0; a < P->W; ++a) all &= P->flag[w * P->W + a];
                if (all) {
                    /* the averaged tables are no longer the ones the visit
                     * counts of this stage describe: H restarts in both cases */
                    average_window(P, w);
                    if (P->sw[w] == P->K) {
                        P->wdone[w] = 1;
                        for (int a = 0; a < P->W; ++a)
                            memset(P->H[w * P->W + a], 0, sizeof(uint64_t) * (size_t)bins_of(P, w));
                    } else {
                        P->sw[w] += 1;
                        reset_window(P, w);
                    }
                }
            }
            all_done &= P->wdone[w];
            if (P->sw[w] < lowest) lowest = P->sw[w];
        }
        P->s = lowest;
        if (all_done) {
            P->done = 1;
            P->r += 1;
            return;
        }
    }
    or_exchange(P, P->r);
    P->r += 1;
}

/* Run up to n intervals (X trials per walker, then a boundary); returns the
 * number of intervals executed (fewer once the run has finished). */
OR_EXPORT int64_t or_run(or_rewl *P, int64_t n) {
    int64_t k = 0;
    for (; k < n && !P->done; ++k) {
        or_sweep(P, P->X);
        or_boundary(P);
    }
    return k;
}

/* ----------------------------- accessors -------------------------------- */
OR_EXPORT void or_info(const or_rewl *P, int *s, int *done, int64_t *r,
                       int *nwalk) {
    *s = P->s; *done = P->done; *r = P->r; *nwalk = P->nwalk;
}

OR_EXPORT void or_window_of(const or_rewl *P, int w, int *lo, int *hi) {
    *lo = P->lo[w];
    *hi = P->hi[w];
}

OR_EXPORT void or_window_rect(const or_rewl *P, int w, int *elo, int *ehi, int *mlo, int *mhi) {
    *elo = P->elo[w];
    *ehi = P->ehi[w];
    *mlo = P->mlo[w];
    *mhi = P->mhi[w];
}

OR_EXPORT int or_n_windows(const or_rewl *P) { return P->n_win; }

/* ------------------------------------------------------------------------ */
/* Windows in both coordinates (the second alternative of Sec. 2, end).       */
/* The D-6 windows in e and in m form a grid of rectangles; a rectangle is    */
/* kept when it holds a realizable state.  The realizable energies at         */
/* magnetization bin m run from e_min(m) to e_max(m): with k = min(m, N - m), */
/* e_min = P_min/2, P_min = min(2 ceil(2 sqrt k), 2L + 2 [L does not divide   */
/* k] when k >= L) the shortest domain wall around k sites on the torus, and  */
/* e_max = 2k (minority spins on one sublattice).  Between them every bin is  */
/* realizable except next to m = N/2 (one below the top at m = N/2 +- 1; the  */
/* bin above the bottom and the two below the top at m = N/2), as exhaustive  */
/* enumeration shows for L = 4 and 6.                                          */
/* ------------------------------------------------------------------------ */
static void envelope(int L, int m, int *emin, int *emax) {
    int N = L * L, k = m < N - m ? m : N - m;
    int pmin = 0;
    if (k > 0) {
        int t = 0;
        while ((int64_t)t * t < 4 * (int64_t)k) ++t;        /* ceil(2 sqrt k) */
        pmin = 2 * t;
        if (k >= L) {
            int band = 2 * L + (k % L ? 2 : 0);
            if (band < pmin) pmin = band;
        }
    }
    *emin = pmin / 2;
    *emax = 2 * k;
}

static int is_hole(int L, int e, int m) {
    int N = L * L, emin, emax;
    envelope(L, m, &emin, &emax);
    if (m == N / 2) return e == emin + 1 || e == emax - 1 || e == emax - 2;
    if (m == N / 2 - 1 || m == N / 2 + 1) return e == emax - 1;
    return 0;
}

static int rect_has_state(int L, int elo, int ehi, int mlo, int mhi) {
    for (int m = mlo; m <= mhi; ++m) {
        int emin, emax;
        envelope(L, m, &emin, &emax);
        for (int e = elo > emin ? elo : emin; e <= (ehi < emax ? ehi : emax); ++e)
            if (!is_hole(L, e, m)) return 1;
    }
    return 0;
}

OR_EXPORT int or_realizable(int L, int e, int m) {
    int emin, emax;
    envelope(L, m, &emin, &emax);
    return e >= emin && e <= emax && !is_hole(L, e, m);
}

OR_EXPORT or_rewl *or_create_2d(int L, int n_e, int pe, int qe, int n_m, int pm, int qm, int W,
                                int K, int flat_num, int flat_den, int64_t X, uint64_t seed,
                                int init) {
    if (L < 2 || (L & 1) || n_e < 1 || n_m < 1 || qe < 1 || pe < 0 || pe >= qe || qm < 1 ||
        pm < 0 || pm >= qm)
        return NULL;
    int N = L * L, n_grid = n_e * n_m;
    int *keep = calloc((size_t)n_grid, sizeof(int));
    int *glo = calloc((size_t)n_grid * 4, sizeof(int));
    if (!keep || !glo) { free(keep); free(glo); return NULL; }
    int n_win = 0;
    for (int ie = 0; ie < n_e; ++ie)
        for (int im = 0; im < n_m; ++im) {
            int *r = glo + 4 * (ie * n_m + im);
            or_window(N, n_e, pe, qe, ie, &r[0], &r[1]);
            or_window(N, n_m, pm, qm, im, &r[2], &r[3]);
            keep[ie * n_m + im] = rect_has_state(L, r[0], r[1], r[2], r[3]) ? n_win++ : -1;
        }
    or_rewl *P = n_win ? or_create(L, n_win, pe, qe, W, K, flat_num, flat_den, X, seed, init) : NULL;
    if (!P) { free(keep); free(glo); return NULL; }
    P->split = 2;
    P->n_pairs = 0;
    for (int ie = 0; ie < n_e; ++ie)
        for (int im = 0; im < n_m; ++im) {
            int w = keep[ie * n_m + im];
            if (w < 0) continue;
            const int *r = glo + 4 * (ie * n_m + im);
            P->elo[w] = r[0]; P->ehi[w] = r[1]; P->mlo[w] = r[2]; P->mhi[w] = r[3];
            P->lo[w] = r[0]; P->hi[w] = r[1];
            if (ie + 1 < n_e && keep[(ie + 1) * n_m + im] >= 0) {
                P->pa[P->n_pairs] = w; P->pb[P->n_pairs] = keep[(ie + 1) * n_m + im];
                P->pdir[P->n_pairs] = 0; P->palong[P->n_pairs] = ie; P->n_pairs += 1;
            }
            if (im + 1 < n_m && keep[ie * n_m + im + 1] >= 0) {
                P->pa[P->n_pairs] = w; P->pb[P->n_pairs] = keep[ie * n_m + im + 1];
                P->pdir[P->n_pairs] = 1; P->palong[P->n_pairs] = im; P->n_pairs += 1;
            }
        }
    free(keep); free(glo);
    if (alloc_tables(P) != 0) { or_destroy(P); return NULL; }
    return P;
}

OR_EXPORT int64_t or_bins_of_walker(const or_rewl *P, int g) {
    return bins_of(P, win_of(P, g));
}

OR_EXPORT void or_get_walker(const or_rewl *P, int g, int64_t *lng,
                             uint64_t *H, int8_t *spins, int *e, int *m,
                             int64_t *t, int64_t *te, int *flag) {
    int64_t nb = bins_of(P, win_of(P, g));
    if (lng) memcpy(lng, P->lng[g], sizeof(int64_t) * (size_t)nb);
    if (H) memcpy(H, P->H[g], sizeof(uint64_t) * (size_t)nb);
    if (spins) memcpy(spins, P->spin + (size_t)g * P->N, (size_t)P->N);
    *e = P->e[g]; *m = P->m[g]; *t = P->t[g]; *te = P->te[g];
    *flag = P->flag[g];
}

/* Overwrite a walker's table and/or configuration (used by statistical tests
 * that freeze ln g, e.g. the detailed-balance check of Eq. 2).  E and M are
 * recomputed from the spins. */
OR_EXPORT void or_set_walker(or_rewl *P, int g, const int64_t *lng,
                             const int8_t *spins) {
    int64_t nb = bins_of(P, win_of(P, g));
    if (lng) memcpy(P->lng[g], lng, sizeof(int64_t) * (size_t)nb);
    if (spins) {
        memcpy(P->spin + (size_t)g * P->N, spins, (size_t)P->N);
        int E, M;
        or_energy(P->spin + (size_t)g * P->N, P->L, &E, &M);
        P->e[g] = (E + 2 * P->N) / 4;
        P->m[g] = (M + P->N) / 2;
    }
}

/* Overwrite a walker's visit histogram H of the current stage (tests of the */
/* flatness rule on hand-made tables). */
OR_EXPORT void or_set_hist(or_rewl *P, int g, const uint64_t *H) {
    memcpy(P->H[g], H, sizeof(uint64_t) * (size_t)bins_of(P, win_of(P, g)));
}

/* Set the stage index s (ln f = 2^-s) of every window and clear the flatness
 * latches; used by statistical tests that run the walk at a fixed, negligible
 * ln f. */
OR_EXPORT void or_set_stage(or_rewl *P, int s) {
    P->s = s;
    for (int w = 0; w < P->n_win; ++w) P->sw[w] = s;
    for (int g = 0; g < P->nwalk; ++g) P->flag[g] = 0;
}

/* Choose how stages advance (before or_init): 0 = all windows together (the
 * paper, Sec. 2), 1 = each window alone, averaging its walkers' ln g. */
/* Choose which coordinate the windows split (before or_init): 0 = energy,
 * 1 = magnetization (the alternative split the paper names in Sec. 2).  The
 * window bounds are the same D-6 formula over [0, N] either way, so the
 * table sizes do not change. */
OR_EXPORT int or_set_split(or_rewl *P, int split) {
    if ((split != 0 && split != 1) || P->split == 2) return -1;
    P->split = split;
    rects_from_split(P);
    return 0;
}

/* Number of host threads the walker loops may use (0 = leave as is);      */
/* returns the number now in effect.  Results do not depend on it.           */
OR_EXPORT int or_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

OR_EXPORT int or_set_sync(or_rewl *P, int sync) {
    if (sync != 0 && sync != 1) return -1;
    P->sync = sync;
    return 0;
}

OR_EXPORT void or_window_state(const or_rewl *P, int w, int *s, int *done) {
    *s = P->sw[w];
    *done = P->wdone[w];
}
