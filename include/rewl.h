/*
 * rewl.h -- C ABI of the MI355X (gfx950) implementation of two-dimensional
 * replica-exchange Wang-Landau sampling (2D-REWL) of the periodic L x L Ising
 * model, after Valentim et al., arXiv:1508.02748.
 *
 * The calls follow the paper's problem statement (Sec. 2): split the energy
 * range into overlapping windows with the full magnetization range, run
 * Wang-Landau walkers in each window (Eq. 1), check flatness and refine ln f,
 * exchange configurations between adjacent windows (Eq. 2), and finally join
 * the per-walker ln g(E,M) pieces (Eq. 3, Eq. 4).  A second family of calls
 * reweights a joint DOS into ln Z(beta, h) and its derivatives.
 *
 * Conventions shared by every call
 *   - Every call returns rewl_status (0 = OK, < 0 = error); rewl_last_error()
 *     gives a message for the calling thread's most recent error.
 *   - Energy bins e = (E + 2N)/4 in [0, N], magnetization bins m = (M + N)/2
 *     in [0, N] (m = number of up spins); N = L*L, E = -sum_<ij> s_i s_j.
 *   - ln g is int64 fixed point in units of 2^-k_final; ln f at stage s is
 *     2^-s, i.e. 2^(k_final - s) units.  H is the visit count of the current
 *     stage.
 *   - Device memory is owned by the caller: rewl_plan_buffer_sizes() says how
 *     many bytes each buffer needs and rewl_plan_bind() lends the library
 *     device pointers (any allocator; the Python binding uses PyTorch) and a
 *     hipStream_t.  The library never frees them; they must outlive the plan.
 *   - All device work is enqueued on the bound stream.  Only rewl_init,
 *     rewl_query, rewl_query_windows, rewl_read_walker, rewl_merge_lng,
 *     rewl_save, rewl_load and rewl_sweep_times synchronise it (and rewl_run
 *     in the plain form, once per interval).
 *   - A plan is not internally synchronised: call it from one host thread at
 *     a time.  Different plans are independent.  The reweighting calls keep
 *     no state.
 *   - Arguments are validated before any device work (REWL_EINVAL).  A HIP
 *     error surfaces as REWL_EDEVICE; after it the plan answers REWL_ESTATE
 *     to every call but rewl_plan_destroy.
 *   - Results are deterministic: with the same problems and seeds every call
 *     sequence gives bit-identical spins, E, M, ln g and H, whatever the
 *     tuning or form (batched / plain), because every random number is a
 *     Philox4x32-10 draw addressed by (seed, walker, attempt index).
 */
#ifndef REWL_H
#define REWL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    REWL_OK = 0,
    REWL_EINVAL = -1,     /* bad argument, nothing was done */
    REWL_ENOMEM = -2,     /* host allocation failed */
    REWL_EDEVICE = -3,    /* a HIP call or kernel failed */
    REWL_ESTATE = -4,     /* plan not bound / in error / entry walk exceeded its cap */
    REWL_EOVERFLOW = -5,  /* ln g would leave int64 headroom, or a bin has 2^31
                             visits in one stage (its 32-bit count could wrap) */
    REWL_ENOTREADY = -6   /* reserved */
} rewl_status;

/* One REWL simulation -- the paper's problem statement (Sec. 2, Sec. 3). */
typedef struct {
    int32_t L;                   /* even, 4..64: periodic L x L, J = 1, h = 0 while sampling */
    int32_t n_windows;           /* >= 1 windows in the split coordinate (energy: full M
                                    range each, Sec. 3) */
    int32_t overlap_num;         /* overlap of neighbouring windows = num/den, */
    int32_t overlap_den;         /*   e.g. 3/4, or 1/2 as in the paper's runs */
    int32_t walkers_per_window;  /* >= 1, independent g and H each (Sec. 2); <= 256 */
    int32_t k_final;             /* ln f runs 2^0 .. 2^-k_final; 0 <= k_final <= 40 */
    int32_t flat_num;            /* flat iff min H >= num/den * mean H over */
    int32_t flat_den;            /*   visited bins; 4/5 = the paper's 80 % */
    int64_t interval;            /* trials per walker between flatness checks and
                                    exchange rounds; 1 .. 2^30 */
    uint64_t seed;               /* Philox key */
    int32_t init;                /* 0: spins Bernoulli(1/2) from Philox; 1: all +1 */
    int32_t stage_sync;          /* REWL_SYNC_PROBLEM (the paper) or REWL_SYNC_WINDOW */
    int32_t split;               /* REWL_SPLIT_ENERGY (the paper's runs),
                                    REWL_SPLIT_MAGNETIZATION or REWL_SPLIT_BOTH; one
                                    value per plan */
    int32_t m_windows;           /* REWL_SPLIT_BOTH: windows along M (>= 1), with */
    int32_t m_overlap_num;       /*   overlap m_overlap_num / m_overlap_den; the fields */
    int32_t m_overlap_den;       /*   above then describe the windows along E; else 0 */
    int32_t reserved;            /* must be 0 */
} rewl_problem;

/* How ln f is refined (rewl_problem.stage_sync).
 *   REWL_SYNC_PROBLEM: once every walker of the problem is flat, all windows
 *     move to the next stage together (Sec. 2); flatness at the last stage
 *     ends the problem.
 *   REWL_SYNC_WINDOW: a window whose walkers are all flat first averages their
 *     ln g -- in every bin some walker of the window has visited, all walkers
 *     take floor(mean over the walkers that visited it), other bins stay 0 --
 *     and moves to its next stage alone; its last stage ends it, after which
 *     its walkers make no trials and its window pairs do not exchange; the
 *     problem ends with its last window.  (The common REWL form the paper
 *     cites, Sec. 1; not the paper's own runs.) */
enum { REWL_SYNC_PROBLEM = 0, REWL_SYNC_WINDOW = 1 };

/* Which coordinate the windows split (rewl_problem.split).
 *   REWL_SPLIT_ENERGY: windows over the energy bins e, each with the full
 *     magnetization range (Sec. 2, Sec. 3; the paper's runs).  A walker's
 *     tables are indexed [e - lo][m].
 *   REWL_SPLIT_MAGNETIZATION: windows over the magnetization bins m with the
 *     same overlapping-window formula, each keeping every energy (the
 *     alternative split named at the end of Sec. 2).  A proposal leaving the
 *     window in m is rejected; the entry walk and the exchange overlap test
 *     use m.  Tables are indexed [e][m - lo].
 *   REWL_SPLIT_BOTH: windows in both coordinates (the second alternative of
 *     Sec. 2): the n_windows energy windows times the m_windows magnetization
 *     windows form a grid of rectangles, of which only those holding a state
 *     are kept (closed-form support of the (e, m) plane: with k = min(m, N-m)
 *     minority spins the energy bins run from half the shortest domain wall
 *     around k sites on the torus to 2k, every bin between holding a state
 *     except three next to m = N/2).  Kept rectangles are numbered e-major
 *     (rewl_window_rect gives them).  A proposal leaving the rectangle is
 *     rejected; the entry walk's distance is the sum of both coordinates'
 *     distances; neighbours exchange along E on rounds r with bit 1 of r
 *     clear and along M otherwise, pairs whose lower window's grid index
 *     along that direction is r (mod 2).  Tables are indexed [e - e_lo][m -
 *     m_lo].
 * All problems of one plan use the same split. */
enum { REWL_SPLIT_ENERGY = 0, REWL_SPLIT_MAGNETIZATION = 1, REWL_SPLIT_BOTH = 2 };

/* Execution form and tuning.  None of these change results. */
enum { REWL_FORM_BATCHED = 0, REWL_FORM_PLAIN = 1 };
typedef struct {
    int32_t form;             /* REWL_FORM_BATCHED: all problems, windows and walkers
                                 in one launch per interval, device-side stage
                                 control, intervals replayed from a HIP graph;
                                 REWL_FORM_PLAIN: one launch per window and a host
                                 round trip per interval */
    int32_t walkers_per_wg;   /* 64, 128 or 256 lanes (= walkers) per workgroup; 0 = auto */
    int32_t graph_intervals;  /* intervals captured per graph (batched); 0 = auto */
    int32_t grid_waves_per_cu;/* persistent grid: at most this many wavefronts per CU, each
                                 running its tiles of walkers in turn; 0 = auto */
    int32_t profile;          /* 1: start with profiling on (see rewl_set_profile) */
    int32_t walkers_per_wave; /* 1..64 lanes of each wavefront carry a walker; fewer spread
                                 a small batch over more CUs; 0 = 64 */
    int32_t table_layout;     /* REWL_LAYOUT_DENSE or REWL_LAYOUT_BAND (below); fixed when
                                 the plan is created */
    int32_t audit_shift;      /* the stage visit counts are audited once per
                                 2^audit_shift stage trials of a walker; 0 = 30 (24 for
                                 packed layouts), else 1..30 (1..24); every interval
                                 must be at most 2^audit_shift.
                                 An audit stops the run (REWL_EOVERFLOW) once a bin has
                                 2^(audit_shift + 1) visits in one stage, so a small
                                 value only tests that guard.  Fixed when the plan is
                                 created. */
} rewl_tuning;

/* How each walker's tables are stored (rewl_tuning.table_layout).  All
 * layouts hold the same values; they differ in memory and addressing only.
 * Bit 0 selects the band, bit 1 packed words.
 *   REWL_LAYOUT_DENSE: every bin of the window's rectangle.
 *   REWL_LAYOUT_BAND (energy split): each row of 4 energy bins keeps only
 *     the magnetization band [ceil(e/2), N - ceil(e/2)] of its lowest energy
 *     e, which holds every realizable state of the row (a state with energy
 *     bin e has at least e/2 minority spins); all rows of a window keep the
 *     width of its widest row.  (magnetization split) each window keeps only
 *     the energy rows up to 2 k_max, k_max the largest minority-spin count
 *     of its magnetization bins.  About half the memory of the dense layout
 *     over all windows.
 *   ..._PACKED: one 64-bit word per bin (8 B instead of 12) holding ln g in
 *     bits 63..26 and a 26-bit stage base in bits 25..0.  Needs k_final <= 24
 *     and interval <= 2^24 (audit_shift <= 24, default 24); a run stops with
 *     REWL_EOVERFLOW once some ln g reaches 2^37 units (at least 8192 in ln g)
 *     or a bin has 2^(audit_shift + 1) visits in one stage. */
enum {
    REWL_LAYOUT_DENSE = 0,
    REWL_LAYOUT_BAND = 1,
    REWL_LAYOUT_DENSE_PACKED = 2,
    REWL_LAYOUT_BAND_PACKED = 3
};

/* Buffers the caller provides (device memory). */
enum {
    REWL_BUF_TABLES = 0,  /* ln g (int64, 8 B per bin) of each walker's window table
                             (4 x 4 tiles of (e, m)), then the stage base (uint32,
                             4 B per bin, same bin order): the stage's visit count
                             is H = (ln g >> (K - s)) - base mod 2^32; 12 B per bin.
                             Packed layouts: one word per bin, 8 B. */
    REWL_BUF_SPINS = 1,   /* bit-packed configurations */
    REWL_BUF_STATE = 2,   /* descriptors, walker and problem state, scratch */
    REWL_NBUF = 3
};

typedef struct rewl_plan rewl_plan;

/* Validate problems, compute windows (Sec. 2, Fig. 1(b)) and buffer sizes.
 * `tuning` may be NULL (batched form, automatic choices).  n_problems >= 1. */
rewl_status rewl_plan_create(const rewl_problem* problems, int32_t n_problems,
                             const rewl_tuning* tuning, rewl_plan** out);
void rewl_plan_destroy(rewl_plan* plan);

/* Bytes per buffer (sizes_out has REWL_NBUF entries). */
rewl_status rewl_plan_buffer_sizes(const rewl_plan* plan, size_t* sizes_out);

/* Lend device buffers (REWL_NBUF pointers, 256-byte aligned, at least the
 * sizes above) and the hipStream_t to enqueue on (NULL = default stream). */
rewl_status rewl_plan_bind(rewl_plan* plan, void* const* dev_ptrs, void* hip_stream);

/* Bounds [lo, hi] of window w of problem prob, in energy bins (energy split)
 * or magnetization bins (magnetization split). */
rewl_status rewl_window_bounds(const rewl_plan* plan, int32_t prob, int32_t w,
                               int32_t* e_lo, int32_t* e_hi);

/* Rectangle [e_lo, e_hi] x [m_lo, m_hi] (energy and magnetization bins) of
 * window w of problem prob, for any split. */
rewl_status rewl_window_rect(const rewl_plan* plan, int32_t prob, int32_t w, int32_t* e_lo,
                             int32_t* e_hi, int32_t* m_lo, int32_t* m_hi);

/* Windows of problem prob (for REWL_SPLIT_BOTH the kept rectangles). */
rewl_status rewl_plan_windows(const rewl_plan* plan, int32_t prob, int32_t* n_windows);

/* Counts of the plan: problems, walkers in total. */
rewl_status rewl_plan_counts(const rewl_plan* plan, int32_t* n_problems, int64_t* n_walkers);

/* Initial configurations and entry of every walker into its window
 * (Metropolis at unit temperature on the distance to the window); zeroes all
 * tables.  Synchronises.  REWL_ESTATE if a walker needs more than 2^40 entry
 * trials. */
rewl_status rewl_init(rewl_plan* plan);

/* n_intervals x { interval trials per walker (Eq. 1 walk), flatness check and
 * ln f reduction, exchange round (Eq. 2) }.  Problems that have finished stop
 * changing.  Enqueued (the plain form synchronises once per interval). */
rewl_status rewl_run(rewl_plan* plan, int64_t n_intervals);

/* The three parts of an interval, separately: n trials per walker of every
 * unfinished problem (enqueued in pieces of at most 2^30 trials, each followed
 * by the audit of the 32-bit stage visit counts); the flatness check and
 * stage advance ("reduce ln f"); the exchange round of the boundary last
 * closed by rewl_reduce_lnf. */
rewl_status rewl_sweep(rewl_plan* plan, int64_t n_trials);
rewl_status rewl_reduce_lnf(rewl_plan* plan);
rewl_status rewl_exchange(rewl_plan* plan);

/* Per problem: stage s (the lowest stage of its windows), done flag, trials
 * made per walker of its first window.  Arrays of n_problems entries; any may
 * be NULL.  Synchronises. */
rewl_status rewl_query(rewl_plan* plan, int32_t* stage_out, int32_t* done_out,
                       int64_t* trials_out);

/* Per window of problem prob (arrays of n_windows): the stage index (ln f =
 * 2^-stage), whether the window has finished, and its walkers' trial count.
 * With REWL_SYNC_PROBLEM all windows share one stage.  Synchronises. */
rewl_status rewl_query_windows(rewl_plan* plan, int32_t prob, int32_t* stage_out, int32_t* done_out,
                               int64_t* trials_out);

/* State of walker a of window w of problem prob.  lng and H (nullable) get the
 * window table with cap_bins entries of room: (hi - lo + 1) x (N + 1)
 * row-major by (e - lo, m) for the energy split, (N + 1) x (hi - lo + 1) by
 * (e, m - lo) for the magnetization split; spins (nullable) gets N bytes +1/-1 in row-major
 * site order; e, m, t (nullable) the current bins and trial count.
 * Synchronises. */
rewl_status rewl_read_walker(rewl_plan* plan, int32_t prob, int32_t w, int32_t a,
                             int64_t* lng, uint64_t* H, size_t cap_bins, int8_t* spins,
                             int32_t* e, int32_t* m, int64_t* t);

/* Joining the fragments of problem prob into one joint DOS (Sec. 2):
 * walkers of a window are aligned on their mean over the bins all of them
 * visited and averaged; Eq. (3) gives each window's ln g(E) = log sum_M g;
 * the matching point E_mat of neighbouring windows minimises the difference
 * of beta(E) = d ln g / dE (central differences (ln g(E+4) - ln g(E-4))/8)
 * over their overlap, at or above the previous matching point, ties to the
 * lowest E; the upper window is shifted by one constant to agree there and
 * Eq. (4) takes the lower window below E_mat and the upper from E_mat on.
 * Other splits (the alternatives of Sec. 2) join in two steps: first the
 * windows sharing one magnetization range, by energy as above, then these
 * magnetization columns along M by the same rule on their marginals over E,
 * ln g(M) = log sum_E g (the column below M_mat from the lower one).  A
 * magnetization split is one window per column; an energy split one column.
 * norm 0: ln g(E = -2N) = ln 2 (the two ground states); 1: sum g = 2^N.
 * Device outputs: lng_out (N+1) x (N+1) float64 by (e, m), -inf where no
 * walker visited; lnge_out (N+1) the marginal ln g(E) of that table;
 * e_mat_out (nullable) the rewl_merge_points matching points: for
 * one-coordinate splits the n_windows - 1 points of consecutive windows (E_mat,
 * or M_mat for magnetization windows); for windows in both coordinates, per
 * window the E_mat at which it starts in its column (-1 for the lowest
 * window of a column), then the M_mat of every column but the first;
 * lng_err_out (nullable) (N+1) x (N+1) error bars: per bin, the standard
 * error of the window average over the walkers that visited it
 * (sqrt(sum (x_a - mean)^2 / (n (n-1))) of the aligned values, i.e. the
 * leave-one-walker-out jackknife error with the alignment held fixed; Sec. 2
 * notes that several walkers per window make error bars possible), taken from
 * the window that supplies the bin in Eq. (4); NaN where fewer than two
 * walkers visited.  `workspace` is device memory of
 * rewl_merge_workspace_size bytes.  Synchronises; REWL_ESTATE when a
 * window's walkers share no visited bin or two pieces have no usable
 * matching point. */
rewl_status rewl_merge_points(const rewl_plan* plan, int32_t prob, int32_t* n_points);
rewl_status rewl_merge_workspace_size(const rewl_plan* plan, int32_t prob, size_t* bytes);
rewl_status rewl_merge_lng(rewl_plan* plan, int32_t prob, int32_t norm, void* workspace, size_t workspace_bytes,
                           double* lng_out, double* lnge_out, int32_t* e_mat_out, double* lng_err_out);

/* Reweighting of a joint DOS (float64 ln g over bins (e, m), -inf = not
 * visited) into ln Z(beta, h) = log sum exp(ln g - beta E + beta h M) at G
 * grid points; all pointers are device pointers.  lng is nE x nM row-major for
 * e = e0 .. e0+nE-1, m = m0 .. m0+nM-1 of a lattice of N spins.  beta, h, lnz
 * have G entries. */
rewl_status rewl_lnz_forward(const double* lng, int32_t N, int32_t e0, int32_t nE,
                             int32_t m0, int32_t nM, const double* beta, const double* h,
                             int64_t G, double* lnz, void* hip_stream);

/* Backward of rewl_lnz_forward.  order 1: with the saved lnz and upstream
 * grad_out, writes grad_beta = g <-E + hM>, grad_h = g beta <M> (each G
 * entries) and, if grad_lng is not NULL, grad_lng = sum_g g p_g(E,M)
 * (nE x nM).  order 2: writes, per grid point, the first moments and the
 * covariances needed for second derivatives into mom (G x 5 doubles:
 * <M>, <U>, Var(U), Var(M), Cov(U,M), U = -E + hM); grad pointers unused. */
rewl_status rewl_lnz_backward(const double* lng, int32_t N, int32_t e0, int32_t nE,
                              int32_t m0, int32_t nM, const double* beta, const double* h,
                              int64_t G, const double* lnz, const double* grad_out,
                              double* grad_beta, double* grad_h, double* grad_lng,
                              double* mom, int32_t order, void* hip_stream);

/* Second order: the backward of rewl_lnz_backward's (grad_beta, grad_h) with
 * respect to (grad_out, beta, h), so that specific heat and susceptibility
 * come out as gradients of gradients (d2 ln Z / d beta2 = Var(U), d2 ln Z /
 * d h2 = beta^2 Var(M), d2 ln Z / d beta d h = <M> + beta Cov(U, M), U = -E
 * + h M).  Inputs per grid point (G entries, device): grad_out g (NULL =
 * all ones) and the upstream gradients a of grad_beta and c of grad_h (each
 * NULL = zeros).  Outputs (G entries each, required):
 *   d_grad_out = a <U> + c beta <M>
 *   d_beta     = g (a Var(U) + c (<M> + beta Cov(U, M)))
 *   d_h        = g (a (<M> + beta Cov(U, M)) + c beta^2 Var(M)).
 * Dependence on ln g is not differentiated.  Enqueued on hip_stream. */
rewl_status rewl_lnz_backward2(const double* lng, int32_t N, int32_t e0, int32_t nE,
                               int32_t m0, int32_t nM, const double* beta, const double* h,
                               int64_t G, const double* lnz, const double* grad_out,
                               const double* up_beta, const double* up_h, double* d_grad_out,
                               double* d_beta, double* d_h, void* hip_stream);

/* Reweighting on a tensor-product grid beta[0..nB) x h[0..nH): lnz[i*nH + j]
 * = ln Z(beta[i], h[j]), the same quantity as rewl_lnz_forward at those
 * points (equal up to the order of rounding).  The sum is factorised through
 * the M columns: A(i, M) = log sum_E exp(ln g - beta_i E) does not depend on
 * h, and ln Z = log sum_M exp(A(i, M) + beta_i h_j M); this needs
 * nB nE nM + nB nH nM exponentials instead of nB nH nE nM.  Geometry as for
 * rewl_lnz_forward; all arrays are device memory; `workspace` holds
 * rewl_lnz_grid_workspace_size bytes (caller-owned, contents not kept
 * between calls).  nB <= 65535.  Enqueued on hip_stream. */
rewl_status rewl_lnz_grid_workspace_size(int32_t nM, int64_t nB, int64_t nH, size_t* bytes);
rewl_status rewl_lnz_grid_forward(const double* lng, int32_t N, int32_t e0, int32_t nE,
                                  int32_t m0, int32_t nM, const double* beta, int64_t nB,
                                  const double* h, int64_t nH, void* workspace, size_t workspace_bytes,
                                  double* lnz, void* hip_stream);

/* rewl_lnz_grid_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the workspace is a fixed array of REWL_NOALLOC_SCRATCH_BYTES of
 * device memory that the library holds on each GPU it runs on until the
 * process ends, so the call allocates nothing.  Needs nB * nM * 8 <=
 * REWL_NOALLOC_SCRATCH_BYTES (REWL_EINVAL otherwise).  All calls on one GPU
 * share that array: calls that overlap in time on one GPU (on different
 * streams, or from several threads without ordering) race and may corrupt
 * each other's results; calls ordered on one stream are safe.  Inputs,
 * outputs and the result as for rewl_lnz_grid_forward (same kernels). */
#define REWL_NOALLOC_SCRATCH_BYTES (64ull << 20)
rewl_status rewl_lnz_grid_forward_noalloc(const double* lng, int32_t N, int32_t e0, int32_t nE,
                                          int32_t m0, int32_t nM, const double* beta, int64_t nB,
                                          const double* h, int64_t nH, double* lnz, void* hip_stream);

/* Backward of rewl_lnz_grid_forward with the saved lnz (nB x nH) and upstream
 * grad_out (nB x nH, NULL = all ones).  grad_beta (nB) = sum_j g_ij <-E + h_j M>_ij
 * and grad_h (nH) = sum_i g_ij beta_i <M>_ij (both or neither); grad_lng
 * (nE x nM, nullable) = sum_ij g_ij p_ij(E, M); mom (nullable, nB x nH x 5)
 * = <M>, <U>, Var(U), Var(M), Cov(U, M) per point, U = -E + h M, as in
 * rewl_lnz_backward order 2.  Variances use the law of total variance over
 * the M columns, with central sums throughout.  At least one output is
 * required. */
rewl_status rewl_lnz_grid_backward(const double* lng, int32_t N, int32_t e0, int32_t nE,
                                   int32_t m0, int32_t nM, const double* beta, int64_t nB,
                                   const double* h, int64_t nH, const double* lnz,
                                   const double* grad_out, void* workspace, size_t workspace_bytes,
                                   double* grad_beta, double* grad_h, double* grad_lng, double* mom,
                                   void* hip_stream);

/* Second order on a tensor-product grid: the backward of
 * rewl_lnz_grid_backward's (grad_beta (nB), grad_h (nH)) given their upstream
 * gradients up_beta (nB) and up_h (nH) (each NULL = zeros) and the first
 * order's grad_out (nB x nH, NULL = all ones).  Per point (i, j) the terms of
 * rewl_lnz_backward2 with a = up_beta[i], c = up_h[j]; outputs d_grad_out
 * (nB x nH), d_beta[i] = sum_j of the point terms, d_h[j] = sum_i of them
 * (fixed summation order).  `workspace` as for rewl_lnz_grid_forward.
 * Enqueued on hip_stream. */
rewl_status rewl_lnz_grid_backward2(const double* lng, int32_t N, int32_t e0, int32_t nE,
                                    int32_t m0, int32_t nM, const double* beta, int64_t nB,
                                    const double* h, int64_t nH, const double* lnz,
                                    const double* grad_out, const double* up_beta,
                                    const double* up_h, void* workspace, size_t workspace_bytes,
                                    double* d_grad_out, double* d_beta, double* d_h,
                                    void* hip_stream);

/* Replace the tuning of a plan (same form); results do not change. */
rewl_status rewl_set_tuning(rewl_plan* plan, const rewl_tuning* tuning);

/* Checkpoint / resume at an interval boundary.  The Philox counters are part
 * of the state, so a resumed run continues bit for bit.  rewl_save writes
 * the problems and all three device buffers into a host blob of
 * rewl_save_size bytes (synchronises); rewl_load restores them into a plan
 * created from the same problems and bound to its own buffers (synchronises);
 * REWL_EINVAL for a truncated blob or one saved from other problems. */
rewl_status rewl_save_size(const rewl_plan* plan, size_t* bytes);
rewl_status rewl_save(rewl_plan* plan, void* blob, size_t cap, size_t* used);
rewl_status rewl_load(rewl_plan* plan, const void* blob, size_t size);

/* Profiling of the batched form: while on, rewl_run enqueues its intervals
 * one launch at a time (not from the graph) with a HIP event pair around
 * every sweep kernel; rewl_sweep_times then gives those kernels' durations
 * (ms) for the most recent rewl_run, in launch order, writing min(cap, count)
 * values and the count, and synchronises.  Results are unchanged. */
rewl_status rewl_set_profile(rewl_plan* plan, int32_t on);
rewl_status rewl_sweep_times(rewl_plan* plan, float* ms, int32_t cap, int32_t* count);

const char* rewl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* REWL_H */
