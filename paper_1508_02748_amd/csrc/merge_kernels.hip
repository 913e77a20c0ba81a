// merge_kernels.hip -- joining the per-walker ln g(E,M) fragments of one REWL
// problem into a joint density of states (Sec. 2, Eq. 3 and Eq. 4), float64.
//
// The windows are joined in two steps.  First, within each magnetization
// column (the windows sharing one magnetization range, ordered by energy),
// along E as the paper joins its energy windows; then the joined columns along
// M in the same way with the roles of E and M exchanged (the alternative
// splits of Sec. 2).  An energy split is one column of all windows; a
// magnetization split has one window per column.
//
//   k_merge_window   one workgroup per window: each walker is aligned on its
//                    mean over the bins every walker of the window has visited
//                    (exact int128 sums), then ln g is averaged over the
//                    walkers that visited each bin, with the standard error of
//                    that average over the walkers (the leave-one-walker-out
//                    jackknife error with the alignment held fixed; NaN below
//                    two walkers) stored after the window's averages.
//   k_merge_marg_rows one wavefront per (window, energy row): Eq. (3) over the
//                    window's magnetizations, ln g(E) = log sum_M g(E, M).
//   k_merge_join_e   one thread per column: for each energy-neighbouring pair
//                    the matching energy E_mat minimises the difference of
//                    beta(E) = d ln g / dE (central differences) over the
//                    overlap, at or above the previous matching point, ties to
//                    the lowest E; the upper window is shifted to agree at E_mat.
//   k_merge_marg_cols one wavefront per (column, magnetization): the joined
//                    column's marginal over E, ln g(M).
//   k_merge_join_m   one thread: the same rule along M between the columns.
//   k_merge_fill     Eq. (4) in both steps: bin (e, m) comes from the column
//                    whose matching interval in m contains m, and within it
//                    from the window whose matching interval in e contains e.
//   k_merge_rows / k_merge_norm   row marginals of the joint table and the
//                    normalisation (ground-state count g(-2N) = 2, or
//                    sum g = 2^N).
#include <hip/hip_runtime.h>

#include <math.h>

#include "rewl_internal.h"

namespace rewl {
namespace {

__device__ __forceinline__ int64_t lng_at(const DevState& S, const WDesc& d, int er, int mc) {
    const int64_t i = table_index_or_none(d, d.e0 + er, d.m0 + mc);
    return i < 0 ? 0 : rewl::lng_at(S, d.table_off + static_cast<uint64_t>(i));
}

struct GeoView {
    const MergeGeo& G;
    __device__ int col(int w) const { return G.iws[G.off_col + w]; }
    __device__ int ematA(int w) const { return G.iws[G.off_ematA + w]; }
    __device__ int first(int c) const { return G.iws[G.off_first + c]; }
    __device__ int count(int c) const { return G.iws[G.off_count + c]; }
    __device__ int cmlo(int c) const { return G.iws[G.off_cmlo + c]; }
    __device__ int cmhi(int c) const { return G.iws[G.off_cmhi + c]; }
    __device__ int mmat(int c) const { return G.iws[G.off_mmat + c]; }
    __device__ int member(int k) const { return G.iws[G.off_members + k]; }
    __device__ int elo(int w) const { return G.iws[G.off_rect + 4 * w]; }
    __device__ int ehi(int w) const { return G.iws[G.off_rect + 4 * w + 1]; }
    __device__ int mlo(int w) const { return G.iws[G.off_rect + 4 * w + 2]; }
    __device__ int mhi(int w) const { return G.iws[G.off_rect + 4 * w + 3]; }
};

__global__ void __launch_bounds__(256) k_merge_window(DevState S, MergeGeo G) {
    const int w = blockIdx.x;
    const GeoView V{G};
    const int W = G.W, nMw = V.mhi(w) - V.mlo(w) + 1;
    const PDesc P = S.pd[G.prob];
    const int g0 = P.walker_off + w * W;
    const int nE = V.ehi(w) - V.elo(w) + 1;
    const int64_t nb = static_cast<int64_t>(nE) * nMw;
    const double unit = ldexp(1.0, -G.K);
    double* shift = G.ws + G.off_shift + static_cast<int64_t>(w) * W;
    for (int e = threadIdx.x; e <= G.N; e += blockDim.x) G.ws[G.off_margA + static_cast<int64_t>(w) * (G.N + 1) + e] = -INFINITY;
    __shared__ unsigned long long red_lo[256], red_hi[256];
    __shared__ long long red_n[256];
    // alignment constants: mean of each walker's ln g over the common bins
    for (int a = 0; a < W; ++a) {
        const WDesc da = S.wd[g0 + a];
        unsigned __int128 acc = 0;
        long long cnt = 0;
        for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
            const int er = static_cast<int>(i / nMw), mc = static_cast<int>(i % nMw);
            bool common = true;
            for (int b = 0; b < W && common; ++b) common = lng_at(S, S.wd[g0 + b], er, mc) > 0;
            if (common) {
                acc += static_cast<unsigned __int128>(static_cast<uint64_t>(lng_at(S, da, er, mc)));
                ++cnt;
            }
        }
        red_lo[threadIdx.x] = static_cast<unsigned long long>(acc);
        red_hi[threadIdx.x] = static_cast<unsigned long long>(acc >> 64);
        red_n[threadIdx.x] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned __int128 tot = 0;
            long long n = 0;
            for (int k = 0; k < static_cast<int>(blockDim.x); ++k) {
                tot += (static_cast<unsigned __int128>(red_hi[k]) << 64) | red_lo[k];
                n += red_n[k];
            }
            // mean in ln units: the exact sum rounded once, divided once
            const double mean = n > 0 ? (static_cast<double>(tot) * unit) / static_cast<double>(n) : 0.0;
            shift[a] = mean;
            if (n == 0) G.iws[0] = 1;
        }
        __syncthreads();
    }
    // window average over the walkers that visited each bin
    double* avg = G.ws + G.avg_off[w];
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
        const int er = static_cast<int>(i / nMw), mc = static_cast<int>(i % nMw);
        double num = 0.0;
        int cnt = 0;
        for (int a = 0; a < W; ++a) {
            const int64_t l = lng_at(S, S.wd[g0 + a], er, mc);
            if (l > 0) {
                num += static_cast<double>(l) * unit - shift[a];
                ++cnt;
            }
        }
        const double mean = cnt > 0 ? num / cnt : -INFINITY;
        avg[i] = mean;
        double ss = 0.0;
        for (int a = 0; a < W; ++a) {
            const int64_t l = lng_at(S, S.wd[g0 + a], er, mc);
            if (l > 0) {
                const double dv = (static_cast<double>(l) * unit - shift[a]) - mean;
                ss += dv * dv;
            }
        }
        avg[nb + i] = cnt > 1 ? sqrt(ss / (static_cast<double>(cnt) * (cnt - 1))) : NAN;
    }
}

// log sum exp of n values x[0], x[stride], ..., one wavefront.
__device__ double wave_lse(const double* x, int n, int64_t stride = 1) {
    const int lane = threadIdx.x & 63;
    double mx = -INFINITY;
    for (int i = lane; i < n; i += 64) mx = fmax(mx, x[i * stride]);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (!(mx > -INFINITY)) return -INFINITY;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += exp(x[i * stride] - mx);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    return mx + log(s);
}

__global__ void __launch_bounds__(64) k_merge_marg_rows(MergeGeo G) {
    const int w = blockIdx.y, er = blockIdx.x;
    const GeoView V{G};
    if (er > V.ehi(w) - V.elo(w)) return;
    const int nMw = V.mhi(w) - V.mlo(w) + 1;
    const double v = wave_lse(G.ws + G.avg_off[w] + static_cast<int64_t>(er) * nMw, nMw);
    if (threadIdx.x == 0) G.ws[G.off_margA + static_cast<int64_t>(w) * (G.N + 1) + V.elo(w) + er] = v;
}

__device__ __forceinline__ double beta_c(const double* g, int x, int N) {
    if (x < 1 || x + 1 > N) return NAN;
    const double a = g[x - 1], b = g[x], c = g[x + 1];
    if (!(a > -INFINITY) || !(b > -INFINITY) || !(c > -INFINITY)) return NAN;
    return (c - a) / 8.0;
}

// Sequential join of n pieces along one coordinate (Eq. 3 - 4): piece k covers
// [lo(k), hi(k)] and has marginal marg(k) (length N + 1, -inf outside).  run is
// scratch of N + 1 values; writes each piece's matching point (its lo for the
// first) and additive constant; returns false when a pair has no usable point.
template <class Lo, class Hi, class Marg>
__device__ bool join_pieces(int n, int N, Lo lo, Hi hi, Marg marg, double* run, int32_t* mat, double* shift) {
    const double* m0 = marg(0);
    for (int x = 0; x <= N; ++x) run[x] = (x >= lo(0) && x <= hi(0)) ? m0[x] : -INFINITY;
    shift[0] = 0.0;
    mat[0] = lo(0);
    int cur_hi = hi(0), prev = 0;
    for (int j = 1; j < n; ++j) {
        const double* mj = marg(j);
        double best = INFINITY;
        int at = -1;
        for (int x = (lo(j) > prev ? lo(j) : prev); x <= cur_hi; ++x) {
            const double bi = beta_c(run, x, N), bj = beta_c(mj, x, N);
            if (isnan(bi) || isnan(bj)) continue;
            const double dd = fabs(bi - bj);
            if (dd < best) {
                best = dd;
                at = x;
            }
        }
        if (at < 0) return false;
        const double c = run[at] - mj[at];
        shift[j] = c;
        mat[j] = at;
        for (int x = at; x <= N; ++x) run[x] = (x <= hi(j)) ? mj[x] + c : -INFINITY;
        cur_hi = hi(j);
        prev = at;
    }
    return true;
}

__global__ void __launch_bounds__(64) k_merge_join_e(MergeGeo G) {
    const int c = blockIdx.x;
    if (threadIdx.x != 0 || c >= G.ncol) return;
    const GeoView V{G};
    const int f = V.first(c), n = V.count(c), N = G.N;
    auto lo = [&](int k) { return V.elo(V.member(f + k)); };
    auto hi = [&](int k) { return V.ehi(V.member(f + k)); };
    auto marg = [&](int k) {
        return static_cast<const double*>(G.ws + G.off_margA + static_cast<int64_t>(V.member(f + k)) * (N + 1));
    };
    // the join writes in member order (staging slots f .. f+n-1), then per window
    int32_t* smat = G.iws + G.off_stage + f;
    double* ssh = G.ws + G.off_stageA + f;
    if (!join_pieces(n, N, lo, hi, marg, G.ws + G.off_runA + static_cast<int64_t>(c) * (N + 1), smat, ssh)) {
        G.iws[0] = 2;
        return;
    }
    for (int k = 0; k < n; ++k) {
        G.iws[G.off_ematA + V.member(f + k)] = smat[k];
        G.ws[G.off_shiftA + V.member(f + k)] = ssh[k];
    }
}

// Value of the column c's joined table at (e, m) (before the join along M), with
// the error of the supplying window.
__device__ __forceinline__ double column_value(const MergeGeo& G, const GeoView& V, int c, int e, int m, double* err) {
    const int f = V.first(c), n = V.count(c);
    int w = V.member(f);
    for (int k = 1; k < n; ++k)
        if (e >= V.ematA(V.member(f + k))) w = V.member(f + k);
    if (e < V.elo(w) || e > V.ehi(w) || m < V.mlo(w) || m > V.mhi(w)) {
        if (err) *err = NAN;
        return -INFINITY;
    }
    const int nMw = V.mhi(w) - V.mlo(w) + 1;
    const int64_t nb = static_cast<int64_t>(V.ehi(w) - V.elo(w) + 1) * nMw;
    const int64_t k = G.avg_off[w] + static_cast<int64_t>(e - V.elo(w)) * nMw + (m - V.mlo(w));
    if (err) *err = G.ws[k + nb];
    return G.ws[k] + G.ws[G.off_shiftA + w];
}

__global__ void __launch_bounds__(64) k_merge_marg_cols(MergeGeo G) {
    const int c = blockIdx.y, mc = blockIdx.x;
    const GeoView V{G};
    const int m = V.cmlo(c) + mc;
    if (m > V.cmhi(c)) return;
    const int lane = threadIdx.x & 63, N = G.N;
    double mx = -INFINITY;
    for (int e = lane; e <= N; e += 64) mx = fmax(mx, column_value(G, V, c, e, m, nullptr));
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    double v = -INFINITY;
    if (mx > -INFINITY) {
        double s = 0.0;
        for (int e = lane; e <= N; e += 64) s += exp(column_value(G, V, c, e, m, nullptr) - mx);
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        v = mx + log(s);
    }
    if (lane == 0) G.ws[G.off_margB + static_cast<int64_t>(c) * (N + 1) + m] = v;
}

// Column marginals start empty; a single column needs no join along M.
__global__ void __launch_bounds__(64) k_merge_init_margB(MergeGeo G) {
    const int c = blockIdx.x;
    for (int m = threadIdx.x; m <= G.N; m += blockDim.x) G.ws[G.off_margB + static_cast<int64_t>(c) * (G.N + 1) + m] = -INFINITY;
    if (c == 0 && threadIdx.x == 0) {
        G.ws[G.off_shiftB] = 0.0;
        G.iws[G.off_mmat] = G.iws[G.off_cmlo];
    }
}

// The matching points, for the caller: one-coordinate splits give the n - 1
// matching points of consecutive windows (E_mat, or M_mat for windows in m);
// windows in both coordinates give, per window, the E_mat at which it starts
// within its column (-1 for the column's lowest window), then the M_mat of
// each column after the first.
__global__ void k_merge_points(MergeGeo G, int split, int32_t* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const GeoView V{G};
    if (split == 0) {
        for (int j = 1; j < G.nwin; ++j) out[j - 1] = V.ematA(j);
    } else if (split == 1) {
        for (int j = 1; j < G.ncol; ++j) out[j - 1] = V.mmat(j);
    } else {
        for (int w = 0; w < G.nwin; ++w) out[w] = V.member(V.first(V.col(w))) == w ? -1 : V.ematA(w);
        for (int j = 1; j < G.ncol; ++j) out[G.nwin + j - 1] = V.mmat(j);
    }
}

__global__ void k_merge_join_m(MergeGeo G) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const GeoView V{G};
    const int N = G.N;
    auto lo = [&](int c) { return V.cmlo(c); };
    auto hi = [&](int c) { return V.cmhi(c); };
    auto marg = [&](int c) { return static_cast<const double*>(G.ws + G.off_margB + static_cast<int64_t>(c) * (N + 1)); };
    if (!join_pieces(G.ncol, N, lo, hi, marg, G.ws + G.off_runB, G.iws + G.off_mmat, G.ws + G.off_shiftB)) G.iws[0] = 2;
}

__global__ void __launch_bounds__(256) k_merge_fill(MergeGeo G, double* out, double* err) {
    const int N = G.N, nM = N + 1;
    const int64_t total = static_cast<int64_t>(nM) * nM;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const GeoView V{G};
    const int e = static_cast<int>(i / nM), m = static_cast<int>(i % nM);
    int c = 0;
    for (int k = 1; k < G.ncol; ++k)
        if (m >= V.mmat(k)) c = k;
    double ev = NAN, v = -INFINITY;
    if (m >= V.cmlo(c) && m <= V.cmhi(c)) {
        v = column_value(G, V, c, e, m, &ev);
        v = v + G.ws[G.off_shiftB + c];
    }
    out[i] = v;
    if (err) err[i] = ev;
}

__global__ void __launch_bounds__(64) k_merge_rows(int N, const double* joint, double* rows) {
    const int e = blockIdx.x;
    const double v = wave_lse(joint + static_cast<int64_t>(e) * (N + 1), N + 1);
    if (threadIdx.x == 0) rows[e] = v;
}

// constant to subtract: ground state  ln g(e=0) - ln 2; or total  LSE - N ln 2
__global__ void __launch_bounds__(64) k_merge_norm(int N, int norm, const double* rows, double* cst) {
    double c;
    if (norm == 0) {
        c = rows[0] - log(2.0);
    } else {
        c = wave_lse(rows, N + 1) - N * log(2.0);
    }
    if (threadIdx.x == 0) cst[0] = c;
}

__global__ void __launch_bounds__(256) k_merge_apply(int N, double* joint, double* rows, const double* cst) {
    const int64_t total = static_cast<int64_t>(N + 1) * (N + 1);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const double c = cst[0];
    if (i < total) joint[i] -= c;
    if (i <= N) rows[i] -= c;
}

}  // namespace

hipError_t launch_merge_points(const MergeGeo& G, int split, int32_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_merge_points, dim3(1), dim3(64), 0, st, G, split, out);
    return hipGetLastError();
}

hipError_t launch_merge(const DevState& S, const MergeGeo& G, int max_nE, int norm, double* lng_out, double* lnge_out,
                        double* err_out, hipStream_t st) {
    const int N = G.N;
    hipLaunchKernelGGL(k_merge_window, dim3(G.nwin), dim3(256), 0, st, S, G);
    hipLaunchKernelGGL(k_merge_marg_rows, dim3(max_nE, G.nwin), dim3(64), 0, st, G);
    hipLaunchKernelGGL(k_merge_join_e, dim3(G.ncol), dim3(64), 0, st, G);
    hipLaunchKernelGGL(k_merge_init_margB, dim3(G.ncol), dim3(64), 0, st, G);
    if (G.ncol > 1) {
        hipLaunchKernelGGL(k_merge_marg_cols, dim3(N + 1, G.ncol), dim3(64), 0, st, G);
        hipLaunchKernelGGL(k_merge_join_m, dim3(1), dim3(64), 0, st, G);
    }
    const int64_t total = static_cast<int64_t>(N + 1) * (N + 1);
    const int blocks = static_cast<int>((total + 255) / 256);
    hipLaunchKernelGGL(k_merge_fill, dim3(blocks), dim3(256), 0, st, G, lng_out, err_out);
    hipLaunchKernelGGL(k_merge_rows, dim3(N + 1), dim3(64), 0, st, N, lng_out, lnge_out);
    hipLaunchKernelGGL(k_merge_norm, dim3(1), dim3(64), 0, st, N, norm, lnge_out, G.ws + G.off_cst);
    hipLaunchKernelGGL(k_merge_apply, dim3(blocks), dim3(256), 0, st, N, lng_out, lnge_out, G.ws + G.off_cst);
    return hipGetLastError();
}

}  // namespace rewl
