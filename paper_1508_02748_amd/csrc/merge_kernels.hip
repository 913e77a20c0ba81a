// merge_kernels.hip -- joining the per-walker ln g(E,M) fragments of one REWL
// problem into a joint density of states (Sec. 2, Eq. 3 and Eq. 4), float64.
//
//   k_merge_window   one workgroup per window: each walker is aligned on its
//                    mean over the bins every walker of the window has visited
//                    (exact int128 sums), then ln g is averaged over the
//                    walkers that visited each bin, with the standard error of
//                    that average over the walkers (the leave-one-walker-out
//                    jackknife error with the alignment held fixed; NaN below
//                    two walkers) stored after the window's averages.
//   k_merge_marginal one wavefront per (window, energy row): Eq. (3),
//                    ln g(E) = log sum_M g(E, M).
//   k_merge_join     one thread: for each neighbouring pair of windows the
//                    matching energy E_mat minimises the difference of
//                    beta(E) = d ln g / dE (central differences) over the
//                    overlap, at or above the previous matching point, ties to
//                    the lowest E; the upper piece is shifted to agree at E_mat.
//   k_merge_fill     Eq. (4): row e of the joint table comes from the piece
//                    whose matching interval contains e.
//   k_merge_rows / k_merge_norm   row marginals of the joint table and the
//                    normalisation (ground-state count g(-2N) = 2, or
//                    sum g = 2^N).
#include <hip/hip_runtime.h>

#include <math.h>

#include "rewl_internal.h"

namespace rewl {
namespace {

__device__ __forceinline__ int64_t lng_at(const DevState& S, const WDesc& d, int er, int m) {
    const int64_t i = table_index_or_none(d, d.e0 + er, d.m0 + m);
    return i < 0 ? 0 : S.lng[d.table_off + i];
}

__global__ void __launch_bounds__(256) k_merge_window(DevState S, MergeGeo G) {
    const int w = blockIdx.x;
    const PDesc P = S.pd[G.prob];
    const int W = P.W, nM = P.N + 1;
    const int g0 = P.walker_off + w * W;
    const WDesc d0 = S.wd[g0];
    const int nE = d0.hi - d0.lo + 1;
    const int64_t nb = static_cast<int64_t>(nE) * nM;
    const double unit = ldexp(1.0, -P.K);
    double* shift = G.ws + G.off_shift + static_cast<int64_t>(w) * W;
    for (int e = threadIdx.x; e < nM; e += blockDim.x) G.ws[G.off_marg + static_cast<int64_t>(w) * nM + e] = -INFINITY;
    __shared__ unsigned long long red_lo[256], red_hi[256];
    __shared__ long long red_n[256];
    // alignment constants: mean of each walker's ln g over the common bins
    for (int a = 0; a < W; ++a) {
        const WDesc da = S.wd[g0 + a];
        unsigned __int128 acc = 0;
        long long cnt = 0;
        for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
            const int er = static_cast<int>(i / nM), m = static_cast<int>(i % nM);
            bool common = true;
            for (int b = 0; b < W && common; ++b) common = lng_at(S, S.wd[g0 + b], er, m) > 0;
            if (common) {
                acc += static_cast<unsigned __int128>(static_cast<uint64_t>(lng_at(S, da, er, m)));
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
            if (n == 0) G.flags[0] = 1;
        }
        __syncthreads();
    }
    // window average over the walkers that visited each bin
    double* avg = G.ws + G.off_avg[w];
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
        const int er = static_cast<int>(i / nM), m = static_cast<int>(i % nM);
        double num = 0.0;
        int cnt = 0;
        for (int a = 0; a < W; ++a) {
            const int64_t l = lng_at(S, S.wd[g0 + a], er, m);
            if (l > 0) {
                num += static_cast<double>(l) * unit - shift[a];
                ++cnt;
            }
        }
        const double mean = cnt > 0 ? num / cnt : -INFINITY;
        avg[i] = mean;
        double ss = 0.0;
        for (int a = 0; a < W; ++a) {
            const int64_t l = lng_at(S, S.wd[g0 + a], er, m);
            if (l > 0) {
                const double dv = (static_cast<double>(l) * unit - shift[a]) - mean;
                ss += dv * dv;
            }
        }
        avg[nb + i] = cnt > 1 ? sqrt(ss / (static_cast<double>(cnt) * (cnt - 1))) : NAN;
    }
}

// log sum exp of n values with stride 1, one wavefront.
__device__ double wave_lse(const double* x, int n) {
    const int lane = threadIdx.x & 63;
    double mx = -INFINITY;
    for (int i = lane; i < n; i += 64) mx = fmax(mx, x[i]);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (!(mx > -INFINITY)) return -INFINITY;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += exp(x[i] - mx);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    return mx + log(s);
}

__global__ void __launch_bounds__(64) k_merge_marginal(DevState S, MergeGeo G) {
    const int w = blockIdx.y, er = blockIdx.x;
    const PDesc P = S.pd[G.prob];
    const WDesc d = S.wd[P.walker_off + w * P.W];
    if (er > d.hi - d.lo) return;
    const int nM = P.N + 1;
    const double v = wave_lse(G.ws + G.off_avg[w] + static_cast<int64_t>(er) * nM, nM);
    if (threadIdx.x == 0) G.ws[G.off_marg + static_cast<int64_t>(w) * nM + d.lo + er] = v;
}

__device__ __forceinline__ double beta_c(const double* g, int e, int N) {
    if (e < 1 || e + 1 > N) return NAN;
    const double a = g[e - 1], b = g[e], c = g[e + 1];
    if (!(a > -INFINITY) || !(b > -INFINITY) || !(c > -INFINITY)) return NAN;
    return (c - a) / 8.0;
}

__global__ void k_merge_join(DevState S, MergeGeo G, int32_t* e_mat_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const PDesc P = S.pd[G.prob];
    const int N = P.N, nM = N + 1, nwin = P.nwin;
    double* mg = G.ws + G.off_mg;   // marginal of the pieces joined so far
    double* marg = G.ws + G.off_marg;
    double* pshift = G.ws + G.off_pshift;
    int32_t* emat = G.emat;
    const WDesc d0 = S.wd[P.walker_off];
    for (int e = 0; e <= N; ++e) mg[e] = (e >= d0.lo && e <= d0.hi) ? marg[e] : -INFINITY;
    pshift[0] = 0.0;
    emat[0] = 0;
    int cur_hi = d0.hi, prev = 0;
    for (int j = 1; j < nwin; ++j) {
        const WDesc dj = S.wd[P.walker_off + j * P.W];
        const double* mj = marg + static_cast<int64_t>(j) * nM;
        double best = INFINITY;
        int at = -1;
        for (int e = (dj.lo > prev ? dj.lo : prev); e <= cur_hi; ++e) {
            const double bi = beta_c(mg, e, N), bj = beta_c(mj, e, N);
            if (isnan(bi) || isnan(bj)) continue;
            const double dd = fabs(bi - bj);
            if (dd < best) {
                best = dd;
                at = e;
            }
        }
        if (at < 0) {
            G.flags[0] = 2;
            return;
        }
        const double c = mg[at] - mj[at];
        pshift[j] = c;
        emat[j] = at;
        if (e_mat_out) e_mat_out[j - 1] = at;
        for (int e = at; e <= N; ++e) mg[e] = (e <= dj.hi) ? mj[e] + c : -INFINITY;
        cur_hi = dj.hi;
        prev = at;
    }
}

__global__ void __launch_bounds__(256) k_merge_fill(DevState S, MergeGeo G, double* out, double* err) {
    const PDesc P = S.pd[G.prob];
    const int N = P.N, nM = N + 1;
    const int64_t total = static_cast<int64_t>(nM) * nM;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int e = static_cast<int>(i / nM), m = static_cast<int>(i % nM);
    int j = 0;
    for (int k = 1; k < P.nwin; ++k)
        if (e >= G.emat[k]) j = k;
    const WDesc d = S.wd[P.walker_off + j * P.W];
    double v = -INFINITY, ev = NAN;
    if (e >= d.lo && e <= d.hi) {
        const int64_t k = G.off_avg[j] + static_cast<int64_t>(e - d.lo) * nM + m;
        v = G.ws[k] + G.ws[G.off_pshift + j];
        ev = G.ws[k + static_cast<int64_t>(d.hi - d.lo + 1) * nM];
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

hipError_t launch_merge(const DevState& S, const MergeGeo& G, int N, int nwin, int max_nE, int norm, double* lng_out,
                        double* lnge_out, int32_t* e_mat_out, double* err_out, hipStream_t st) {
    hipLaunchKernelGGL(k_merge_window, dim3(nwin), dim3(256), 0, st, S, G);
    hipLaunchKernelGGL(k_merge_marginal, dim3(max_nE, nwin), dim3(64), 0, st, S, G);
    hipLaunchKernelGGL(k_merge_join, dim3(1), dim3(64), 0, st, S, G, e_mat_out);
    const int64_t total = static_cast<int64_t>(N + 1) * (N + 1);
    const int blocks = static_cast<int>((total + 255) / 256);
    hipLaunchKernelGGL(k_merge_fill, dim3(blocks), dim3(256), 0, st, S, G, lng_out, err_out);
    hipLaunchKernelGGL(k_merge_rows, dim3(N + 1), dim3(64), 0, st, N, lng_out, lnge_out);
    hipLaunchKernelGGL(k_merge_norm, dim3(1), dim3(64), 0, st, N, norm, lnge_out, G.ws + G.off_cst);
    hipLaunchKernelGGL(k_merge_apply, dim3(blocks), dim3(256), 0, st, N, lng_out, lnge_out, G.ws + G.off_cst);
    return hipGetLastError();
}

}  // namespace rewl
