// lnz_kernels.hip -- reweighting of a joint density of states g(E,M) into
// ln Z(beta, h) = log sum_{(E,M)} exp(ln g(E,M) - beta E + beta h M) and its
// derivatives, in float64 on gfx950.
//
// One thread per grid point (beta, h).  ln Z takes one pass over the bins (an
// exponential sum kept relative to the running maximum), reading them through
// scalar loads since every lane of a wavefront walks the same bins.  The
// moment and d/d ln g kernels stream the table through LDS in chunks of 256
// bins, each bin read once per workgroup and broadcast to its 256 threads, and
// reuse the saved ln Z as the shift.  Unvisited bins hold -inf and contribute
// zero.
#include <hip/hip_runtime.h>

#include <math.h>

#include "rewl_internal.h"

namespace rewl {
namespace {

constexpr int TILE = 256;

// Every exponential below is of d <= 0: a term relative to the largest term of
// its sum (or to the sum itself).  Terms with d <= -80 are skipped: e^-80 <
// 2e-35, so even 2^32 skipped terms change a sum by less than 1e-25 of its
// largest term, far below float64 rounding.  The branch lets a wavefront skip
// the exponential when none of its lanes needs it.
constexpr double CUT = -80.0;

struct Geo {
    const double* lng;
    int N, e0, nE, m0, nM;
};

// Energy and magnetization of table entry i = ie * nM + im.
__device__ __forceinline__ void em_of(const Geo& g, int64_t i, double& E, double& M) {
    const int ie = static_cast<int>(i / g.nM);
    const int im = static_cast<int>(i - static_cast<int64_t>(ie) * g.nM);
    E = 4.0 * (g.e0 + ie) - 2.0 * g.N;
    M = 2.0 * (g.m0 + im) - 1.0 * g.N;
}

// One term of the one-pass sum: the sum is kept relative to the largest term
// met so far and rescaled when a larger one appears.
__device__ __forceinline__ void lse_step(double x, double& mx, double& sum) {
    if (x > mx) {
        sum = (mx - x > CUT ? sum * exp(mx - x) : 0.0) + 1.0;
        mx = x;
    } else {
        const double d = x - mx;
        if (d > CUT) sum += exp(d);
    }
}

__global__ void __launch_bounds__(TILE) k_lnz_fwd(Geo geo, const double* __restrict__ beta,
                                                   const double* __restrict__ hf, int64_t G,
                                                   double* __restrict__ lnz) {
    const int64_t gp = static_cast<int64_t>(blockIdx.x) * TILE + threadIdx.x;
    const bool on = gp < G;
    const double b = on ? beta[gp] : 0.0;
    const double bh = on ? b * hf[gp] : 0.0;
    // Every lane walks the same bins in the same order, so the bin values are
    // uniform across the wavefront: they come through scalar loads, eight at a
    // time, and E, M are exact integer-valued doubles stepped per bin.  Only
    // the per-point arithmetic runs on the vector unit.
    const double* __restrict__ lg = geo.lng;
    const int nM = geo.nM;
    double mx = -INFINITY, sum = 0.0;
    for (int ie = 0; ie < geo.nE; ++ie) {
        const double bE = b * (4.0 * (geo.e0 + ie) - 2.0 * geo.N);
        const double* __restrict__ row = lg + static_cast<int64_t>(ie) * nM;
        double M = 2.0 * geo.m0 - 1.0 * geo.N;
        int im = 0;
        for (; im + 8 <= nM; im += 8) {
            double l[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) l[k] = row[im + k];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                lse_step(l[k] - bE + bh * M, mx, sum);
                M += 2.0;
            }
        }
        for (; im < nM; ++im) {
            lse_step(row[im] - bE + bh * M, mx, sum);
            M += 2.0;
        }
    }
    if (on) lnz[gp] = mx + log(sum);
}

// Per grid point, with p = exp(ln g - beta E + beta h M - ln Z) and
// U = -E + h M: <M>, <U> in a first pass, then Var(U), Var(M), Cov(U, M) as
// central sums about those means in a second pass (no cancellation of large
// raw moments at low temperature or strong field).
// With upstream gradients a = up_b, c = up_h of (grad_beta, grad_h) it also
// writes the second-order terms of the backward of the first-order backward
// (d2 != nullptr): with g = grad_out and cross = <M> + beta Cov(U, M),
//   d grad_out = a <U> + c beta <M>
//   d beta     = g (a Var(U) + c cross)
//   d h        = g (a cross + c beta^2 Var(M)).
__global__ void __launch_bounds__(TILE) k_lnz_mom(Geo geo, const double* beta, const double* hf, int64_t G,
                                                   const double* lnz, const double* gout, double* mom,
                                                   double* gbeta, double* gh, const double* up_b,
                                                   const double* up_h, double* d_go, double* d_b, double* d_h) {
    __shared__ double sl[TILE], sE[TILE], sM[TILE];
    const int64_t gp = static_cast<int64_t>(blockIdx.x) * TILE + threadIdx.x;
    const bool on = gp < G;
    const double b = on ? beta[gp] : 0.0;
    const double h = on ? hf[gp] : 0.0;
    const double bh = b * h;
    const double z = on ? lnz[gp] : 0.0;
    const int64_t nb = static_cast<int64_t>(geo.nE) * geo.nM;
    double s0 = 0, sU = 0, sM1 = 0;
    double mU = 0, mM = 0, sUU = 0, sMM = 0, sUM = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t base = 0; base < nb; base += TILE) {
            const int64_t i = base + threadIdx.x;
            double E = 0, M = 0, l = -INFINITY;
            if (i < nb) {
                l = geo.lng[i];
                em_of(geo, i, E, M);
            }
            __syncthreads();
            sl[threadIdx.x] = l;
            sE[threadIdx.x] = E;
            sM[threadIdx.x] = M;
            __syncthreads();
            const int n = static_cast<int>(nb - base < TILE ? nb - base : TILE);
            for (int j = 0; j < n; ++j) {
                const double d = (sl[j] - b * sE[j] + bh * sM[j]) - z;
                if (!(d > CUT)) continue;
                const double p = exp(d);
                const double U = -sE[j] + h * sM[j];
                if (pass == 0) {
                    s0 += p;
                    sU += p * U;
                    sM1 += p * sM[j];
                } else {
                    const double du = U - mU, dm = sM[j] - mM;
                    sUU += p * du * du;
                    sMM += p * dm * dm;
                    sUM += p * du * dm;
                }
            }
        }
        if (pass == 0) {
            mU = sU / s0;
            mM = sM1 / s0;
        }
    }
    if (!on) return;
    const double vU = sUU / s0, vM = sMM / s0, cUM = sUM / s0;
    if (mom) {
        mom[5 * gp + 0] = mM;
        mom[5 * gp + 1] = mU;
        mom[5 * gp + 2] = vU;
        mom[5 * gp + 3] = vM;
        mom[5 * gp + 4] = cUM;
    }
    const double go = gout ? gout[gp] : 1.0;
    if (gbeta) gbeta[gp] = go * mU;
    if (gh) gh[gp] = go * b * mM;
    if (d_go) {
        const double a = up_b ? up_b[gp] : 0.0, c = up_h ? up_h[gp] : 0.0;
        const double cross = mM + b * cUM;
        d_go[gp] = a * mU + c * (b * mM);
        d_b[gp] = go * (a * vU + c * cross);
        d_h[gp] = go * (a * cross + c * (b * b * vM));
    }
}

// grad ln g(E,M) = sum_g grad_out_g p_g(E,M): one thread per bin, grid points
// staged through LDS.
__global__ void __launch_bounds__(TILE) k_lnz_glng(Geo geo, const double* beta, const double* hf, int64_t G,
                                                    const double* lnz, const double* gout, double* glng) {
    __shared__ double sb[TILE], sbh[TILE], sz[TILE], sg[TILE];
    const int64_t nb = static_cast<int64_t>(geo.nE) * geo.nM;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * TILE + threadIdx.x;
    double E = 0, M = 0, l = -INFINITY;
    if (i < nb) {
        l = geo.lng[i];
        em_of(geo, i, E, M);
    }
    double acc = 0.0;
    for (int64_t base = 0; base < G; base += TILE) {
        const int64_t k = base + threadIdx.x;
        __syncthreads();
        if (k < G) {
            sb[threadIdx.x] = beta[k];
            sbh[threadIdx.x] = beta[k] * hf[k];
            sz[threadIdx.x] = lnz[k];
            sg[threadIdx.x] = gout ? gout[k] : 1.0;
        }
        __syncthreads();
        const int n = static_cast<int>(G - base < TILE ? G - base : TILE);
        for (int j = 0; j < n; ++j) {
            const double d = l - sb[j] * E + sbh[j] * M - sz[j];
            if (d > CUT) acc += sg[j] * exp(d);
        }
    }
    if (i < nb) glng[i] = acc;
}


// ------------------------------------------------------------------ tensor-product grids
// For a grid beta_i x h_j the sum factorises through the M columns:
//   A(i, M)  = log sum_E exp(ln g(E, M) - beta_i E)            (independent of h)
//   ln Z(i,j) = log sum_M exp(A(i, M) + beta_i h_j M)
// so the exponentials cost nB nE nM + nB nH nM instead of nB nH nE nM.  The
// backward needs, per column, the conditional mean and variance of E at
// beta_i (law of total variance), and for d/d ln g the column weights
//   c(i, M) = sum_j grad_out(i,j) exp(A(i, M) + beta_i h_j M - ln Z(i,j)),
// so that d ln Z / d ln g(E, M) summed over the grid is
//   sum_i exp(ln g(E, M) - beta_i E - A(i, M)) c(i, M).

constexpr int GB = 8;  // beta values per thread in the column pass

// One thread per (column M, block of GB betas); consecutive threads read
// consecutive M of one energy row, so every row load is coalesced.
__global__ void __launch_bounds__(TILE) k_grid_cols(Geo geo, const double* beta, int64_t nB, double* A,
                                                     double* u1, double* u2) {
    const int im = blockIdx.x * TILE + threadIdx.x;
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * GB;
    if (im >= geo.nM) return;
    double b[GB], mx[GB], s0[GB], s1[GB];
#pragma unroll
    for (int k = 0; k < GB; ++k) {
        b[k] = i0 + k < nB ? beta[i0 + k] : 0.0;
        mx[k] = -INFINITY;
        s0[k] = 0.0;
        s1[k] = 0.0;
    }
    const double* col = geo.lng + im;
    for (int ie = 0; ie < geo.nE; ++ie) {
        const double l = col[static_cast<int64_t>(ie) * geo.nM];
        if (l == -INFINITY) continue;
        const double E = 4.0 * (geo.e0 + ie) - 2.0 * geo.N;
#pragma unroll
        for (int k = 0; k < GB; ++k) mx[k] = fmax(mx[k], l - b[k] * E);
    }
    if (mx[0] == -INFINITY) {  // an empty column is empty at every beta
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            if (i0 + k >= nB) break;
            const int64_t o = (i0 + k) * geo.nM + im;
            A[o] = -INFINITY;
            if (u1) {
                u1[o] = 0.0;
                u2[o] = 0.0;
            }
        }
        return;
    }
    for (int ie = 0; ie < geo.nE; ++ie) {
        const double l = col[static_cast<int64_t>(ie) * geo.nM];
        if (l == -INFINITY) continue;
        const double E = 4.0 * (geo.e0 + ie) - 2.0 * geo.N;
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            const double d = (l - b[k] * E) - mx[k];
            if (d > CUT) {
                const double w = exp(d);
                s0[k] += w;
                s1[k] += w * E;
            }
        }
    }
    if (u1) {
        double mean[GB], s2[GB];
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            mean[k] = s1[k] / s0[k];
            s2[k] = 0.0;
        }
        for (int ie = 0; ie < geo.nE; ++ie) {
            const double l = col[static_cast<int64_t>(ie) * geo.nM];
            if (l == -INFINITY) continue;
            const double E = 4.0 * (geo.e0 + ie) - 2.0 * geo.N;
#pragma unroll
            for (int k = 0; k < GB; ++k) {
                const double x = (l - b[k] * E) - mx[k];
                if (x > CUT) {
                    const double d = E - mean[k];
                    s2[k] += exp(x) * d * d;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            if (i0 + k >= nB) break;
            const int64_t o = (i0 + k) * geo.nM + im;
            u1[o] = mean[k];
            u2[o] = s2[k] / s0[k];
        }
    }
#pragma unroll
    for (int k = 0; k < GB; ++k) {
        if (i0 + k >= nB) break;
        A[(i0 + k) * geo.nM + im] = mx[k] + log(s0[k]);
    }
}

// ln Z(i, j): one workgroup per (beta_i, 256 h values); the row A(i, .) is
// staged through LDS in chunks and broadcast to the workgroup.
__global__ void __launch_bounds__(TILE) k_grid_rows(const double* A, int N, int m0, int nM, const double* beta,
                                                     const double* hf, int64_t nH, double* lnz) {
    __shared__ double sa[TILE];
    const int64_t i = blockIdx.x;
    const int64_t j = static_cast<int64_t>(blockIdx.y) * TILE + threadIdx.x;
    const bool on = j < nH;
    const double bh = on ? beta[i] * hf[j] : 0.0;
    const double* row = A + i * nM;
    double mx = -INFINITY, sum = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int base = 0; base < nM; base += TILE) {
            const int k = base + threadIdx.x;
            __syncthreads();
            sa[threadIdx.x] = k < nM ? row[k] : -INFINITY;
            __syncthreads();
            const int n = nM - base < TILE ? nM - base : TILE;
            for (int q = 0; q < n; ++q) {
                const double M = 2.0 * (m0 + base + q) - 1.0 * N;
                const double x = sa[q] + bh * M;
                if (pass == 0) mx = fmax(mx, x);
                else if (x - mx > CUT) sum += exp(x - mx);
            }
        }
    }
    if (on) lnz[i * nH + j] = mx + log(sum);
}

// Per grid point (i, j), from the column statistics: with p_M = exp(A(i,M) +
// beta_i h_j M - ln Z) and the conditional mean of U = -E + h M in column M,
// ubar = -u1 + h M: <M>, <U>, then Var(U) = sum p (u2 + (ubar - <U>)^2),
// Var(M), Cov(U, M) = sum p (ubar - <U>)(M - <M>) about those means.  Also
// the per-point terms of the gradients: tb = g <U>, th = g beta <M>; or, for
// the second order (d_go != nullptr, upstream a_i = up_b[i], c_j = up_h[j]),
// d grad_out = a_i <U> + c_j beta_i <M> and the per-point terms of d beta and
// d h, tb = g (a_i Var(U) + c_j cross), th = g (a_i cross + c_j beta_i^2
// Var(M)) with cross = <M> + beta_i Cov(U, M), summed over j and i afterwards.
__global__ void __launch_bounds__(TILE) k_grid_mom(const double* A, const double* u1, const double* u2, int N,
                                                    int m0, int nM, const double* beta, const double* hf,
                                                    int64_t nH, const double* lnz, const double* gout,
                                                    double* mom, double* tb, double* th, const double* up_b,
                                                    const double* up_h, double* d_go) {
    __shared__ double sa[TILE], s1[TILE], s2[TILE];
    const int64_t i = blockIdx.x;
    const int64_t j = static_cast<int64_t>(blockIdx.y) * TILE + threadIdx.x;
    const bool on = j < nH;
    const double b = beta[i];
    const double h = on ? hf[j] : 0.0;
    const double bh = b * h;
    const double z = on ? lnz[i * nH + j] : 0.0;
    const int64_t r0 = i * nM;
    double c0 = 0, cU = 0, cM = 0, mU = 0, mM = 0, vU = 0, vM = 0, cUM = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int base = 0; base < nM; base += TILE) {
            const int k = base + threadIdx.x;
            __syncthreads();
            sa[threadIdx.x] = k < nM ? A[r0 + k] : -INFINITY;
            s1[threadIdx.x] = k < nM ? u1[r0 + k] : 0.0;
            s2[threadIdx.x] = k < nM ? u2[r0 + k] : 0.0;
            __syncthreads();
            const int n = nM - base < TILE ? nM - base : TILE;
            for (int q = 0; q < n; ++q) {
                if (sa[q] == -INFINITY) continue;
                const double M = 2.0 * (m0 + base + q) - 1.0 * N;
                const double dz = sa[q] + bh * M - z;
                if (!(dz > CUT)) continue;
                const double p = exp(dz);
                const double ub = -s1[q] + h * M;
                if (pass == 0) {
                    c0 += p;
                    cU += p * ub;
                    cM += p * M;
                } else {
                    const double du = ub - mU, dm = M - mM;
                    vU += p * (s2[q] + du * du);
                    vM += p * dm * dm;
                    cUM += p * du * dm;
                }
            }
        }
        if (pass == 0) {
            mU = cU / c0;
            mM = cM / c0;
        }
    }
    if (!on) return;
    const int64_t o = i * nH + j;
    if (mom) {
        mom[5 * o + 0] = mM;
        mom[5 * o + 1] = mU;
        mom[5 * o + 2] = vU / c0;
        mom[5 * o + 3] = vM / c0;
        mom[5 * o + 4] = cUM / c0;
    }
    const double go = gout ? gout[o] : 1.0;
    if (d_go) {
        const double a = up_b ? up_b[i] : 0.0, c = up_h ? up_h[j] : 0.0;
        const double vUn = vU / c0, vMn = vM / c0, cross = mM + b * (cUM / c0);
        d_go[o] = a * mU + c * (b * mM);
        tb[o] = go * (a * vUn + c * cross);
        th[o] = go * (a * cross + c * (b * b * vMn));
    } else if (tb) {
        tb[o] = go * mU;
        th[o] = go * b * mM;
    }
}

// grad_beta(i) = sum_j tb(i, j): one thread per beta_i, fixed order.
__global__ void __launch_bounds__(TILE) k_grid_sum_rows(const double* tb, int64_t nB, int64_t nH, double* gbeta) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * TILE + threadIdx.x;
    if (i >= nB) return;
    double s = 0.0;
    for (int64_t j = 0; j < nH; ++j) s += tb[i * nH + j];
    gbeta[i] = s;
}

// grad_h(j) = sum_i th(i, j): a workgroup per 64 columns, its four waves
// summing every fourth row, then the four partial sums in a fixed order.
__global__ void __launch_bounds__(TILE) k_grid_sum_cols(const double* th, int64_t nB, int64_t nH, double* gh) {
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    double s = 0.0;
    if (j < nH)
        for (int64_t i = wave; i < nB; i += 4) s += th[i * nH + j];
    part[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && j < nH) gh[j] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// c(i, M) = sum_j grad_out(i, j) exp(A(i, M) + beta_i h_j M - ln Z(i, j)):
// one thread per (i, M), the (h_j, ln Z(i, j), grad_out(i, j)) row staged in LDS.
__global__ void __launch_bounds__(TILE) k_grid_colw(const double* A, int N, int m0, int nM, const double* beta,
                                                     const double* hf, int64_t nH, const double* lnz,
                                                     const double* gout, double* cw) {
    __shared__ double sh[TILE], sz[TILE], sg[TILE];
    const int64_t i = blockIdx.y;
    const int im = blockIdx.x * TILE + threadIdx.x;
    const bool on = im < nM;
    const double a = on ? A[i * nM + im] : -INFINITY;
    const double bM = beta[i] * (2.0 * (m0 + im) - 1.0 * N);
    double acc = 0.0;
    for (int64_t base = 0; base < nH; base += TILE) {
        const int64_t k = base + threadIdx.x;
        __syncthreads();
        if (k < nH) {
            sh[threadIdx.x] = hf[k];
            sz[threadIdx.x] = lnz[i * nH + k];
            sg[threadIdx.x] = gout ? gout[i * nH + k] : 1.0;
        }
        __syncthreads();
        if (a == -INFINITY) continue;
        const int n = static_cast<int>(nH - base < TILE ? nH - base : TILE);
        for (int q = 0; q < n; ++q) {
            const double d = a + bM * sh[q] - sz[q];
            if (d > CUT) acc += sg[q] * exp(d);
        }
    }
    if (on) cw[i * nM + im] = acc;
}

// grad ln g(E, M) = sum_i exp(ln g(E, M) - beta_i E - A(i, M)) c(i, M): one
// thread per bin; A and c are read along M (coalesced), beta from LDS.
__global__ void __launch_bounds__(TILE) k_grid_glng(Geo geo, const double* beta, int64_t nB, const double* A,
                                                     const double* cw, double* glng) {
    __shared__ double sb[TILE];
    const int64_t nb = static_cast<int64_t>(geo.nE) * geo.nM;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * TILE + threadIdx.x;
    double E = 0, M = 0, l = -INFINITY;
    int im = 0;
    if (idx < nb) {
        l = geo.lng[idx];
        em_of(geo, idx, E, M);
        im = static_cast<int>(idx % geo.nM);
    }
    double acc = 0.0;
    for (int64_t base = 0; base < nB; base += TILE) {
        const int64_t k = base + threadIdx.x;
        __syncthreads();
        if (k < nB) sb[threadIdx.x] = beta[k];
        __syncthreads();
        if (l == -INFINITY) continue;
        const int n = static_cast<int>(nB - base < TILE ? nB - base : TILE);
        for (int q = 0; q < n; ++q) {
            const int64_t o = (base + q) * geo.nM + im;
            const double d = l - sb[q] * E - A[o];
            if (d > CUT) acc += exp(d) * cw[o];
        }
    }
    if (idx < nb) glng[idx] = acc;
}

int nblk(int64_t n) { return static_cast<int>((n + TILE - 1) / TILE); }

}  // namespace

hipError_t launch_lnz_forward(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                              const double* h, int64_t G, double* lnz, hipStream_t st) {
    if (G <= 0) return hipSuccess;
    Geo geo{lng, N, e0, nE, m0, nM};
    hipLaunchKernelGGL(k_lnz_fwd, dim3(nblk(G)), dim3(TILE), 0, st, geo, beta, h, G, lnz);
    return hipGetLastError();
}

hipError_t launch_lnz_moments(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                              const double* h, int64_t G, const double* lnz, const double* gout, double* mom,
                              double* gbeta, double* gh, hipStream_t st) {
    if (G <= 0) return hipSuccess;
    Geo geo{lng, N, e0, nE, m0, nM};
    hipLaunchKernelGGL(k_lnz_mom, dim3(nblk(G)), dim3(TILE), 0, st, geo, beta, h, G, lnz, gout, mom, gbeta, gh,
                       static_cast<const double*>(nullptr), static_cast<const double*>(nullptr),
                       static_cast<double*>(nullptr), static_cast<double*>(nullptr), static_cast<double*>(nullptr));
    return hipGetLastError();
}

hipError_t launch_lnz_second(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                             const double* h, int64_t G, const double* lnz, const double* gout, const double* up_b,
                             const double* up_h, double* d_go, double* d_b, double* d_h, hipStream_t st) {
    if (G <= 0) return hipSuccess;
    Geo geo{lng, N, e0, nE, m0, nM};
    hipLaunchKernelGGL(k_lnz_mom, dim3(nblk(G)), dim3(TILE), 0, st, geo, beta, h, G, lnz, gout,
                       static_cast<double*>(nullptr), static_cast<double*>(nullptr), static_cast<double*>(nullptr),
                       up_b, up_h, d_go, d_b, d_h);
    return hipGetLastError();
}

hipError_t launch_lnz_grad_lng(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                               const double* h, int64_t G, const double* lnz, const double* grad_out,
                               double* grad_lng, hipStream_t st) {
    const int64_t nb = static_cast<int64_t>(nE) * nM;
    if (nb <= 0) return hipSuccess;
    Geo geo{lng, N, e0, nE, m0, nM};
    hipLaunchKernelGGL(k_lnz_glng, dim3(nblk(nb)), dim3(TILE), 0, st, geo, beta, h, G, lnz, grad_out, grad_lng);
    return hipGetLastError();
}

hipError_t launch_lnz_grid_forward(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                                   int64_t nB, const double* h, int64_t nH, double* A, double* lnz, hipStream_t st) {
    if (nB <= 0 || nH <= 0) return hipSuccess;
    Geo geo{lng, N, e0, nE, m0, nM};
    hipLaunchKernelGGL(k_grid_cols, dim3(nblk(nM), static_cast<unsigned>((nB + GB - 1) / GB)), dim3(TILE), 0, st,
                       geo, beta, nB, A, static_cast<double*>(nullptr), static_cast<double*>(nullptr));
    hipLaunchKernelGGL(k_grid_rows, dim3(static_cast<unsigned>(nB), nblk(nH)), dim3(TILE), 0, st, A, N, m0, nM, beta,
                       h, nH, lnz);
    return hipGetLastError();
}

hipError_t launch_lnz_grid_backward(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                                    int64_t nB, const double* h, int64_t nH, const double* lnz, const double* gout,
                                    double* A, double* u1, double* u2, double* cw, double* tb, double* th,
                                    double* gbeta, double* gh, double* glng, double* mom, hipStream_t st) {
    if (nB <= 0 || nH <= 0) return hipSuccess;
    Geo geo{lng, N, e0, nE, m0, nM};
    hipLaunchKernelGGL(k_grid_cols, dim3(nblk(nM), static_cast<unsigned>((nB + GB - 1) / GB)), dim3(TILE), 0, st,
                       geo, beta, nB, A, u1, u2);
    if (mom || tb)
        hipLaunchKernelGGL(k_grid_mom, dim3(static_cast<unsigned>(nB), nblk(nH)), dim3(TILE), 0, st, A, u1, u2, N,
                           m0, nM, beta, h, nH, lnz, gout, mom, tb, th, static_cast<const double*>(nullptr),
                           static_cast<const double*>(nullptr), static_cast<double*>(nullptr));
    if (tb) {
        hipLaunchKernelGGL(k_grid_sum_rows, dim3(nblk(nB)), dim3(TILE), 0, st, tb, nB, nH, gbeta);
        hipLaunchKernelGGL(k_grid_sum_cols, dim3(static_cast<unsigned>((nH + 63) / 64)), dim3(TILE), 0, st, th, nB,
                           nH, gh);
    }
    if (glng) {
        hipLaunchKernelGGL(k_grid_colw, dim3(nblk(nM), static_cast<unsigned>(nB)), dim3(TILE), 0, st, A, N, m0, nM,
                           beta, h, nH, lnz, gout, cw);
        const int64_t nb = static_cast<int64_t>(nE) * nM;
        hipLaunchKernelGGL(k_grid_glng, dim3(nblk(nb)), dim3(TILE), 0, st, geo, beta, nB, A, cw, glng);
    }
    return hipGetLastError();
}

hipError_t launch_lnz_grid_second(const double* lng, int N, int e0, int nE, int m0, int nM, const double* beta,
                                  int64_t nB, const double* h, int64_t nH, const double* lnz, const double* gout,
                                  const double* up_b, const double* up_h, double* A, double* u1, double* u2,
                                  double* tb, double* th, double* d_go, double* d_b, double* d_h, hipStream_t st) {
    if (nB <= 0 || nH <= 0) return hipSuccess;
    Geo geo{lng, N, e0, nE, m0, nM};
    hipLaunchKernelGGL(k_grid_cols, dim3(nblk(nM), static_cast<unsigned>((nB + GB - 1) / GB)), dim3(TILE), 0, st,
                       geo, beta, nB, A, u1, u2);
    hipLaunchKernelGGL(k_grid_mom, dim3(static_cast<unsigned>(nB), nblk(nH)), dim3(TILE), 0, st, A, u1, u2, N, m0,
                       nM, beta, h, nH, lnz, gout, static_cast<double*>(nullptr), tb, th, up_b, up_h, d_go);
    hipLaunchKernelGGL(k_grid_sum_rows, dim3(nblk(nB)), dim3(TILE), 0, st, tb, nB, nH, d_b);
    hipLaunchKernelGGL(k_grid_sum_cols, dim3(static_cast<unsigned>((nH + 63) / 64)), dim3(TILE), 0, st, th, nB, nH,
                       d_h);
    return hipGetLastError();
}

}  // namespace rewl
