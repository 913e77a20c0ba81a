// lnz_kernels.hip -- reweighting of a joint density of states g(E,M) into
// ln Z(beta, h) = log sum_{(E,M)} exp(ln g(E,M) - beta E + beta h M) and its
// derivatives, in float64 on gfx950.
//
// One thread per grid point (beta, h); a workgroup of 256 grid points streams
// the ln g table through LDS in chunks of 256 bins, so every bin is read from
// HBM once per workgroup and broadcast to its 256 threads.  ln Z takes two
// passes (maximum, then the shifted exponential sum); the moments pass reuses
// the saved ln Z as the shift.  Unvisited bins hold -inf and contribute zero.
#include <hip/hip_runtime.h>

#include <math.h>

#include "rewl_internal.h"

namespace rewl {
namespace {

constexpr int TILE = 256;

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

__global__ void __launch_bounds__(TILE) k_lnz_fwd(Geo geo, const double* beta, const double* hf, int64_t G,
                                                   double* lnz) {
    __shared__ double sl[TILE], sE[TILE], sM[TILE];
    const int64_t gp = static_cast<int64_t>(blockIdx.x) * TILE + threadIdx.x;
    const bool on = gp < G;
    const double b = on ? beta[gp] : 0.0;
    const double bh = on ? b * hf[gp] : 0.0;
    const int64_t nb = static_cast<int64_t>(geo.nE) * geo.nM;
    double mx = -INFINITY;
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
            const double x = sl[j] - b * sE[j] + bh * sM[j];
            mx = fmax(mx, x);
        }
    }
    double sum = 0.0;
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
            const double x = sl[j] - b * sE[j] + bh * sM[j];
            sum += exp(x - mx);
        }
    }
    if (on) lnz[gp] = mx + log(sum);
}

// Per grid point, with p = exp(ln g - beta E + beta h M - ln Z) and
// U = -E + h M: <M>, <U> in a first pass, then Var(U), Var(M), Cov(U, M) as
// central sums about those means in a second pass (no cancellation of large
// raw moments at low temperature or strong field).
__global__ void __launch_bounds__(TILE) k_lnz_mom(Geo geo, const double* beta, const double* hf, int64_t G,
                                                   const double* lnz, const double* gout, double* mom,
                                                   double* gbeta, double* gh) {
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
                const double x = sl[j] - b * sE[j] + bh * sM[j];
                const double p = exp(x - z);
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
        for (int j = 0; j < n; ++j) acc += sg[j] * exp(l - sb[j] * E + sbh[j] * M - sz[j]);
    }
    if (i < nb) glng[i] = acc;
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
    hipLaunchKernelGGL(k_lnz_mom, dim3(nblk(G)), dim3(TILE), 0, st, geo, beta, h, G, lnz, gout, mom, gbeta, gh);
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

}  // namespace rewl
