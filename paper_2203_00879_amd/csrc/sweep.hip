// sweep.hip -- derivative kernels and convective NSE sweeps (FP64).
#include "kernels.hpp"
#include "sweep.hpp"

namespace nopcs {

// ---------------------------------------------------------------------------
// Standalone first / second derivative along DIR (nopcs_derivative).
// ---------------------------------------------------------------------------
template <int DIR, int NMAX>
__global__ __launch_bounds__((SweepCfg<DIR, NMAX>::NT)) void k_deriv(const double *__restrict__ f, double *d1,
                                                                     double *d2, SweepGeom g, LinePlanDev pl) {
    using C = SweepCfg<DIR, NMAX>;
    __shared__ double F[C::LDS];
    const int npa = (g.nA + C::P - 1) / C::P;
    const int pencil = xcd_swizzle(blockIdx.x, gridDim.x);
    const int pa = pencil % npa, pb = pencil / npa;
    const int l0 = pa * C::P;
    const int np = min(C::P, g.nA - l0);
    const long long base = (long long)l0 * g.sA + (long long)pb * g.sB;
    const int n = g.n;
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        const int q = threadIdx.x + s * C::NT;
        if (q < C::P * n) {
            int l, i;
            C::owned(q, n, l, i);
            if (l < np) F[C::idx(l, i)] = f[base + l * g.sA + i * g.sD];
        }
    }
    __syncthreads();
    lds_line_solve<DIR, NMAX>(F, pl, np);
    if (d1) {
#pragma unroll
        for (int s = 0; s < C::PTS; ++s) {
            const int q = threadIdx.x + s * C::NT;
            if (q < C::P * n) {
                int l, i;
                C::owned(q, n, l, i);
                if (l < np) d1[base + l * g.sA + i * g.sD] = F[C::idx(l, i)];
            }
        }
    }
    if (d2) {
        lds_line_solve<DIR, NMAX>(F, pl, np);
#pragma unroll
        for (int s = 0; s < C::PTS; ++s) {
            const int q = threadIdx.x + s * C::NT;
            if (q < C::P * n) {
                int l, i;
                C::owned(q, n, l, i);
                if (l < np) d2[base + l * g.sA + i * g.sD] = F[C::idx(l, i)];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Convective sweep along DIR: for each of the 5 flux components of ge3-ge5,
//   mode ACCUM:  R_c <- R_c - D_DIR(flux_c)
//   mode RK:     k = R_c - D_DIR(flux_c), then the classical RK4 register update
// ---------------------------------------------------------------------------
template <int DIR, int NMAX, int MODE>
__global__ __launch_bounds__((SweepCfg<DIR, NMAX>::NT)) void k_nse_sweep(NseSweepArgs a, SweepGeom g, LinePlanDev pl) {
    using C = SweepCfg<DIR, NMAX>;
    __shared__ double F[C::LDS];
    const int npa = (g.nA + C::P - 1) / C::P;
    const int pencil = xcd_swizzle(blockIdx.x, gridDim.x);
    const int pa = pencil % npa, pb = pencil / npa;
    const int l0 = pa * C::P;
    const int np = min(C::P, g.nA - l0);
    const long long base = (long long)l0 * g.sA + (long long)pb * g.sB;
    const int n = g.n;
    const long long N3 = a.N3;
    const NdConst &c = a.c;

    // fluxes of the owned points, kept in registers across the 5 components
    double flux[5][C::PTS];
    long long addr[C::PTS];
    bool own[C::PTS];
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        const int q = threadIdx.x + s * C::NT;
        own[s] = false;
        addr[s] = 0;
        if (q < C::P * n) {
            int l, i;
            C::owned(q, n, l, i);
            if (l < np) {
                own[s] = true;
                addr[s] = base + l * g.sA + i * g.sD;
            }
        }
        if (own[s]) {
            const long long o = addr[s];
            const double rho = a.Qin[o], mx = a.Qin[N3 + o], my = a.Qin[2 * N3 + o], mz = a.Qin[3 * N3 + o],
                         Ep = a.Qin[4 * N3 + o];
            const Prim pr = prim_from(c, rho, mx, my, mz, Ep);
            const double ud = DIR == 0 ? pr.u : DIR == 1 ? pr.v : pr.w;
            const double md = DIR == 0 ? mx : DIR == 1 ? my : mz;
            flux[0][s] = md;
            flux[1][s] = DIR == 0 ? mx * ud + pr.pp : mx * ud;
            flux[2][s] = DIR == 1 ? my * ud + pr.pp : my * ud;
            flux[3][s] = DIR == 2 ? mz * ud + pr.pp : mz * ud;
            flux[4][s] = ((Ep + pr.pp) + c.H) * ud;
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) flux[k][s] = 0.0;
        }
    }

#pragma unroll
    for (int comp = 0; comp < 5; ++comp) {
        if (comp > 0) __syncthreads();   // previous component's results consumed
#pragma unroll
        for (int s = 0; s < C::PTS; ++s) {
            if (own[s]) {
                const int q = threadIdx.x + s * C::NT;
                int l, i;
                C::owned(q, n, l, i);
                F[C::idx(l, i)] = flux[comp][s];
            }
        }
        __syncthreads();
        lds_line_solve<DIR, NMAX>(F, pl, np);
#pragma unroll
        for (int s = 0; s < C::PTS; ++s) {
            if (!own[s]) continue;
            const int q = threadIdx.x + s * C::NT;
            int l, i;
            C::owned(q, n, l, i);
            const double df = F[C::idx(l, i)];
            const long long o = comp * N3 + addr[s];
            if (MODE == MODE_ACCUM) {
                a.R[o] = a.R[o] - df;
            } else {
                const double kv = a.R[o] - df;
                if (a.stage == 0) {
                    a.K[o] = kv;
                    a.Qs[o] = a.Qn[o] + a.half_dt * kv;
                } else if (a.stage == 1) {
                    a.K[o] = a.K[o] + 2.0 * kv;
                    a.Qs[o] = a.Qn[o] + a.half_dt * kv;
                } else if (a.stage == 2) {
                    a.K[o] = a.K[o] + 2.0 * kv;
                    a.Qs[o] = a.Qn[o] + a.dt * kv;
                } else {
                    a.Qn[o] = a.Qn[o] + a.sixth_dt * (a.K[o] + kv);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <int DIR, int NMAX>
static hipError_t launch_deriv_t(const double *f, double *d1, double *d2, const SweepGeom &g, const LinePlanDev &pl,
                                 hipStream_t st) {
    using C = SweepCfg<DIR, NMAX>;
    const int npa = (g.nA + C::P - 1) / C::P;
    const long long blocks = (long long)npa * g.nB;
    hipLaunchKernelGGL((k_deriv<DIR, NMAX>), dim3((unsigned)blocks), dim3(C::NT), 0, st, f, d1, d2, g, pl);
    return hipGetLastError();
}

template <int DIR, int NMAX>
static hipError_t launch_sweep_t(const NseSweepArgs &a, const SweepGeom &g, const LinePlanDev &pl, int mode,
                                 hipStream_t st) {
    using C = SweepCfg<DIR, NMAX>;
    const int npa = (g.nA + C::P - 1) / C::P;
    const long long blocks = (long long)npa * g.nB;
    if (mode == MODE_ACCUM)
        hipLaunchKernelGGL((k_nse_sweep<DIR, NMAX, MODE_ACCUM>), dim3((unsigned)blocks), dim3(C::NT), 0, st, a, g, pl);
    else
        hipLaunchKernelGGL((k_nse_sweep<DIR, NMAX, MODE_RK>), dim3((unsigned)blocks), dim3(C::NT), 0, st, a, g, pl);
    return hipGetLastError();
}

int nmax_class(int n) {
    if (n <= 64) return 64;
    if (n <= 128) return 128;
    if (n <= 256) return 256;
    if (n <= 512) return 512;
    if (n <= 1024) return 1024;
    return 0;
}

int sweep_lines_per_block(int dir, int n) {
    switch (nmax_class(n)) {
        case 64: return dir == 0 ? SweepCfg<0, 64>::P : SweepCfg<1, 64>::P;
        case 128: return dir == 0 ? SweepCfg<0, 128>::P : SweepCfg<1, 128>::P;
        case 256: return dir == 0 ? SweepCfg<0, 256>::P : SweepCfg<1, 256>::P;
        case 512: return dir == 0 ? SweepCfg<0, 512>::P : SweepCfg<1, 512>::P;
        case 1024: return dir == 0 ? SweepCfg<0, 1024>::P : SweepCfg<1, 1024>::P;
    }
    return 0;
}

int sweep_threads_per_block(int dir, int n) {
    switch (nmax_class(n)) {
        case 64: return dir == 0 ? SweepCfg<0, 64>::NT : SweepCfg<1, 64>::NT;
        case 128: return dir == 0 ? SweepCfg<0, 128>::NT : SweepCfg<1, 128>::NT;
        case 256: return dir == 0 ? SweepCfg<0, 256>::NT : SweepCfg<1, 256>::NT;
        case 512: return dir == 0 ? SweepCfg<0, 512>::NT : SweepCfg<1, 512>::NT;
        case 1024: return dir == 0 ? SweepCfg<0, 1024>::NT : SweepCfg<1, 1024>::NT;
    }
    return 0;
}

#define NOPCS_DISPATCH_NMAX(DIRV, NM, CALL)     \
    switch (NM) {                               \
        case 64: { constexpr int NMX = 64; CALL; } \
        case 128: { constexpr int NMX = 128; CALL; } \
        case 256: { constexpr int NMX = 256; CALL; } \
        case 512: { constexpr int NMX = 512; CALL; } \
        case 1024: { constexpr int NMX = 1024; CALL; } \
        default: return hipErrorInvalidValue;  \
    }

hipError_t launch_deriv(int dir, const double *f, double *d1, double *d2, const SweepGeom &g, const LinePlanDev &pl,
                        hipStream_t st) {
    const int nm = nmax_class(g.n);
    if (dir == 0) { NOPCS_DISPATCH_NMAX(0, nm, return (launch_deriv_t<0, NMX>(f, d1, d2, g, pl, st))); }
    if (dir == 1) { NOPCS_DISPATCH_NMAX(1, nm, return (launch_deriv_t<1, NMX>(f, d1, d2, g, pl, st))); }
    NOPCS_DISPATCH_NMAX(2, nm, return (launch_deriv_t<2, NMX>(f, d1, d2, g, pl, st)));
}

hipError_t launch_nse_sweep(int dir, int mode, const NseSweepArgs &a, const SweepGeom &g, const LinePlanDev &pl,
                            hipStream_t st) {
    const int nm = nmax_class(g.n);
    if (dir == 0) { NOPCS_DISPATCH_NMAX(0, nm, return (launch_sweep_t<0, NMX>(a, g, pl, mode, st))); }
    if (dir == 1) { NOPCS_DISPATCH_NMAX(1, nm, return (launch_sweep_t<1, NMX>(a, g, pl, mode, st))); }
    NOPCS_DISPATCH_NMAX(2, nm, return (launch_sweep_t<2, NMX>(a, g, pl, mode, st)));
}

}  // namespace nopcs
