// cvisc.hip -- point-wise kernels of the D1-based (compact) viscous variant of
// the right-hand side of ge17: the viscous fluxes Ev, Fv, Gv (ge6-ge8 with the
// stresses of ge19 and bv1-bv3, the heat flux of ge20) built from gradients
// that the compact first derivative supplies, and the assembly of their
// divergence with the gravity source (ge8a).  The derivatives in between are
// the sweep kernels' compact first derivative.  Every expression is formed as
// in the explicit viscous kernel, in the same order.
#include "cvisc.hpp"

namespace nopcs {

namespace {

int pw_blocks(long long N) {
    const long long b = (N + 255) / 256;
    return (int)(b < (1 << 30) ? b : (1 << 30));
}

__global__ void __launch_bounds__(256) k_cv_prims(const double *__restrict__ Q, long long N, long long S, NdConst c,
                                                  double *__restrict__ P) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += step) {
        const Prim q = prim_from(c, Q[i], Q[N + i], Q[2 * N + i], Q[3 * N + i], Q[4 * N + i]);
        P[i] = q.u;
        P[S + i] = q.v;
        P[2 * S + i] = q.w;
        P[3 * S + i] = q.T;
    }
}

__global__ void __launch_bounds__(256) k_cv_flux(const double *__restrict__ P, const double *__restrict__ G,
                                                 long long N, long long S, NdConst c, double *__restrict__ F) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += step) {
        double g[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int d = 0; d < 3; ++d) g[a][d] = G[(3 * a + d) * S + i];
        const double u = P[i], v = P[S + i], w = P[2 * S + i], T = P[3 * S + i];
        const double m = mu_of(c, T), b = beta_of(c, T);
        const double A = (4.0 / 3.0) * m + b, B = b - (2.0 / 3.0) * m;
        const double txx = (A * g[0][0] + B * (g[1][1] + g[2][2])) * c.iRe;
        const double tyy = (A * g[1][1] + B * (g[0][0] + g[2][2])) * c.iRe;
        const double tzz = (A * g[2][2] + B * (g[0][0] + g[1][1])) * c.iRe;
        const double txy = m * (g[0][1] + g[1][0]) * c.iRe;
        const double txz = m * (g[0][2] + g[2][0]) * c.iRe;
        const double tyz = m * (g[1][2] + g[2][1]) * c.iRe;
        const double q3[3] = {-c.kappa * m * g[3][0], -c.kappa * m * g[3][1], -c.kappa * m * g[3][2]};
        const double t[3][3] = {{txx, txy, txz}, {txy, tyy, tyz}, {txz, tyz, tzz}};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            F[(4 * d + 0) * S + i] = t[d][0];
            F[(4 * d + 1) * S + i] = t[d][1];
            F[(4 * d + 2) * S + i] = t[d][2];
            F[(4 * d + 3) * S + i] = u * t[d][0] + v * t[d][1] + w * t[d][2] - q3[d];
        }
    }
}

__global__ void __launch_bounds__(256) k_cv_assemble(const double *__restrict__ Q, const double *__restrict__ DF,
                                                     long long N, long long S, NdConst c, double *__restrict__ R) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += step) {
        double acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = (DF[q * S + i] + DF[(4 + q) * S + i]) + DF[(8 + q) * S + i];
        R[i] = 0.0;
        R[N + i] = acc[0];
        R[2 * N + i] = acc[1] - c.ghat * Q[i];
        R[3 * N + i] = acc[2];
        R[4 * N + i] = acc[3] - c.ghat * Q[2 * N + i];
    }
}

}  // namespace

hipError_t launch_cv_prims(const double *Q, long long N, long long S, const NdConst &c, double *P, hipStream_t st) {
    hipLaunchKernelGGL(k_cv_prims, dim3(pw_blocks(N)), dim3(256), 0, st, Q, N, S, c, P);
    return hipGetLastError();
}

hipError_t launch_cv_flux(const double *P, const double *G, long long N, long long S, const NdConst &c, double *F,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_cv_flux, dim3(pw_blocks(N)), dim3(256), 0, st, P, G, N, S, c, F);
    return hipGetLastError();
}

hipError_t launch_cv_assemble(const double *Q, const double *DF, long long N, long long S, const NdConst &c,
                              double *R, hipStream_t st) {
    hipLaunchKernelGGL(k_cv_assemble, dim3(pw_blocks(N)), dim3(256), 0, st, Q, DF, N, S, c, R);
    return hipGetLastError();
}

}  // namespace nopcs
