// diag.hip -- kernels of the flow diagnostics.
//  * Vorticity budget (Eq. eqn12_1): the primitive fields whose gradients enter
//    it, and the vorticity with the three source terms of the inviscid
//    vorticity transport equation built from those gradients.  The derivatives
//    in between are the compact first derivative of the sweep kernels.
//  * Disturbance pressure p - p_h (Section 4) and the amplitude spectrum of one
//    line of it (a direct DFT; lines hold at most a few thousand points).
#include "diag.hpp"

namespace nopcs {

namespace {

// u, v, w = (rho u, rho v, rho w) / rho and p' = (gamma - 1)(E' - rho |V|^2 / 2)
// (ge12, ge13), into four fields of stride S
__global__ void __launch_bounds__(256) k_vort_prims(const double *__restrict__ Q, long long N, long long S,
                                                    double gm1, double *__restrict__ P) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += step) {
        const double r = Q[i];
        const double m0 = Q[N + i], m1 = Q[2 * N + i], m2 = Q[3 * N + i];
        const double u = m0 / r, v = m1 / r, w = m2 / r;
        const double ke = 0.5 * ((m0 * u + m1 * v) + m2 * w);
        P[i] = u;
        P[S + i] = v;
        P[2 * S + i] = w;
        P[3 * S + i] = gm1 * (Q[4 * N + i] - ke);
    }
}

// G: 15 fields of stride S: dV_i/dx_j at 3 i + j, d rho/dx_j at 9 + j,
// dp'/dx_j at 12 + j.  out: 12 fields of stride N: omega, (omega . grad) V,
// -omega div V, (grad rho x grad p') / rho^2.
__global__ void __launch_bounds__(256) k_vort_combine(const double *__restrict__ Q, const double *__restrict__ G,
                                                      long long N, long long S, double *__restrict__ out) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += step) {
        double g[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) g[a][b] = G[(3 * a + b) * S + i];
        const double om[3] = {g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]};
        const double div = (g[0][0] + g[1][1]) + g[2][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            out[a * N + i] = om[a];
            out[(3 + a) * N + i] = (om[0] * g[a][0] + om[1] * g[a][1]) + om[2] * g[a][2];
            out[(6 + a) * N + i] = -(om[a] * div);
        }
        const double gr0 = G[9 * S + i], gr1 = G[10 * S + i], gr2 = G[11 * S + i];
        const double gp0 = G[12 * S + i], gp1 = G[13 * S + i], gp2 = G[14 * S + i];
        const double r = Q[i];
        const double r2 = r * r;
        out[9 * N + i] = (gr1 * gp2 - gr2 * gp1) / r2;
        out[10 * N + i] = (gr2 * gp0 - gr0 * gp2) / r2;
        out[11 * N + i] = (gr0 * gp1 - gr1 * gp0) / r2;
    }
}

// out = p'(Q) - p'(Q0) = (gamma - 1)((E' - E'_0) - (k - k_0)), k = rho |V|^2 / 2
__global__ void __launch_bounds__(256) k_disturbance_pressure(const double *__restrict__ Q,
                                                              const double *__restrict__ Q0, long long N, double gm1,
                                                              double *__restrict__ out) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += step) {
        const double r = Q[i], m0 = Q[N + i], m1 = Q[2 * N + i], m2 = Q[3 * N + i];
        const double k = 0.5 * ((m0 * (m0 / r) + m1 * (m1 / r)) + m2 * (m2 / r));
        const double r0 = Q0[i], n0 = Q0[N + i], n1 = Q0[2 * N + i], n2 = Q0[3 * N + i];
        const double k0 = 0.5 * ((n0 * (n0 / r0) + n1 * (n1 / r0)) + n2 * (n2 / r0));
        out[i] = gm1 * ((Q[4 * N + i] - Q0[4 * N + i]) - (k - k0));
    }
}

// amp[k] = |sum_j f[j stride] exp(-2 pi i j k / n)| / n, one block per k.  The
// phase index j k mod n is exact in integers, so every twiddle is one
// sincospi of an argument in [0, 2).
constexpr int kSpecThreads = 256;
__global__ void __launch_bounds__(kSpecThreads) k_line_spectrum(const double *__restrict__ f, int n, long long stride,
                                                                double *__restrict__ amp) {
    __shared__ double sre[kSpecThreads], sim[kSpecThreads];
    const int k = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int j = threadIdx.x; j < n; j += kSpecThreads) {
        const long long m = ((long long)j * k) % n;
        double s, c;
        sincospi(2.0 * (double)m / (double)n, &s, &c);
        const double v = f[(long long)j * stride];
        re = fma_(v, c, re);
        im = fma_(-v, s, im);
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int w = kSpecThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sre[threadIdx.x] += sre[threadIdx.x + w];
            sim[threadIdx.x] += sim[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) amp[k] = sqrt(sre[0] * sre[0] + sim[0] * sim[0]) / (double)n;
}

int pointwise_blocks(long long N) {
    const long long b = (N + 255) / 256;
    return (int)(b < (1 << 30) ? b : (1 << 30));
}

}  // namespace

hipError_t launch_vort_prims(const double *Q, long long N, long long S, double gm1, double *P, hipStream_t st) {
    hipLaunchKernelGGL(k_vort_prims, dim3(pointwise_blocks(N)), dim3(256), 0, st, Q, N, S, gm1, P);
    return hipGetLastError();
}

hipError_t launch_vort_combine(const double *Q, const double *G, long long N, long long S, double *out,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_vort_combine, dim3(pointwise_blocks(N)), dim3(256), 0, st, Q, G, N, S, out);
    return hipGetLastError();
}

hipError_t launch_disturbance_pressure(const double *Q, const double *Q0, long long N, double gm1, double *out,
                                      hipStream_t st) {
    hipLaunchKernelGGL(k_disturbance_pressure, dim3(pointwise_blocks(N)), dim3(256), 0, st, Q, Q0, N, gm1, out);
    return hipGetLastError();
}

hipError_t launch_line_spectrum(const double *f, int n, long long stride, double *amp, hipStream_t st) {
    hipLaunchKernelGGL(k_line_spectrum, dim3(n / 2 + 1), dim3(kSpecThreads), 0, st, f, n, stride, amp);
    return hipGetLastError();
}

}  // namespace nopcs
