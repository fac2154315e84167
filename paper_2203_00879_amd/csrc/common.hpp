// common.hpp -- shared definitions of libnopcs: non-dimensional constants,
// point-wise physics (device), error reporting and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/nopcs.h"

// LDS index checks: nothing on the GPU; abort in the host (CPU) build of the
// kernels that the test-suite runs under AddressSanitizer.
#ifdef NOPCS_CPU_EMUL
#include <cstdio>
#include <cstdlib>
#define NOPCS_LDS_BOUND(i, n)                                                                         \
    do {                                                                                              \
        if ((long long)(i) < 0 || (long long)(i) >= (long long)(n)) {                                 \
            std::fprintf(stderr, "LDS index %lld outside [0, %lld) at %s:%d\n", (long long)(i),       \
                         (long long)(n), __FILE__, __LINE__);                                         \
            std::abort();                                                                             \
        }                                                                                             \
    } while (0)
#else
#define NOPCS_LDS_BOUND(i, n) \
    do {                      \
    } while (0)
#endif

// A value known to be the same in every lane of a wavefront, moved to a scalar
// register (the host build of the kernels runs lanes as threads: no-op).
#ifdef NOPCS_CPU_EMUL
#define NOPCS_UNIFORM(x) (x)
#else
#define NOPCS_UNIFORM(x) __builtin_amdgcn_readfirstlane(x)
#endif

// Read-only table the kernels index with wave-uniform indices: through the
// constant address space the compiler uses scalar loads (scalar cache, no wait
// on the vector memory counter).  The tables are written before the launch and
// never during it.
#ifdef NOPCS_CPU_EMUL
#define NOPCS_SCALAR_PTR(T, p) ((const T *)(p))
#else
#define NOPCS_SCALAR_PTR(T, p) ((const T __attribute__((address_space(4))) *)(p))
#endif

namespace nopcs {

// OUCS3 scheme with eta = 0 (Section 3, entries of A and B after Eq. CS:AfpBf):
// alpha f'_{i-1} + f'_i + alpha f'_{i+1} = [b1 (f_{i+1}-f_{i-1}) + b2 (f_{i+2}-f_{i-2})] / h
constexpr double kAlpha = 0.3793894912;
constexpr double kB1 = 0.7877868952;
constexpr double kB2 = 0.045801298;
// Semi-bandwidth of the equivalent explicit operator C = A^-1 B in FP64 (Section 3).
constexpr int kNb = 48;
constexpr int kTaps = 2 * kNb + 1;

// Non-dimensional constants of Section 2 (ge14-ge20), computed on the host from SI.
struct NdConst {
    double gamma, gm1, Rh, M2, Re, iRe, Pr, St, mu_s, kappa, Eref, H, ghat, mub_a, mub_b, T_s;
    int viscous;
};

inline NdConst make_nd(const nse_params &p) {
    NdConst o;
    const double gl = p.g * p.L;
    const double Us = std::sqrt(gl);
    o.gamma = p.gamma;
    o.gm1 = p.gamma - 1.0;
    o.Rh = p.R_gas * p.T_s / gl;                          // R* T_s / U_s^2
    o.M2 = gl / (p.gamma * p.R_gas * p.T_s);             // U_s^2 / (gamma R* T_s)
    const double r = p.T_s / p.T_ref;                    // Sutherland at T_s
    o.mu_s = p.mu_ref * r * std::sqrt(r) * (p.T_ref + p.S_suth) / (p.T_s + p.S_suth);
    o.Re = p.rho_s * Us * p.L / o.mu_s;
    o.iRe = 1.0 / o.Re;
    o.Pr = p.Pr;
    o.St = p.S_suth / p.T_s;
    o.kappa = 1.0 / ((p.gamma - 1.0) * p.Pr * o.Re * o.M2);  // heat-flux factor of ge20
    o.Eref = o.Rh / (p.gamma - 1.0);
    o.H = o.Eref + o.Rh;
    o.ghat = p.gravity ? 1.0 : 0.0;                      // g L / U_s^2
    o.mub_a = p.mub_a;
    o.mub_b = p.mub_b;
    o.T_s = p.T_s;
    o.viscous = p.viscous ? 1 : 0;
    return o;
}

// ---------------------------------------------------------------------------
// Point-wise physics.  Operation order is fixed (no contraction: the library is
// built with -ffp-contract=off) so that results are reproducible bit for bit.
// ---------------------------------------------------------------------------
struct Prim {
    double u, v, w, pp, T;
};

// Q = [rho, rho u, rho v, rho w, E'] -> velocity, p' = p - Rh, T (ge12, ge13)
__host__ __device__ inline Prim prim_from(const NdConst &c, double rho, double mx, double my, double mz, double Ep) {
    Prim q;
    const double ri = 1.0 / rho;
    q.u = mx * ri;
    q.v = my * ri;
    q.w = mz * ri;
    const double ke = 0.5 * (mx * q.u + my * q.v + mz * q.w);
    q.pp = (c.gamma - 1.0) * (Ep - ke);
    q.T = (q.pp + c.Rh) / (rho * c.Rh);
    return q;
}

// a * b + c with one rounding (the build disables implicit contraction, so
// every fused multiply-add of the kernels is written out with these)
__host__ __device__ inline double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ inline float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Sutherland's law relative to T_s, mu/mu_s (Section 2).
__host__ __device__ inline double mu_of(const NdConst &c, double T) {
    return T * sqrt(T) * (1.0 + c.St) / (T + c.St);
}

// Bulk viscosity regression (eq. reg) relative to mu_s.
__host__ __device__ inline double beta_of(const NdConst &c, double T) {
    return (c.mub_a * (T * c.T_s) - c.mub_b) / c.mu_s;
}

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
const char *get_error();

#define NOPCS_HIP_CHECK(expr)                                                            \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ::nopcs::set_error(std::string(#expr " failed: ") + hipGetErrorString(e_)); \
            return NOPCS_EDEVICE;                                                        \
        }                                                                                \
    } while (0)

// blockIdx -> work item, so that consecutive work items land on the same XCD
// (blocks are dispatched round-robin over the 8 XCDs of the MI355X; neighbouring
// pencils then share their L2).
__device__ inline int xcd_swizzle(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, local = b >> 3;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

}  // namespace nopcs
