// cvisc.hpp -- host launchers of the point-wise kernels of the D1-based
// (compact) viscous variant of the right-hand side.
#pragma once

#include "common.hpp"

namespace nopcs {

// Q (5 fields of N) -> u, v, w, T (4 fields of stride S >= N)
hipError_t launch_cv_prims(const double *Q, long long N, long long S, const NdConst &c, double *P, hipStream_t st);
// primitives P and their 12 gradients G (G[3a + d] = d P_a / d x_d, stride S)
// -> the 12 viscous flux components F[4d + q] (Ev, Fv, Gv; stride S)
hipError_t launch_cv_flux(const double *P, const double *G, long long N, long long S, const NdConst &c, double *F,
                          hipStream_t st);
// R (5 fields of N) = divergence of the fluxes from DF[4d + q] = D_d F[4d + q]
// (stride S), plus the gravity source of Q
hipError_t launch_cv_assemble(const double *Q, const double *DF, long long N, long long S, const NdConst &c,
                              double *R, hipStream_t st);

}  // namespace nopcs
