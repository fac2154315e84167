// vort.hpp -- host launchers of the point-wise parts of the vorticity budget.
#pragma once

#include "common.hpp"

namespace nopcs {

// Q (5 fields of N) -> u, v, w, p' (4 fields of stride S >= N)
hipError_t launch_vort_prims(const double *Q, long long N, long long S, double gm1, double *P, hipStream_t st);
// Q and the 15 gradient fields G (stride S) -> 12 output fields of stride N
hipError_t launch_vort_combine(const double *Q, const double *G, long long N, long long S, double *out,
                               hipStream_t st);

}  // namespace nopcs
