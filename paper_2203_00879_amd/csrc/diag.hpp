// diag.hpp -- host launchers of the diagnostics kernels.
#pragma once

#include "common.hpp"

namespace nopcs {

// Q (5 fields of N) -> u, v, w, p' (4 fields of stride S >= N)
hipError_t launch_vort_prims(const double *Q, long long N, long long S, double gm1, double *P, hipStream_t st);
// Q and the 15 gradient fields G (stride S) -> 12 output fields of stride N
hipError_t launch_vort_combine(const double *Q, const double *G, long long N, long long S, double *out,
                               hipStream_t st);

// out (N) = p'(Q) - p'(Q0) for two 5-field states of N points
hipError_t launch_disturbance_pressure(const double *Q, const double *Q0, long long N, double gm1, double *out,
                                      hipStream_t st);
// amp (n / 2 + 1) = DFT amplitudes / n of f[j stride], j < n
hipError_t launch_line_spectrum(const double *f, int n, long long stride, double *amp, hipStream_t st);

}  // namespace nopcs
