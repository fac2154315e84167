// dmarch.hpp -- first derivative of one field along y or z as a line march.
#pragma once

#include "plan.hpp"

namespace nopcs {

// true if the first derivative along dir can run as a closure pass and a line
// march with this plan (dir 1 or 2, runs of at most 32 unknowns, at most 8
// closure slots per row)
bool dmarch_usable(int dir, const LinePlanDev &pl);
// device bytes of the closure values of every line (0: the plan has no closure rows)
size_t dmarch_closure_bytes(const int n[3], int dir, const LinePlanDev &pl);
// d1 <- D_dir f for every line along dir of an n[0] x n[1] x n[2] field;
// clo: dmarch_closure_bytes of device scratch (the closure values)
hipError_t launch_dmarch(int dir, const double *f, double *d1, double *clo, const int n[3], const LinePlanDev &pl,
                         hipStream_t st);

}  // namespace nopcs
