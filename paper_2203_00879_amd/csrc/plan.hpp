// plan.hpp -- per-line-length plans of the NOHAP segmented compact solve.
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace nopcs {

// Row kinds of one line.
enum : uint8_t { ROW_COMPACT = 0, ROW_WALL = 1, ROW_CLOSURE = 2 };

// Line operators with a plan: the OUCS3 first derivative (Section 3) and the
// implicit low-pass filter (Section 4; fourth-order tridiagonal compact filter
// with coefficient alpha_f, wall rows unfiltered).
enum : int { OP_D1 = 0, OP_FILTER = 1 };

// Right-hand side of the filter: af fh_{i-1} + fh_i + af fh_{i+1} =
// a0 f_i + (a1/2)(f_{i+1} + f_{i-1}) + (a2/2)(f_{i+2} + f_{i-2}), fourth order.
struct FilterCoefs {
    double a0, a1h, a2h;   // a0, a1 / 2, a2 / 2
};
inline FilterCoefs filter_coefs(double af) {
    FilterCoefs c;
    c.a0 = 5.0 / 8.0 + 0.75 * af;
    c.a1h = 0.5 * (0.5 + af);
    c.a2h = 0.5 * (-1.0 / 8.0 + 0.25 * af);
    return c;
}

// Device view of a line plan (passed by value to kernels).
struct LinePlanDev {
    int op;                // OP_D1 or OP_FILTER
    double alpha;          // off-diagonal of A (kAlpha, or the filter's alpha_f)
    FilterCoefs fc;        // OP_FILTER: right-hand side coefficients
    int n;                 // points on the line
    int nrun;              // Thomas runs (maximal sets of compact rows between known rows)
    int ncl;               // closure rows
    double ih;             // 1/h
    const int2 *runs;      // [nrun] (lo, hi): known rows bounding the run; unknowns lo+1..hi-1
    const int2 *run_slot;  // [nrun] known-row slots of lo and hi
    const short *kslot;    // [n] known-row slot of each row (-1: compact row); slots 0..3 are the
                           // wall rows 0, 1, n-2, n-1, slot 4 + q is closure q
    const int *cl_row;     // [ncl] row index e of each closure
    const int *cl_j0;      // [ncl] first tap column
    const int *cl_len;     // [ncl] number of taps (<= 97)
    const double *rden;    // [n] reciprocal elimination pivots 1 / (1 - alpha c'_{k-1}), k = 1..
    const double *cp;      // [n] c'_k = alpha / den_k
    const float *rden32;   // FP32 copies
    const float *cp32;
    const double *cl_coefA;// [64][ncl][2] closure q's taps on the 128 rows from 32 * (cl_j0[q] / 32):
                           // row a at [a / 2][q][a % 2], 0 outside the tap window
    // ---- line-march tables (sweeps that stream along the line) ----
    int max_m;             // longest run (unknowns)
    int ngrp;              // run groups (consecutive runs marched by one thread)
    int k1_S;              // closure accumulator slots (0: more than kMaxSlots needed)
    const int2 *grp;       // [ngrp] (first run, one past the last run)
    const int *run_own;    // [nrun] known rows whose R update this run makes: bit 0 lo, 1 hi,
                           // 2 row 0, 3 row n-1
    const int *k1_rec;     // [n * k1_S] per row j and slot s: -1 or q | t << 12 | flags (kRec*)
    const double *k1_w;    // [n * k1_S] the tap coefficient C_{e,j} * h of that record (0 if none)
    int k1_nev;            // rows with slot events (in order)
    const int *k1_evrow;   // [k1_nev] those rows
    const int *k1_evmask;  // [3 k1_nev] bit s: slot s opens / meets its closure row / closes there
    const double *cl_wsum; // [ncl] sum of the closure's taps (ascending order)
};

// Closure-slot record flags (line-march closure pass).
constexpr int kRecOpen = 1 << 20;   // first tap: the slot's sum starts at this row
constexpr int kRecRow = 1 << 21;    // this row is the closure row e itself
constexpr int kRecClose = 1 << 22;  // last tap: the closure value is complete
constexpr int kMaxSlots = 16;

// Host description (kept for tests and for building the device copy).
struct LinePlanHost {
    int op = OP_D1;
    double alpha = kAlpha;
    int n = 0, nseg = 0, sub_len = 0;
    std::vector<int> seg_lo;          // user segment starts
    std::vector<int2> runs, run_slot;
    std::vector<short> kslot;
    std::vector<int> cl_row, cl_j0, cl_len;
    std::vector<double> cl_coef;      // ncl * kTaps
    std::vector<uint8_t> row_kind;
    std::vector<double> den, rden, cp;
    int max_m = 0, k1_S = 0;
    std::vector<int2> grp;
    std::vector<int> run_own, k1_rec, k1_evrow, k1_evmask;
    std::vector<double> k1_w, cl_wsum;
};

// Run groups of the line-march sweeps: about kGroupRows rows, at most
// kGroupRuns runs each.
constexpr int kGroupRows = 128;
constexpr int kGroupRuns = 4;

// Build the plan of a line of n points cut into nseg user segments; each user
// segment is further cut into pieces of at most sub_len points (0 = no extra cuts).
// Returns false with an error message on invalid input.
bool build_line_plan(int n, int nseg, int sub_len, LinePlanHost &out, std::string &err, int op = OP_D1,
                     double alpha_f = 0.0);

// Kind of every row of a line of n points cut into nseg user segments and
// pieces of at most sub_len points (host only; valid n, nseg assumed).
std::vector<uint8_t> row_kinds(int n, int nseg, int sub_len);

// Segment starts of an even split (the first n % nseg segments one point longer).
std::vector<int> even_segments(int n, int nseg);

// Cached device plan for (device, n, nseg, sub_len, len) -> LinePlanDev, built
// (and its device memory allocated) on first use; lookup_only: never build,
// NOPCS_EINVAL if the plan is not cached yet.
int get_line_plan(int n, int nseg, int sub_len, double len, LinePlanDev *out, bool lookup_only = false,
                  int op = OP_D1, double alpha_f = 0.0);

// Free all cached device plans of the current device.
void release_line_plans();

}  // namespace nopcs
