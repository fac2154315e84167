// kernels.hpp -- kernel argument blocks and host launchers of libnopcs.
#pragma once

#include "batch.hpp"
#include "common.hpp"
#include "plan.hpp"
#include "sweep.hpp"

namespace nopcs {

struct NseSweepArgs {
    const double *Qin;  // stage input state (5 fields)
    void *R;            // right-hand side accumulator (5 fields; FP64, or FP32 when r32)
    bool r32;           // R stored in FP32 (mixed precision)
    double *Qn;         // RK: state at the start of the step (in/out at the last stage)
    double *K;          // RK: k1 + 2 k2 + 2 k3 accumulator
    double *Qs;         // RK: next stage state
    long long N3;       // points per field
    int stage;          // 0..3
    double dt, half_dt, sixth_dt;
    NdConst c;
};

// RK4 stage update fused into the last convective sweep: the sweep's
// k = R - f' goes straight into the stage registers instead of R.  The next
// stage state goes to S, which must not be the sweep's input state: in FP64 it
// is R itself (each point's R is read and then written by one thread only), in
// mixed precision (FP32 R) a second FP64 stage buffer.
struct RkFuse {
    double *K;          // k1 + 2 k2 + 2 k3 accumulator
    double *Qn;         // state at the start of the step (in/out at the last stage)
    double *S;          // next stage state (stages 0-2; in FP64 it must be R)
    int stage;          // 0..3
    double dt, half_dt, sixth_dt;
};

int nmax_class(int n);
int sweep_lines_per_block(int dir, int n);
int sweep_threads_per_block(int dir, int n);
int sweep_known_rows_max(int n);

// Every stepping launcher below either launches for one box or, given a
// collector, adds its box to phase `phase` of a batched step (batch.hpp).
hipError_t launch_deriv(int dir, const double *f, double *d1, double *d2, const SweepGeom &g, const LinePlanDev &pl,
                        hipStream_t st);
// implicit filter of one field along dir with a filter plan (out may equal f)
hipError_t launch_filter(int dir, const double *f, double *out, const SweepGeom &g, const LinePlanDev &pl,
                         hipStream_t st);
// R <- R - D_dir(convective flux) for the 5 components (one launch per direction)
hipError_t launch_nse_sweep(int dir, const NseSweepArgs &a, const SweepGeom &g, const LinePlanDev &pl,
                            hipStream_t st, BatchCollector *col = nullptr, int phase = 0);

// RK4 register update of stage a.stage from R (point-wise over 5 fields)
hipError_t launch_rk_update(const NseSweepArgs &a, hipStream_t st, BatchCollector *col = nullptr, int phase = 0);

// Line-march sweeps along y (dir 1) and z (dir 2): geometry of the lines.
struct MarchGeom {
    int nx, no, n, nxc;     // lines along x, lines along the other axis, points per line, x chunks
    long long sD, sO, N3;   // strides of the line direction and of the other axis; points per field
};
// true if the plan's runs and closure slots fit the march kernels
bool march_usable(int dir, const LinePlanDev &pl);
// doubles of the closure array of one march sweep
size_t march_closure_elems(const int n[3], int dir, int ncl);
// Arguments of the line-march kernels (one box).
struct ClosureArgs {
    const double *Q;
    double *clo;
    MarchGeom g;
    LinePlanDev pl;
    NdConst c;
};
struct MarchArgs {
    const double *Q;
    void *R;          // FP64 or FP32, as the kernel instantiation says
    const double *clo;
    MarchGeom g;
    LinePlanDev pl;
    NdConst c;
    RkFuse F;
};
// closure rows of the 5 convective flux components along dir into clo
// (march_closure_elems doubles); nothing to do without closure rows
hipError_t launch_march_closures(int dir, const double *Q, double *clo, const int n[3], const LinePlanDev &pl,
                                 const NdConst &c, hipStream_t st, BatchCollector *col = nullptr, int phase = 0);
// R <- R - D_dir(convective flux) for the 5 components, closures from clo;
// r32: R is stored in FP32; c32: the elimination runs in FP32
hipError_t launch_march_runs(int dir, const double *Q, void *R, bool r32, bool c32, const double *clo, const int n[3],
                             const LinePlanDev &pl, const NdConst &c, hipStream_t st, const RkFuse *rk = nullptr,
                             BatchCollector *col = nullptr, int phase = 0);

// Planes per z chunk of the viscous kernel on an n[0] x n[1] x n[2] box
// (set_visc_z_chunk(0) restores the default).
int visc_z_chunk(const int n[3]);
void set_visc_z_chunk(int planes);
int visc_z_chunk_setting();   // 0: the default rule

// Viscous fluxes (explicit second order) + gravity source: R = div(Fv) + S.
hipError_t launch_visc(const double *Q, void *R, bool r32, const int n[3], const double ih[3], const NdConst &c,
                       hipStream_t st, BatchCollector *col = nullptr, int phase = 0);

// Wall conditions on one face pair (dir 0, 1, 2) of state Q.
hipError_t launch_bc(double *Q, const int n[3], int dir, const NdConst &c, hipStream_t st,
                     BatchCollector *col = nullptr, int phase = 0);

}  // namespace nopcs
