/*
 * nopcs.h -- C ABI of libnopcs.so, the MI355X (gfx950) implementation of the
 * non-overlapping parallel compact scheme (NOHAP closure on OUCS3) and of the
 * compressible Navier-Stokes stepping that consumes it, after "Ultrasound
 * Triggering of Rayleigh-Taylor Instability: Solution of Compressible
 * Navier-Stokes Equation by a Non-Overlapping Parallel Compact Scheme"
 * (Sundaram, Sengupta & Sengupta).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Fields live in device memory (HBM), FP64, structure-of-arrays, x fastest:
 *    element (i, j, k) of a field is at offset i + n[0] * (j + n[1] * k).
 *    y is the vertical direction; gravity acts along -y.
 *  - A state Q holds 5 such fields back to back: rho, rho u, rho v, rho w, E',
 *    non-dimensional (Section 2, eqs. ge14-ge15; velocity scale sqrt(g L),
 *    pressure scale rho_s g L).  E' = rho e_t - Rh / (gamma - 1) with
 *    Rh = R T_s / (g L): the total energy minus the constant energy of the
 *    reference state p = Rh (an exact shift that keeps low-Mach round-off small).
 *  - Nodes sit on the walls: the spacing along d is h_d = len[d] / (n[d] - 1).
 *  - Every call is asynchronous on the HIP stream passed in (NULL = the null
 *    stream); the caller owns all buffers passed in and must keep them alive
 *    until the stream has run the work.  The library never frees them.
 *  - Return value: NOPCS_OK (0) or a negative NOPCS_E* code; nothing throws
 *    across the ABI.  Argument errors are reported synchronously and launch
 *    nothing; nopcs_last_error() gives a message for the calling thread.
 *    Device faults surface at the next synchronising call.
 *  - The library owns cached per-grid plans (segment tables, closure rows,
 *    elimination tables) in device memory; nopcs_release_plans() frees them.
 */
#ifndef NOPCS_H
#define NOPCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NOPCS_OK = 0,
    NOPCS_EINVAL = -1,     /* invalid argument (sizes, segments, pointers, precision) */
    NOPCS_ENOMEM = -2,     /* device or host allocation failed, or over the HBM budget */
    NOPCS_EDEVICE = -3,    /* a HIP runtime call failed */
    NOPCS_EAGAIN = -4,     /* request still pending (solver_poll) */
    NOPCS_ENOTFOUND = -5,  /* unknown or already released request id */
    NOPCS_ENONFINITE = -6, /* a request's final state holds NaN or Inf */
    NOPCS_EBUSY = -7       /* request queue full */
};

enum {
    NOPCS_FP64 = 0,   /* every step in FP64 */
    NOPCS_MIXED = 1   /* rk_step: the Thomas eliminations of the y and z sweeps run in
                         FP32 on (B f)_i rounded once from FP64; the x sweep (and any
                         line that falls back to the LDS pencil) stages and solves in
                         FP32 each flux less its line's first-row value; the viscous
                         differences, stresses, heat fluxes and their divergence run
                         in FP32 from primitives rounded once; the RHS register is
                         FP32.  Closure rows, wall rows, the gravity source and the
                         RK registers (state, accumulator, stage state) stay FP64.
                         nse_rhs, whose R is the caller's FP64 array: only the y and
                         z eliminations (line marches) run in FP32. */
};

/* Uniform box.  n[d] >= 8 points along x, y, z; len[d] > 0 non-dimensional edge
 * (units of L); nseg[d] >= 1 non-overlapping segments along d (Section 3, Fig. 2),
 * split as evenly as possible (the first n % nseg segments get one extra point),
 * each segment at least 4 points long. */
typedef struct {
    int32_t n[3];
    double len[3];
    int32_t nseg[3];
} nopcs_grid;

/* Physical parameters in SI units (Section 2); the library non-dimensionalizes:
 * U_s = sqrt(g L), Rh = R_gas T_s / (g L), M^2 = g L / (gamma R_gas T_s),
 * mu_s = Sutherland(T_s) with (mu_ref, T_ref, S_suth), Re = rho_s U_s L / mu_s,
 * bulk viscosity mu_b = mub_a T* - mub_b [Pa s] (eq. reg: mub_a = 3.381e-4,
 * mub_b = 7.383e-4).  viscous = 0 drops the viscous fluxes, gravity = 0 the
 * source term ge8a. */
typedef struct {
    double gamma, R_gas, g, L, T_s, rho_s, Pr, mu_ref, T_ref, S_suth, mub_a, mub_b;
    int32_t viscous, gravity;
} nse_params;

/* Message of the last failed call on this thread ("" if none). */
const char *nopcs_last_error(void);

/* ABI version (major * 100 + minor). */
int nopcs_version(void);

/* Free every cached plan on the current device (not thread-safe against
 * concurrent calls). */
int nopcs_release_plans(void);

/* Workspace (device bytes) needed by nse_rhs and rk_step for this grid and
 * precision: three 5-field registers (the RK4 accumulator, the stage state and
 * the right-hand side, FP64, the last FP32 under NOPCS_MIXED; nse_rhs leaves
 * them untouched), then the closure array of the sweeps along y and z (5
 * components x closure rows x lines, the larger direction), and under
 * NOPCS_MIXED a second FP64 stage register.  When the z sweep carries the RK4
 * update it writes the next stage state over the right-hand side (FP64) or
 * into the other stage register (mixed), so registers swap roles between
 * stages; their contents between calls are unspecified.  Depends on the piece
 * length in force (nopcs_set_piece_length).  Host only; returns 0 on invalid
 * input. */
size_t nopcs_workspace_bytes(const nopcs_grid *grid, int precision);

/*
 * nopcs_line_plan -- host-only introspection of the segmented line plan that
 * nopcs_derivative uses along a line of n points cut into nseg segments
 * (Section 3, Fig. 2), each further cut into pieces of at most piece_len points
 * (0: no extra cuts; -1: the library's own choice for this n).
 * Outputs (each may be NULL; cap bounds every array):
 *   *nrun, runs[2*r] = (lo, hi): known rows bounding each Thomas run (unknowns lo+1..hi-1);
 *   *ncl, rows[q]: closure rows; coef[97*q + t]: C_{e, e-48+t} * h (0 outside the line)
 *   with C the global A^-1 B (Eqs. CS:fpCf, CS:fpCf_i).
 * Returns NOPCS_OK, NOPCS_EINVAL (bad n/nseg) or NOPCS_ENOMEM (cap too small).
 * Touches no device.
 */
int nopcs_line_plan(int32_t n, int32_t nseg, int32_t piece_len, int32_t cap, int32_t *nrun, int32_t *runs,
                    int32_t *ncl, int32_t *rows, double *coef);

/*
 * nopcs_derivative -- first and/or second derivative along one direction.
 *
 * Computes f' from the OUCS3 compact scheme [A]{f'} = [B]{f} (Section 3,
 * Eq. CS:AfpBf; interior A = (alpha, 1, alpha), B antisymmetric with b1, b2)
 * with the NOHAP sub-domain closure: each line along `dir` is cut into
 * grid->nseg[dir] non-overlapping segments; the first and last point of every
 * segment that is not a wall row take the truncated equivalent explicit value
 * f'_e = sum_{|k|<=48} C_{e,e+k} f_{e+k} with C the row of the global
 * A^-1 B (Eqs. CS:fpCf and CS:fpCf_i), and the remaining rows of each segment
 * are solved independently by the Thomas algorithm.  The result equals the
 * sequential single-domain solve up to round-off (Section 3).  Rows 0 and
 * n-1 use the second-order one-sided difference and rows 1 and n-2 the
 * second-order central difference (the physical-boundary closure, which the
 * paper cites without giving).  The second derivative is the same operator
 * applied twice.  The library may cut segments further into shorter
 * independent pieces with the same closure; results change by round-off only.
 *
 * dir: 0 = x, 1 = y, 2 = z.  precision: NOPCS_FP64 (NOPCS_MIXED is rejected here).
 * f: device, n0*n1*n2 doubles (read only).  d1, d2: device outputs of the same
 * size, either may be NULL but not both; they must not overlap f.
 * The first derivative alone (d2 NULL) along y or z on a box with at least
 * 2^17 lines along dir runs as a closure pass and a line march (one thread per
 * line), with the closure values in scratch taken with hipMallocAsync on
 * hip_stream and freed there (8 bytes per closure row and line); every other
 * case runs as a staged pencil solve in LDS (see nopcs_set_deriv_form).
 */
int nopcs_derivative(const nopcs_grid *grid, int dir, int precision, const double *f, double *d1, double *d2,
                     void *hip_stream);

/*
 * nopcs_set_deriv_form -- how nopcs_derivative, nopcs_vorticity_budget and the
 * compact viscous variant (nse_rhs_compact_viscous, rk_step_compact_viscous)
 * compute first derivatives alone along y or z: 0 (the default) the line march
 * on boxes with at least 2^17 lines along the direction and the pencil solve on
 * smaller ones; 1 always the pencil solve; 2 always the line march (where the
 * plan allows: runs of at most 32 unknowns and at most 8 closure slots per
 * row, else the pencil).  The forms differ by rounding order only.  A call
 * that marches takes its closure values (8 bytes per closure row and line of
 * the larger marching direction) with hipMallocAsync on its stream and frees
 * them there.  Process-wide; NOPCS_EINVAL for other values.
 */
int nopcs_set_deriv_form(int32_t form);

/*
 * nopcs_vorticity_workspace_bytes -- bytes of device workspace that
 * nopcs_vorticity_budget needs for this grid (19 fields, each rounded up to
 * 32 doubles); 0 (with an error message) for an invalid grid.
 */
size_t nopcs_vorticity_workspace_bytes(const nopcs_grid *grid);

/*
 * nopcs_vorticity_budget -- vorticity and the three source terms on the right of
 * the inviscid vorticity transport equation (Eq. eqn12_1), the terms the
 * paper's analysis of RTI onset compares (Section 5): vortex stretching
 * (omega . grad) V, dilatation -omega (div V) and the baroclinic term
 * (grad rho x grad p) / rho^2.
 *
 * V = (rho u, rho v, rho w) / rho and p' = (gamma - 1)(E' - rho |V|^2 / 2)
 * (ge12, ge13; the reference pressure is constant and drops out of grad p).
 * Every derivative is the compact first derivative of nopcs_derivative along
 * x, y or z (with grid->nseg segments), so all 15 gradients share its accuracy.
 *
 * params: only gamma is used (all fields are still checked).  Q: device state,
 * 5 fields of n0*n1*n2 doubles (read only).  out: device output, 12 fields of
 * n0*n1*n2 doubles: omega_x, omega_y, omega_z, stretching (x, y, z),
 * dilatation (x, y, z), baroclinic (x, y, z); must not overlap Q or ws.  ws:
 * device workspace of at least nopcs_vorticity_workspace_bytes(grid) bytes,
 * 256-byte aligned (NOPCS_EINVAL otherwise); its contents on return are
 * unspecified.  Work is queued on hip_stream; the call does not wait for it.
 */
int nopcs_vorticity_budget(const nse_params *params, const nopcs_grid *grid, const double *Q, double *out, void *ws,
                           size_t ws_bytes, void *hip_stream);

/*
 * nopcs_disturbance_pressure -- the disturbance pressure of Section 4: the
 * pressure of state Q minus that of a reference state Q0 (the initial,
 * hydrostatic box), out = (gamma - 1)((E' - E'_0) - (K - K_0)) with
 * K = (rho u u + rho v v + rho w w) / 2 (ge12, ge13), i.e. p(Q) - p(Q0) formed
 * without the two large pressures.  Q, Q0: device states (5 fields of
 * n0*n1*n2 doubles, read only); out: device, n0*n1*n2 doubles, must not overlap
 * them.  params: only gamma is used.  Asynchronous on hip_stream.
 */
int nopcs_disturbance_pressure(const nse_params *params, const nopcs_grid *grid, const double *Q, const double *Q0,
                               double *out, void *hip_stream);

/*
 * nopcs_line_spectrum -- amplitude spectrum of one line of samples, as the
 * paper takes of the disturbance pressure along y (Section 4):
 *   amp[k] = |sum_{j<n} f[j*stride] exp(-2 pi i j k / n)| / n,  k = 0 .. n/2,
 * by a direct transform (one block per k; phases reduced exactly in integers).
 * f: device, read at f[j*stride] for j < n (the caller guarantees those
 * elements exist); amp: device, n/2 + 1 doubles.  2 <= n <= 16384 and
 * stride >= 1, else NOPCS_EINVAL.  Asynchronous on hip_stream.
 */
int nopcs_line_spectrum(const double *f, int32_t n, int64_t stride, double *amp, void *hip_stream);

/*
 * nse_rhs -- right-hand side of the non-dimensional compressible NSE (ge17):
 *   R = dEv/dx + dFv/dy + dGv/dz + S - (dE/dx + dF/dy + dG/dz)
 * with convective fluxes ge3-ge5 differentiated by the NOHAP compact scheme
 * (as nopcs_derivative), viscous fluxes ge6-ge8 with the stresses of ge19 and
 * bv1-bv3 (bulk viscosity from eq. reg, no Stokes hypothesis), heat flux ge20
 * and gravity source ge8a, the viscous terms by second-order explicit
 * differences (Section 4), central inside and one-sided on wall nodes.
 *
 * Q: device state (5 fields, read only); R: device output (5 fields), must not
 * overlap Q.  ws: device workspace of at least nopcs_workspace_bytes(grid,
 * precision) bytes, 256-byte aligned, not overlapping Q or R (NOPCS_EINVAL
 * otherwise); its contents on return are unspecified.
 */
int nse_rhs(const nse_params *params, const nopcs_grid *grid, int precision, const double *Q, double *R, void *ws,
            size_t ws_bytes, void *hip_stream);

/*
 * nse_rhs_noalloc -- nse_rhs for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same kernels and the same result as nse_rhs (bit for bit),
 * with no workspace argument: the only scratch nse_rhs needs, the closure
 * array of the y and z line marches (5 components x closure rows x lines
 * doubles of the larger direction), lives in a static device array of
 * NOPCS_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and never builds a plan: the grid's line plans
 * must already be cached on the current device by an earlier call with the
 * same grid and piece lengths (nse_rhs, rk_step, nopcs_derivative, ...),
 * else NOPCS_EINVAL.  Grids whose closure array exceeds the static array
 * (about 256^3 with the default pieces) get NOPCS_EINVAL with a message, before
 * any device work.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (nothing in it needs clearing: each closure
 * value is written before it is read): calls that overlap on one GPU -- on
 * different streams or from different threads -- race and must not be
 * issued.  Q: device state (5 fields, read only); R: device output (5 fields),
 * not overlapping Q.  Asynchronous on hip_stream.
 */
#define NOPCS_NOALLOC_SCRATCH_BYTES (64u << 20)
int nse_rhs_noalloc(const nse_params *params, const nopcs_grid *grid, int precision, const double *Q, double *R,
                    void *hip_stream);

/*
 * nopcs_compact_viscous_workspace_bytes -- bytes of device workspace that
 * nse_rhs_compact_viscous needs: nopcs_workspace_bytes(grid, NOPCS_FP64) plus
 * 28 fields (u, v, w, T, 12 gradients, 12 viscous flux components), each
 * rounded up to 32 doubles; 0 (with an error message) for an invalid grid.
 */
size_t nopcs_compact_viscous_workspace_bytes(const nopcs_grid *grid);

/*
 * nse_rhs_compact_viscous -- the right-hand side of ge17 as nse_rhs, with the
 * viscous terms differentiated by the compact first derivative instead of the
 * explicit second-order differences: the gradients of u, v, w and T inside Ev,
 * Fv, Gv (ge6-ge8, ge19, ge20, bv1-bv3) and the divergence of those fluxes
 * each take the NOHAP compact D1 of nopcs_derivative along x, y or z (with
 * grid->nseg segments).  This is the D1-based viscous variant of the paper's
 * own setup (Section 4 uses the explicit scheme, which nse_rhs implements).
 * Convective terms and the gravity source are as in nse_rhs; FP64 only.
 *
 * Q: device state (5 fields, read only); R: device output (5 fields), must not
 * overlap Q or ws.  ws: device workspace of at least
 * nopcs_compact_viscous_workspace_bytes(grid) bytes, 256-byte aligned
 * (NOPCS_EINVAL otherwise); its contents on return are unspecified.
 */
int nse_rhs_compact_viscous(const nse_params *params, const nopcs_grid *grid, const double *Q, double *R, void *ws,
                            size_t ws_bytes, void *hip_stream);

/*
 * rk_step -- advance Q by nsteps steps of the classical four-stage RK4
 * (Section 4) at fixed dt (non-dimensional time, units of sqrt(L/g)):
 *   k1 = R(Q), k2 = R(Q + dt/2 k1), k3 = R(Q + dt/2 k2), k4 = R(Q + dt k3),
 *   Q <- Q + dt/6 (k1 + 2 k2 + 2 k3 + k4),
 * applying the wall conditions of the closed, adiabatic box (Section 2) to
 * every stage state and to the new state: zero momentum; wall temperature
 * from the one-sided second-order normal derivative of T set to zero; wall
 * density evolved by continuity; E' from the equation of state.  Faces are
 * treated in the order x, y, z.
 *
 * Q: device state, in/out, 16-byte aligned.  ws: device workspace of at least
 * nopcs_workspace_bytes(grid, precision) bytes, 256-byte aligned.
 */
int rk_step(const nse_params *params, const nopcs_grid *grid, int precision, double *Q, double dt, int32_t nsteps,
            void *ws, size_t ws_bytes, void *hip_stream);

/*
 * nopcs_filter -- the implicit 3D filter of Section 4, in place on a state.
 * The paper applies an implicit filter with filtering coefficient 0.135 every
 * 50 steps and cites it without printing it; it is read here as the
 * fourth-order tridiagonal compact filter
 *   af fh_{i-1} + fh_i + af fh_{i+1}
 *       = a0 f_i + (a1/2)(f_{i+1} + f_{i-1}) + (a2/2)(f_{i+2} + f_{i-2}),
 *   a0 = 5/8 + 3 af / 4,  a1 = 1/2 + af,  a2 = -1/8 + af / 4,
 * on rows 2 .. n-3 of every line (rows 0, 1, n-2, n-1 unfiltered), solved
 * with the NOHAP closure of Section 3 exactly as nopcs_derivative solves the
 * derivative: each segment end takes the truncated row (|j - e| <= 48) of the
 * global A_f^-1 B_f, the rest of each segment is an independent Thomas run;
 * the result equals the one-segment solve up to round-off.  Every one of the
 * 5 fields is filtered along x, then y, then z, then the wall conditions of
 * rk_step are applied.  alpha_f (0.135 in the paper) must lie in (-0.5, 0.5).
 * Q: device state, 5 fields, in/out.  Asynchronous on hip_stream.
 */
int nopcs_filter(const nse_params *params, const nopcs_grid *grid, double alpha_f, double *Q, void *hip_stream);

/*
 * rk_step_filtered -- rk_step with the implicit filter of nopcs_filter
 * applied after every filter_every-th step, counting from this call's first
 * step (Section 4: every 50 steps, alpha_f = 0.135); filter_every = 0 never
 * filters.  Arguments otherwise as rk_step.
 */
int rk_step_filtered(const nse_params *params, const nopcs_grid *grid, int precision, double *Q, double dt,
                     int32_t nsteps, int32_t filter_every, double alpha_f, void *ws, size_t ws_bytes,
                     void *hip_stream);

/*
 * rk_step_compact_viscous -- rk_step in FP64 with the right-hand side of
 * nse_rhs_compact_viscous (viscous terms by the compact first derivative):
 * the same four stages, registers and wall conditions.  ws: at least
 * nopcs_compact_viscous_workspace_bytes(grid) bytes, 256-byte aligned; Q
 * 16-byte aligned.  Launches directly (no graph replay).
 */
int rk_step_compact_viscous(const nse_params *params, const nopcs_grid *grid, double *Q, double dt, int32_t nsteps,
                            void *ws, size_t ws_bytes, void *hip_stream);

/*
 * rk_step_batch -- rk_step for a batch of independent boxes of any sizes, all
 * with the same parameters and precision, each with its own dt (box.dt, or the
 * call's dt where box.dt is 0).  Boxes too small to fill the device alone
 * (under 2^21 points) share their launches: one launch per stage kernel and
 * configuration covers all of them, its blocks taking their (box, block)
 * items from a device table of the boxes' arguments; each larger box runs its
 * own launches.  The step is captured once as a HIP graph holding one branch
 * per large box and one for the shared launches (cached per batch: boxes,
 * their states, workspaces and dt, parameters, precision, piece lengths and
 * mode) and each of the nsteps steps is one replay on hip_stream
 * (nopcs_set_batch_mode selects other arrangements).  Every box gets exactly
 * the result of rk_step on it alone (its blocks run the single-box kernels'
 * arithmetic).  1 <= nbox <= NOPCS_MAX_BATCH; each box: a valid grid, Q
 * 16-byte aligned, ws of at least nopcs_workspace_bytes(grid, precision)
 * bytes, 256-byte aligned, dt >= 0; no two boxes may share a state or a
 * workspace.  NOPCS_EINVAL on argument errors (before any device work).
 */
#define NOPCS_MAX_BATCH 64
typedef struct {
    nopcs_grid grid;
    double *Q;               /* device state, in/out */
    void *ws;                /* device workspace of this box */
    size_t ws_bytes;
    double dt;               /* this box's step; 0: the call's dt */
} nopcs_box;

int rk_step_batch(const nse_params *params, int32_t nbox, const nopcs_box *boxes, int precision, double dt,
                  int32_t nsteps, void *hip_stream);

/*
 * nopcs_set_batch_mode -- how rk_step_batch runs a step: 0 every box in the
 * shared launches, replayed as a graph; 1 one graph branch per box holding
 * that box's own launches (the boxes overlap on the device through the
 * branches); 2 every box in the shared launches, issued directly on
 * hip_stream every step without a graph; 3 (the default) shared launches for
 * the small boxes and a branch for each large one, as above.  Every mode gives
 * every box its lone result.  Process-wide; NOPCS_EINVAL for other values.
 */
int nopcs_set_batch_mode(int32_t mode);

/* ------------------------------------------------------------------------ */
/* Tuning.                                                                    */
/* ------------------------------------------------------------------------ */
/*
 * nopcs_set_piece_length -- length of the extra cuts that the library makes
 * inside every NOHAP segment along direction dir (0, 1, 2) before solving, in
 * points: -1 restores the library's own choice (no cuts for n <= 64, else 32),
 * 0 makes no extra cuts (one Thomas run per segment, the sequential order of
 * Section 3), and a value >= 8 cuts every segment into pieces of at most that
 * many points, each closed like a segment end (Eqs. CS:fpCf, CS:fpCf_i).
 * Results change by round-off only.  The setting is process-wide and applies
 * to calls made after it returns; plans already built for other lengths stay
 * cached.  A later call whose grid then needs more known rows per line than a
 * block holds fails with NOPCS_EINVAL.  Returns NOPCS_OK or NOPCS_EINVAL.
 * Touches no device.
 */
int nopcs_set_piece_length(int32_t dir, int32_t piece_len);

/*
 * nopcs_autotune -- choose the piece length of each direction for this box by
 * timing rk_step (one untimed step, then two timed with HIP events on
 * hip_stream) on a scratch copy of Q for each candidate (n <= 64: 0, 16, 32;
 * longer lines: 16, 24, 32 points), one direction after the other, and leave
 * the fastest set with nopcs_set_piece_length (process-wide); then the
 * viscous kernel's z chunk (16, 32, 64, 128 planes, nopcs_set_visc_chunk).  Candidates whose
 * closure array would not fit ws_bytes are skipped.  Q is not modified; the
 * call allocates and frees a 5-field scratch state and synchronises hip_stream.
 * piece_out[3]: the lengths in force on return.  Results of later calls change
 * by round-off only.
 */
/*
 * nopcs_set_visc_chunk -- planes per z chunk of the viscous kernel (one block
 * marches a 28 x 12-column tile over that many planes, re-reading two planes
 * at each chunk end): 0 restores the default (64 planes, halved down to 16
 * while the box would have fewer than 1024 blocks), else 8..1024 (larger than
 * nz means one chunk).  Results do not
 * depend on it (every plane is computed by one chunk with the same
 * arithmetic).  Process-wide; NOPCS_EINVAL outside the range.
 * nopcs_visc_chunk -- the chunk in force for this grid, or NOPCS_EINVAL.
 */
int nopcs_set_visc_chunk(int32_t planes);
int32_t nopcs_visc_chunk(const nopcs_grid *grid);

int nopcs_autotune(const nse_params *params, const nopcs_grid *grid, int precision, const double *Q, void *ws,
                   size_t ws_bytes, void *hip_stream, int32_t piece_out[3]);

/*
 * nopcs_set_graphs -- on != 0: rk_step captures one RK4 step (all its kernel
 * launches) into a HIP graph on a private stream, the first time it sees a given
 * (device, state pointer, workspace pointer, box, parameters, precision, dt,
 * piece lengths), and replays that graph nsteps times on the caller's stream;
 * results are bit for bit those of the launches themselves.  Graphs are cached
 * (at most 64 by default, nopcs_set_graph_cache_limit) and freed by
 * nopcs_release_plans.  Kernel timing
 * (nopcs_timing_*) does not see launches inside graphs.  on == 0 (the default)
 * launches every kernel directly.  Process-wide; returns NOPCS_OK.
 */
int nopcs_set_graphs(int32_t on);

/*
 * nopcs_set_graph_cache_limit -- the number of cached steps (graphs of
 * rk_step and rk_step_batch, and the collected launches of batch mode 2) the
 * library keeps, 1..4096 (default 64).  When a new step would exceed it, the
 * least recently replayed entries are freed, each after its replays have run;
 * lowering the limit frees entries at once the same way.  A serving loop whose
 * batches change often holds one entry per batch it has seen, each with its
 * device tables (a few KB) and graph.  Process-wide; NOPCS_EINVAL outside the
 * range.
 */
int nopcs_set_graph_cache_limit(int32_t n);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of many boxes on one GPU.                    */
/* ------------------------------------------------------------------------ */
typedef struct nopcs_solver nopcs_solver;

typedef struct {
    size_t hbm_budget_bytes; /* device bytes the solver may hold for resident requests */
    int32_t max_slots;       /* maximum requests resident on the device at once */
    int32_t max_queue;       /* maximum requests waiting for admission */
    int32_t device;          /* HIP device ordinal */
    int32_t batched;         /* 0: each resident request steps on its own stream;
                                1: all resident requests step together through
                                rk_step_batch, one batch in flight at a time
                                (switched off on the GPU: solver_create answers
                                NOPCS_EINVAL; only the CPU build of the
                                kernels runs it) */
} solver_config;

typedef struct {
    nse_params params;
    nopcs_grid grid;
    int32_t nsteps;          /* RK4 steps to run, >= 1 */
    int32_t precision;       /* NOPCS_FP64 or NOPCS_MIXED */
    double dt;               /* fixed non-dimensional step, > 0 */
    const double *Q0_host;   /* initial state, host, 5*n0*n1*n2 doubles; copied at submit */
} solve_request;

typedef struct {
    int32_t status;          /* NOPCS_OK, NOPCS_EAGAIN or an error */
    int32_t steps_done;
    double t_submit, t_admit, t_done; /* seconds on the solver's monotonic clock */
} solve_result;

/* Create a solver: one stream per slot (default priority) and a worker thread that
 * admits queued requests in arrival order while a slot is free and their device
 * footprint (state + nopcs_workspace_bytes) fits hbm_budget_bytes, and keeps every
 * resident request advancing in chunks of RK4 steps (continuous batching): on the
 * request's own stream (batched = 0), or, with batched = 1, in batched steps over
 * every resident request (rk_step_batch per group of requests with the same
 * parameters and precision; a chunk advances every member by the steps the
 * member closest to its end has left, at most 8).  Either way a request's
 * arithmetic is that of rk_step on its box alone, in the request's precision,
 * NOPCS_FP64 or NOPCS_MIXED.  *out is owned by the caller until solver_destroy. */
int solver_create(const solver_config *cfg, nopcs_solver **out);

/* Queue a request (non-blocking; the initial state is copied).  NOPCS_EBUSY if the
 * queue is full; NOPCS_ENOMEM if the request alone exceeds the HBM budget. */
int solver_submit(nopcs_solver *s, const solve_request *req, uint64_t *id_out);

/* NOPCS_EAGAIN while pending; once finished, copies the final state into Q_out_host
 * (5*n0*n1*n2 doubles, may be NULL), fills *out, releases the request and returns
 * its status (NOPCS_OK or NOPCS_ENONFINITE).  Unknown / released id: NOPCS_ENOTFOUND. */
int solver_poll(nopcs_solver *s, uint64_t id, double *Q_out_host, solve_result *out);

/* Seconds on the solver's monotonic clock (the clock of solve_result). */
double solver_now(nopcs_solver *s);

/* Stop the admission thread, drop pending requests and free device memory. */
int solver_destroy(nopcs_solver *s);

/* ------------------------------------------------------------------------ */
/* Kernel timing (instrumentation).                                           */
/* ------------------------------------------------------------------------ */
enum {
    NOPCS_K_VISCOUS = 0,  /* viscous fluxes + gravity source (writes R)          */
    NOPCS_K_SWEEP_X = 1,  /* convective x sweep (R -= D_x E)                      */
    NOPCS_K_SWEEP_Y = 2,  /* convective y sweep (R -= D_y F)                      */
    NOPCS_K_SWEEP_Z = 3,  /* convective z sweep (R -= D_z G; in rk_step with the  */
                          /* z line march it also makes the RK4 update)           */
    NOPCS_K_WALL = 4,     /* wall conditions (one launch per face pair)          */
    NOPCS_K_DERIV = 5,    /* standalone derivative; the vorticity budget's 15     */
                          /* first derivatives                                    */
    NOPCS_K_RK = 6,       /* RK4 register update of one stage (when not fused)    */
    NOPCS_K_CLOSURE_Y = 7,/* closure rows of the y sweep (line-march pass)         */
    NOPCS_K_CLOSURE_Z = 8,/* closure rows of the z sweep (line-march pass)         */
    NOPCS_K_VORT = 9,     /* diagnostics: point-wise parts of the vorticity       */
                          /* budget, disturbance pressure, line spectrum          */
    NOPCS_K_FILTER = 10,  /* implicit filter along one direction (one field)      */
    NOPCS_K_COUNT = 11
};

/* on != 0: from now on every kernel launched by this library is bracketed by a
 * pair of HIP events recorded on the stream it is launched on; previous records
 * and totals are cleared.  on == 0 stops recording (totals are kept). */
int nopcs_timing_enable(int on);

/* Per-kernel totals of the recorded launches: waits for the recorded events,
 * adds their durations and returns the totals since the last enable.
 * kernel: one of NOPCS_K_*; total_ms, launches may be NULL. */
int nopcs_timing_read(int32_t kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* NOPCS_H */
