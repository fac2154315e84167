// march.hip -- convective sweeps along y and z that stream along the line.
//
// Lines along y and z are strided in memory.  Staging whole lines in LDS gives
// narrow pencils (a few consecutive x per row, scattered over many DRAM pages);
// here a block owns 128 neighbouring lines (consecutive x, so every load and
// store is one 1 KB row; 512-byte rows measured 25-30 % slower) and walks
// along the line direction, two wavefronts per flux component:
//
//   k_closure_march  one pass over the rows that carry taps accumulates every
//       closure row of the NOHAP split (Eqs. CS:fpCf, CS:fpCf_i) in a few
//       register slots,
//         f'_e = [sum_j C_ej (f_j - f_r) - (f_e - f_r) sum_j C_ej] / h,
//       with f_r the flux at the line's first row.  In exact arithmetic this is
//       sum_j C_ej (f_j - f_e) (the form the LDS sweeps use); both vanish
//       exactly for a constant field.  Results go to a small array
//       [component][closure][line].
//   k_march_sweep  walks a group of consecutive Thomas runs of a line: (B f)_i
//       from a five-value register window, forward elimination with the
//       tabulated reciprocal pivots (Section 3) into registers (runs of <= 32
//       unknowns),
//       back substitution fused with R -= f'.  The known rows bounding the runs
//       come from the closure pass or from the explicit wall rows.
//
// Rows of the state reach the block through a two-chunk LDS ring: the threads
// of component w fetch field w of the next few rows into registers while the
// block works on the current chunk, and publish them at the chunk boundary
// (one barrier per chunk).  Every thread forms its own flux component from the
// staged row.
// Arithmetic of the walls, the runs and the R update is operation for
// operation that of the LDS sweeps.
#include "kernels.hpp"

namespace nopcs {

namespace {

constexpr int MW = 128;     // lines per block (consecutive x; two wavefronts per component)
constexpr int MRL = 32;     // longest run a thread keeps in registers
constexpr int NCOMP = 5;    // flux components (one row of MW threads each) = state fields
constexpr int CHC = 4;      // rows per LDS chunk: closure pass
constexpr int CHM = 4;      // rows per LDS chunk: run march

// Convective flux component comp along DIR (ge3-ge5) from the staged row of
// one line.  Field 0 of a staged row holds 1/rho (the density threads take
// the reciprocal once per row when they publish); the products are those of
// prim_from, so the fluxes equal the LDS sweeps' bit for bit.
template <int DIR>
__device__ inline double flux_row(const double (*L)[MW], int lane, int comp, const NdConst &c) {
    if (comp == 0) return L[DIR + 1][lane];
    const double ri = L[0][lane], md = L[DIR + 1][lane];
    if (comp == 4 || comp == DIR + 1) {
        const double mx = L[1][lane], my = L[2][lane], mz = L[3][lane], Ep = L[4][lane];
        const double u = mx * ri, v = my * ri, w = mz * ri;
        const double ke = 0.5 * (mx * u + my * v + mz * w);
        const double pp = (c.gamma - 1.0) * (Ep - ke);
        const double ud = DIR == 1 ? v : w;
        if (comp == 4) return ((Ep + pp) + c.H) * ud;
        return md * ud + pp;
    }
    const double ud = md * ri;
    return L[comp][lane] * ud;
}

// Rows [row0, rowN] of the block's MW lines pass through a two-chunk LDS ring
// and are read strictly in order through next().  PF chunks are in flight in
// registers while the block works on the chunk in LDS (PF = 2 measured slower
// than 1 for both marches).
template <int CH, int PF = 1>
struct RowPipe {
    double (*L)[CH][NCOMP][MW];   // [2][CH][field][lane]
    const double *src;            // this thread's field at row 0 of its line (a valid
                                  // address also for lanes past the last line)
    long long sD;
    int row0, rowN, lane, field;
    int u, k;                     // next row to read: slot u of chunk k
    double pre[PF][CH];           // the next PF chunks, in flight
    // unconditional loads (no branches: the compiler's memory waits stay
    // precise); rows past rowN repeat row rowN and are never used.  The row
    // offset steps by sD (a uniform select stops it at rowN).
    __device__ void fetch(int rb, double (&dst)[CH]) {
        long long off = sD * min(rb, rowN);
#pragma unroll
        for (int v = 0; v < CH; ++v) {
            dst[v] = src[off];
            off += rb + v < rowN ? sD : 0;
        }
    }
    // field 0 (density) is published as 1/rho, the only form flux_row uses
    __device__ void publish(double (&val)[CH], int buf) {
        if (field == 0) {
#pragma unroll
            for (int v = 0; v < CH; ++v) val[v] = 1.0 / val[v];
        }
#pragma unroll
        for (int v = 0; v < CH; ++v) L[buf][v][field][lane] = val[v];
    }
    // before the first read: chunk 0 in LDS, chunks 1 .. PF in flight
    __device__ void start() {
        double c0[CH];
        fetch(row0, c0);
#pragma unroll
        for (int p = 0; p < PF; ++p) fetch(row0 + (p + 1) * CH, pre[p]);
        publish(c0, 0);
        u = 0;
        k = 0;
        __syncthreads();
    }
    // staged fields of the next row; the first read of chunk k >= 1 publishes
    // it and starts fetching chunk k + PF (uniform: every wavefront of the
    // block reads the same rows)
    __device__ const double (*next())[MW] {
        if (u == CH) {
            u = 0;
            ++k;
            publish(pre[0], k & 1);
            __syncthreads();
#pragma unroll
            for (int p = 0; p + 1 < PF; ++p)
#pragma unroll
                for (int v = 0; v < CH; ++v) pre[p][v] = pre[p + 1][v];
            fetch(row0 + (k + PF) * CH, pre[PF - 1]);
        }
        NOPCS_LDS_BOUND(u, CH);
        NOPCS_LDS_BOUND(k * CH + u, rowN - row0 + 1 + CH);
        return L[k & 1][u++];
    }
};

// ---------------------------------------------------------------------------
// Closure pass
// ---------------------------------------------------------------------------
template <int DIR, int S>
__device__ inline void closure_march_body(const double *__restrict__ Q, double *__restrict__ clo, const MarchGeom &g,
                                          const LinePlanDev &pl, const NdConst &c, int b) {
    __shared__ double L[2][CHC][NCOMP][MW];
    const int xc = b % g.nxc, o = b / g.nxc;
    const int lane = threadIdx.x;
    const int x = xc * MW + lane;
    const int comp = NOPCS_UNIFORM((int)threadIdx.y);
    const bool ok = x < g.nx;
    const long long base = x + g.sO * o;
    const long long nlines = (long long)g.nx * g.no;
    const long long line = x + (long long)g.nx * o;
    const auto cl_j0 = NOPCS_SCALAR_PTR(int, pl.cl_j0);
    const auto cl_len = NOPCS_SCALAR_PTR(int, pl.cl_len);
    const auto k1_rec = NOPCS_SCALAR_PTR(int, pl.k1_rec);
    const auto k1_w = NOPCS_SCALAR_PTR(double, pl.k1_w);
    const auto cl_wsum = NOPCS_SCALAR_PTR(double, pl.cl_wsum);
    const int jlo = cl_j0[0];
    const int jhi = cl_j0[pl.ncl - 1] + cl_len[pl.ncl - 1] - 1;
    RowPipe<CHC> P;
    P.L = L;
    P.src = Q + comp * g.N3 + (ok ? base : 0);
    P.sD = g.sD;
    P.row0 = jlo;
    P.rowN = jhi;
    P.lane = lane;
    P.field = comp;
    P.start();
    const auto ev_row = NOPCS_SCALAR_PTR(int, pl.k1_evrow);
    const auto ev_msk = NOPCS_SCALAR_PTR(int, pl.k1_evmask);
    // slot sums against one reference per line, the flux f_r of the first row:
    //   acc_s = sum_j C_ej (f_j - f_r) - (f_e - f_r) sum_j C_ej,
    // the second term taken when the slot meets its closure row e; equal to
    // sum_j C_ej (f_j - f_e) in real arithmetic and zero for a constant field
    double acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0;
    double fref = 0.0;
    // every slot accumulates every row (an idle slot carries a zero tap, which
    // leaves its sum unchanged); slots open, meet their closure row and close
    // only on the listed event rows, handled outside the plain row loop
    auto accumulate = [&](int j, double g) {
        const auto wj = k1_w + (size_t)j * S;
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = fma_(wj[s], g, acc[s]);
    };
    int j = jlo;
    for (int e = 0; e < pl.k1_nev; ++e) {
        const int je = ev_row[e];
        for (; j < je; ++j) accumulate(j, flux_row<DIR>(P.next(), lane, comp, c) - fref);
        const double f = flux_row<DIR>(P.next(), lane, comp, c);
        if (e == 0) fref = f;   // the first event row is the line's first row (a slot opens there)
        const double g = f - fref;
        const int open = ev_msk[3 * e], erow = ev_msk[3 * e + 1], close = ev_msk[3 * e + 2];
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (open & (1 << s)) acc[s] = 0.0;
        accumulate(j, g);
        const auto rec = k1_rec + (size_t)j * S;
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (erow & (1 << s)) acc[s] = acc[s] - g * cl_wsum[rec[s] & 0xfff];
        if (close) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (close & (1 << s)) {
                    const int qi = rec[s] & 0xfff;
                    if (ok) clo[((long long)comp * pl.ncl + qi) * nlines + line] = acc[s] * pl.ih;
                }
            }
        }
        ++j;
    }
}

// Closure pass with one thread per line: each thread streams its own line,
// loads the 5 state fields of a row itself, forms the 5 flux components and
// accumulates every slot of every component in registers -- no LDS, no
// barriers; the fields of the next CPL rows are in flight in registers.  The
// arithmetic (1/rho, the flux products, each slot's sum in row order) is that
// of k_closure_march, so the closure values are the same bit for bit.  Used for
// plans of at most 8 slots (5 x 8 accumulators).
constexpr int CLW = 128;   // lines per block
constexpr int CPL = 4;     // rows in flight per thread

template <int DIR>
__device__ inline void closure_line_body(const double *__restrict__ Q, double *__restrict__ clo, const MarchGeom &g,
                                         const LinePlanDev &pl, const NdConst &c, int b) {
    constexpr int S = 8;
    const int nxb = (g.nx + CLW - 1) / CLW;
    const int xc = b % nxb, o = b / nxb;
    const int x = xc * CLW + (int)threadIdx.x;
    const bool ok = x < g.nx;
    const long long base = (ok ? x : 0) + g.sO * o;
    const long long nlines = (long long)g.nx * g.no;
    const long long line = x + (long long)g.nx * o;
    const auto cl_j0 = NOPCS_SCALAR_PTR(int, pl.cl_j0);
    const auto cl_len = NOPCS_SCALAR_PTR(int, pl.cl_len);
    const auto k1_rec = NOPCS_SCALAR_PTR(int, pl.k1_rec);
    const auto k1_w = NOPCS_SCALAR_PTR(double, pl.k1_w);
    const auto cl_wsum = NOPCS_SCALAR_PTR(double, pl.cl_wsum);
    const auto ev_row = NOPCS_SCALAR_PTR(int, pl.k1_evrow);
    const auto ev_msk = NOPCS_SCALAR_PTR(int, pl.k1_evmask);
    const int jlo = cl_j0[0];
    const int jhi = cl_j0[pl.ncl - 1] + cl_len[pl.ncl - 1] - 1;
    const long long sD = g.sD, N3 = g.N3;
    // the 5 fields of row j (rows past jhi repeat jhi; unconditional loads)
    auto load = [&](int j, double (&q)[NCOMP]) {
        const long long off = base + sD * min(j, jhi);
#pragma unroll
        for (int f = 0; f < NCOMP; ++f) q[f] = Q[f * N3 + off];
    };
    // the 5 flux components of a row (the products of flux_row)
    auto fluxes = [&](const double (&q)[NCOMP], double (&fx)[NCOMP]) {
        const double ri = 1.0 / q[0];
        const double mx = q[1], my = q[2], mz = q[3], Ep = q[4];
        const double md = DIR == 1 ? my : mz;
        const double u = mx * ri, v = my * ri, w = mz * ri;
        const double ke = 0.5 * (mx * u + my * v + mz * w);
        const double pp = (c.gamma - 1.0) * (Ep - ke);
        const double ud = DIR == 1 ? v : w;
        const double uo = md * ri;   // the form flux_row uses for the passive components
        fx[0] = md;
        fx[1] = mx * uo;
        fx[2] = DIR == 1 ? md * ud + pp : my * uo;
        fx[3] = DIR == 2 ? md * ud + pp : mz * uo;
        fx[4] = ((Ep + pp) + c.H) * ud;
    };
    double acc[NCOMP][S];
#pragma unroll
    for (int k = 0; k < NCOMP; ++k)
#pragma unroll
        for (int s = 0; s < S; ++s) acc[k][s] = 0.0;
    double fref[NCOMP] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double ring[CPL][NCOMP];
#pragma unroll
    for (int u = 0; u < CPL; ++u) load(jlo + u, ring[u]);
    int e = 0;
    int jev = ev_row[0];   // the first event row is jlo (a slot opens there)
    for (int j0 = jlo; j0 <= jhi; j0 += CPL) {
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            const int j = j0 + u;
            double q[NCOMP];
#pragma unroll
            for (int f = 0; f < NCOMP; ++f) q[f] = ring[u][f];
            load(j + CPL, ring[u]);
            if (j > jhi) continue;   // uniform
            double fx[NCOMP];
            fluxes(q, fx);
            const auto wj = k1_w + (size_t)j * S;
            if (j != jev) {
#pragma unroll
                for (int k = 0; k < NCOMP; ++k) {
                    const double gk = fx[k] - fref[k];
#pragma unroll
                    for (int s = 0; s < S; ++s) acc[k][s] = fma_(wj[s], gk, acc[k][s]);
                }
                continue;
            }
            // event row: slots open, meet their closure row or close here
            if (e == 0) {
#pragma unroll
                for (int k = 0; k < NCOMP; ++k) fref[k] = fx[k];
            }
            const int open = ev_msk[3 * e], erow = ev_msk[3 * e + 1], close = ev_msk[3 * e + 2];
            const auto rec = k1_rec + (size_t)j * S;
#pragma unroll
            for (int k = 0; k < NCOMP; ++k) {
                const double gk = fx[k] - fref[k];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (open & (1 << s)) acc[k][s] = 0.0;
                    acc[k][s] = fma_(wj[s], gk, acc[k][s]);
                    if (erow & (1 << s)) acc[k][s] = acc[k][s] - gk * cl_wsum[rec[s] & 0xfff];
                }
            }
            if (close) {
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (close & (1 << s)) {
                        const int qi = rec[s] & 0xfff;
#pragma unroll
                        for (int k = 0; k < NCOMP; ++k)
                            if (ok) clo[((long long)k * pl.ncl + qi) * nlines + line] = acc[k][s] * pl.ih;
                    }
                }
            }
            ++e;
            jev = e < pl.k1_nev ? ev_row[e] : -1;
        }
    }
}

// ---------------------------------------------------------------------------
// Run march
// ---------------------------------------------------------------------------
// TR: storage type of R; TC: arithmetic of the elimination (B f is formed in
// FP64 from the FP64 window and rounded once; known rows stay FP64).
// RKS >= 0: RK4 stage RKS fused into the epilogue, see RkFuse (R and the
// elimination both FP64, or both FP32).
template <int DIR, bool FULL, class TR, class TC, int RKS>
__device__ inline void march_sweep_body(const double *__restrict__ Q, TR *R, const double *__restrict__ clo,
                                        const MarchGeom &g, const LinePlanDev &pl, const NdConst &c, const RkFuse &F,
                                        int b) {
    static_assert(RKS < 0 || sizeof(TR) == sizeof(TC), "the fused RK update: FP64 or mixed precision");
    __shared__ double L[2][CHM][NCOMP][MW];
    __shared__ double KV[2 * kGroupRuns][NCOMP][MW];   // closure values bounding the group's runs
    const int xc = b % g.nxc, rest = b / g.nxc, o = rest % g.no, grp = rest / g.no;
    const int lane = threadIdx.x;
    const int x = xc * MW + lane;
    const int comp = NOPCS_UNIFORM((int)threadIdx.y);
    const bool ok = FULL || x < g.nx;   // FULL: nx is a multiple of MW
    const int n = g.n;
    const double ih = pl.ih;
    const long long sD = g.sD;
    const long long base = x + g.sO * o;
    const long long nlines = (long long)g.nx * g.no;
    const long long line = x + (long long)g.nx * o;
    TR *Rc = R + comp * g.N3 + (ok ? base : 0);   // this component's R at row 0 of the line
    const double *clc = clo + (long long)comp * pl.ncl * nlines + (ok ? line : 0);
    // int2 tables read as int pairs through the scalar path
    const auto runs_i = NOPCS_SCALAR_PTR(int, pl.runs);
    const auto slot_i = NOPCS_SCALAR_PTR(int, pl.run_slot);
    const auto grp_i = NOPCS_SCALAR_PTR(int, pl.grp);
    auto runs = [&](int r) { return make_int2(runs_i[2 * r], runs_i[2 * r + 1]); };
    auto run_slot = [&](int r) { return make_int2(slot_i[2 * r], slot_i[2 * r + 1]); };
    const auto run_own = NOPCS_SCALAR_PTR(int, pl.run_own);
    const auto rden = NOPCS_SCALAR_PTR(TC, (sizeof(TC) == 8 ? (const void *)pl.rden : (const void *)pl.rden32));
    const auto cp = NOPCS_SCALAR_PTR(TC, (sizeof(TC) == 8 ? (const void *)pl.cp : (const void *)pl.cp32));
    const int2 gr = make_int2(grp_i[2 * grp], grp_i[2 * grp + 1]);
    const int lo0 = runs(gr.x).x;

    // closure values of the group's run bounds, read once into LDS (each
    // thread reads back only what it wrote)
    for (int r = gr.x; r < gr.y; ++r) {
        const int2 slot = run_slot(r);
        const int j = 2 * (r - gr.x);
        NOPCS_LDS_BOUND(j + 1, 2 * kGroupRuns);
        if (slot.x >= 4) KV[j][comp][lane] = ok ? clc[(long long)(slot.x - 4) * nlines] : 0.0;
        if (slot.y >= 4) KV[j + 1][comp][lane] = ok ? clc[(long long)(slot.y - 4) * nlines] : 0.0;
    }
    RowPipe<CHM> P;
    P.L = L;
    P.src = Q + comp * g.N3 + (ok ? base : 0);
    P.sD = sD;
    P.row0 = lo0 - 1;
    P.rowN = runs(gr.y - 1).y + 1;
    P.lane = lane;
    P.field = comp;
    P.start();

    // window: w0..w4 = f(i-2) .. f(i+2) for the row i about to be solved
    int i = lo0 + 1;
    double w0 = flux_row<DIR>(P.next(), lane, comp, c);
    double w1 = flux_row<DIR>(P.next(), lane, comp, c);
    double w2 = flux_row<DIR>(P.next(), lane, comp, c);
    double w3 = flux_row<DIR>(P.next(), lane, comp, c);
    double w4 = flux_row<DIR>(P.next(), lane, comp, c);
    auto advance = [&]() {
        w0 = w1;
        w1 = w2;
        w2 = w3;
        w3 = w4;
        w4 = flux_row<DIR>(P.next(), lane, comp, c);   // row i + 3 (a dummy past the group's last row)
        ++i;
    };

    // Fused RK4 stage (RKS >= 0): back substitution in place, then per row
    // k = R - f' and the register update of RKS (operation for operation that
    // of k_rk_update, k rounded from R's type to FP64 as there); stage 0-2 write
    // K and the next stage state S, stage 3 writes Qn.  Rows are fetched RB
    // steps ahead at clamped rows; steps past the run store nothing.
    double *const Kc = RKS >= 0 ? F.K + comp * g.N3 + (ok ? base : 0) : nullptr;
    double *const Nc = RKS >= 0 ? F.Qn + comp * g.N3 + (ok ? base : 0) : nullptr;
    // FP64: the next stage state goes over R (same element offsets as Rc);
    // mixed precision: into F.S
    double *const Sm = RKS < 0 || RKS == 3 || sizeof(TR) == 8 ? nullptr : F.S + comp * g.N3 + (ok ? base : 0);
    auto store_s = [&](long long off, double v) {
        if constexpr (sizeof(TR) == 8) reinterpret_cast<double *>(Rc)[off] = v;
        else Sm[off] = v;
    };
    auto rk_point = [&](long long off, double rv, double kk, double qn, double x) {
        const double kv = double(TR(TR(rv) - TR(x)));   // R - f' in R's type, as the unfused march
        if constexpr (RKS == 0) {
            Kc[off] = kv;
            store_s(off, qn + F.half_dt * kv);
        } else if constexpr (RKS == 1) {
            Kc[off] = kk + 2.0 * kv;
            store_s(off, qn + F.half_dt * kv);
        } else if constexpr (RKS == 2) {
            Kc[off] = kk + 2.0 * kv;
            store_s(off, qn + F.dt * kv);
        } else {
            Nc[off] = qn + F.sixth_dt * (kk + kv);
        }
    };
    auto rk_epilogue = [&](TC (&d)[MRL], int m, int lo, int hi, int own, double xlo, double xhi, double v0,
                           double vn) {
        TC xn = TC(0);
#pragma unroll
        for (int t = MRL - 1; t >= 0; --t) {
            const int k = t + 1;
            const TC xs = k == m ? d[t] : fma_(-cp[min(k, m)], xn, d[t]);   // k > m: unused, read in range
            d[t] = t < m ? xs : TC(0);
            xn = d[t];
        }
        constexpr int RB = 4;
        auto rrow = [&](int t) { return sD * (lo + 1 + (t < m ? t : m - 1)); };
        // the known rows this run may update (rows outside lo+1 .. hi-1)
        const long long klo = sD * lo, khi = sD * hi, kn = sD * (n - 1);
        auto known_rows = [&]() {
            const double rlo = double(Rc[klo]), rhi = double(Rc[khi]), r0 = double(Rc[0]), rn = double(Rc[kn]);
            const double klo_k = RKS > 0 ? Kc[klo] : 0.0, khi_k = RKS > 0 ? Kc[khi] : 0.0;
            const double k0_k = RKS > 0 ? Kc[0] : 0.0, kn_k = RKS > 0 ? Kc[kn] : 0.0;
            const double qlo = Nc[klo], qhi = Nc[khi], q0 = Nc[0], qnn = Nc[kn];
            if (ok) {
                if (own & 1) rk_point(klo, rlo, klo_k, qlo, xlo);
                if (own & 2) rk_point(khi, rhi, khi_k, qhi, xhi);
                if (own & 4) rk_point(0, r0, k0_k, q0, v0);
                if (own & 8) rk_point(kn, rn, kn_k, qnn, vn);
            }
        };
        // the known rows first, so that their operands do not stay live through
        // the row loop (each row is read and written by this thread only; this
        // keeps the FP64 stage kernels within their registers, without spills)
        known_rows();
        double fr[RB], fk[RB], fq[RB];
#pragma unroll
        for (int t = 0; t < RB; ++t) {
            fr[t] = double(Rc[rrow(t)]);
            fk[t] = RKS > 0 ? Kc[rrow(t)] : 0.0;
            fq[t] = Nc[rrow(t)];
        }
#pragma unroll
        for (int t = 0; t < MRL; ++t) {
            const double rv = fr[t % RB], kk = fk[t % RB], qn = fq[t % RB];
            if (t + RB < MRL) {
                fr[t % RB] = double(Rc[rrow(t + RB)]);
                if (RKS > 0) fk[t % RB] = Kc[rrow(t + RB)];
                fq[t % RB] = Nc[rrow(t + RB)];
            }
            if (ok && t < m) rk_point(rrow(t), rv, kk, qn, double(d[t]));
        }
    };

    for (int r = gr.x; r < gr.y; ++r) {
        const int2 run = runs(r);
        const int lo = run.x, hi = run.y, m = hi - lo - 1;
        while (i < lo + 1) advance();
        const int2 slot = run_slot(r);
        const int own = run_own[r];
        // known rows: closures from the closure pass, rows 1 and n-2 central,
        // rows 0 and n-1 one-sided (the formulas of the LDS sweeps)
        double xlo = 0.0, xhi = 0.0, v0 = 0.0, vn = 0.0;
        if (slot.x >= 4) xlo = KV[2 * (r - gr.x)][comp][lane];
        else xlo = 0.5 * ih * (w2 - w0);   // row 1 (i = 2)
        if (slot.y >= 4) xhi = KV[2 * (r - gr.x) + 1][comp][lane];
        if (own & 4) v0 = 0.5 * ih * (4.0 * (w1 - w0) - (w2 - w0));   // row 0 (i = 2)
        TC d[MRL];
#pragma unroll
        for (int t = 0; t < MRL; ++t) d[t] = TC(0);
        TC dprev = TC(0);
        const TC alpha = TC(kAlpha);
#pragma unroll
        for (int t = 0; t < MRL; ++t) {
            if (t < m) {
                const int k = t + 1;
                const double rr64 = ih * (kB1 * (w3 - w1) + kB2 * (w4 - w0));
                TC rr = TC(rr64);
                if (k == 1) rr = rr - alpha * TC(xlo);
                if (k == m) {
                    if (slot.y < 4) xhi = 0.5 * ih * (w4 - w2);   // row n-2 (i = n-3)
                    if (own & 8) {
                        const double fl = w4;                         // row n-1
                        vn = -0.5 * ih * (4.0 * (w3 - fl) - (w2 - fl));
                    }
                    rr = rr - alpha * TC(xhi);
                }
                // (r_k - alpha d_{k-1}) / den_k as r_k / den_k - c'_k d_{k-1}
                const TC dp = fma_(-cp[k], dprev, rr * rden[k]);
                d[t] = dp;
                dprev = dp;
                advance();
            }
        }
        if constexpr (RKS >= 0) {
            rk_epilogue(d, m, lo, hi, own, xlo, xhi, v0, vn);
            continue;
        }
        // back substitution (x_m = d_m, x_k = d_k - c'_k x_{k+1}) fused with
        // R -= f'.  The loop is straight-line over MRL steps so that memory
        // waits stay precise: steps t >= m use x = 0 on the run's last row,
        // which rewrites that row's original value before its real update.
        // R rows are fetched RA steps ahead, each load issued before the store
        // that follows it.
        constexpr int RA = 8;
        auto rrow = [&](int t) { return sD * (lo + 1 + (t < m ? t : m - 1)); };
        TR ring[RA];
#pragma unroll
        for (int t = MRL - RA; t < MRL; ++t) ring[t % RA] = Rc[rrow(t)];
        // R of the known rows this run may update (rows outside lo+1 .. hi-1)
        const TR rlo = Rc[sD * lo], rhi = Rc[sD * hi], r0 = Rc[0], rn = Rc[sD * (n - 1)];
        TC xn = TC(0);
#pragma unroll
        for (int t = MRL - 1; t >= 0; --t) {
            const int k = t + 1;
            const TC xs = k == m ? d[t] : fma_(-cp[min(k, m)], xn, d[t]);   // k > m: unused, read in range
            const TC xk = t < m ? xs : TC(0);
            xn = xk;
            const TR nv = ring[t % RA] - TR(xk);
            if (t - RA >= 0) ring[t % RA] = Rc[rrow(t - RA)];
            if (ok) Rc[rrow(t)] = nv;
        }
        if (ok) {
            if (own & 1) Rc[sD * lo] = rlo - TR(xlo);
            if (own & 2) Rc[sD * hi] = rhi - TR(xhi);
            if (own & 4) Rc[0] = r0 - TR(v0);
            if (own & 8) Rc[sD * (n - 1)] = rn - TR(vn);
        }
    }
}

// ---------------------------------------------------------------------------
// Kernels: one box (block b of its own grid) or a batch of boxes (a walk over
// a table of boxes, see batch.hpp); both run the bodies above.
// ---------------------------------------------------------------------------
template <int DIR, int S>
struct ClosureMarchBody {
    using Args = ClosureArgs;
    __device__ static void run(const Args &a, int b, int) { closure_march_body<DIR, S>(a.Q, a.clo, a.g, a.pl, a.c, b); }
};
template <int DIR>
struct ClosureLineBody {
    using Args = ClosureArgs;
    __device__ static void run(const Args &a, int b, int) { closure_line_body<DIR>(a.Q, a.clo, a.g, a.pl, a.c, b); }
};
template <int DIR, bool FULL, class TR, class TC, int RKS>
struct MarchBody {
    using Args = MarchArgs;
    __device__ static void run(const Args &a, int b, int) {
        march_sweep_body<DIR, FULL, TR, TC, RKS>(a.Q, static_cast<TR *>(a.R), a.clo, a.g, a.pl, a.c, a.F, b);
    }
};

}  // namespace

bool march_usable(int dir, const LinePlanDev &pl) {
    if (dir != 1 && dir != 2) return false;
    if (pl.nrun < 1 || pl.max_m > MRL || pl.max_m < 1) return false;
    if (pl.ncl > 0 && pl.k1_S != 8 && pl.k1_S != kMaxSlots) return false;
    return pl.ngrp >= 1;
}

size_t march_closure_elems(const int n[3], int dir, int ncl) {
    const size_t lines = (size_t)n[0] * n[1] * n[2] / (size_t)n[dir];
    return (size_t)NCOMP * (size_t)ncl * lines;
}

MarchGeom march_geom(const int n[3], int dir) {
    MarchGeom g;
    g.nx = n[0];
    g.n = n[dir];
    g.N3 = (long long)n[0] * n[1] * n[2];
    if (dir == 1) {
        g.no = n[2];
        g.sD = n[0];
        g.sO = (long long)n[0] * n[1];
    } else {
        g.no = n[1];
        g.sD = (long long)n[0] * n[1];
        g.sO = n[0];
    }
    g.nxc = (n[0] + MW - 1) / MW;
    return g;
}

hipError_t launch_march_closures(int dir, const double *Q, double *clo, const int n[3], const LinePlanDev &pl,
                                 const NdConst &c, hipStream_t st, BatchCollector *col, int phase) {
    if (pl.ncl == 0) return hipSuccess;
    const ClosureArgs a{Q, clo, march_geom(n, dir), pl, c};
    // at most 8 slots: one thread per line; 16 slots: the LDS ring pass
    if (pl.k1_S == 8) {
        const int blocks = ((a.g.nx + CLW - 1) / CLW) * a.g.no;
        if (dir == 1) return run_body<ClosureLineBody<1>, CLW>(a, blocks, dim3(CLW), st, col, phase);
        if (dir == 2) return run_body<ClosureLineBody<2>, CLW>(a, blocks, dim3(CLW), st, col, phase);
        return hipErrorInvalidValue;
    }
    const int blocks = a.g.nxc * a.g.no;
    const dim3 blk(MW, NCOMP);
    if (dir == 1) return run_body<ClosureMarchBody<1, kMaxSlots>, MW * NCOMP>(a, blocks, blk, st, col, phase);
    if (dir == 2) return run_body<ClosureMarchBody<2, kMaxSlots>, MW * NCOMP>(a, blocks, blk, st, col, phase);
    return hipErrorInvalidValue;
}

// the run march of one instantiation for one box (or added to a batch)
template <int DIR, class TR, class TC, int RKS>
static hipError_t march_go(const MarchArgs &a, hipStream_t st, BatchCollector *col, int phase) {
    const int blocks = (int)((long long)a.g.nxc * a.g.no * a.pl.ngrp);
    const dim3 blk(MW, NCOMP);
    if (a.g.nx % MW == 0)   // FULL: every lane holds a line
        return run_body<MarchBody<DIR, true, TR, TC, RKS>, MW * NCOMP>(a, blocks, blk, st, col, phase);
    return run_body<MarchBody<DIR, false, TR, TC, RKS>, MW * NCOMP>(a, blocks, blk, st, col, phase);
}

template <class T>
static hipError_t march_rk_go(const MarchArgs &a, int stage, hipStream_t st, BatchCollector *col, int phase) {
    switch (stage) {
        case 0: return march_go<2, T, T, 0>(a, st, col, phase);
        case 1: return march_go<2, T, T, 1>(a, st, col, phase);
        case 2: return march_go<2, T, T, 2>(a, st, col, phase);
        case 3: return march_go<2, T, T, 3>(a, st, col, phase);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_march_runs(int dir, const double *Q, void *R, bool r32, bool c32, const double *clo, const int n[3],
                             const LinePlanDev &pl, const NdConst &c, hipStream_t st, const RkFuse *rk,
                             BatchCollector *col, int phase) {
    MarchArgs a{Q, R, clo, march_geom(n, dir), pl, c, RkFuse{}};
    if (rk) {
        // z sweep with the RK4 stage update fused (R and the elimination both
        // FP64 or both FP32)
        if (dir != 2 || r32 != c32) return hipErrorInvalidValue;
        a.F = *rk;
        return r32 ? march_rk_go<float>(a, rk->stage, st, col, phase) : march_rk_go<double>(a, rk->stage, st, col, phase);
    }
    if (dir == 1) {
        if (!c32) return march_go<1, double, double, -1>(a, st, col, phase);
        if (!r32) return march_go<1, double, float, -1>(a, st, col, phase);
        return march_go<1, float, float, -1>(a, st, col, phase);
    }
    if (dir == 2) {
        if (!c32) return march_go<2, double, double, -1>(a, st, col, phase);
        if (!r32) return march_go<2, double, float, -1>(a, st, col, phase);
        return march_go<2, float, float, -1>(a, st, col, phase);
    }
    return hipErrorInvalidValue;
}

}  // namespace nopcs
