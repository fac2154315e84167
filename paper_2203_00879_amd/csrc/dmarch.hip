// dmarch.hip -- first derivative of one field along y or z as a line march
// (Section 3, Fig. 2).  A closure pass streams every line once and sums the
// closure rows (rows of the global A^-1 B at the piece cuts, Eqs. CS:fpCf and
// CS:fpCf_i) into per-line values; the march then streams every line again and
// solves the Thomas runs between the known rows, writing the derivative.  One
// thread owns one line; the lines of a block are consecutive in x, so each row
// a wavefront reads or writes is one contiguous segment, and no LDS staging or
// barrier is needed.  The arithmetic is that of the right-hand side's line
// march, with the field in place of a flux component and d1 = x in place of
// R -= x, so both agree with the LDS pencil solve up to rounding order.
#include "dmarch.hpp"

#include "kernels.hpp"

namespace nopcs {

namespace {

constexpr int DW = 128;    // lines per block (consecutive x)
constexpr int DRF = 8;     // closure pass: rows in flight per thread
constexpr int DMRL = 32;   // longest run a thread keeps in registers
constexpr int DRB = 8;     // run march: rows fetched ahead
constexpr int DS = 8;      // closure slots per row

struct DGeom {
    int nx, no, n, nxc;    // lines along x, lines along the other axis, points per line, x chunks
    long long sD, sO;      // strides of the line direction and of the other axis
};

DGeom dgeom(const int n[3], int dir) {
    DGeom g;
    g.nx = n[0];
    g.n = n[dir];
    if (dir == 1) {
        g.no = n[2];
        g.sD = n[0];
        g.sO = (long long)n[0] * n[1];
    } else {
        g.no = n[1];
        g.sD = (long long)n[0] * n[1];
        g.sO = n[0];
    }
    g.nxc = (n[0] + DW - 1) / DW;
    return g;
}

// Closure values of every line: slot s of a row sums C_{e,j} h (f_j - f_ref)
// over the taps j of the closure it serves (f_ref: the field at the first
// event row, which keeps the sums small), the closure row e itself subtracts
// (f_e - f_ref) times the closure's tap sum, and the completed slot, times
// 1/h, is the closure value.  Event rows (slots opening, meeting their row,
// closing) come from the plan in row order.
__global__ __launch_bounds__(DW) void k_dclosure(const double *__restrict__ f, double *__restrict__ clo, DGeom g,
                                                 LinePlanDev pl) {
    const int xc = (int)(blockIdx.x % (unsigned)g.nxc), o = (int)(blockIdx.x / (unsigned)g.nxc);
    const int x = xc * DW + (int)threadIdx.x;
    const bool ok = x < g.nx;
    const long long base = (ok ? x : 0) + g.sO * o;
    const long long nlines = (long long)g.nx * g.no;
    const long long line = (long long)x + (long long)g.nx * o;
    const auto cl_j0 = NOPCS_SCALAR_PTR(int, pl.cl_j0);
    const auto cl_len = NOPCS_SCALAR_PTR(int, pl.cl_len);
    const auto k1_rec = NOPCS_SCALAR_PTR(int, pl.k1_rec);
    const auto k1_w = NOPCS_SCALAR_PTR(double, pl.k1_w);
    const auto cl_wsum = NOPCS_SCALAR_PTR(double, pl.cl_wsum);
    const auto ev_row = NOPCS_SCALAR_PTR(int, pl.k1_evrow);
    const auto ev_msk = NOPCS_SCALAR_PTR(int, pl.k1_evmask);
    const int jlo = cl_j0[0];
    const int jhi = cl_j0[pl.ncl - 1] + cl_len[pl.ncl - 1] - 1;
    const double *const src = f + base;
    // rows past jhi repeat jhi (unconditional loads; never used)
    auto ld = [&](int j) { return src[g.sD * min(j, jhi)]; };
    double acc[DS];
#pragma unroll
    for (int s = 0; s < DS; ++s) acc[s] = 0.0;
    double fref = 0.0;
    double ring[DRF];
#pragma unroll
    for (int u = 0; u < DRF; ++u) ring[u] = ld(jlo + u);
    int e = 0;
    int jev = ev_row[0];   // the first event row is jlo (a slot opens there)
    for (int j0 = jlo; j0 <= jhi; j0 += DRF) {
#pragma unroll
        for (int u = 0; u < DRF; ++u) {
            const int j = j0 + u;
            const double fv = ring[u];
            ring[u] = ld(j + DRF);
            if (j > jhi) continue;   // uniform
            const auto wj = k1_w + (size_t)j * DS;
            if (j != jev) {
                const double gk = fv - fref;
#pragma unroll
                for (int s = 0; s < DS; ++s) acc[s] = fma_(wj[s], gk, acc[s]);
                continue;
            }
            if (e == 0) fref = fv;
            const int open = ev_msk[3 * e], erow = ev_msk[3 * e + 1], close = ev_msk[3 * e + 2];
            const auto rec = k1_rec + (size_t)j * DS;
            const double gk = fv - fref;
#pragma unroll
            for (int s = 0; s < DS; ++s) {
                if (open & (1 << s)) acc[s] = 0.0;
                acc[s] = fma_(wj[s], gk, acc[s]);
                if (erow & (1 << s)) acc[s] = acc[s] - gk * cl_wsum[rec[s] & 0xfff];
            }
            if (close) {
#pragma unroll
                for (int s = 0; s < DS; ++s)
                    if ((close & (1 << s)) && ok) clo[(long long)(rec[s] & 0xfff) * nlines + line] = acc[s] * pl.ih;
            }
            ++e;
            jev = e < pl.k1_nev ? ev_row[e] : -1;
        }
    }
}

// The runs of one group of one line: forward elimination with the closure
// and wall values as known rows (reciprocal pivots), back substitution, and
// the known rows this run owns.  Rows are read DRB steps ahead at clamped
// indices (unconditional loads); steps past the run compute nothing that is
// stored.
__global__ __launch_bounds__(DW) void k_dmarch(const double *__restrict__ f, double *__restrict__ d1,
                                               const double *__restrict__ clo, DGeom g, LinePlanDev pl) {
    __shared__ double KV[2 * kGroupRuns][DW];   // closure values bounding the group's runs (per thread)
    const int xc = (int)(blockIdx.x % (unsigned)g.nxc);
    const int rest = (int)(blockIdx.x / (unsigned)g.nxc), o = rest % g.no, grp = rest / g.no;
    const int lane = (int)threadIdx.x;
    const int x = xc * DW + lane;
    const bool ok = x < g.nx;
    const int n = g.n;
    const double ih = pl.ih;
    const long long sD = g.sD;
    const long long base = (ok ? x : 0) + g.sO * o;
    const long long nlines = (long long)g.nx * g.no;
    const long long line = (long long)x + (long long)g.nx * o;
    const double *const src = f + base;
    double *const dst = d1 + base;
    const auto runs_i = NOPCS_SCALAR_PTR(int, pl.runs);
    const auto slot_i = NOPCS_SCALAR_PTR(int, pl.run_slot);
    const auto grp_i = NOPCS_SCALAR_PTR(int, pl.grp);
    const auto run_own = NOPCS_SCALAR_PTR(int, pl.run_own);
    const auto rden = NOPCS_SCALAR_PTR(double, pl.rden);
    const auto cp = NOPCS_SCALAR_PTR(double, pl.cp);
    const int g0 = grp_i[2 * grp], g1 = grp_i[2 * grp + 1];
    // rows 0 .. n-1 only: a run's window starts at lo - 1 >= 0 (rows 0 and 1 are known)
    auto ld = [&](int row) { return src[sD * min(row, n - 1)]; };
    for (int r = g0; r < g1; ++r) {
        const int sx = slot_i[2 * r], sy = slot_i[2 * r + 1];
        const int j = 2 * (r - g0);
        NOPCS_LDS_BOUND(j + 1, 2 * kGroupRuns);
        if (sx >= 4) KV[j][lane] = ok ? clo[(long long)(sx - 4) * nlines + line] : 0.0;
        if (sy >= 4) KV[j + 1][lane] = ok ? clo[(long long)(sy - 4) * nlines + line] : 0.0;
    }
    const double alpha = kAlpha;
    for (int r = g0; r < g1; ++r) {
        const int lo = runs_i[2 * r], hi = runs_i[2 * r + 1], m = hi - lo - 1;
        const int sx = slot_i[2 * r], sy = slot_i[2 * r + 1];
        const int own = run_own[r];
        // window w0..w4 = f(i-2) .. f(i+2) for the row i = lo + 1 about to be solved
        double w0 = ld(lo - 1), w1 = ld(lo), w2 = ld(lo + 1), w3 = ld(lo + 2), w4 = ld(lo + 3);
        double ring[DRB];
#pragma unroll
        for (int t = 0; t < DRB; ++t) ring[t] = ld(lo + 4 + t);
        // known rows: closures from the closure pass, rows 1 and n-2 central,
        // rows 0 and n-1 one-sided
        double xlo, xhi = 0.0, v0 = 0.0, vn = 0.0;
        if (sx >= 4) xlo = KV[2 * (r - g0)][lane];
        else xlo = 0.5 * ih * (w2 - w0);   // row 1
        if (sy >= 4) xhi = KV[2 * (r - g0) + 1][lane];
        if (own & 4) v0 = 0.5 * ih * (4.0 * (w1 - w0) - (w2 - w0));   // row 0
        double d[DMRL];
        double dprev = 0.0;
#pragma unroll
        for (int t = 0; t < DMRL; ++t) {
            const int k = t + 1;
            double rr = ih * (kB1 * (w3 - w1) + kB2 * (w4 - w0));
            if (k == 1) rr = rr - alpha * xlo;
            if (k == m) {
                if (sy < 4) xhi = 0.5 * ih * (w4 - w2);   // row n-2
                if (own & 8) {
                    const double fl = w4;                  // row n-1
                    vn = -0.5 * ih * (4.0 * (w3 - fl) - (w2 - fl));
                }
                rr = rr - alpha * xhi;
            }
            // (r_k - alpha d_{k-1}) / den_k as r_k / den_k - c'_k d_{k-1}
            const double dp = fma_(-cp[min(k, m)], dprev, rr * rden[min(k, m)]);
            d[t] = t < m ? dp : 0.0;
            if (t < m) dprev = dp;
            w0 = w1;
            w1 = w2;
            w2 = w3;
            w3 = w4;
            w4 = ring[t % DRB];
            ring[t % DRB] = ld(lo + 4 + t + DRB);
        }
        // back substitution: x_m = d_m, x_k = d_k - c'_k x_{k+1}
        double xn = 0.0;
#pragma unroll
        for (int t = DMRL - 1; t >= 0; --t) {
            const int k = t + 1;
            const double xs = k == m ? d[t] : fma_(-cp[min(k, m)], xn, d[t]);
            const double xk = t < m ? xs : 0.0;
            xn = xk;
            if (ok && t < m) dst[sD * (lo + 1 + t)] = xk;
        }
        if (ok) {
            if (own & 1) dst[sD * lo] = xlo;
            if (own & 2) dst[sD * hi] = xhi;
            if (own & 4) dst[0] = v0;
            if (own & 8) dst[sD * (n - 1)] = vn;
        }
    }
}

}  // namespace

bool dmarch_usable(int dir, const LinePlanDev &pl) {
    if (dir != 1 && dir != 2) return false;
    if (pl.op != OP_D1 || !march_usable(dir, pl) || pl.max_m > DMRL) return false;
    return pl.ncl == 0 || pl.k1_S == DS;
}

size_t dmarch_closure_bytes(const int n[3], int dir, const LinePlanDev &pl) {
    const size_t lines = (size_t)n[0] * n[1] * n[2] / (size_t)n[dir];
    return (size_t)pl.ncl * lines * sizeof(double);
}

hipError_t launch_dmarch(int dir, const double *f, double *d1, double *clo, const int n[3], const LinePlanDev &pl,
                         hipStream_t st) {
    if (!dmarch_usable(dir, pl) || (pl.ncl > 0 && !clo)) return hipErrorInvalidValue;
    const DGeom g = dgeom(n, dir);
    if (pl.ncl > 0) {
        const long long blocks = (long long)g.nxc * g.no;
        hipLaunchKernelGGL(k_dclosure, dim3((unsigned)blocks), dim3(DW), 0, st, f, clo, g, pl);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const long long blocks = (long long)g.nxc * g.no * pl.ngrp;
    hipLaunchKernelGGL(k_dmarch, dim3((unsigned)blocks), dim3(DW), 0, st, f, d1, clo, g, pl);
    return hipGetLastError();
}

}  // namespace nopcs
