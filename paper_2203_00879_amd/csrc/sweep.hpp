// sweep.hpp -- LDS-staged pencil sweeps of the NOHAP compact first derivative.
//
// A workgroup stages a pencil of P lines (full length along the sweep
// direction) of one field in LDS and evaluates the segmented compact solve
// there (Section 3):
//   A: every thread forms (B f)_i for the compact rows it owns and the explicit
//      wall rows; closure threads form the truncated equivalent explicit sums
//      f'_e = sum_j C_{e,j} (f_j - f_e) / h of the segment ends (Eq. CS:fpCf_i,
//      global rows of C; the f_e shift is exact for the untruncated row and
//      makes constant fields differentiate to exactly zero);
//   B: results written back in place;
//   C: one thread per (line, run) runs the Thomas algorithm with tabulated
//      pivots on the compact rows between two known rows.
// Lines along x are contiguous in HBM, lines along y and z are gathered P at a
// time from neighbouring x positions so every HBM access is a coalesced row.
#pragma once

#include "common.hpp"
#include "plan.hpp"

namespace nopcs {

template <int DIR, int NMAX>
struct SweepCfg {
    static constexpr int P = DIR == 0 ? (NMAX <= 128 ? 16 : 2048 / NMAX) : (NMAX <= 256 ? 16 : 4096 / NMAX);
    static constexpr int NT = DIR == 0 ? 256 : (NMAX <= 64 ? 128 : NMAX <= 128 ? 256 : 512);
    static constexpr int PTS = (P * NMAX + NT - 1) / NT;   // points owned per thread
    static constexpr int CLPT = 4;                          // closures per thread (max)
    static constexpr int PITCH = NMAX + NMAX / 16 + 1;      // x layout: padded line pitch
    static constexpr int LDS = DIR == 0 ? P * PITCH : NMAX * P;
    __device__ static int idx(int l, int i) {
        if (DIR == 0) return l * PITCH + i + (i >> 4);
        return i * P + l;
    }
    // owned point s of thread t: pencil-local (line, position)
    __device__ static void owned(int q, int n, int &l, int &i) {
        if (DIR == 0) { l = q / n; i = q - l * n; }
        else { i = q / P; l = q - i * P; }
    }
};

// Strides of the sweep direction (D), the pencil direction (A: lines of one
// pencil) and the remaining direction (B) in elements.
struct SweepGeom {
    long long sD, sA, sB;
    int nA, nB, n;
};

inline SweepGeom sweep_geom(const int n[3], int dir) {
    const long long sx = 1, sy = n[0], sz = (long long)n[0] * n[1];
    SweepGeom g;
    if (dir == 0) { g.sD = sx; g.sA = sy; g.sB = sz; g.nA = n[1]; g.nB = n[2]; }
    else if (dir == 1) { g.sD = sy; g.sA = sx; g.sB = sz; g.nA = n[0]; g.nB = n[2]; }
    else { g.sD = sz; g.sA = sx; g.sB = sy; g.nA = n[0]; g.nB = n[1]; }
    g.n = n[dir];
    return g;
}

// Segmented compact solve of the P staged lines in F (FP64).  All threads of
// the block must call it; it ends with a barrier and leaves f' in F.
template <int DIR, int NMAX>
__device__ inline void lds_line_solve(double *F, const LinePlanDev &pl, int np) {
    using C = SweepCfg<DIR, NMAX>;
    const int tid = threadIdx.x;
    const int n = pl.n;
    const double ih = pl.ih;
    double dreg[C::PTS];
    double creg[C::CLPT];
    // ---- A: explicit parts, reading F ----
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        const int q = tid + s * C::NT;
        dreg[s] = 0.0;
        if (q < C::P * n) {
            int l, i;
            C::owned(q, n, l, i);
            if (l < np) {
                const uint8_t kind = pl.row_kind[i];
                if (kind == ROW_COMPACT) {
                    dreg[s] = ih * (kB1 * (F[C::idx(l, i + 1)] - F[C::idx(l, i - 1)]) +
                                    kB2 * (F[C::idx(l, i + 2)] - F[C::idx(l, i - 2)]));
                } else if (kind == ROW_WALL) {
                    if (i == 0) {
                        const double f0 = F[C::idx(l, 0)];
                        dreg[s] = 0.5 * ih * (4.0 * (F[C::idx(l, 1)] - f0) - (F[C::idx(l, 2)] - f0));
                    } else if (i == 1) {
                        dreg[s] = 0.5 * ih * (F[C::idx(l, 2)] - F[C::idx(l, 0)]);
                    } else if (i == n - 2) {
                        dreg[s] = 0.5 * ih * (F[C::idx(l, n - 1)] - F[C::idx(l, n - 3)]);
                    } else {
                        const double fl = F[C::idx(l, n - 1)];
                        dreg[s] = -0.5 * ih * (4.0 * (F[C::idx(l, n - 2)] - fl) - (F[C::idx(l, n - 3)] - fl));
                    }
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < C::CLPT; ++c) {
        const int q = tid + c * C::NT;
        creg[c] = 0.0;
        if (q < C::P * pl.ncl) {
            const int l = q % C::P, e = q / C::P;
            if (l < np) {
                const int row = pl.cl_row[e], j0 = pl.cl_j0[e], len = pl.cl_len[e];
                const double *coef = pl.cl_coef + (size_t)e * kTaps;
                const double fe = F[C::idx(l, row)];
                double acc = 0.0;
                for (int t = 0; t < len; ++t) acc += coef[t] * (F[C::idx(l, j0 + t)] - fe);
                creg[c] = acc * ih;
            }
        }
    }
    __syncthreads();
    // ---- B: write back ----
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        const int q = tid + s * C::NT;
        if (q < C::P * n) {
            int l, i;
            C::owned(q, n, l, i);
            if (l < np && pl.row_kind[i] != ROW_CLOSURE) F[C::idx(l, i)] = dreg[s];
        }
    }
#pragma unroll
    for (int c = 0; c < C::CLPT; ++c) {
        const int q = tid + c * C::NT;
        if (q < C::P * pl.ncl) {
            const int l = q % C::P, e = q / C::P;
            if (l < np) F[C::idx(l, pl.cl_row[e])] = creg[c];
        }
    }
    __syncthreads();
    // ---- C: Thomas on every run, known end rows lo and hi ----
    for (int q = tid; q < C::P * pl.nrun; q += C::NT) {
        const int l = q % C::P, r = q / C::P;
        if (l >= np) continue;
        const int2 run = pl.runs[r];
        const int lo = run.x, hi = run.y, m = hi - lo - 1;
        const double xlo = F[C::idx(l, lo)], xhi = F[C::idx(l, hi)];
        double dprev = 0.0;
        for (int k = 1; k <= m; ++k) {
            const int i = lo + k;
            double rr = F[C::idx(l, i)];
            if (k == 1) rr = rr - kAlpha * xlo;
            if (k == m) rr = rr - kAlpha * xhi;
            const double dp = (rr - kAlpha * dprev) / pl.den[k];
            F[C::idx(l, i)] = dp;
            dprev = dp;
        }
        double xnext = dprev;
        for (int k = m - 1; k >= 1; --k) {
            const int i = lo + k;
            const double x = F[C::idx(l, i)] - pl.cp[k] * xnext;
            F[C::idx(l, i)] = x;
            xnext = x;
        }
    }
    __syncthreads();
}

}  // namespace nopcs
