// sweep.hpp -- LDS-staged pencil sweeps of the NOHAP compact first derivative.
//
// A workgroup stages a pencil of P full lines along the sweep direction, for up
// to G field components at once, in LDS and evaluates the segmented compact
// solve of Section 3 there, in three phases separated by barriers:
//   A  known rows: the explicit wall rows and the segment-end (closure) rows
//      f'_e = sum_j C_{e,j} (f_j - f_e) / h with C the global A^-1 B truncated
//      to |j - e| <= 48 (Eqs. CS:fpCf, CS:fpCf_i; the f_e shift is exact for the
//      untruncated row and makes constant fields differentiate to exactly 0),
//      walked over aligned 32-row blocks with a per-plan coefficient table.
//      Results go to a side array KN, so known rows of F keep their f values.
//   C  one thread per (line, run) -- a run is the set of compact rows between
//      two known rows -- forms (B f)_i from a five-point register window and
//      runs the Thomas algorithm (tabulated reciprocal pivots) with the known rows as
//      boundary values, overwriting the run's rows of F with f'.  The rows just
//      outside a run are known rows and are never overwritten, so runs need no
//      halo exchange.
//   E  owned points read f' (from F or KN) and apply the caller's epilogue.
// Lines along x are contiguous in HBM; lines along y and z are gathered P at a
// time from neighbouring x positions so every HBM access is a coalesced row.
#pragma once

#include "common.hpp"
#include "plan.hpp"

namespace nopcs {

template <int DIR, int NMAX, int PW = 0, int NTH = 256>
struct SweepCfg {
    // lines per pencil: every configuration keeps the block within 64 KB of LDS;
    // PW > 0 sets it (a single-component kernel can afford wider pencils)
    static constexpr int P = PW > 0 ? PW : NMAX <= 128 ? 1024 / NMAX : 2048 / NMAX;
    static constexpr int NT = NTH;                                   // threads per block
    static constexpr int PTS = (P * NMAX) / NT;                      // owned slots per thread
    static constexpr int G = 2;                                      // components per LDS pass
    static constexpr int KMAX = NMAX <= 128 ? NMAX / 2 + 4 : NMAX / 8 + 8;
    static constexpr int PAD = (NMAX >> 5) * 2 + 2;
    static constexpr int PITCH = NMAX + PAD + 1;                     // x layout line pitch
    static constexpr int FSZ = DIR == 0 ? P * PITCH : NMAX * P + PAD;
    static constexpr int RSTEP = DIR == 0 ? 1 : P;                   // LDS step between rows of a line
    // LDS index of (line l, position i) inside one component buffer; the
    // 2-double step every 32 positions spreads concurrent runs over the banks
    __device__ static int fidx(int l, int i) {
        const int ix = DIR == 0 ? l * PITCH + i + ((i >> 5) << 1) : i * P + l + ((i >> 5) << 1);
        NOPCS_LDS_BOUND(l, P);
        NOPCS_LDS_BOUND(i, NMAX);
        NOPCS_LDS_BOUND(ix, FSZ);
        return ix;
    }
    // index of (known-row slot s, line l) inside one component of KN
    __device__ static int kidx(int s, int l) {
        NOPCS_LDS_BOUND(s, KMAX);
        NOPCS_LDS_BOUND(l, P);
        return s * P + l;
    }
    // owned slot q -> (line, position); valid when l < lines and i < n
    __device__ static void owned(int q, int &l, int &i) {
        if (DIR == 0) { l = q / NMAX; i = q % NMAX; }
        else { l = q % P; i = q / P; }
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

// Phases A and C for NC components staged in F[c].  Known-row values land in
// KN(c)[slot * P + l] (FP64).  All threads of the block call it; it ends with
// a barrier; f' is then in F (compact rows) and KN (known rows).
// TF = float (mixed precision): F holds FP32 values; the closure and wall rows
// are still summed in FP64 from them, the Thomas runs eliminate in FP32 with
// the plan's FP32 pivot tables.
// OP = OP_FILTER applies the plan's implicit filter instead of the first
// derivative: closure rows f_e + sum_j C_ej (f_j - f_e) (the filter's rows sum
// to 1), wall rows unfiltered, interior right-hand side
// a0 f_i + a1/2 (f_{i+1} + f_{i-1}) + a2/2 (f_{i+2} + f_{i-2}), A = (af, 1, af).
template <int DIR, int NMAX, int NC, int PW = 0, int OP = OP_D1, int NTH = 256, class TF = double>
__device__ inline void lds_line_solve(TF *Fb, double *KNb, const LinePlanDev &pl, int np) {
    using C = SweepCfg<DIR, NMAX, PW, NTH>;
    constexpr int KS = C::P * C::KMAX;
    auto F = [&](int c) -> TF * { return Fb + c * C::FSZ; };
    auto KN = [&](int c) -> double * { return KNb + c * KS; };
    constexpr bool FILT = OP == OP_FILTER;
    static_assert(!FILT || sizeof(TF) == 8, "the filter runs in FP64");
    const int tid = threadIdx.x;
    const int n = pl.n;
    const double ih = pl.ih;
    const double alpha = FILT ? pl.alpha : kAlpha;
    const TF ih_t = TF(ih), alpha_t = TF(alpha), b1_t = TF(kB1), b2_t = TF(kB2);
    const double fa0 = pl.fc.a0, fa1 = pl.fc.a1h, fa2 = pl.fc.a2h;
    // interior right-hand side of row i from the window f_{i-2} .. f_{i+2}
    auto rhs5 = [&](TF w0, TF w1, TF w2, TF w3, TF w4) -> TF {
        if constexpr (FILT) return fa0 * w2 + fa1 * (w1 + w3) + fa2 * (w0 + w4);
        else return ih_t * (b1_t * (w3 - w1) + b2_t * (w4 - w0));
    };
    // plan tables through the scalar path where the index is wave-uniform
    const auto runs_i = NOPCS_SCALAR_PTR(int, pl.runs);
    const auto slot_i = NOPCS_SCALAR_PTR(int, pl.run_slot);
    const TF *const rden_v = sizeof(TF) == 8 ? (const TF *)(const void *)pl.rden : (const TF *)(const void *)pl.rden32;
    const TF *const cp_v = sizeof(TF) == 8 ? (const TF *)(const void *)pl.cp : (const TF *)(const void *)pl.cp32;
    const auto rden = NOPCS_SCALAR_PTR(TF, rden_v);
    const auto cp = NOPCS_SCALAR_PTR(TF, cp_v);
    // rows n .. (n rounded up to 32) - 1 of every staged line read as zeros
    // (phase A walks whole 32-row blocks)
    const int ntail = ((n + 31) & ~31) - n;
    if (ntail > 0) {
        for (int q = tid; q < NC * C::P * ntail; q += C::NT) {
            const int c = q / (C::P * ntail), rest = q - c * (C::P * ntail);
            F(c)[C::fidx(rest % C::P, n + rest / C::P)] = TF(0);
        }
        __syncthreads();
    }
    // ---- A: known rows, one thread per (component, line, row); the closure
    // items come first so that every thread has at most one of them ----
    const int ncl = pl.ncl;
    const int ncli = NC * C::P * ncl;
    for (int q = tid; q < ncli + NC * C::P * 4; q += C::NT) {
        const bool clo = q < ncli;
        const int w = clo ? q : q - ncli;
        const int l = w % C::P, rest = w / C::P;
        const int c = rest % NC, s = rest / NC;     // s: closure index, or wall slot 0..3
        if (l >= np) continue;
        const TF *f = F(c);
        double v;
        if (clo) {
            // f'_e = sum_t C_{e,j0+t} (f_{j0+t} - f_e) / h, walked over the aligned
            // 32-row blocks that the tap window touches: inside a block the LDS
            // offsets of the rows are compile-time constants, the table holds the
            // taps of a block row pair in one 16-byte entry (zeros outside the
            // window; rows past the line's end are zero in F), and the entries of
            // the closures of a wavefront are adjacent.  Two interleaved partial
            // sums; the loads of TB rows are issued before the first is used.
            constexpr int TB = 8;
            constexpr int RS = C::RSTEP;
            const int row = pl.cl_row[s], j0 = pl.cl_j0[s], len = pl.cl_len[s];
            const int b0 = j0 >> 5, nb = ((j0 + len - 1) >> 5) - b0 + 1;   // 1..4 blocks
            const double2 *ctab = reinterpret_cast<const double2 *>(pl.cl_coefA);
            const double fe = double(f[C::fidx(l, row)]);
            double a0 = 0.0, a1 = 0.0;
            for (int bb = 0; bb < 4; ++bb) {
                if (bb >= nb) break;
                const int r0 = (b0 + bb) << 5;
                const TF *fb = f + C::fidx(l, r0);
                NOPCS_LDS_BOUND(C::fidx(l, r0) + 31 * RS, C::FSZ);
                const unsigned cofs = (unsigned)(16 * bb * ncl + s);
#pragma unroll
                for (int j8 = 0; j8 < 32; j8 += TB) {
                    double2 cf[TB / 2];
                    double fv[TB];
#pragma unroll
                    for (int u = 0; u < TB / 2; ++u) cf[u] = (ctab + (size_t)(j8 / 2 + u) * ncl)[cofs];
#pragma unroll
                    for (int u = 0; u < TB; ++u) fv[u] = double(fb[(j8 + u) * RS]) - fe;
#pragma unroll
                    for (int u = 0; u < TB / 2; ++u) {
                        a0 = fma_(cf[u].x, fv[2 * u], a0);
                        a1 = fma_(cf[u].y, fv[2 * u + 1], a1);
                    }
                }
            }
            v = FILT ? fe + (a0 + a1) : (a0 + a1) * ih;
        } else if (FILT) {
            v = double(f[C::fidx(l, s == 0 ? 0 : s == 1 ? 1 : s == 2 ? n - 2 : n - 1)]);
        } else if (s == 0) {
            const double f0 = double(f[C::fidx(l, 0)]);
            v = 0.5 * ih * (4.0 * (double(f[C::fidx(l, 1)]) - f0) - (double(f[C::fidx(l, 2)]) - f0));
        } else if (s == 1) {
            v = 0.5 * ih * (double(f[C::fidx(l, 2)]) - double(f[C::fidx(l, 0)]));
        } else if (s == 2) {
            v = 0.5 * ih * (double(f[C::fidx(l, n - 1)]) - double(f[C::fidx(l, n - 3)]));
        } else {
            const double fl = double(f[C::fidx(l, n - 1)]);
            v = -0.5 * ih * (4.0 * (double(f[C::fidx(l, n - 2)]) - fl) - (double(f[C::fidx(l, n - 3)]) - fl));
        }
        KN(c)[C::kidx(clo ? 4 + s : s, l)] = v;
    }
    __syncthreads();
    // ---- C: B f and Thomas on every run, one thread per (component, line, run) ----
    // Forward: d_k = (r_k - alpha d_{k-1}) / den_k as r_k * (1/den_k) - c'_k d_{k-1}
    // (c'_k = alpha / den_k), one fused multiply-add on the recurrence.  Both
    // loops count k uniformly across the wavefront (table entries come through
    // scalar loads issued one step ahead); LDS reads sit at clamped rows.
    const int kmax = pl.max_m;
    for (int q = tid; q < NC * C::P * pl.nrun; q += C::NT) {
        const int c = q / (C::P * pl.nrun), rest = q - c * (C::P * pl.nrun);
        const int l = rest % C::P, r = rest / C::P;
        if (l >= np) continue;
        TF *f = F(c);
        const double *kn = KN(c);
        const int lo = runs_i[2 * r], hi = runs_i[2 * r + 1], m = hi - lo - 1;
        const TF xlo = TF(kn[C::kidx(slot_i[2 * r], l)]);
        const TF xhi = TF(kn[C::kidx(slot_i[2 * r + 1], l)]);
        // window f_{i-2} .. f_{i+2} at i = lo + 1; rows lo - 1 and hi + 1 are
        // known rows (closures and walls come in adjacent pairs), whose F keeps f
        TF w0 = f[C::fidx(l, lo - 1)];
        TF w1 = f[C::fidx(l, lo)];
        TF w2 = f[C::fidx(l, lo + 1)];
        TF w3 = f[C::fidx(l, min(lo + 2, hi + 1))];
        TF w4 = f[C::fidx(l, min(lo + 3, hi + 1))];
        // row k = 1 (every lane starts there) with the lower known value; the
        // upper known value enters row m after the loop: d_m gains
        // -alpha x_hi / den_m, the only place where it appears
        TF dprev;
        {
            const TF fn = f[C::fidx(l, min(lo + 4, hi + 1))];
            TF rr = rhs5(w0, w1, w2, w3, w4);
            rr = rr - alpha_t * xlo;
            dprev = rr * rden[1];
            f[C::fidx(l, lo + 1)] = dprev;
            w0 = w1;
            w1 = w2;
            w2 = w3;
            w3 = w4;
            w4 = fn;
        }
        TF cpk = cp[2], rdk = rden[2];
#pragma unroll 2
        for (int k = 2; k <= m; ++k) {
            const int i = lo + k;
            const TF fn = f[C::fidx(l, min(i + 3, hi + 1))];
            const TF cpn = cp[k + 1], rdn = rden[k + 1];
            const TF rr = rhs5(w0, w1, w2, w3, w4);
            const TF dp = fma_(-cpk, dprev, rr * rdk);
            f[C::fidx(l, i)] = dp;
            dprev = dp;
            cpk = cpn;
            rdk = rdn;
            w0 = w1;
            w1 = w2;
            w2 = w3;
            w3 = w4;
            w4 = fn;
        }
        dprev = fma_(-alpha_t * xhi, rden_v[m], dprev);
        f[C::fidx(l, lo + m)] = dprev;
        // backward: x_m = d_m, x_k = d_k - c'_k x_{k+1}; k runs from the plan's
        // longest run down, lanes of shorter runs wait until k < m
        TF fcur = f[C::fidx(l, lo + max(min(kmax - 1, m - 1), 1))];
        cpk = cp[max(kmax - 1, 1)];
        for (int k = kmax - 1; k >= 1; --k) {
            const TF fnx = f[C::fidx(l, lo + max(min(k - 1, m - 1), 1))];
            const TF cpx = cp[max(k - 1, 1)];
            if (k < m) {
                const TF x = fma_(-cpk, dprev, fcur);
                f[C::fidx(l, lo + k)] = x;
                dprev = x;
            }
            fcur = fnx;
            cpk = cpx;
        }
    }
    __syncthreads();
}

// f' of component c at (l, i) after lds_line_solve; ks = pl.kslot[i] (the
// known-row slot of row i, -1 for a compact row), read once by the caller
template <int DIR, int NMAX, int PW = 0, int NTH = 256, class TF = double>
__device__ inline double lds_result(const TF *Fb, const double *KNb, int c, int ks, int l, int i) {
    using C = SweepCfg<DIR, NMAX, PW, NTH>;
    return ks < 0 ? double(Fb[c * C::FSZ + C::fidx(l, i)]) : KNb[c * C::P * C::KMAX + C::kidx(ks, l)];
}

// known-row slots of a thread's owned points (clamped index: always a valid read)
template <int DIR, int NMAX, int PW = 0, int NTH = 256>
__device__ inline void owned_slots(const LinePlanDev &pl, int ks[SweepCfg<DIR, NMAX, PW, NTH>::PTS]) {
    using C = SweepCfg<DIR, NMAX, PW, NTH>;
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        int l, i;
        C::owned(threadIdx.x + s * C::NT, l, i);
        ks[s] = pl.kslot[min(i, pl.n - 1)];
    }
}

}  // namespace nopcs
