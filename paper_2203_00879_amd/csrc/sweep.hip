// sweep.hip -- derivative kernels and convective NSE sweeps (FP64).
#include "kernels.hpp"
#include "sweep.hpp"

namespace nopcs {

namespace {

// pencil `pencil` of a sweep: first line, valid lines, base element offset
template <class C>
__device__ inline void pencil_at(const SweepGeom &g, int pencil, int &np, long long &base) {
    const int npa = (g.nA + C::P - 1) / C::P;
    const int pa = pencil % npa, pb = pencil / npa;
    const int l0 = pa * C::P;
    np = min(C::P, g.nA - l0);
    base = (long long)l0 * g.sA + (long long)pb * g.sB;
}

// pencil of this block (single-box launches)
template <class C>
__device__ inline void pencil_of(const SweepGeom &g, int &np, long long &base) {
    pencil_at<C>(g, xcd_swizzle(blockIdx.x, gridDim.x), np, base);
}

template <class C>
__device__ inline int wall_row(int s, int n) {
    return s == 0 ? 0 : s == 1 ? 1 : s == 2 ? n - 2 : n - 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Standalone first / second derivative along DIR (nopcs_derivative).
// ---------------------------------------------------------------------------
// Lines per pencil of the standalone derivative: along y and z the lines of a
// pencil are neighbours in x, so every row is one contiguous run of P values;
// with a single LDS component the pencil holds 8192 values: 32 lines of up to
// 256 points, 16 of 512, 8 of 1024.
template <int DIR, int NMAX>
constexpr int deriv_pencil_width() {
    return DIR == 0 || NMAX <= 128 ? 0 : 8192 / NMAX;
}
// threads per block of the standalone single-field pencil kernels: along y
// and z 512 threads stage 8192 values (16 lines of 512 points, 128-byte rows;
// 75 KB of LDS, two blocks per CU at 107 VGPRs), 256 elsewhere
template <int DIR, int NMAX>
constexpr int deriv_threads() {
    return DIR == 0 || NMAX <= 128 ? 256 : 512;
}

template <int DIR, int NMAX>
__global__ __launch_bounds__((deriv_threads<DIR, NMAX>())) void k_deriv(const double *__restrict__ f, double *d1,
                                                                      double *d2, SweepGeom g, LinePlanDev pl) {
    constexpr int PW = deriv_pencil_width<DIR, NMAX>();
    constexpr int NTH = deriv_threads<DIR, NMAX>();
    using C = SweepCfg<DIR, NMAX, PW, NTH>;
    __shared__ double F[C::FSZ];
    __shared__ double KN[C::P * C::KMAX];
    int np;
    long long base;
    pencil_of<C>(g, np, base);
    const int n = g.n;
    int ks[C::PTS];
    owned_slots<DIR, NMAX, PW, NTH>(pl, ks);
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        int l, i;
        C::owned(threadIdx.x + s * C::NT, l, i);
        if (l < np && i < n) F[C::fidx(l, i)] = f[base + l * g.sA + i * g.sD];
    }
    __syncthreads();
    lds_line_solve<DIR, NMAX, 1, PW, OP_D1, NTH>(F, KN, pl, np);
    if (d1) {
#pragma unroll
        for (int s = 0; s < C::PTS; ++s) {
            int l, i;
            C::owned(threadIdx.x + s * C::NT, l, i);
            if (l < np && i < n) d1[base + l * g.sA + i * g.sD] = lds_result<DIR, NMAX, PW, NTH>(F, KN, 0, ks[s], l, i);
        }
    }
    if (d2) {
        // put the known rows' f' back into F, then differentiate again
        const int nk = 4 + pl.ncl;
        for (int q = threadIdx.x; q < C::P * nk; q += C::NT) {
            const int l = q % C::P, s = q / C::P;
            if (l >= np) continue;
            const int row = s < 4 ? wall_row<C>(s, n) : pl.cl_row[s - 4];
            F[C::fidx(l, row)] = KN[C::kidx(s, l)];
        }
        __syncthreads();
        lds_line_solve<DIR, NMAX, 1, PW, OP_D1, NTH>(F, KN, pl, np);
#pragma unroll
        for (int s = 0; s < C::PTS; ++s) {
            int l, i;
            C::owned(threadIdx.x + s * C::NT, l, i);
            if (l < np && i < n) d2[base + l * g.sA + i * g.sD] = lds_result<DIR, NMAX, PW, NTH>(F, KN, 0, ks[s], l, i);
        }
    }
}

// ---------------------------------------------------------------------------
// Implicit filter along DIR of one field, in place (out may equal f: a block
// reads its whole pencil before it writes any of it, and pencils are disjoint).
// ---------------------------------------------------------------------------
template <int DIR, int NMAX>
__global__ __launch_bounds__((deriv_threads<DIR, NMAX>())) void k_filter(const double *f, double *out, SweepGeom g,
                                                                         LinePlanDev pl) {
    constexpr int PW = deriv_pencil_width<DIR, NMAX>();
    constexpr int NTH = deriv_threads<DIR, NMAX>();
    using C = SweepCfg<DIR, NMAX, PW, NTH>;
    __shared__ double F[C::FSZ];
    __shared__ double KN[C::P * C::KMAX];
    int np;
    long long base;
    pencil_of<C>(g, np, base);
    const int n = g.n;
    int ks[C::PTS];
    owned_slots<DIR, NMAX, PW, NTH>(pl, ks);
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        int l, i;
        C::owned(threadIdx.x + s * C::NT, l, i);
        if (l < np && i < n) F[C::fidx(l, i)] = f[base + l * g.sA + i * g.sD];
    }
    __syncthreads();
    lds_line_solve<DIR, NMAX, 1, PW, OP_FILTER, NTH>(F, KN, pl, np);
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        int l, i;
        C::owned(threadIdx.x + s * C::NT, l, i);
        if (l < np && i < n) out[base + l * g.sA + i * g.sD] = lds_result<DIR, NMAX, PW, NTH>(F, KN, 0, ks[s], l, i);
    }
}

// ---------------------------------------------------------------------------
// Convective sweep along DIR: R_c <- R_c - D_DIR(flux_c) for the 5 flux
// components of ge3-ge5, staged C::G components at a time.
// ---------------------------------------------------------------------------
namespace {

// TF = float (mixed precision): the group is staged in FP32 as the offset
// fluxes of nse_sweep_body (flux less FREF, its line's first-row value,
// rounded once) and solved in FP32.  FREF is written before a barrier of the
// caller that precedes the first group.
template <int DIR, int NMAX, int C0, int NC, class TR, class TF>
__device__ inline void nse_group(const NseSweepArgs &a, const SweepGeom &g, const LinePlanDev &pl, int np,
                                 long long base, double (&flux)[5][SweepCfg<DIR, NMAX>::PTS],
                                 const int (&ks)[SweepCfg<DIR, NMAX>::PTS], TF *F, double *KN,
                                 const double (*FREF)[SweepCfg<DIR, NMAX>::P]) {
    using C = SweepCfg<DIR, NMAX>;
    const int n = g.n;
    const long long N3 = a.N3;
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        int l, i;
        C::owned(threadIdx.x + s * C::NT, l, i);
        if (l < np && i < n) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if constexpr (sizeof(TF) == 8) F[c * C::FSZ + C::fidx(l, i)] = flux[C0 + c][s];
                else F[c * C::FSZ + C::fidx(l, i)] = TF(flux[C0 + c][s] - FREF[C0 + c][l]);
            }
        }
    }
    __syncthreads();
    lds_line_solve<DIR, NMAX, NC, 0, OP_D1, C::NT, TF>(F, KN, pl, np);
    // R of the owned points; unconditional loads at clamped indices (no branch
    // makes the compiler drain the loads in flight), unused values dropped
    TR *const R = static_cast<TR *>(a.R);
    TR rv[NC][C::PTS];
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        int l, i;
        C::owned(threadIdx.x + s * C::NT, l, i);
        const long long o = base + min(l, np - 1) * g.sA + min(i, n - 1) * g.sD;
#pragma unroll
        for (int c = 0; c < NC; ++c) rv[c][s] = R[(C0 + c) * N3 + o];
    }
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        int l, i;
        C::owned(threadIdx.x + s * C::NT, l, i);
        if (!(l < np && i < n)) continue;
        const long long o = base + l * g.sA + i * g.sD;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            R[(C0 + c) * N3 + o] = rv[c][s] - TR(lds_result<DIR, NMAX, 0, C::NT, TF>(F, KN, c, ks[s], l, i));
    }
}

}  // namespace

// TR = float (mixed precision): R in FP32, and the line solves in FP32 on
// offset fluxes: each flux component less its value at the line's first row
// (FREF, FP64), rounded once.  The derivative of a constant is exactly zero in
// every row type (interior B f, the shifted closure sums, the wall
// differences), so the offset changes nothing but the size of what FP32
// carries: the line's own variation (for the pressure in the momentum flux,
// the hydrostatic level of the line drops out).  Known rows stay FP64.
template <int DIR, int NMAX, class TR>
__device__ inline void nse_sweep_body(const NseSweepArgs &a, const SweepGeom &g, const LinePlanDev &pl, int b) {
    using C = SweepCfg<DIR, NMAX>;
    using TF = TR;
    __shared__ TF F[C::G * C::FSZ];
    __shared__ double KN[C::G * C::P * C::KMAX];
    __shared__ double FREF[sizeof(TF) == 8 ? 1 : 5][C::P];
    int np;
    long long base;
    pencil_at<C>(g, b, np, base);
    const int n = g.n;
    const long long N3 = a.N3;
    const NdConst &c = a.c;
    // convective fluxes of the owned points (ge3-ge5), kept in registers
    // (loads at clamped indices, unconditional: see nse_group; points outside
    // the pencil are never stored)
    double flux[5][C::PTS];
#pragma unroll
    for (int s = 0; s < C::PTS; ++s) {
        int l, i;
        C::owned(threadIdx.x + s * C::NT, l, i);
        const long long o = base + min(l, np - 1) * g.sA + min(i, n - 1) * g.sD;
        const double rho = a.Qin[o], mx = a.Qin[N3 + o], my = a.Qin[2 * N3 + o], mz = a.Qin[3 * N3 + o],
                     Ep = a.Qin[4 * N3 + o];
        const Prim pr = prim_from(c, rho, mx, my, mz, Ep);
        const double ud = DIR == 0 ? pr.u : DIR == 1 ? pr.v : pr.w;
        flux[0][s] = DIR == 0 ? mx : DIR == 1 ? my : mz;
        flux[1][s] = DIR == 0 ? mx * ud + pr.pp : mx * ud;
        flux[2][s] = DIR == 1 ? my * ud + pr.pp : my * ud;
        flux[3][s] = DIR == 2 ? mz * ud + pr.pp : mz * ud;
        flux[4][s] = ((Ep + pr.pp) + c.H) * ud;
        if constexpr (sizeof(TF) != 8) {
            // the offsets: fluxes of the first row of every line
            if (i == 0 && l < np) {
#pragma unroll
                for (int q = 0; q < 5; ++q) FREF[q][l] = flux[q][s];
            }
        }
    }
    int ks[C::PTS];
    owned_slots<DIR, NMAX>(pl, ks);
    static_assert(C::G == 2, "component grouping below assumes groups {0,1}, {2,3} and {4}");
    if constexpr (sizeof(TF) != 8) __syncthreads();   // FREF published
    nse_group<DIR, NMAX, 0, 2, TR, TF>(a, g, pl, np, base, flux, ks, F, KN, FREF);
    __syncthreads();
    nse_group<DIR, NMAX, 2, 2, TR, TF>(a, g, pl, np, base, flux, ks, F, KN, FREF);
    __syncthreads();
    nse_group<DIR, NMAX, 4, 1, TR, TF>(a, g, pl, np, base, flux, ks, F, KN, FREF);
}

// ---------------------------------------------------------------------------
// RK4 register update
// ---------------------------------------------------------------------------
namespace {
// one element: the stage's register updates, k = R
template <int STAGE>
__device__ inline void rk_elem(double kv, double &K, double &Qs, double &Qn, const NseSweepArgs &a) {
    if (STAGE == 0) {
        K = kv;
        Qs = Qn + a.half_dt * kv;
    } else if (STAGE == 1) {
        K = K + 2.0 * kv;
        Qs = Qn + a.half_dt * kv;
    } else if (STAGE == 2) {
        K = K + 2.0 * kv;
        Qs = Qn + a.dt * kv;
    } else {
        Qn = Qn + a.sixth_dt * (K + kv);
    }
}

// two neighbouring elements per thread and iteration (16-byte accesses); the
// registers must be 16-byte aligned, an odd tail element is done separately
template <class TR> struct Pair;
template <> struct Pair<double> { using T = double2; };
template <> struct Pair<float> { using T = float2; };

template <int STAGE, class TR>
__device__ inline void rk_update_body(const NseSweepArgs &a, long long total, int b, int nb) {
    const long long npair = total >> 1;
    const long long stride = (long long)nb * 256;
    const TR *const R = static_cast<const TR *>(a.R);
    const auto *R2 = reinterpret_cast<const typename Pair<TR>::T *>(R);
    double2 *K2 = reinterpret_cast<double2 *>(a.K);
    double2 *S2 = reinterpret_cast<double2 *>(a.Qs);
    double2 *N2 = reinterpret_cast<double2 *>(a.Qn);
    for (long long p = (long long)b * 256 + threadIdx.x; p < npair; p += stride) {
        const auto kr = R2[p];
        const double2 kv = make_double2(double(kr.x), double(kr.y));
        double2 kk = STAGE == 0 ? make_double2(0.0, 0.0) : K2[p];
        double2 qn = N2[p];
        double2 qs;
        rk_elem<STAGE>(kv.x, kk.x, qs.x, qn.x, a);
        rk_elem<STAGE>(kv.y, kk.y, qs.y, qn.y, a);
        if (STAGE < 3) {
            K2[p] = kk;
            S2[p] = qs;
        } else {
            N2[p] = qn;
        }
    }
    if ((total & 1) && b == 0 && threadIdx.x == 0) {
        const long long o = total - 1;
        double kk = STAGE == 0 ? 0.0 : a.K[o], qs = 0.0, qn = a.Qn[o];
        rk_elem<STAGE>(double(R[o]), kk, qs, qn, a);
        if (STAGE < 3) {
            a.K[o] = kk;
            a.Qs[o] = qs;
        } else {
            a.Qn[o] = qn;
        }
    }
}
}  // namespace

struct SweepArgs {
    NseSweepArgs a;
    SweepGeom g;
    LinePlanDev pl;
};
template <int DIR, int NMAX, class TR>
struct SweepBody {
    using Args = SweepArgs;
    // the FP32 x sweep capped at 128 VGPRs: four blocks per CU instead of three
    // (at 512 and 1024 points a few registers spill; 512^3: 4.34 -> 3.86 ms)
    static constexpr int kMinWaves = DIR == 0 && sizeof(TR) == 4 ? 4 : 1;
    __device__ static void run(const Args &x, int b, int) { nse_sweep_body<DIR, NMAX, TR>(x.a, x.g, x.pl, b); }
};
struct RkUpdArgs {
    NseSweepArgs a;
    long long total;
};
template <int STAGE, class TR>
struct RkUpdBody {
    using Args = RkUpdArgs;
    __device__ static void run(const Args &x, int b, int nb) { rk_update_body<STAGE, TR>(x.a, x.total, b, nb); }
};

// Classical RK4 register update of one stage (Section 4), point-wise over the
// 5 fields:  k = R;  stage 0: K = k, Qs = Qn + dt/2 k;  stage 1: K += 2k,
// Qs = Qn + dt/2 k;  stage 2: K += 2k, Qs = Qn + dt k;  stage 3:
// Qn = Qn + dt/6 (K + k).
hipError_t launch_rk_update(const NseSweepArgs &a, hipStream_t st, BatchCollector *col, int phase) {
    const long long total = 5 * a.N3;
    const bool aligned = ((reinterpret_cast<uintptr_t>(a.R) | reinterpret_cast<uintptr_t>(a.K) |
                           reinterpret_cast<uintptr_t>(a.Qs) | reinterpret_cast<uintptr_t>(a.Qn)) & 15) == 0;
    if (!aligned) return hipErrorInvalidValue;   // the library's own buffers are 256-byte aligned
    long long blocks = ((total >> 1) + 255) / 256;
    if (blocks > 256 * 32) blocks = 256 * 32;
    if (blocks < 1) blocks = 1;
    const RkUpdArgs x{a, total};
    const int nb = (int)blocks;
    const dim3 blk(256);
    if (a.r32) {
        switch (a.stage) {
            case 0: return run_body<RkUpdBody<0, float>, 256>(x, nb, blk, st, col, phase);
            case 1: return run_body<RkUpdBody<1, float>, 256>(x, nb, blk, st, col, phase);
            case 2: return run_body<RkUpdBody<2, float>, 256>(x, nb, blk, st, col, phase);
            default: return run_body<RkUpdBody<3, float>, 256>(x, nb, blk, st, col, phase);
        }
    }
    switch (a.stage) {
        case 0: return run_body<RkUpdBody<0, double>, 256>(x, nb, blk, st, col, phase);
        case 1: return run_body<RkUpdBody<1, double>, 256>(x, nb, blk, st, col, phase);
        case 2: return run_body<RkUpdBody<2, double>, 256>(x, nb, blk, st, col, phase);
        default: return run_body<RkUpdBody<3, double>, 256>(x, nb, blk, st, col, phase);
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <int DIR, int NMAX>
static hipError_t launch_deriv_t(const double *f, double *d1, double *d2, const SweepGeom &g, const LinePlanDev &pl,
                                 hipStream_t st) {
    using C = SweepCfg<DIR, NMAX, deriv_pencil_width<DIR, NMAX>(), deriv_threads<DIR, NMAX>()>;
    const int npa = (g.nA + C::P - 1) / C::P;
    const long long blocks = (long long)npa * g.nB;
    hipLaunchKernelGGL((k_deriv<DIR, NMAX>), dim3((unsigned)blocks), dim3(C::NT), 0, st, f, d1, d2, g, pl);
    return hipGetLastError();
}

template <int DIR, int NMAX>
static hipError_t launch_filter_t(const double *f, double *out, const SweepGeom &g, const LinePlanDev &pl,
                                  hipStream_t st) {
    using C = SweepCfg<DIR, NMAX, deriv_pencil_width<DIR, NMAX>(), deriv_threads<DIR, NMAX>()>;
    const int npa = (g.nA + C::P - 1) / C::P;
    const long long blocks = (long long)npa * g.nB;
    hipLaunchKernelGGL((k_filter<DIR, NMAX>), dim3((unsigned)blocks), dim3(C::NT), 0, st, f, out, g, pl);
    return hipGetLastError();
}

template <int DIR, int NMAX>
static hipError_t launch_sweep_t(const NseSweepArgs &a, const SweepGeom &g, const LinePlanDev &pl, hipStream_t st,
                                 BatchCollector *col, int phase) {
    using C = SweepCfg<DIR, NMAX>;
    const int npa = (g.nA + C::P - 1) / C::P;
    const int blocks = (int)((long long)npa * g.nB);
    const SweepArgs x{a, g, pl};
    if (a.r32) return run_body<SweepBody<DIR, NMAX, float>, C::NT>(x, blocks, dim3(C::NT), st, col, phase);
    return run_body<SweepBody<DIR, NMAX, double>, C::NT>(x, blocks, dim3(C::NT), st, col, phase);
}

int nmax_class(int n) {
    if (n <= 64) return 64;
    if (n <= 128) return 128;
    if (n <= 256) return 256;
    if (n <= 512) return 512;
    if (n <= 1024) return 1024;
    return 0;
}

#define NOPCS_NMAX_SWITCH(NM, EXPR)                        \
    switch (NM) {                                          \
        case 64: { constexpr int NMX = 64; EXPR; }         \
        case 128: { constexpr int NMX = 128; EXPR; }       \
        case 256: { constexpr int NMX = 256; EXPR; }       \
        case 512: { constexpr int NMX = 512; EXPR; }       \
        case 1024: { constexpr int NMX = 1024; EXPR; }     \
        default: break;                                    \
    }

int sweep_lines_per_block(int dir, int n) {
    (void)dir;
    NOPCS_NMAX_SWITCH(nmax_class(n), return (SweepCfg<1, NMX>::P));
    return 0;
}

int sweep_threads_per_block(int dir, int n) {
    (void)dir;
    NOPCS_NMAX_SWITCH(nmax_class(n), return (SweepCfg<1, NMX>::NT));
    return 0;
}

int sweep_known_rows_max(int n) {
    NOPCS_NMAX_SWITCH(nmax_class(n), return (SweepCfg<1, NMX>::KMAX));
    return 0;
}

hipError_t launch_deriv(int dir, const double *f, double *d1, double *d2, const SweepGeom &g, const LinePlanDev &pl,
                        hipStream_t st) {
    const int nm = nmax_class(g.n);
    if (dir == 0) { NOPCS_NMAX_SWITCH(nm, return (launch_deriv_t<0, NMX>(f, d1, d2, g, pl, st))); }
    else if (dir == 1) { NOPCS_NMAX_SWITCH(nm, return (launch_deriv_t<1, NMX>(f, d1, d2, g, pl, st))); }
    else { NOPCS_NMAX_SWITCH(nm, return (launch_deriv_t<2, NMX>(f, d1, d2, g, pl, st))); }
    return hipErrorInvalidValue;
}

hipError_t launch_filter(int dir, const double *f, double *out, const SweepGeom &g, const LinePlanDev &pl,
                         hipStream_t st) {
    if (pl.op != OP_FILTER) return hipErrorInvalidValue;
    const int nm = nmax_class(g.n);
    if (dir == 0) { NOPCS_NMAX_SWITCH(nm, return (launch_filter_t<0, NMX>(f, out, g, pl, st))); }
    else if (dir == 1) { NOPCS_NMAX_SWITCH(nm, return (launch_filter_t<1, NMX>(f, out, g, pl, st))); }
    else { NOPCS_NMAX_SWITCH(nm, return (launch_filter_t<2, NMX>(f, out, g, pl, st))); }
    return hipErrorInvalidValue;
}

hipError_t launch_nse_sweep(int dir, const NseSweepArgs &a, const SweepGeom &g, const LinePlanDev &pl,
                            hipStream_t st, BatchCollector *col, int phase) {
    const int nm = nmax_class(g.n);
    if (dir == 0) { NOPCS_NMAX_SWITCH(nm, return (launch_sweep_t<0, NMX>(a, g, pl, st, col, phase))); }
    else if (dir == 1) { NOPCS_NMAX_SWITCH(nm, return (launch_sweep_t<1, NMX>(a, g, pl, st, col, phase))); }
    else { NOPCS_NMAX_SWITCH(nm, return (launch_sweep_t<2, NMX>(a, g, pl, st, col, phase))); }
    return hipErrorInvalidValue;
}

}  // namespace nopcs
