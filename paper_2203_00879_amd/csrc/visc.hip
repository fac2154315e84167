// visc.hip -- viscous terms and gravity source of ge17, explicit second order.
//
// R = dEv/dx + dFv/dy + dGv/dz + S  (ge6-ge8, ge8a, ge19, ge20, bv1-bv3)
// The velocity and temperature gradients inside Ev, Fv, Gv and the outer
// divergence both use second-order differences: central inside, one-sided on
// wall nodes (Section 4).
//
// One block owns a CTX x CTY tile of output columns plus a two-column halo and
// marches along z over a chunk of planes; one thread per column, one barrier
// per plane (primitives and fluxes of plane k in LDS buffer k mod 2 while the
// divergence of plane k-1 reads the other buffer).  Each thread
// keeps the primitives (u, v, w, T) of its own column for planes k-1..k+1 in
// registers (planes k-2 and k+2 are loaded again at the walls), so z
// differences need no shared memory.  Per plane, every column
// publishes its primitives in LDS once; every node then evaluates its gradients,
// mu, beta and the flux vectors it contributes (Ev at x-neighbours, Fv at
// y-neighbours, Gv at the column itself) exactly once.  The x and y parts of
// the divergence are taken from LDS at plane k; the z part is finished one
// plane later from a three-plane register history of Gv.  Each state value is
// read from HBM about 1.8 times (tile halo of 32 x 16 columns for 28 x 12
// outputs, the z-chunk overlap, the planes loaded ahead of a chunk's end),
// each flux vector computed once.
// Tiles at the high end of x and y are shifted inward (overlapping their
// neighbour, which writes identical values) so that the one-sided wall
// stencils stay inside the halo.  The summation order is that of the oracle:
// (dEv/dx + dFv/dy) + dGv/dz, then the source.
// Mixed precision (R in FP32): the primitives are formed in FP64 from the
// state and rounded once; their differences, the stresses, heat fluxes and
// the divergence run in FP32 (mu and beta from the rounded temperature in
// FP64), with one plane in flight: 128 VGPRs and 48 KB of LDS, two blocks
// per CU instead of one.
#include <algorithm>
#include <atomic>

#include "kernels.hpp"

namespace nopcs {

namespace {
// Planes of raw state in flight ahead of the window (1, 2 or 3).  A block of
// 512 threads holds its CU alone (two waves per SIMD), so registers up to 256
// per thread cost no occupancy: three planes in flight (231 VGPRs) hide more
// of the load latency than one (166): 4.39 -> 4.08 ms at 512^3.
// The FP32 form (mixed precision) keeps one plane in flight instead, so that
// two blocks share a CU (at most 128 VGPRs, see ViscBody).
constexpr int VPF64 = 3, VPF32 = 1;
static_assert(VPF64 >= 1 && VPF64 <= 3 && VPF32 >= 1 && VPF32 <= 3, "one to three planes in flight");
// Outputs per block (CTX x CTY) and columns per block (with a two-point halo).
constexpr int CTX = 28, CTY = 12, CX = CTX + 4, CY = CTY + 4, CNT = CX * CY;

struct VArgs {
    const double *Q;
    void *R;        // TR[5 N3]
    int nx, ny, nz, ntx, nty, zc;
    long long N3;
    double ihx, ihy, ihz;
    NdConst c;
};

// second-order derivative from three values along an axis: f(-1), f(+1)
// inside, or the one-sided form at a wall node (f0 on the wall, f1, f2 inward;
// the high wall flips the sign)
template <class T>
__device__ inline T d2c(T fm, T fp, T ih) { return T(0.5) * ih * (fp - fm); }
template <class T>
__device__ inline T d2w(T f0, T f1, T f2, T ih, bool high) {
    const T v = T(0.5) * ih * (T(4.0) * (f1 - f0) - (f2 - f0));
    return high ? -v : v;
}

// derivative of LDS field P at slot o along x (st = 1) or y (st = CX); g is
// the node's global index along that axis.  WALL: the node may lie on a wall.
template <bool WALL, class T>
__device__ inline T dplane(const T *P, int o, int st, int g, int n, T ih) {
    if (WALL) {
        if (g == 0) {
            NOPCS_LDS_BOUND(o + 2 * st, CNT);
            return d2w(P[o], P[o + st], P[o + 2 * st], ih, false);
        }
        if (g == n - 1) {
            NOPCS_LDS_BOUND(o - 2 * st, CNT);
            return d2w(P[o], P[o - st], P[o - 2 * st], ih, true);
        }
    }
    NOPCS_LDS_BOUND(o - st, CNT);
    NOPCS_LDS_BOUND(o + st, CNT);
    return d2c(P[o - st], P[o + st], ih);
}

// z derivative at plane k from the column window w = planes k-1, k, k+1; the
// walls also need plane k+2 (fp2, bottom) or k-2 (fm2, top)
template <class T>
__device__ inline T dz(const T w[3], T fm2, T fp2, int k, int nz, T ih) {
    if (k == 0) return d2w(w[1], w[2], fp2, ih, false);
    if (k == nz - 1) return d2w(w[1], w[0], fm2, ih, true);
    return d2c(w[0], w[2], ih);
}

// One block's march over planes k0..k1-1 (see the file header).  S holds, per
// column slot: u, v, w, T of plane k (fields 0-3), Ev (4-7) and Fv (8-11).
// Output columns with gi < own_i or gj < own_j belong to the neighbouring tile.
// TV: arithmetic of the primitives' differences, the stresses and fluxes and
// the divergence (FP64; FP32 in mixed precision, where R is FP32 too); the
// state is read and turned into primitives in FP64, the gravity source and
// mu, beta are formed in FP64.
template <bool WALL, class TR, class TV>
__device__ inline void visc_march(const VArgs &A, TV *S, int i0, int j0, int own_i, int own_j, int k0,
                                  int k1) {
    constexpr int VPF = sizeof(TV) == 8 ? VPF64 : VPF32;
    TR *const R = static_cast<TR *>(A.R);
    const NdConst &c = A.c;
    const double *Q = A.Q;
    const long long N3 = A.N3;
    const long long plane = (long long)A.nx * A.ny;
    const int tid = threadIdx.x;
    const int ci = tid % CX, cj = tid / CX;
    const int gi = i0 - 2 + ci, gj = j0 - 2 + cj;
    const bool indom = !WALL || (gi >= 0 && gi < A.nx && gj >= 0 && gj < A.ny);
    const bool inx = ci >= 2 && ci <= CTX + 1, iny = cj >= 2 && cj <= CTY + 1;
    const bool center = indom && inx && iny && gi >= own_i && gj >= own_j;
    const bool needE = indom && ci >= 1 && ci <= CTX + 2 && iny;   // includes every center
    const bool needF = indom && cj >= 1 && cj <= CTY + 2 && inx;
    const long long col = indom ? gi + (long long)A.nx * gj : 0;
    // S holds two buffers of 12 fields (planes of even and odd k), each per
    // column slot: u, v, w, T of the plane (fields 0-3), Ev (4-7), Fv (8-11)
    constexpr int SB = 12 * CNT;

    // raw state of one plane of this column (a benign dummy outside the box);
    // the loads are unconditional (clamped address, select afterwards) so that
    // no branch makes the compiler drain the loads in flight
    auto load = [&](int p, double q[5]) {
        const bool in = indom && p >= 0 && p < A.nz;
        const long long o = col + plane * min(max(p, 0), A.nz - 1);
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const double v = Q[f * N3 + o];
            q[f] = in ? v : (f == 0 ? 1.0 : 0.0);
        }
    };
    auto prim = [&](const double q[5], TV &u, TV &v, TV &w, TV &T) {
        const Prim pr = prim_from(c, q[0], q[1], q[2], q[3], q[4]);
        u = TV(pr.u);
        v = TV(pr.v);
        w = TV(pr.w);
        T = TV(pr.T);
    };
    const TV ihx = TV(A.ihx), ihy = TV(A.ihy), ihz = TV(A.ihz), iRe = TV(c.iRe), kap = TV(c.kappa);
    // R of plane k: the divergence plus the gravity source (rho and rho v of that plane)
    auto write_R = [&](int k, const TV acc[4], double rho, double my) {
        const long long o = col + plane * k;
        R[o] = TR(0.0);
        R[N3 + o] = TR(acc[0]);
        R[2 * N3 + o] = TR(acc[1] - c.ghat * rho);
        R[3 * N3 + o] = TR(acc[2]);
        R[4 * N3 + o] = TR(acc[3] - c.ghat * my);
    };

    // planes whose node fluxes are needed: k0-1 .. k1, and nz-3 for the top wall
    const int kb = max(0, min(k0 - 1, A.nz - 3)), ke = min(A.nz - 1, k1);
    // window before the first shift: planes kb-2, kb-1, kb; raw states of
    // kb+1 (rawA) and, with two planes in flight, kb+2 (rawB)
    TV wu[3], wv[3], ww[3], wT[3];
    double wr[3], wy[3], raw[5], rawB[5], rawC[5];
#pragma unroll
    for (int s = 1; s < 3; ++s) {
        load(kb - 2 + s, raw);
        prim(raw, wu[s], wv[s], ww[s], wT[s]);
        wr[s] = raw[0];
        wy[s] = raw[2];
    }
    load(kb + 1, raw);
    if (VPF >= 2) load(kb + 2, rawB);
    if (VPF == 3) load(kb + 3, rawC);
    // G history (planes k-2, k-1, k)
    TV G[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    // dEv/dx + dFv/dy at plane p from the fluxes in buffer p & 1
    auto xy_part = [&](int p, TV part[4]) {
        const TV *Sc = S + (p & 1) * SB;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            part[q] = dplane<WALL>(Sc + (4 + q) * CNT, tid, 1, gi, A.nx, ihx) +
                      dplane<WALL>(Sc + (8 + q) * CNT, tid, CX, gj, A.ny, ihy);
    };

    // plane k; cur holds the raw state of plane k+1 and receives that of
    // k+1+VPF; nxt (two or three planes in flight) holds k+2.  With VPF
    // planes the loop is unrolled VPF times and the buffers trade roles, so
    // no register copy waits for a load in flight.
    auto plane_step = [&](int k, double (&cur)[5], double (&nxt)[5]) {
        // window -> planes k-1, k, k+1; the raw state of k+1+VPF stays in flight
        // while this plane is processed
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            wu[s] = wu[s + 1];
            wv[s] = wv[s + 1];
            ww[s] = ww[s + 1];
            wT[s] = wT[s + 1];
            wr[s] = wr[s + 1];
            wy[s] = wy[s + 1];
        }
        prim(cur, wu[2], wv[2], ww[2], wT[2]);
        wr[2] = cur[0];
        wy[2] = cur[2];
        load(k + 1 + VPF, cur);
        // one barrier per plane: the primitives and fluxes of plane k go to
        // buffer k & 1 while the divergence of plane k-1 reads buffer (k-1) & 1
        TV *const Sb = S + (k & 1) * SB;
        TV *const Pu = Sb, *const Pv = Sb + CNT, *const Pw = Sb + 2 * CNT, *const PT = Sb + 3 * CNT;
        Pu[tid] = wu[1];
        Pv[tid] = wv[1];
        Pw[tid] = ww[1];
        PT[tid] = wT[1];
        __syncthreads();
        // ---- node fluxes at (column, plane k): each computed once ----
        TV Gk[4] = {0, 0, 0, 0};
        if (needE || needF) {
            TV um2 = 0, vm2 = 0, wm2 = 0, Tm2 = 0, up2 = 0, vp2 = 0, wp2 = 0, Tp2 = 0;
            if (k == 0) prim(VPF == 1 ? cur : nxt, up2, vp2, wp2, Tp2);
            if (k == A.nz - 1) {
                double q2[5];
                load(k - 2, q2);
                prim(q2, um2, vm2, wm2, Tm2);
            }
            const TV u = wu[1], v = wv[1], w = ww[1], T = wT[1];
            const TV m = TV(mu_of(c, double(T))), bb = TV(beta_of(c, double(T)));
            const TV Aa = TV(4.0 / 3.0) * m + bb, Bb = bb - TV(2.0 / 3.0) * m;
            // the stress tensor first (bv1-bv3), so that the nine velocity
            // gradients die early; each entry is formed exactly as the oracle does
            TV txx, tyy, tzz;
            {
                const TV ux = dplane<WALL>(Pu, tid, 1, gi, A.nx, ihx);
                const TV vy = dplane<WALL>(Pv, tid, CX, gj, A.ny, ihy);
                const TV wz = dz(ww, wm2, wp2, k, A.nz, ihz);
                txx = (Aa * ux + Bb * (vy + wz)) * iRe;
                tyy = (Aa * vy + Bb * (ux + wz)) * iRe;
                tzz = (Aa * wz + Bb * (ux + vy)) * iRe;
            }
            const TV txy = m * (dplane<WALL>(Pu, tid, CX, gj, A.ny, ihy) + dplane<WALL>(Pv, tid, 1, gi, A.nx, ihx)) * iRe;
            const TV txz = m * (dz(wu, um2, up2, k, A.nz, ihz) + dplane<WALL>(Pw, tid, 1, gi, A.nx, ihx)) * iRe;
            const TV tyz = m * (dz(wv, vm2, vp2, k, A.nz, ihz) + dplane<WALL>(Pw, tid, CX, gj, A.ny, ihy)) * iRe;
            if (needE) {
                const TV qx = -kap * m * dplane<WALL>(PT, tid, 1, gi, A.nx, ihx);
                Sb[4 * CNT + tid] = txx;
                Sb[5 * CNT + tid] = txy;
                Sb[6 * CNT + tid] = txz;
                Sb[7 * CNT + tid] = u * txx + v * txy + w * txz - qx;
            }
            if (needF) {
                const TV qy = -kap * m * dplane<WALL>(PT, tid, CX, gj, A.ny, ihy);
                Sb[8 * CNT + tid] = txy;
                Sb[9 * CNT + tid] = tyy;
                Sb[10 * CNT + tid] = tyz;
                Sb[11 * CNT + tid] = u * txy + v * tyy + w * tyz - qy;
            }
            if (center) {
                const TV qz = -kap * m * dz(wT, Tm2, Tp2, k, A.nz, ihz);
                Gk[0] = txz;
                Gk[1] = tyz;
                Gk[2] = tzz;
                Gk[3] = u * txz + v * tyz + w * tzz - qz;
            }
        }
        if (center) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                G[0][q] = G[1][q];
                G[1][q] = G[2][q];
                G[2][q] = Gk[q];
            }
            // plane k-1: its fluxes were written before this plane's barrier
            const bool own_prev = k - 1 >= k0 && k - 1 < k1 && k - 1 >= kb;
            TV part[4] = {0, 0, 0, 0};
            if (own_prev) xy_part(k - 1, part);
            // finish plane k-1 (inside): needs G(k) - G(k-2)
            if (own_prev && k - 1 >= 1 && k - 1 <= A.nz - 2) {
                TV acc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = part[q] + d2c(G[0][q], G[2][q], ihz);
                write_R(k - 1, acc, wr[0], wy[0]);
            }
            // the bottom wall plane waits for G(0), G(1), G(2); its x-y part is
            // parked in R, where only this thread reads it back
            if (own_prev && k - 1 == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) R[(q + 1) * N3 + col] = TR(part[q]);
            }
            if (k == 2 && k0 == 0) {
                TV acc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[q] = TV(R[(q + 1) * N3 + col]) + d2w(G[0][q], G[1][q], G[2][q], ihz, false);
                write_R(0, acc, Q[col], Q[2 * N3 + col]);
            }
        }
    };
    if (VPF == 1) {
#pragma nounroll
        for (int k = kb; k <= ke; ++k) plane_step(k, raw, raw);
    } else if (VPF == 2) {
#pragma nounroll
        for (int k = kb; k <= ke; k += 2) {
            plane_step(k, raw, rawB);
            if (k + 1 <= ke) plane_step(k + 1, rawB, raw);
        }
    } else {
#pragma nounroll
        for (int k = kb; k <= ke; k += 3) {
            plane_step(k, raw, rawB);
            if (k + 1 <= ke) plane_step(k + 1, rawB, rawC);
            if (k + 2 <= ke) plane_step(k + 2, rawC, raw);
        }
    }
    // the top wall plane nz-1 (its fluxes written by the last plane step) is
    // finished with G(nz-1), G(nz-2), G(nz-3)
    if (ke == A.nz - 1 && ke < k1) {
        __syncthreads();
        if (center) {
            TV part[4], acc[4];
            xy_part(ke, part);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = part[q] + d2w(G[2][q], G[1][q], G[0][q], ihz, true);
            write_R(ke, acc, wr[1], wy[1]);
        }
    }
}

template <class TR>
__device__ inline void visc_body(const VArgs &A, int b) {
    const int tt = b % A.ntx, rest = b / A.ntx, ty = rest % A.nty, tz = rest / A.nty;
    const int own_i = tt * CTX, own_j = ty * CTY;
    const int i0 = min(own_i, max(0, A.nx - CTX));
    const int j0 = min(own_j, max(0, A.ny - CTY));
    const int k0 = tz * A.zc, k1 = min(A.nz, k0 + A.zc);
    if (!A.c.viscous) {
        const int ci = threadIdx.x % CX, cj = threadIdx.x / CX;
        const int gi = i0 - 2 + ci, gj = j0 - 2 + cj;
        if (ci < 2 || ci > CTX + 1 || cj < 2 || cj > CTY + 1 || gi < own_i || gj < own_j || gi >= A.nx ||
            gj >= A.ny)
            return;
        const long long N3 = A.N3;
        TR *const R = static_cast<TR *>(A.R);
        for (int k = k0; k < k1; ++k) {
            const long long o = gi + (long long)A.nx * (gj + (long long)A.ny * k);
            R[o] = TR(0.0);
            R[N3 + o] = TR(0.0);
            R[2 * N3 + o] = TR(0.0 - A.c.ghat * A.Q[o]);
            R[3 * N3 + o] = TR(0.0);
            R[4 * N3 + o] = TR(0.0 - A.c.ghat * A.Q[2 * N3 + o]);
        }
        return;
    }
    using TV = TR;
    __shared__ TV S[2 * 12 * CNT];
    // every column and every flux node of the tile off the x and y walls
    const bool interior = i0 >= 2 && i0 + CTX + 2 <= A.nx && j0 >= 2 && j0 + CTY + 2 <= A.ny;
    if (interior) visc_march<false, TR, TV>(A, S, i0, j0, own_i, own_j, k0, k1);
    else visc_march<true, TR, TV>(A, S, i0, j0, own_i, own_j, k0, k1);
}

template <class TR>
struct ViscBody {
    using Args = VArgs;
    // FP32 form: four waves per SIMD (two 512-thread blocks per CU)
    static constexpr int kMinWaves = sizeof(TR) == 4 ? 4 : 1;
    __device__ static void run(const Args &a, int b, int) { visc_body<TR>(a, b); }
};
}  // namespace

// Planes per z chunk of the viscous kernel: the setting (> 0), else 64,
// halved (down to 16) while the grid would have fewer than 1024 blocks (four
// per CU: at 192^3 a 64-plane chunk leaves 336).  Each output plane is
// computed by one chunk with the same arithmetic, so results do not depend on
// it.
static std::atomic<int> g_visc_chunk{0};
int visc_z_chunk(const int n[3]) {
    const int v = g_visc_chunk.load();
    if (v > 0) return std::min(v, n[2]);
    const long long tiles = (long long)((n[0] + CTX - 1) / CTX) * ((n[1] + CTY - 1) / CTY);
    int zc = 64;
    while (zc > 16 && tiles * ((n[2] + zc - 1) / zc) < 1024) zc /= 2;
    return std::min(zc, n[2]);
}
void set_visc_z_chunk(int planes) { g_visc_chunk.store(planes); }
int visc_z_chunk_setting() { return g_visc_chunk.load(); }

hipError_t launch_visc(const double *Q, void *R, bool r32, const int n[3], const double ih[3], const NdConst &c,
                       hipStream_t st, BatchCollector *col, int phase) {
    VArgs A;
    A.Q = Q;
    A.R = R;
    A.nx = n[0];
    A.ny = n[1];
    A.nz = n[2];
    A.ntx = (n[0] + CTX - 1) / CTX;
    A.nty = (n[1] + CTY - 1) / CTY;
    A.zc = visc_z_chunk(n);
    A.N3 = (long long)n[0] * n[1] * n[2];
    A.ihx = ih[0];
    A.ihy = ih[1];
    A.ihz = ih[2];
    A.c = c;
    const int ntz = (n[2] + A.zc - 1) / A.zc;
    const int blocks = (int)((long long)A.ntx * A.nty * ntz);
    if (r32) return run_body<ViscBody<float>, CNT>(A, blocks, dim3(CNT), st, col, phase);
    return run_body<ViscBody<double>, CNT>(A, blocks, dim3(CNT), st, col, phase);
}

// ---------------------------------------------------------------------------
// Wall conditions of the closed adiabatic box (Section 2), one face pair.
// ---------------------------------------------------------------------------
namespace {
struct BcArgs {
    double *Q;
    int nx, ny, nz, dir;
    long long N3;
    NdConst c;
};
__device__ inline void bc_body(const BcArgs &A, int blk) {
    double *const Q = A.Q;
    const int nx = A.nx, ny = A.ny, nz = A.nz, dir = A.dir;
    const long long N3 = A.N3;
    const NdConst &c = A.c;
    const int n[3] = {nx, ny, nz};
    const long long st[3] = {1, nx, (long long)nx * ny};
    const int a = dir == 0 ? 1 : 0, bb = dir == 2 ? 1 : 2;
    const long long nface = (long long)n[a] * n[bb];
    const long long t = (long long)blk * 256 + threadIdx.x;
    if (t >= 2 * nface) return;
    const int side = t >= nface ? 1 : 0;
    const long long l = t - side * nface;
    const long long ia = l % n[a], ib = l / n[a];
    const int iw = side ? n[dir] - 1 : 0;
    const long long inward = side ? -st[dir] : st[dir];
    const long long o = ia * st[a] + ib * st[bb] + (long long)iw * st[dir];
    auto temp = [&](long long p) {
        return prim_from(c, Q[p], Q[N3 + p], Q[2 * N3 + p], Q[3 * N3 + p], Q[4 * N3 + p]).T;
    };
    const double T1 = temp(o + inward), T2 = temp(o + 2 * inward);
    const double Tw = T1 + (T1 - T2) / 3.0;   // one-sided dT/dn = 0
    const double rho = Q[o];
    Q[N3 + o] = 0.0;
    Q[2 * N3 + o] = 0.0;
    Q[3 * N3 + o] = 0.0;
    Q[4 * N3 + o] = (rho * c.Rh * Tw - c.Rh) / (c.gamma - 1.0);
}
struct BcBody {
    using Args = BcArgs;
    // every node of the face pair is independent: block b takes nodes 256 b ..
    __device__ static void run(const Args &a, int b, int) { bc_body(a, b); }
};
}  // namespace

hipError_t launch_bc(double *Q, const int n[3], int dir, const NdConst &c, hipStream_t st, BatchCollector *col,
                     int phase) {
    const int a = dir == 0 ? 1 : 0, b = dir == 2 ? 1 : 2;
    const long long tot = 2LL * n[a] * n[b];
    const BcArgs x{Q, n[0], n[1], n[2], dir, (long long)n[0] * n[1] * n[2], c};
    return run_body<BcBody, 256>(x, (int)((tot + 255) / 256), dim3(256), st, col, phase);
}

}  // namespace nopcs
