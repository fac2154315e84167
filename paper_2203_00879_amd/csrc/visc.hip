// visc.hip -- viscous terms and gravity source of ge17, explicit second order.
//
// R = dEv/dx + dFv/dy + dGv/dz + S  (ge6-ge8, ge8a, ge19, ge20, bv1-bv3)
// The velocity and temperature gradients inside Ev, Fv, Gv and the outer
// divergence both use second-order differences: central inside, one-sided on
// wall nodes (Section 4).  One block owns a TX x TY tile of an x-y plane and
// marches along z over a chunk of planes; the primitives (u, v, w, T) of five
// consecutive planes with a two-point halo sit in an LDS ring, so every state
// value is read from HBM about once per block.  Tiles at the high end of x
// and y are shifted inward (overlapping their neighbour) so that the one-sided
// wall stencils, which reach three points inward, stay inside the halo.
#include "kernels.hpp"

namespace nopcs {

namespace {
constexpr int VTX = 32, VTY = 6, VLX = VTX + 4, VLY = VTY + 4, VPL = VLX * VLY, VRING = 5;
constexpr int VNT = VTX * VTY;

struct VArgs {
    const double *Q;
    double *R;
    int nx, ny, nz, ntx, nty, zc;
    long long N3;
    double ihx, ihy, ihz;
    NdConst c;
};

struct Ring {
    double (*S)[4][VPL];
    __device__ double at(int a, int li, int lj, int p) const {
        NOPCS_LDS_BOUND(li, VLX);
        NOPCS_LDS_BOUND(lj, VLY);
        NOPCS_LDS_BOUND(p, 1 << 30);
        return S[p % VRING][a][lj * VLX + li];
    }
};

// second-order derivative of primitive a along axis e at local node (li, lj, p)
__device__ inline double grad(const Ring &r, int a, int e, int li, int lj, int p, int gidx, int n, double ih) {
    auto f = [&](int o) -> double {
        return e == 0 ? r.at(a, li + o, lj, p) : e == 1 ? r.at(a, li, lj + o, p) : r.at(a, li, lj, p + o);
    };
    if (gidx == 0) {
        const double f0 = f(0);
        return 0.5 * ih * (4.0 * (f(1) - f0) - (f(2) - f0));
    }
    if (gidx == n - 1) {
        const double f0 = f(0);
        return -0.5 * ih * (4.0 * (f(-1) - f0) - (f(-2) - f0));
    }
    return 0.5 * ih * (f(1) - f(-1));
}

// viscous flux vector along d (Ev, Fv or Gv; components 1..4) at a local node
__device__ inline void vflux(const Ring &r, const VArgs &A, int d, int li, int lj, int p, int gi, int gj, int gk,
                             double out[4]) {
    const NdConst &c = A.c;
    const double u = r.at(0, li, lj, p), v = r.at(1, li, lj, p), w = r.at(2, li, lj, p), T = r.at(3, li, lj, p);
    const double m = mu_of(c, T), b = beta_of(c, T);
    const double Aa = (4.0 / 3.0) * m + b, Bb = b - (2.0 / 3.0) * m;
    auto gx = [&](int a) { return grad(r, a, 0, li, lj, p, gi, A.nx, A.ihx); };
    auto gy = [&](int a) { return grad(r, a, 1, li, lj, p, gj, A.ny, A.ihy); };
    auto gz = [&](int a) { return grad(r, a, 2, li, lj, p, gk, A.nz, A.ihz); };
    if (d == 0) {
        const double ux = gx(0), vx = gx(1), wx = gx(2), Tx = gx(3);
        const double uy = gy(0), vy = gy(1), uz = gz(0), wz = gz(2);
        const double txx = (Aa * ux + Bb * (vy + wz)) * c.iRe;
        const double txy = m * (uy + vx) * c.iRe;
        const double txz = m * (uz + wx) * c.iRe;
        const double qx = -c.kappa * m * Tx;
        out[0] = txx; out[1] = txy; out[2] = txz;
        out[3] = u * txx + v * txy + w * txz - qx;
    } else if (d == 1) {
        const double uy = gy(0), vy = gy(1), wy = gy(2), Ty = gy(3);
        const double ux = gx(0), vx = gx(1), vz = gz(1), wz = gz(2);
        const double txy = m * (uy + vx) * c.iRe;
        const double tyy = (Aa * vy + Bb * (ux + wz)) * c.iRe;
        const double tyz = m * (vz + wy) * c.iRe;
        const double qy = -c.kappa * m * Ty;
        out[0] = txy; out[1] = tyy; out[2] = tyz;
        out[3] = u * txy + v * tyy + w * tyz - qy;
    } else {
        const double uz = gz(0), vz = gz(1), wz = gz(2), Tz = gz(3);
        const double ux = gx(0), wx = gx(2), vy = gy(1), wy = gy(2);
        const double txz = m * (uz + wx) * c.iRe;
        const double tyz = m * (vz + wy) * c.iRe;
        const double tzz = (Aa * wz + Bb * (ux + vy)) * c.iRe;
        const double qz = -c.kappa * m * Tz;
        out[0] = txz; out[1] = tyz; out[2] = tzz;
        out[3] = u * txz + v * tyz + w * tzz - qz;
    }
}

// divergence contribution d(flux_d)/dx_d at the output node, all 4 components
__device__ inline void vdiv(const Ring &r, const VArgs &A, int d, int li, int lj, int p, int gi, int gj, int gk,
                            double acc[4]) {
    const int gidx = d == 0 ? gi : d == 1 ? gj : gk;
    const int n = d == 0 ? A.nx : d == 1 ? A.ny : A.nz;
    const double ih = d == 0 ? A.ihx : d == 1 ? A.ihy : A.ihz;
    auto node = [&](int o, double out[4]) {
        vflux(r, A, d, li + (d == 0 ? o : 0), lj + (d == 1 ? o : 0), p + (d == 2 ? o : 0), gi + (d == 0 ? o : 0),
              gj + (d == 1 ? o : 0), gk + (d == 2 ? o : 0), out);
    };
    double f0[4], f1[4], f2[4];
    if (gidx == 0) {
        node(0, f0); node(1, f1); node(2, f2);
        for (int q = 0; q < 4; ++q) acc[q] = 0.5 * ih * (4.0 * (f1[q] - f0[q]) - (f2[q] - f0[q]));
    } else if (gidx == n - 1) {
        node(0, f0); node(-1, f1); node(-2, f2);
        for (int q = 0; q < 4; ++q) acc[q] = -0.5 * ih * (4.0 * (f1[q] - f0[q]) - (f2[q] - f0[q]));
    } else {
        node(1, f1); node(-1, f0);
        for (int q = 0; q < 4; ++q) acc[q] = 0.5 * ih * (f1[q] - f0[q]);
    }
}

__global__ __launch_bounds__(VNT) void k_visc(VArgs A) {
    const int b = blockIdx.x;
    const int tt = b % A.ntx, rest = b / A.ntx, ty = rest % A.nty, tz = rest / A.nty;
    const int i0 = min(tt * VTX, max(0, A.nx - VTX));
    const int j0 = min(ty * VTY, max(0, A.ny - VTY));
    const int k0 = tz * A.zc, k1 = min(A.nz, k0 + A.zc);
    const int tid = threadIdx.x;
    const int gi = i0 + tid % VTX, gj = j0 + tid / VTX;
    const bool valid = gi < A.nx && gj < A.ny;
    const long long N3 = A.N3;
    const NdConst &c = A.c;
    const double *Q = A.Q;

    if (!c.viscous) {
        for (int k = k0; k < k1; ++k) {
            if (!valid) continue;
            const long long o = gi + (long long)A.nx * (gj + (long long)A.ny * k);
            A.R[o] = 0.0;
            A.R[N3 + o] = 0.0;
            A.R[2 * N3 + o] = 0.0 - c.ghat * Q[o];
            A.R[3 * N3 + o] = 0.0;
            A.R[4 * N3 + o] = 0.0 - c.ghat * Q[2 * N3 + o];
        }
        return;
    }

    __shared__ double S[VRING][4][VPL];
    Ring r{S};
    auto load_plane = [&](int p) {
        for (int q = tid; q < VPL; q += VNT) {
            const int li = q % VLX, lj = q / VLX;
            const int x = i0 - 2 + li, y = j0 - 2 + lj;
            if (x < 0 || x >= A.nx || y < 0 || y >= A.ny) continue;
            const long long o = x + (long long)A.nx * (y + (long long)A.ny * p);
            const Prim pr = prim_from(c, Q[o], Q[N3 + o], Q[2 * N3 + o], Q[3 * N3 + o], Q[4 * N3 + o]);
            const int slot = p % VRING;
            S[slot][0][q] = pr.u;
            S[slot][1][q] = pr.v;
            S[slot][2][q] = pr.w;
            S[slot][3][q] = pr.T;
        }
    };
    const int lo = max(0, min(k0 - 2, A.nz - 4));
    int loaded = min(A.nz - 1, max(k0 + 2, 3));
    for (int p = lo; p <= loaded; ++p) load_plane(p);
    __syncthreads();
    const int li = tid % VTX + 2, lj = tid / VTX + 2;
    for (int k = k0; k < k1; ++k) {
        const int target = min(A.nz - 1, max(k + 2, 3));
        if (loaded < target) {
            while (loaded < target) load_plane(++loaded);
            __syncthreads();
        }
        if (valid) {
            double ax[4], ay[4], az[4];
            vdiv(r, A, 0, li, lj, k, gi, gj, k, ax);
            vdiv(r, A, 1, li, lj, k, gi, gj, k, ay);
            vdiv(r, A, 2, li, lj, k, gi, gj, k, az);
            const long long o = gi + (long long)A.nx * (gj + (long long)A.ny * k);
            double acc[4];
            for (int q = 0; q < 4; ++q) acc[q] = ax[q] + ay[q] + az[q];
            A.R[o] = 0.0;
            A.R[N3 + o] = acc[0];
            A.R[2 * N3 + o] = acc[1] - c.ghat * Q[o];
            A.R[3 * N3 + o] = acc[2];
            A.R[4 * N3 + o] = acc[3] - c.ghat * Q[2 * N3 + o];
        }
        __syncthreads();
    }
}
}  // namespace

hipError_t launch_visc(const double *Q, double *R, const int n[3], const double ih[3], const NdConst &c,
                       hipStream_t st) {
    VArgs A;
    A.Q = Q;
    A.R = R;
    A.nx = n[0];
    A.ny = n[1];
    A.nz = n[2];
    A.ntx = (n[0] + VTX - 1) / VTX;
    A.nty = (n[1] + VTY - 1) / VTY;
    A.zc = n[2] <= 64 ? 16 : 32;
    A.N3 = (long long)n[0] * n[1] * n[2];
    A.ihx = ih[0];
    A.ihy = ih[1];
    A.ihz = ih[2];
    A.c = c;
    const int ntz = (n[2] + A.zc - 1) / A.zc;
    const long long blocks = (long long)A.ntx * A.nty * ntz;
    hipLaunchKernelGGL(k_visc, dim3((unsigned)blocks), dim3(VNT), 0, st, A);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wall conditions of the closed adiabatic box (Section 2), one face pair.
// ---------------------------------------------------------------------------
namespace {
__global__ void k_bc(double *Q, int nx, int ny, int nz, int dir, long long N3, NdConst c) {
    const int n[3] = {nx, ny, nz};
    const long long st[3] = {1, nx, (long long)nx * ny};
    const int a = dir == 0 ? 1 : 0, bb = dir == 2 ? 1 : 2;
    const long long nface = (long long)n[a] * n[bb];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
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
}  // namespace

hipError_t launch_bc(double *Q, const int n[3], int dir, const NdConst &c, hipStream_t st) {
    const int a = dir == 0 ? 1 : 0, b = dir == 2 ? 1 : 2;
    const long long tot = 2LL * n[a] * n[b];
    const int nt = 256;
    hipLaunchKernelGGL(k_bc, dim3((unsigned)((tot + nt - 1) / nt)), dim3(nt), 0, st, Q, n[0], n[1], n[2], dir,
                       (long long)n[0] * n[1] * n[2], c);
    return hipGetLastError();
}

}  // namespace nopcs
