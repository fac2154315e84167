// Host driver of the CPU build of libnopcs (kernels run through the CPU HIP
// stand-in under AddressSanitizer).  Test infrastructure only.
//   driver deriv nx ny nz sx sy sz lx ly lz dir  in out        (in: N, out: d1 then d2)
//   driver rhs   nx ny nz sx sy sz lx ly lz viscous gravity in out   (in/out: 5N)
//   driver rk    nx ny nz sx sy sz lx ly lz viscous gravity dt nsteps in out
//   driver plan  n nseg piece_len                            (prints the line-march tables)
// Environment: NOPCS_EMUL_PIECE sets the extra-cut length of every direction.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nopcs.h"
#include "../../paper_2203_00879_amd/csrc/plan.hpp"
#include "hip/hip_runtime.h"

// device-like buffers: guarded on both sides
struct Buf {
    double *p;
    size_t n;
    explicit Buf(size_t n_) : p((double *)emu_guarded_alloc(n_ * sizeof(double))), n(n_) {}
    ~Buf() { emu_guarded_free(p); }
};

static std::vector<double> read_raw(const char *path, size_t n) {
    std::vector<double> v(n);
    FILE *f = std::fopen(path, "rb");
    if (!f || std::fread(v.data(), sizeof(double), n, f) != n) { std::fprintf(stderr, "read %s failed\n", path); std::exit(3); }
    std::fclose(f);
    return v;
}
static void write_raw(const char *path, const double *p, size_t n) {
    FILE *f = std::fopen(path, "wb");
    if (!f || std::fwrite(p, sizeof(double), n, f) != n) { std::fprintf(stderr, "write %s failed\n", path); std::exit(3); }
    std::fclose(f);
}

int main(int argc, char **argv) {
    if (argc < 2) { std::fprintf(stderr, "usage\n"); return 2; }
    const std::string mode = argv[1];
    if (mode == "plan" && argc >= 5) {  // driver plan n nseg piece: line-march tables of one line plan
        nopcs::LinePlanHost P;
        std::string err;
        if (!nopcs::build_line_plan(std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]), P, err)) return 1;
        std::printf("nrun %zu ncl %zu max_m %d k1_S %d ngrp %zu\n", P.runs.size(), P.cl_row.size(), P.max_m, P.k1_S,
                    P.grp.size());
        return 0;
    }
    if (argc < 11) { std::fprintf(stderr, "usage\n"); return 2; }
    // NOPCS_EMUL_PIECE: extra-cut length for all directions (-1 default, 0 none)
    if (const char *pc = std::getenv("NOPCS_EMUL_PIECE"))
        for (int d = 0; d < 3; ++d)
            if (nopcs_set_piece_length(d, std::atoi(pc)) != NOPCS_OK) return 2;
    nopcs_grid g;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = std::atoi(argv[2 + d]);
        g.nseg[d] = std::atoi(argv[5 + d]);
        g.len[d] = std::atof(argv[8 + d]);
    }
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    nse_params p;
    p.gamma = 1.4; p.R_gas = 287.0; p.g = 9.81; p.L = 0.15; p.T_s = 300.0; p.rho_s = 101325.0 / (287.0 * 300.0);
    p.Pr = 0.712; p.mu_ref = 1.716e-5; p.T_ref = 273.15; p.S_suth = 110.4; p.mub_a = 3.381e-4; p.mub_b = 7.383e-4;
    int rc = 0;
    if (mode == "deriv") {
        const int dir = std::atoi(argv[11]);
        std::vector<double> fh = read_raw(argv[12], N);
        Buf f(N), d1(N), d2(N);
        std::memcpy(f.p, fh.data(), N * sizeof(double));
        rc = nopcs_derivative(&g, dir, NOPCS_FP64, f.p, d1.p, d2.p, nullptr);
        if (rc == 0) {
            std::vector<double> out(2 * N);
            std::memcpy(out.data(), d1.p, N * sizeof(double));
            std::memcpy(out.data() + N, d2.p, N * sizeof(double));
            write_raw(argv[13], out.data(), 2 * N);
        }
    } else if (mode == "rhs") {
        p.viscous = std::atoi(argv[11]);
        p.gravity = std::atoi(argv[12]);
        std::vector<double> Qh = read_raw(argv[13], 5 * N);
        Buf Q(5 * N), R(5 * N);
        std::memcpy(Q.p, Qh.data(), 5 * N * sizeof(double));
        const size_t wsb = nopcs_workspace_bytes(&g, NOPCS_FP64);
        Buf ws((wsb + 7) / 8);
        rc = nse_rhs(&p, &g, NOPCS_FP64, Q.p, R.p, ws.p, wsb, nullptr);
        if (rc == 0) write_raw(argv[14], R.p, 5 * N);
    } else if (mode == "rk") {
        p.viscous = std::atoi(argv[11]);
        p.gravity = std::atoi(argv[12]);
        const double dt = std::atof(argv[13]);
        const int nsteps = std::atoi(argv[14]);
        std::vector<double> Qh = read_raw(argv[15], 5 * N);
        Buf Q(5 * N);
        std::memcpy(Q.p, Qh.data(), 5 * N * sizeof(double));
        const size_t wsb = nopcs_workspace_bytes(&g, NOPCS_FP64);
        Buf ws((wsb + 7) / 8);
        rc = rk_step(&p, &g, NOPCS_FP64, Q.p, dt, nsteps, ws.p, wsb, nullptr);
        if (rc == 0) write_raw(argv[16], Q.p, 5 * N);
    } else {
        return 2;
    }
    if (rc != 0) std::fprintf(stderr, "call failed: %d %s\n", rc, nopcs_last_error());
    nopcs_release_plans();
    return rc == 0 ? 0 : 1;
}
