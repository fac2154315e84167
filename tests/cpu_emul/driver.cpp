// Host driver of the CPU build of libnopcs (kernels run through the CPU HIP
// stand-in under AddressSanitizer).  Test infrastructure only.
//   driver deriv nx ny nz sx sy sz lx ly lz dir  in out        (in: N, out: d1 then d2)
//   driver rhs   nx ny nz sx sy sz lx ly lz viscous gravity in out   (in/out: 5N)
//   driver rk    nx ny nz sx sy sz lx ly lz viscous gravity dt nsteps in out
//   driver filter nx ny nz sx sy sz lx ly lz af every dt nsteps in out  (nopcs_filter if nsteps is 0,
//                                                              else rk_step_filtered; in/out: 5N)
//   driver plan  n nseg piece_len                            (prints the line-march tables)
//   driver serve | serve_batched          (scripted checks of the serving runtime; per-request streams
//                                          or batched chunks)
//   driver batch [modes]               (batched stepping of uneven boxes against each box's lone step,
//                                       in the listed batch modes, default 2013)
// Environment: NOPCS_EMUL_PIECE sets the extra-cut length of every direction;
// NOPCS_EMUL_PRECISION=1 runs rhs and rk in mixed precision.
#include <chrono>
#include <random>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nopcs.h"

namespace nopcs {
size_t graph_cache_entries();   // cached RK4 steps (library-internal)
}
#include "../../paper_2203_00879_amd/csrc/plan.hpp"
#include "hip/hip_runtime.h"

// Context switch of the emulated device threads (x86-64 System V): saves the
// callee-saved registers, MXCSR and the x87 control word on the current stack,
// stores the stack pointer in *save_sp and resumes the context saved at new_sp.
asm(R"(
    .text
    .globl emu_ctx_switch
    .type emu_ctx_switch, @function
emu_ctx_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    subq $8, %rsp
    stmxcsr (%rsp)
    fnstcw 4(%rsp)
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    ldmxcsr (%rsp)
    fldcw 4(%rsp)
    addq $8, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_ctx_switch, .-emu_ctx_switch
    .section .note.GNU-stack,"",@progbits
    .text
)");

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

static nse_params air_params() {
    nse_params p;
    p.gamma = 1.4; p.R_gas = 287.0; p.g = 9.81; p.L = 0.15; p.T_s = 300.0; p.rho_s = 101325.0 / (287.0 * 300.0);
    p.Pr = 0.712; p.mu_ref = 1.716e-5; p.T_ref = 273.15; p.S_suth = 110.4; p.mub_a = 3.381e-4; p.mub_b = 7.383e-4;
    p.viscous = 1; p.gravity = 1;
    return p;
}

// a smooth non-dimensional state on an n^3 box (rho ~ 1, small velocities, E' ~ 0)
static std::vector<double> test_state(int n, int seed) {
    const size_t N = (size_t)n * n * n;
    std::vector<double> q(5 * N);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const size_t o = i + (size_t)n * (j + (size_t)n * k);
                const double a = 0.3 * (seed + 1), x = (double)i / (n - 1), y = (double)j / (n - 1), z = (double)k / (n - 1);
                q[o] = 1.0 + 0.05 * std::sin(6.0 * x + a) * std::cos(5.0 * y - a) * std::sin(4.0 * z + 1.0);
                q[N + o] = 0.01 * std::sin(3.0 * y + a) * x * (1 - x);
                q[2 * N + o] = 0.01 * std::cos(2.0 * z - a) * y * (1 - y);
                q[3 * N + o] = 0.01 * std::sin(4.0 * x + 2 * a) * z * (1 - z);
                q[4 * N + o] = 50.0 * std::cos(3.0 * x - a) * std::sin(2.0 * y + z);
            }
    return q;
}

#define SERVE_CHECK(cond, what)                                          \
    do {                                                                 \
        if (!(cond)) {                                                   \
            std::fprintf(stderr, "serve check failed: %s\n", what);     \
            return 1;                                                    \
        }                                                                \
        std::printf("ok %s\n", what);                                   \
    } while (0)

// Scripted checks of the serving runtime on 8^3 boxes.
static int serve_checks(int batched) {
    const int n = 8, nsteps = 1;
    const double dt = 1e-5;
    nse_params p = air_params();
    nopcs_grid g;
    for (int d = 0; d < 3; ++d) { g.n[d] = n; g.nseg[d] = 1; g.len[d] = 1.0; }
    const size_t N5 = 5 * (size_t)n * n * n;
    const size_t wsb = nopcs_workspace_bytes(&g, NOPCS_FP64);
    const size_t fp = ((N5 * sizeof(double) + 255) & ~(size_t)255) + wsb;
    // references: rk_step on each state alone (before any solver thread runs
    // kernels); the three requests of check 1 run 1, 6 and 11 steps (several
    // chunks of at most 8 steps, members leaving the batch at different times)
    const int steps_of[3] = {1, 6, 11};
    std::vector<std::vector<double>> q0(3), ref(3);
    for (int r = 0; r < 3; ++r) {
        q0[r] = test_state(n, r);
        Buf Q(N5), ws((wsb + 7) / 8);
        std::memcpy(Q.p, q0[r].data(), N5 * sizeof(double));
        if (rk_step(&p, &g, NOPCS_FP64, Q.p, dt, steps_of[r], ws.p, wsb, nullptr) != NOPCS_OK) return 1;
        ref[r].assign(Q.p, Q.p + N5);
    }
    solve_request rq{};
    rq.params = p; rq.grid = g; rq.nsteps = nsteps; rq.precision = NOPCS_FP64; rq.dt = dt;
    // 1. three requests on two slots: every result equals its box run alone, bit for bit
    {
        solver_config cfg{2 * fp, 2, 16, 0, batched};
        nopcs_solver *s = nullptr;
        SERVE_CHECK(solver_create(&cfg, &s) == NOPCS_OK, "create");
        uint64_t id[3];
        for (int r = 0; r < 3; ++r) {
            rq.Q0_host = q0[r].data();
            rq.nsteps = steps_of[r];
            SERVE_CHECK(solver_submit(s, &rq, &id[r]) == NOPCS_OK, "submit");
        }
        rq.nsteps = nsteps;
        std::vector<double> out(N5);
        solve_result res{};
        for (int r = 0; r < 3; ++r) {
            int rc;
            while ((rc = solver_poll(s, id[r], out.data(), &res)) == NOPCS_EAGAIN) std::this_thread::sleep_for(std::chrono::milliseconds(5));
            SERVE_CHECK(rc == NOPCS_OK && res.steps_done == steps_of[r], "request done");
            SERVE_CHECK(std::memcmp(out.data(), ref[r].data(), N5 * sizeof(double)) == 0, "mix equals alone bit for bit");
            SERVE_CHECK(res.t_submit <= res.t_admit && res.t_admit <= res.t_done, "timestamps ordered");
        }
        SERVE_CHECK(solver_poll(s, id[0], nullptr, &res) == NOPCS_ENOTFOUND, "released id not found");
        SERVE_CHECK(solver_destroy(s) == NOPCS_OK, "destroy");
    }
    // 2. budget for one box: admission strictly in arrival order; a non-finite box is flagged
    {
        solver_config cfg{fp, 4, 16, 0, batched};
        nopcs_solver *s = nullptr;
        SERVE_CHECK(solver_create(&cfg, &s) == NOPCS_OK, "create (one box budget)");
        std::vector<double> bad = q0[1];
        bad[7] = std::nan("");
        uint64_t id[3];
        const double *src[3] = {q0[0].data(), bad.data(), q0[2].data()};
        for (int r = 0; r < 3; ++r) {
            rq.Q0_host = src[r];
            SERVE_CHECK(solver_submit(s, &rq, &id[r]) == NOPCS_OK, "submit (one box budget)");
        }
        solve_result res[3];
        int rc[3];
        for (int r = 0; r < 3; ++r)
            while ((rc[r] = solver_poll(s, id[r], nullptr, &res[r])) == NOPCS_EAGAIN) std::this_thread::sleep_for(std::chrono::milliseconds(5));
        SERVE_CHECK(rc[0] == NOPCS_OK && rc[2] == NOPCS_OK, "finite boxes ok");
        SERVE_CHECK(rc[1] == NOPCS_ENONFINITE, "non-finite box flagged");
        SERVE_CHECK(res[0].t_done <= res[1].t_admit && res[1].t_done <= res[2].t_admit, "admitted in arrival order, one at a time");
        SERVE_CHECK(solver_destroy(s) == NOPCS_OK, "destroy (one box budget)");
    }
    // 3. argument and capacity errors; destroy with work pending
    {
        solver_config cfg{fp, 1, 1, 0, batched};
        nopcs_solver *s = nullptr;
        SERVE_CHECK(solver_create(&cfg, &s) == NOPCS_OK, "create (queue of one)");
        uint64_t id = 0;
        rq.Q0_host = q0[0].data();
        rq.nsteps = 0;
        SERVE_CHECK(solver_submit(s, &rq, &id) == NOPCS_EINVAL, "nsteps 0 rejected");
        rq.nsteps = 8;   // one chunk: keeps the slot busy while the queue fills
        rq.precision = 7;
        SERVE_CHECK(solver_submit(s, &rq, &id) == NOPCS_EINVAL, "unknown precision rejected");
        rq.precision = NOPCS_FP64;
        nopcs_grid big = g;
        big.n[0] = 16;
        solve_request rb = rq;
        rb.grid = big;
        SERVE_CHECK(solver_submit(s, &rb, &id) == NOPCS_ENOMEM, "over-budget box rejected");
        int busy = 0;
        for (int k = 0; k < 8 && !busy; ++k) busy = solver_submit(s, &rq, &id) == NOPCS_EBUSY;
        SERVE_CHECK(busy, "full queue answers EBUSY");
        SERVE_CHECK(solver_poll(s, 987654321ULL, nullptr, nullptr) == NOPCS_ENOTFOUND, "unknown id");
        SERVE_CHECK(solver_destroy(s) == NOPCS_OK, "destroy with pending work");
        solver_config badcfg{fp, 0, 1, 0, batched};
        SERVE_CHECK(solver_create(&badcfg, &s) == NOPCS_EINVAL, "zero slots rejected");
    }
    // 4. a stream of 8 requests on 4 slots, each with its own dt and 1-3
    //    steps (requests joining and leaving batches at every chunk): every
    //    result equals its box run alone, bit for bit
    {
        const int nr = 8;
        std::vector<std::vector<double>> want(nr);
        std::vector<double> dts(nr);
        std::vector<int> nst(nr);
        for (int r = 0; r < nr; ++r) {
            dts[r] = 1e-5 * (1.0 + 0.013 * r);
            nst[r] = 1 + r % 3;
            Buf Q(N5), ws((wsb + 7) / 8);
            std::memcpy(Q.p, q0[r % 3].data(), N5 * sizeof(double));
            if (rk_step(&p, &g, NOPCS_FP64, Q.p, dts[r], nst[r], ws.p, wsb, nullptr) != NOPCS_OK) return 1;
            want[r].assign(Q.p, Q.p + N5);
        }
        solver_config cfg{4 * fp, 4, nr, 0, batched};
        nopcs_solver *s = nullptr;
        SERVE_CHECK(solver_create(&cfg, &s) == NOPCS_OK, "create (stream)");
        std::vector<uint64_t> id(nr);
        bool all_sub = true;
        for (int r = 0; r < nr; ++r) {
            solve_request q = rq;
            q.Q0_host = q0[r % 3].data();
            q.dt = dts[r];
            q.nsteps = nst[r];
            all_sub = all_sub && solver_submit(s, &q, &id[r]) == NOPCS_OK;
        }
        SERVE_CHECK(all_sub, "stream submitted");
        std::vector<double> out(N5);
        bool same = true;
        for (int r = 0; r < nr; ++r) {
            solve_result res{};
            int rc;
            while ((rc = solver_poll(s, id[r], out.data(), &res)) == NOPCS_EAGAIN) std::this_thread::sleep_for(std::chrono::milliseconds(2));
            same = same && rc == NOPCS_OK && res.steps_done == nst[r] &&
                   std::memcmp(out.data(), want[r].data(), N5 * sizeof(double)) == 0;
        }
        SERVE_CHECK(same, "stream of 8 equals alone bit for bit");
        SERVE_CHECK(solver_destroy(s) == NOPCS_OK, "destroy (stream)");
    }
    return 0;
}

// a smooth state on an nx x ny x nz box (as test_state, any shape)
static std::vector<double> box_state(const int n[3], int seed) {
    const size_t N = (size_t)n[0] * n[1] * n[2];
    std::vector<double> q(5 * N);
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                const size_t o = i + (size_t)n[0] * (j + (size_t)n[1] * k);
                const double a = 0.3 * (seed + 1), x = (double)i / (n[0] - 1), y = (double)j / (n[1] - 1),
                             z = (double)k / (n[2] - 1);
                q[o] = 1.0 + 0.05 * std::sin(6.0 * x + a) * std::cos(5.0 * y - a) * std::sin(4.0 * z + 1.0);
                q[N + o] = 0.01 * std::sin(3.0 * y + a) * x * (1 - x);
                q[2 * N + o] = 0.01 * std::cos(2.0 * z - a) * y * (1 - y);
                q[3 * N + o] = 0.01 * std::sin(4.0 * x + 2 * a) * z * (1 - z);
                q[4 * N + o] = 50.0 * std::cos(3.0 * x - a) * std::sin(2.0 * y + z);
            }
    return q;
}

// Batched stepping (rk_step_batch, direct launches) of uneven boxes against
// rk_step on each box alone: every box bit for bit.
static int batch_checks(int prec, const std::string &mode_list) {
    struct Shape { int n[3], s[3]; double dt; };
    const Shape shapes[] = {{{8, 8, 8}, {1, 1, 1}, 1e-5},
                            {{16, 12, 10}, {2, 1, 1}, 2e-5},
                            {{16, 12, 10}, {2, 1, 1}, 0.0},   // the call's dt
                            {{20, 18, 27}, {1, 2, 3}, 1e-5},
                            {{9, 70, 11}, {1, 2, 1}, 3e-5}};
    const int nb = sizeof shapes / sizeof shapes[0], nsteps = 1;
    const double dt_call = 1.5e-5;
    nse_params p = air_params();
    std::vector<nopcs_grid> g(nb);
    std::vector<std::vector<double>> q0(nb), ref(nb);
    std::vector<Buf *> Q(nb), W(nb);
    std::vector<size_t> wsb(nb), n5(nb);
    for (int b = 0; b < nb; ++b) {
        for (int d = 0; d < 3; ++d) {
            g[b].n[d] = shapes[b].n[d];
            g[b].nseg[d] = shapes[b].s[d];
            g[b].len[d] = 1.0 + 0.25 * d;
        }
        n5[b] = 5 * (size_t)g[b].n[0] * g[b].n[1] * g[b].n[2];
        wsb[b] = nopcs_workspace_bytes(&g[b], prec);
        q0[b] = box_state(g[b].n, b);
        Q[b] = new Buf(n5[b]);
        W[b] = new Buf((wsb[b] + 7) / 8);
        std::memcpy(Q[b]->p, q0[b].data(), n5[b] * sizeof(double));
        const double dt = shapes[b].dt > 0 ? shapes[b].dt : dt_call;
        if (rk_step(&p, &g[b], prec, Q[b]->p, dt, nsteps, W[b]->p, wsb[b], nullptr) != NOPCS_OK) {
            std::fprintf(stderr, "lone rk_step failed: %s\n", nopcs_last_error());
            return 1;
        }
        ref[b].assign(Q[b]->p, Q[b]->p + n5[b]);
        std::memcpy(Q[b]->p, q0[b].data(), n5[b] * sizeof(double));
    }
    std::vector<nopcs_box> boxes(nb);
    for (int b = 0; b < nb; ++b) boxes[b] = nopcs_box{g[b], Q[b]->p, W[b]->p, wsb[b], shapes[b].dt};
    int rc = NOPCS_OK;
    std::vector<int> modes;
    for (char ch : mode_list) modes.push_back(ch - '0');
    const int nrep = 2 * (int)modes.size();
    for (int rep = 0; rep < nrep && rc == NOPCS_OK; ++rep) {   // per mode: the second call replays the cached step
        if (rep % 2 == 0) rc = nopcs_set_batch_mode(modes[rep / 2]);
        for (int b = 0; b < nb; ++b) std::memcpy(Q[b]->p, q0[b].data(), n5[b] * sizeof(double));
        if (rc == NOPCS_OK) rc = rk_step_batch(&p, nb, boxes.data(), prec, dt_call, nsteps, nullptr);
        for (int b = 0; b < nb && rc == NOPCS_OK; ++b) {
            if (std::memcmp(Q[b]->p, ref[b].data(), n5[b] * sizeof(double)) != 0) {
                size_t bad = 0;
                while (Q[b]->p[bad] == ref[b][bad]) ++bad;
                std::fprintf(stderr, "box %d differs from its lone step at %zu: %.17g vs %.17g\n", b, bad, Q[b]->p[bad],
                             ref[b][bad]);
                rc = 1;
            }
        }
        if (rc == NOPCS_OK)
            std::printf("ok batch mode %d call %d: %d boxes bit-identical to their lone steps\n", modes[rep / 2],
                        rep % 2, nb);
    }
    if (rc > 1) std::fprintf(stderr, "rk_step_batch failed: %d %s\n", rc, nopcs_last_error());
    // equal grids whose padding bytes differ (memory a C caller never wrote)
    // reuse the cached step: a batch and a lone graph step, each called twice
    if (rc == NOPCS_OK) {
        std::vector<nopcs_box> junk = boxes;
        for (int b = 0; b < nb; ++b) {
            std::memset(static_cast<void *>(&junk[b].grid), 0xA5 + b, sizeof(nopcs_grid));
            for (int d = 0; d < 3; ++d) {
                junk[b].grid.n[d] = g[b].n[d];
                junk[b].grid.len[d] = g[b].len[d];
                junk[b].grid.nseg[d] = g[b].nseg[d];
            }
        }
        const size_t before = nopcs::graph_cache_entries();
        rc = rk_step_batch(&p, nb, junk.data(), prec, dt_call, nsteps, nullptr);
        const size_t after_batch = nopcs::graph_cache_entries();
        if (rc == NOPCS_OK) rc = nopcs_set_graphs(1);
        if (rc == NOPCS_OK) rc = rk_step(&p, &g[1], prec, Q[1]->p, dt_call, 1, W[1]->p, wsb[1], nullptr);
        const size_t after_lone = nopcs::graph_cache_entries();
        if (rc == NOPCS_OK) rc = rk_step(&p, &junk[1].grid, prec, Q[1]->p, dt_call, 1, W[1]->p, wsb[1], nullptr);
        const size_t after_junk = nopcs::graph_cache_entries();
        (void)nopcs_set_graphs(0);
        if (rc == NOPCS_OK && (after_batch != before || after_lone != before + 1 || after_junk != after_lone)) {
            std::fprintf(stderr, "graph cache keyed by padding: %zu %zu %zu %zu entries\n", before, after_batch,
                         after_lone, after_junk);
            rc = 1;
        }
        if (rc == NOPCS_OK) std::printf("ok grids differing in padding only reuse the cached steps\n");
    }
    // more distinct batches than the cache holds (limit lowered to 3): every
    // call a new step (the first box's workspace moved by 256 bytes each time,
    // which changes no result), so cached steps are evicted while new ones are
    // made; each call checked against the lone steps
    const int nchurn = 8;
    if (rc == NOPCS_OK && nopcs_set_graph_cache_limit(3) != NOPCS_OK) rc = 1;
    std::vector<std::vector<double>> lone(2);
    Buf wbig((wsb[0] + 256 * nchurn + 7) / 8);
    for (int b = 0; b < 2 && rc == NOPCS_OK; ++b) {
        std::memcpy(Q[b]->p, q0[b].data(), n5[b] * sizeof(double));
        rc = rk_step(&p, &g[b], prec, Q[b]->p, dt_call, 1, W[b]->p, wsb[b], nullptr);
        lone[b].assign(Q[b]->p, Q[b]->p + n5[b]);
    }
    for (int c = 0; c < nchurn && rc == NOPCS_OK; ++c) {
        nopcs_box two[2] = {boxes[0], boxes[1]};
        two[0].dt = two[1].dt = 0.0;
        two[0].ws = reinterpret_cast<char *>(wbig.p) + 256 * (size_t)c;
        for (int b = 0; b < 2; ++b) std::memcpy(Q[b]->p, q0[b].data(), n5[b] * sizeof(double));
        rc = nopcs_set_batch_mode(c % 4);
        if (rc == NOPCS_OK) rc = rk_step_batch(&p, 2, two, prec, dt_call, 1, nullptr);
        for (int b = 0; b < 2 && rc == NOPCS_OK; ++b)
            if (std::memcmp(Q[b]->p, lone[b].data(), n5[b] * sizeof(double)) != 0) {
                std::fprintf(stderr, "churn call %d: box %d differs from its lone step\n", c, b);
                rc = 1;
            }
    }
    if (rc == NOPCS_OK) std::printf("ok %d distinct batches through the cache\n", nchurn);
    if (nopcs_set_graph_cache_limit(0) != NOPCS_EINVAL || nopcs_set_graph_cache_limit(64) != NOPCS_OK) rc = 1;
    (void)nopcs_set_batch_mode(3);
    // errors: duplicate state, misaligned workspace, negative dt
    if (rc == NOPCS_OK) {
        std::vector<nopcs_box> bad = boxes;
        bad[1].Q = bad[0].Q;
        bad[1].grid = bad[0].grid;
        if (rk_step_batch(&p, 2, bad.data(), prec, dt_call, 1, nullptr) != NOPCS_EINVAL) rc = 1;
        bad = boxes;
        bad[0].ws = static_cast<char *>(bad[0].ws) + 8;
        if (rk_step_batch(&p, 1, bad.data(), prec, dt_call, 1, nullptr) != NOPCS_EINVAL) rc = 1;
        bad = boxes;
        bad[0].dt = -1.0;
        if (rk_step_batch(&p, 1, bad.data(), prec, dt_call, 1, nullptr) != NOPCS_EINVAL) rc = 1;
        if (rk_step_batch(&p, 0, boxes.data(), prec, dt_call, 1, nullptr) != NOPCS_EINVAL) rc = 1;
        if (nopcs_set_batch_mode(4) != NOPCS_EINVAL) rc = 1;
        std::printf(rc == NOPCS_OK ? "ok batch argument errors\n" : "batch argument errors not reported\n");
    }
    for (int b = 0; b < nb; ++b) { delete Q[b]; delete W[b]; }
    nopcs_release_plans();
    return rc == NOPCS_OK ? 0 : 1;
}

// A stream like the serving benchmark's on the CPU build: requests of
// uneven small boxes arrive over time (seeded), every pending request polled
// every millisecond, half of them in mixed precision, each with its own dt
// and 1-20 steps; every result against its lone rk_step, bit for bit.
static int serve_stress(int batched, int nr) {
    std::mt19937 rng(4);
    const int sizes[4][3] = {{8, 8, 8}, {12, 10, 9}, {16, 16, 12}, {9, 20, 10}};
    const int segs[4][3] = {{1, 1, 1}, {1, 2, 1}, {2, 1, 1}, {1, 2, 1}};
    nse_params p = air_params();
    struct W { nopcs_grid g; std::vector<double> q0, want; int steps, prec; double dt, t; };
    std::vector<W> w(nr);
    double t = 0.0;
    for (int r = 0; r < nr; ++r) {
        const int k = (int)(rng() % 4);
        for (int d = 0; d < 3; ++d) { w[r].g.n[d] = sizes[k][d]; w[r].g.nseg[d] = segs[k][d]; w[r].g.len[d] = 1.0; }
        w[r].q0 = box_state(w[r].g.n, r);
        w[r].steps = 1 + (int)(rng() % 20);
        w[r].prec = (r % 2) ? NOPCS_MIXED : NOPCS_FP64;
        w[r].dt = 1e-5 * (1.0 + 0.01 * (double)(rng() % 50));
        t += 0.002 * (double)(rng() % 20);
        w[r].t = t;
        const size_t n5 = w[r].q0.size();
        const size_t wsb = nopcs_workspace_bytes(&w[r].g, w[r].prec);
        Buf Q(n5), ws((wsb + 7) / 8);
        std::memcpy(Q.p, w[r].q0.data(), n5 * sizeof(double));
        if (rk_step(&p, &w[r].g, w[r].prec, Q.p, w[r].dt, w[r].steps, ws.p, wsb, nullptr) != NOPCS_OK) return 1;
        w[r].want.assign(Q.p, Q.p + n5);
    }
    solver_config cfg{(size_t)1 << 32, 8, nr, 0, batched};
    nopcs_solver *s = nullptr;
    SERVE_CHECK(solver_create(&cfg, &s) == NOPCS_OK, "create (stress)");
    std::vector<uint64_t> id(nr);
    std::vector<int> state(nr, 0);   // 0 not submitted, 1 pending, 2 done
    int done = 0, k = 0;
    bool same = true;
    const auto t0 = std::chrono::steady_clock::now();
    while (done < nr) {
        const double now = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        while (k < nr && w[k].t <= now) {
            solve_request q{};
            q.params = p; q.grid = w[k].g; q.nsteps = w[k].steps; q.precision = w[k].prec; q.dt = w[k].dt;
            q.Q0_host = w[k].q0.data();
            if (solver_submit(s, &q, &id[k]) != NOPCS_OK) { std::fprintf(stderr, "submit %d failed\n", k); return 1; }
            state[k++] = 1;
        }
        for (int r = 0; r < k; ++r) {
            if (state[r] != 1) continue;
            std::vector<double> out(w[r].q0.size());
            solve_result res{};
            const int rc = solver_poll(s, id[r], out.data(), &res);
            if (rc == NOPCS_EAGAIN) continue;
            state[r] = 2;
            ++done;
            if (rc != NOPCS_OK || res.steps_done != w[r].steps ||
                std::memcmp(out.data(), w[r].want.data(), out.size() * sizeof(double)) != 0) {
                std::fprintf(stderr, "request %d: status %d, steps %d of %d, or result differs\n", r, rc,
                             res.steps_done, w[r].steps);
                same = false;
            }
        }
        std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    SERVE_CHECK(same, "stress stream equals alone bit for bit");
    SERVE_CHECK(solver_destroy(s) == NOPCS_OK, "destroy (stress)");
    return 0;
}

int main(int argc, char **argv) {
    if (argc < 2) { std::fprintf(stderr, "usage\n"); return 2; }
    const std::string mode = argv[1];
    // NOPCS_EMUL_DERIV_FORM: the form of first derivatives alone (0 by size, 1 pencil, 2 line march)
    if (const char *e = std::getenv("NOPCS_EMUL_DERIV_FORM"))
        if (nopcs_set_deriv_form(std::atoi(e)) != NOPCS_OK) return 2;
    if (mode == "plan" && argc >= 5) {  // driver plan n nseg piece: line-march tables of one line plan
        nopcs::LinePlanHost P;
        std::string err;
        if (!nopcs::build_line_plan(std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]), P, err)) return 1;
        std::printf("nrun %zu ncl %zu max_m %d k1_S %d ngrp %zu\n", P.runs.size(), P.cl_row.size(), P.max_m, P.k1_S,
                    P.grp.size());
        return 0;
    }
    if (mode == "serve_stress" && argc >= 4) {   // driver serve_stress batched nrequests
        const int rc = serve_stress(std::atoi(argv[2]), std::atoi(argv[3]));
        nopcs_release_plans();
        return rc;
    }
    if (mode == "serve" || mode == "serve_batched") {
        const int rc = serve_checks(mode == "serve_batched");
        nopcs_release_plans();   // cached batch launches included
        return rc;
    }
    if (mode == "batch") {   // driver batch [modes, e.g. 2013]
        const char *pe = std::getenv("NOPCS_EMUL_PRECISION");
        return batch_checks(pe && std::atoi(pe) == 1 ? NOPCS_MIXED : NOPCS_FP64, argc > 2 ? argv[2] : "2013");
    }
    if (argc < 11) { std::fprintf(stderr, "usage\n"); return 2; }
    // NOPCS_EMUL_VISC_CHUNK: planes per z chunk of the viscous kernel (0 default)
    if (const char *vc = std::getenv("NOPCS_EMUL_VISC_CHUNK"))
        if (nopcs_set_visc_chunk(std::atoi(vc)) != NOPCS_OK) return 2;
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
    // NOPCS_EMUL_PRECISION=1: mixed precision for rhs and rk
    const char *pe = std::getenv("NOPCS_EMUL_PRECISION");
    const int prec = pe && std::atoi(pe) == 1 ? NOPCS_MIXED : NOPCS_FP64;
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
    } else if (mode == "deriv1") {
        // the first derivative alone (line march along y and z), then the same
        // through the pencil solve: both written, march first
        const int dir = std::atoi(argv[11]);
        std::vector<double> fh = read_raw(argv[12], N);
        Buf f(N), a(N), b(N);
        std::memcpy(f.p, fh.data(), N * sizeof(double));
        rc = nopcs_set_deriv_form(2);
        if (rc == 0) rc = nopcs_derivative(&g, dir, NOPCS_FP64, f.p, a.p, nullptr, nullptr);
        if (rc == 0) rc = nopcs_set_deriv_form(1);
        if (rc == 0) rc = nopcs_derivative(&g, dir, NOPCS_FP64, f.p, b.p, nullptr, nullptr);
        if (nopcs_set_deriv_form(3) != NOPCS_EINVAL) rc = 1;
        (void)nopcs_set_deriv_form(0);
        if (rc == 0) {
            std::vector<double> out(2 * N);
            std::memcpy(out.data(), a.p, N * sizeof(double));
            std::memcpy(out.data() + N, b.p, N * sizeof(double));
            write_raw(argv[13], out.data(), 2 * N);
        }
    } else if (mode == "rhs") {
        p.viscous = std::atoi(argv[11]);
        p.gravity = std::atoi(argv[12]);
        std::vector<double> Qh = read_raw(argv[13], 5 * N);
        Buf Q(5 * N), R(5 * N);
        std::memcpy(Q.p, Qh.data(), 5 * N * sizeof(double));
        const size_t wsb = nopcs_workspace_bytes(&g, prec);
        Buf ws((wsb + 7) / 8);
        rc = nse_rhs(&p, &g, prec, Q.p, R.p, ws.p, wsb, nullptr);
        if (rc == 0) write_raw(argv[14], R.p, 5 * N);
    } else if (mode == "rk") {
        p.viscous = std::atoi(argv[11]);
        p.gravity = std::atoi(argv[12]);
        const double dt = std::atof(argv[13]);
        const int nsteps = std::atoi(argv[14]);
        std::vector<double> Qh = read_raw(argv[15], 5 * N);
        Buf Q(5 * N);
        std::memcpy(Q.p, Qh.data(), 5 * N * sizeof(double));
        const size_t wsb = nopcs_workspace_bytes(&g, prec);
        Buf ws((wsb + 7) / 8);
        rc = rk_step(&p, &g, prec, Q.p, dt, nsteps, ws.p, wsb, nullptr);
        if (rc == 0) write_raw(argv[16], Q.p, 5 * N);
    } else if (mode == "cvisc") {
        p.viscous = std::atoi(argv[11]);
        p.gravity = std::atoi(argv[12]);
        std::vector<double> Qh = read_raw(argv[13], 5 * N);
        Buf Q(5 * N), R(5 * N);
        std::memcpy(Q.p, Qh.data(), 5 * N * sizeof(double));
        const size_t wsb = nopcs_compact_viscous_workspace_bytes(&g);
        Buf ws((wsb + 7) / 8);
        // argv[15] (optional): dt and steps "dt:n" -> rk_step_compact_viscous instead
        if (argc > 15) {
            const double dt = std::atof(argv[15]);
            const int nst = std::atoi(std::strchr(argv[15], ':') + 1);
            rc = rk_step_compact_viscous(&p, &g, Q.p, dt, nst, ws.p, wsb, nullptr);
            if (rc == 0) write_raw(argv[14], Q.p, 5 * N);
        } else {
            rc = nse_rhs_compact_viscous(&p, &g, Q.p, R.p, ws.p, wsb, nullptr);
            if (rc == 0) write_raw(argv[14], R.p, 5 * N);
        }
    } else if (mode == "filter") {   // driver filter ... af every dt nsteps in out: nopcs_filter (nsteps 0) or
                                     // rk_step_filtered
        p.viscous = 1;
        p.gravity = 1;
        const double af = std::atof(argv[11]);
        const int every = std::atoi(argv[12]);
        const double dt = std::atof(argv[13]);
        const int nsteps = std::atoi(argv[14]);
        std::vector<double> Qh = read_raw(argv[15], 5 * N);
        Buf Q(5 * N);
        std::memcpy(Q.p, Qh.data(), 5 * N * sizeof(double));
        if (nsteps == 0) {
            rc = nopcs_filter(&p, &g, af, Q.p, nullptr);
        } else {
            const size_t wsb = nopcs_workspace_bytes(&g, prec);
            Buf ws((wsb + 7) / 8);
            rc = rk_step_filtered(&p, &g, prec, Q.p, dt, nsteps, every, af, ws.p, wsb, nullptr);
        }
        if (rc == 0) write_raw(argv[16], Q.p, 5 * N);
    } else if (mode == "vort") {
        std::vector<double> Qh = read_raw(argv[11], 5 * N);
        Buf Q(5 * N), out(12 * N);
        std::memcpy(Q.p, Qh.data(), 5 * N * sizeof(double));
        const size_t wsb = nopcs_vorticity_workspace_bytes(&g);
        Buf ws((wsb + 7) / 8);
        rc = nopcs_vorticity_budget(&p, &g, Q.p, out.p, ws.p, wsb, nullptr);
        if (rc == 0) write_raw(argv[12], out.p, 12 * N);
    } else if (mode == "dpress") {   // disturbance pressure and the spectrum of its centre line along y
        std::vector<double> Qh = read_raw(argv[11], 5 * N), Q0h = read_raw(argv[12], 5 * N);
        Buf Q(5 * N), Q0(5 * N), dp(N);
        std::memcpy(Q.p, Qh.data(), 5 * N * sizeof(double));
        std::memcpy(Q0.p, Q0h.data(), 5 * N * sizeof(double));
        const int ny = g.n[1];
        Buf amp(ny / 2 + 1);
        rc = nopcs_disturbance_pressure(&p, &g, Q.p, Q0.p, dp.p, nullptr);
        const size_t c0 = ((size_t)(g.n[2] / 2) * ny) * g.n[0] + g.n[0] / 2;
        if (rc == 0) rc = nopcs_line_spectrum(dp.p + c0, ny, g.n[0], amp.p, nullptr);
        if (rc == 0) {
            write_raw(argv[13], dp.p, N);
            write_raw(argv[14], amp.p, ny / 2 + 1);
        }
    } else {
        return 2;
    }
    if (rc != 0) std::fprintf(stderr, "call failed: %d %s\n", rc, nopcs_last_error());
    nopcs_release_plans();
    return rc == 0 ? 0 : 1;
}
