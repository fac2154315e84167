// api.hip -- C ABI entry points of libnopcs (declared in include/nopcs.h).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "cvisc.hpp"
#include "diag.hpp"
#include "dmarch.hpp"

namespace nopcs {

// nopcs_set_deriv_form: how nopcs_derivative computes the first derivative
// alone along y or z (0: by the box size, 1: pencil solve, 2: line march)
static std::atomic<int> g_deriv_form{0};
// lines along the direction from which the line march is the faster form
// (512^3: 0.70 against 0.95 ms along y; 384^3, 147456 lines: 0.38 against
// 0.45; 256^3, 65536 lines: 0.16 against 0.10)
constexpr long long kDerivMarchLines = 1LL << 17;

// cached RK4 steps (graphs or direct batched launches) across devices; not
// part of the C ABI (the CPU build's checks of the step cache read it)
size_t graph_cache_entries();

namespace {
thread_local std::string g_err;
}
void set_error(const std::string &msg) { g_err = msg; }
const char *get_error() { return g_err.c_str(); }

// Length of the extra cuts inside each user segment.  Short lines keep a single
// run per segment (sequential Thomas order); long lines are cut so that a pencil
// has enough independent runs for its threads.  Overridable for tuning.
static std::atomic<int> g_piece_len[3] = {-1, -1, -1};

int piece_length(int dir, int n) {
    const int pl = g_piece_len[dir].load();
    if (pl >= 0) return pl;
    return n <= 64 ? 0 : 32;
}

static bool check_grid(const nopcs_grid *g) {
    if (!g) { set_error("grid is NULL"); return false; }
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 8 || g->n[d] > 1024) {
            set_error("grid n[" + std::to_string(d) + "] must be in [8, 1024], got " + std::to_string(g->n[d]));
            return false;
        }
        if (!(g->len[d] > 0.0) || !std::isfinite(g->len[d])) {
            set_error("grid len[" + std::to_string(d) + "] must be positive and finite");
            return false;
        }
        if (g->nseg[d] < 1 || g->n[d] < 4 * g->nseg[d]) {
            set_error("grid nseg[" + std::to_string(d) + "] must be >= 1 with segments of >= 4 points");
            return false;
        }
    }
    return true;
}

static bool check_params(const nse_params *p) {
    if (!p) { set_error("params is NULL"); return false; }
    const double v[] = {p->gamma, p->R_gas, p->g, p->L, p->T_s, p->rho_s, p->Pr, p->mu_ref, p->T_ref};
    for (double x : v)
        if (!(x > 0.0) || !std::isfinite(x)) {
            set_error("physical parameters must be positive and finite");
            return false;
        }
    if (!(p->gamma > 1.0)) { set_error("gamma must exceed 1"); return false; }
    if (!std::isfinite(p->S_suth) || !std::isfinite(p->mub_a) || !std::isfinite(p->mub_b)) {
        set_error("viscosity constants must be finite");
        return false;
    }
    return true;
}

static int get_plans(const nopcs_grid *g, LinePlanDev pl[3], bool lookup_only = false) {
    for (int d = 0; d < 3; ++d) {
        const int rc = get_line_plan(g->n[d], g->nseg[d], piece_length(d, g->n[d]), g->len[d], &pl[d], lookup_only);
        if (rc != NOPCS_OK) return rc;
        if (4 + pl[d].ncl > sweep_known_rows_max(g->n[d])) {
            set_error("too many segments along direction " + std::to_string(d) + " for " +
                      std::to_string(g->n[d]) + " points");
            return NOPCS_EINVAL;
        }
    }
    return NOPCS_OK;
}

static size_t field_elems(const nopcs_grid *g) { return (size_t)g->n[0] * g->n[1] * g->n[2]; }
// Stride of the scratch fields of the vorticity budget (u, v, w, p' and 15
// gradients) and of the D1-based viscous variant: each field is padded to a
// multiple of 32 doubles so that every field starts 256-byte aligned.
static long long field_stride(const nopcs_grid *g) { return ((long long)field_elems(g) + 31) / 32 * 32; }

// ---------------------------------------------------------------------------
// Event timing of kernel launches (instrumentation only).
// ---------------------------------------------------------------------------
namespace {
struct TimingRec {
    int id;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimingRec> g_recs;
double g_total_ms[NOPCS_K_COUNT];
long long g_launches[NOPCS_K_COUNT];

int drain_timing() {
    for (auto &r : g_recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            set_error("timing event query failed");
            return NOPCS_EDEVICE;
        }
        g_total_ms[r.id] += ms;
        g_launches[r.id] += 1;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_recs.clear();
    return NOPCS_OK;
}
}  // namespace

// Launch through f() bracketed by events when timing is on.
static thread_local bool t_capturing = false;   // inside a graph capture: no event records

template <class F>
static hipError_t timed_impl(int id, hipStream_t st, F &&f);

static thread_local bool t_no_alloc = false;    // inside nse_rhs_noalloc: no event objects either

template <class F>
static hipError_t timed(int id, hipStream_t st, F &&f) {
    if (t_capturing || t_no_alloc) return f();
    return timed_impl(id, st, std::forward<F>(f));
}

// launches collected into a batch are not timed one by one
template <class F>
static hipError_t timed(int id, hipStream_t st, const BatchCollector *col, F &&f) {
    if (col) return f();
    return timed(id, st, std::forward<F>(f));
}

template <class F>
static hipError_t timed_impl(int id, hipStream_t st, F &&f) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        on = g_timing;
    }
    if (!on) return f();
    TimingRec r{id, nullptr, nullptr};
    hipError_t e = hipEventCreate(&r.a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&r.b);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(r.a, st)) != hipSuccess) return e;
    if ((e = f()) != hipSuccess) return e;
    if ((e = hipEventRecord(r.b, st)) != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_tmu);
    g_recs.push_back(r);
    return hipSuccess;
}

// How a call computes first derivatives alone: along y and z the closure pass
// and line march where the form setting and the box size choose it and the
// plan allows (never inside a graph capture or the allocation-free entry
// point: the march takes stream-ordered scratch), the LDS pencil solve
// otherwise.  The scratch holds the closure values of the largest marching
// direction and is released on the stream when the object goes.
struct D1Forms {
    bool march[3] = {false, false, false};
    double *clo = nullptr;
    hipStream_t st = nullptr;
    D1Forms(const nopcs_grid *grid, const LinePlanDev pl[3], hipStream_t s) : st(s) {
        const int form = g_deriv_form.load();
        if (t_capturing || t_no_alloc) return;
        for (int d = 1; d < 3; ++d) {
            const long long lines = (long long)field_elems(grid) / grid->n[d];
            march[d] = (form == 2 || (form == 0 && lines >= kDerivMarchLines)) && dmarch_usable(d, pl[d]);
        }
    }
    D1Forms(const D1Forms &) = delete;
    D1Forms &operator=(const D1Forms &) = delete;
    ~D1Forms() {
        if (clo) (void)hipFreeAsync(clo, st);
    }
    // scratch for the marching directions (only: one direction, -1: both)
    hipError_t alloc(const nopcs_grid *grid, const LinePlanDev pl[3], int only = -1) {
        size_t b = 0;
        for (int d = 1; d < 3; ++d)
            if (march[d] && (only < 0 || only == d)) b = std::max(b, dmarch_closure_bytes(grid->n, d, pl[d]));
        return b ? hipMallocAsync(reinterpret_cast<void **>(&clo), b, st) : hipSuccess;
    }
    hipError_t launch(int d, const double *f, double *d1, const nopcs_grid *grid, const LinePlanDev pl[3]) const {
        if (march[d]) return launch_dmarch(d, f, d1, clo, grid->n, pl[d], st);
        return launch_deriv(d, f, d1, nullptr, sweep_geom(grid->n, d), pl[d], st);
    }
};

}  // namespace nopcs

using namespace nopcs;

// one 5-field FP64 state, 256-byte aligned
static size_t state_bytes(const nopcs_grid *grid) {
    return ((5 * field_elems(grid) * sizeof(double)) + 255) & ~(size_t)255;
}

// closure array of the line-march sweeps along y and z (one is live at a time)
static size_t closure_bytes(const nopcs_grid *grid) {
    size_t most = 0;
    for (int d = 1; d <= 2; ++d) {
        const std::vector<uint8_t> kind = row_kinds(grid->n[d], grid->nseg[d], piece_length(d, grid->n[d]));
        int ncl = 0;
        for (uint8_t k : kind) ncl += k == ROW_CLOSURE;
        most = std::max(most, march_closure_elems(grid->n, d, ncl));
    }
    return ((most * sizeof(double)) + 255) & ~(size_t)255;
}

// convective sweep along d: line march (y, z) when the plan allows, LDS pencils
// otherwise.  c32: the march eliminates in FP32 (mixed precision).
// Phases of a batched RK4 step (the launches of one stage, in order; see
// batch.hpp): launches of different boxes in one phase are independent.
enum : int { PH_VISC = 0, PH_X = 1, PH_Y_CLOSURE = 2, PH_Y = 3, PH_Z_CLOSURE = 4, PH_Z = 5, PH_RK = 6, PH_WALL = 7,
             PH_PER_STAGE = 16 };

static int conv_sweep(int d, const NseSweepArgs &a, const nopcs_grid *grid, const LinePlanDev &pl, double *clo,
                      bool c32, hipStream_t st, const RkFuse *rk = nullptr, BatchCollector *col = nullptr,
                      int phase0 = 0) {
    const int ph_closure = phase0 + (d == 1 ? PH_Y_CLOSURE : PH_Z_CLOSURE);
    const int ph_runs = phase0 + (d == 0 ? PH_X : d == 1 ? PH_Y : PH_Z);
    if (clo && march_usable(d, pl)) {
        NOPCS_HIP_CHECK(timed(NOPCS_K_CLOSURE_Y + (d - 1), st, col, [&] {
            return launch_march_closures(d, a.Qin, clo, grid->n, pl, a.c, st, col, ph_closure);
        }));
        NOPCS_HIP_CHECK(timed(NOPCS_K_SWEEP_X + d, st, col, [&] {
            return launch_march_runs(d, a.Qin, a.R, a.r32, c32, clo, grid->n, pl, a.c, st, rk, col, ph_runs);
        }));
        return NOPCS_OK;
    }
    if (rk) {
        set_error("internal: fused RK update requested on a sweep without the line march");
        return NOPCS_EINVAL;
    }
    NOPCS_HIP_CHECK(timed(NOPCS_K_SWEEP_X + d, st, col,
                          [&] { return launch_nse_sweep(d, a, sweep_geom(grid->n, d), pl, st, col, ph_runs); }));
    return NOPCS_OK;
}

// One classical RK4 step (Section 4): per stage the viscous terms and source,
// the three convective sweeps, the register update and the wall conditions.
// Viscous terms and gravity source by the compact first derivative (the
// D1-based variant) into R, FP64: point-wise u, v, w, T into X, their 12
// gradients, the 12 flux components, the 12 flux derivatives along their own
// directions, then the divergence plus source.  X: 28 fields of
// field_stride(grid) doubles.  Without viscous terms: the source alone, as in
// the explicit path.
static int compact_visc_into(const NdConst &c, const nopcs_grid *grid, const LinePlanDev pl[3], const double *Q,
                             double *R, double *X, hipStream_t st) {
    if (!c.viscous) {
        double ih[3];
        for (int d = 0; d < 3; ++d) ih[d] = (double)(grid->n[d] - 1) / grid->len[d];
        NOPCS_HIP_CHECK(timed(NOPCS_K_VISCOUS, st, [&] { return launch_visc(Q, R, false, grid->n, ih, c, st); }));
        return NOPCS_OK;
    }
    const long long N = (long long)field_elems(grid), S = field_stride(grid);
    double *P = X, *G = X + 4 * S, *F = X + 16 * S;
    D1Forms fm(grid, pl, st);
    NOPCS_HIP_CHECK(fm.alloc(grid, pl));
    NOPCS_HIP_CHECK(timed(NOPCS_K_VISCOUS, st, [&] { return launch_cv_prims(Q, N, S, c, P, st); }));
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) {
            double *dst = G + (3 * a + d) * S;
            const double *src = P + a * S;
            NOPCS_HIP_CHECK(timed(NOPCS_K_DERIV, st, [&] { return fm.launch(d, src, dst, grid, pl); }));
        }
    NOPCS_HIP_CHECK(timed(NOPCS_K_VISCOUS, st, [&] { return launch_cv_flux(P, G, N, S, c, F, st); }));
    // D_d of flux component 4d + q into the gradient slots
    for (int d = 0; d < 3; ++d)
        for (int q = 0; q < 4; ++q) {
            double *dst = G + (4 * d + q) * S;
            const double *src = F + (4 * d + q) * S;
            NOPCS_HIP_CHECK(timed(NOPCS_K_DERIV, st, [&] { return fm.launch(d, src, dst, grid, pl); }));
        }
    NOPCS_HIP_CHECK(timed(NOPCS_K_VISCOUS, st, [&] { return launch_cv_assemble(Q, G, N, S, c, R, st); }));
    return NOPCS_OK;
}

static int launch_step(const nse_params &params, const nopcs_grid *grid, int precision, double *Q, double dt, void *ws,
                       const LinePlanDev pl[3], hipStream_t st, double *cvx = nullptr,
                       BatchCollector *col = nullptr) {
    const NdConst c = make_nd(params);
    const size_t N = field_elems(grid);
    const size_t reg = state_bytes(grid);
    double *K = reinterpret_cast<double *>(ws);
    double *Qs = reinterpret_cast<double *>(static_cast<char *>(ws) + reg);
    void *R = static_cast<char *>(ws) + 2 * reg;   // FP64, or FP32 in mixed precision
    double *clo = reinterpret_cast<double *>(static_cast<char *>(ws) + 3 * reg);
    const bool mixed = precision == NOPCS_MIXED;
    double ih[3];
    for (int d = 0; d < 3; ++d) ih[d] = (double)(grid->n[d] - 1) / grid->len[d];
    NseSweepArgs a{};
    a.R = R;
    a.r32 = mixed;
    a.Qn = Q;
    a.K = K;
    a.Qs = Qs;
    a.N3 = (long long)N;
    a.c = c;
    a.dt = dt;
    a.half_dt = 0.5 * dt;
    a.sixth_dt = dt / 6.0;
    // With the z line march the stage update rides on the z sweep (RkFuse),
    // which must not write the state it reads.  FP64: the next stage state goes
    // over R, and the two FP64 registers (Qs, R) swap roles every stage.  Mixed
    // precision (FP32 R): the next stage state alternates between Qs and a
    // second FP64 stage register.
    const bool fuse = march_usable(2, pl[2]);
    double *Qs2 = reinterpret_cast<double *>(static_cast<char *>(ws) + 3 * reg + closure_bytes(grid));
    double *B[2] = {Qs, mixed ? Qs2 : static_cast<double *>(R)};
    for (int stage = 0; stage < 4; ++stage) {
        // FP64: R in B[(s + 1) % 2], input B[s % 2]; mixed: R fixed, input
        // B[(s + 1) % 2], output B[s % 2]
        void *Rs = fuse && !mixed ? static_cast<void *>(B[(stage + 1) & 1]) : R;
        double *Sout = !fuse ? Qs : mixed ? B[stage & 1] : B[(stage + 1) & 1];
        const double *Qin = stage == 0 ? Q : !fuse ? Qs : mixed ? B[(stage + 1) & 1] : B[stage & 1];
        a.Qin = Qin;
        a.R = Rs;
        a.stage = stage;
        const int ph = stage * PH_PER_STAGE;   // phases of this stage in a batched step
        if (cvx) {   // D1-based viscous variant (FP64 only; never batched)
            if (col) {
                set_error("internal: the D1-based viscous variant is not batched");
                return NOPCS_EINVAL;
            }
            const int rc = compact_visc_into(c, grid, pl, Qin, static_cast<double *>(Rs), cvx, st);
            if (rc != NOPCS_OK) return rc;
        } else {
            NOPCS_HIP_CHECK(timed(NOPCS_K_VISCOUS, st, col,
                                  [&] { return launch_visc(Qin, Rs, mixed, grid->n, ih, c, st, col, ph + PH_VISC); }));
        }
        if (fuse) {
            const RkFuse F{K, Q, Sout, stage, dt, 0.5 * dt, dt / 6.0};
            for (int d = 0; d < 3; ++d) {
                const int rc = conv_sweep(d, a, grid, pl[d], clo, mixed, st, d == 2 ? &F : nullptr, col, ph);
                if (rc != NOPCS_OK) return rc;
            }
        } else {
            for (int d = 0; d < 3; ++d) {
                const int rc = conv_sweep(d, a, grid, pl[d], clo, mixed, st, nullptr, col, ph);
                if (rc != NOPCS_OK) return rc;
            }
            NOPCS_HIP_CHECK(timed(NOPCS_K_RK, st, col, [&] { return launch_rk_update(a, st, col, ph + PH_RK); }));
        }
        double *Qout = stage == 3 ? Q : Sout;
        for (int d = 0; d < 3; ++d)
            NOPCS_HIP_CHECK(timed(NOPCS_K_WALL, st, col,
                                  [&] { return launch_bc(Qout, grid->n, d, c, st, col, ph + PH_WALL + d); }));
    }
    return NOPCS_OK;
}

// ---------------------------------------------------------------------------
// HIP graphs of one RK4 step: captured once per (device, state, workspace, box,
// parameters, precision, dt, piece lengths) on a private stream and replayed on
// the caller's stream.  Kernel timing is not recorded inside graphs.
// ---------------------------------------------------------------------------
static std::atomic<int> g_graphs{0};
namespace {
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;   // recorded after the entry's latest replay
    void *tables = nullptr;      // device tables of a batched step (owned)
    std::vector<BatchLaunch> launches;   // a batched step launched directly (no graph)
    uint64_t last_use = 0;               // g_graph_clock at the latest replay
};
std::mutex g_gmu;
std::map<std::string, GraphEntry> g_graph_cache;
std::map<int, hipStream_t> g_capture_stream;
// branch streams and fork/join events of batched steps, per device
std::map<int, std::vector<hipStream_t>> g_branch_streams;
std::map<int, std::vector<hipEvent_t>> g_branch_events;
std::atomic<int> g_max_graphs{64};   // entries the cache holds (nopcs_set_graph_cache_limit)
uint64_t g_graph_clock = 0;          // use counter for least-recently-used eviction (under g_gmu)

template <class T>
void put_bytes(std::string &k, const T &v) {
    k.append(reinterpret_cast<const char *>(&v), sizeof v);
}
// the grid field by field: its padding bytes (after n and nseg) are whatever
// the caller's memory held and must not make equal grids differ
void put_grid(std::string &k, const nopcs_grid &g) {
    for (int d = 0; d < 3; ++d) {
        put_bytes(k, g.n[d]);
        put_bytes(k, g.len[d]);
        put_bytes(k, g.nseg[d]);
    }
}

// Destroy an entry once its replays have run (the executable may still be
// queued on a caller's stream).
void drop_graph(GraphEntry &e) {
    if (e.done) {
        (void)hipEventSynchronize(e.done);
        (void)hipEventDestroy(e.done);
    }
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    if (e.tables) (void)hipFree(e.tables);
    e.exec = nullptr;
    e.graph = nullptr;
    e.done = nullptr;
    e.tables = nullptr;
}

// Replay a cached executable nsteps times on st and record its completion
// event; the caller holds g_gmu, so no other thread can evict the entry
// between the lookup and the launches.
int replay(GraphEntry &e, int nsteps, hipStream_t st) {
    e.last_use = ++g_graph_clock;
    for (int step = 0; step < nsteps; ++step) {
        if (e.exec) {
            NOPCS_HIP_CHECK(hipGraphLaunch(e.exec, st));
        } else {
            for (const BatchLaunch &L : e.launches)
                NOPCS_HIP_CHECK(L.launch(static_cast<char *>(e.tables) + L.dev_off, L.ntab, L.total, L.blk, st));
        }
    }
    NOPCS_HIP_CHECK(hipEventRecord(e.done, st));
    return NOPCS_OK;
}

// Make room for `room` more entries: the least recently used go (each after
// its replays have run).
void evict_if_full(size_t room = 1) {
    const size_t cap = (size_t)g_max_graphs.load();
    while (!g_graph_cache.empty() && g_graph_cache.size() + room > cap) {
        auto lru = g_graph_cache.begin();
        for (auto it = g_graph_cache.begin(); it != g_graph_cache.end(); ++it)
            if (it->second.last_use < lru->second.last_use) lru = it;
        drop_graph(lru->second);
        g_graph_cache.erase(lru);
    }
}

// Instantiate a captured graph into an entry with its completion event.
int instantiate(GraphEntry &e) {
    if (hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(e.graph);
        e.graph = nullptr;
        set_error("hipGraphInstantiate failed");
        return NOPCS_EDEVICE;
    }
    if (hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGraphExecDestroy(e.exec);
        (void)hipGraphDestroy(e.graph);
        e.exec = nullptr;
        e.graph = nullptr;
        set_error("hipEventCreateWithFlags failed");
        return NOPCS_EDEVICE;
    }
    return NOPCS_OK;
}
}  // namespace

size_t nopcs::graph_cache_entries() {
    std::lock_guard<std::mutex> lk(g_gmu);
    return g_graph_cache.size();
}

static void release_graphs() {
    std::lock_guard<std::mutex> lk(g_gmu);
    for (auto &kv : g_graph_cache) drop_graph(kv.second);
    g_graph_cache.clear();
    for (auto &kv : g_branch_streams)
        for (hipStream_t x : kv.second) (void)hipStreamDestroy(x);
    for (auto &kv : g_branch_events)
        for (hipEvent_t x : kv.second) (void)hipEventDestroy(x);
    for (auto &kv : g_capture_stream)
        if (kv.second) (void)hipStreamDestroy(kv.second);
    g_branch_streams.clear();
    g_branch_events.clear();
    g_capture_stream.clear();
}

static int step_graph(const nse_params &params, const nopcs_grid *grid, int precision, double *Q, double dt, void *ws,
                      const LinePlanDev pl[3], int nsteps, hipStream_t st) {
    int dev = 0;
    NOPCS_HIP_CHECK(hipGetDevice(&dev));
    std::string key;
    put_bytes(key, dev);
    put_bytes(key, Q);
    put_bytes(key, ws);
    put_grid(key, *grid);
    put_bytes(key, params);
    put_bytes(key, precision);
    put_bytes(key, dt);
    for (int d = 0; d < 3; ++d) put_bytes(key, piece_length(d, grid->n[d]));
    put_bytes(key, visc_z_chunk(grid->n));
    std::lock_guard<std::mutex> lk(g_gmu);
    auto it = g_graph_cache.find(key);
    if (it != g_graph_cache.end()) return replay(it->second, nsteps, st);
    evict_if_full();
    hipStream_t &cs = g_capture_stream[dev];
    if (!cs) NOPCS_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    GraphEntry e;
    NOPCS_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    t_capturing = true;
    const int rc = launch_step(params, grid, precision, Q, dt, ws, pl, cs);
    t_capturing = false;
    const hipError_t ec = hipStreamEndCapture(cs, &e.graph);
    if (rc != NOPCS_OK) {
        if (e.graph) (void)hipGraphDestroy(e.graph);
        return rc;
    }
    NOPCS_HIP_CHECK(ec);
    const int ri = instantiate(e);
    if (ri != NOPCS_OK) return ri;
    return replay(g_graph_cache[key] = e, nsteps, st);
}

extern "C" {

const char *nopcs_last_error(void) { return get_error(); }

int nopcs_version(void) { return 100; }

int nopcs_release_plans(void) {
    release_graphs();   // graphs reference plan memory
    release_line_plans();
    return NOPCS_OK;
}

size_t nopcs_workspace_bytes(const nopcs_grid *grid, int precision) {
    if (!check_grid(grid) || (precision != NOPCS_FP64 && precision != NOPCS_MIXED)) return 0;
    // mixed precision: a second FP64 stage register after the closure array
    // (the z sweep that carries the RK4 update writes the next stage state there)
    return (precision == NOPCS_MIXED ? 4 : 3) * state_bytes(grid) + closure_bytes(grid);
}

int nopcs_line_plan(int32_t n, int32_t nseg, int32_t piece_len, int32_t cap, int32_t *nrun, int32_t *runs,
                    int32_t *ncl, int32_t *rows, double *coef) {
    if (piece_len < -1) { set_error("piece_len must be >= -1"); return NOPCS_EINVAL; }
    LinePlanHost P;
    std::string err;
    const int len = piece_len == -1 ? piece_length(1, n) : piece_len;
    if (!build_line_plan(n, nseg, len, P, err)) { set_error(err); return NOPCS_EINVAL; }
    const int nr = (int)P.runs.size(), nc = (int)P.cl_row.size();
    if (nrun) *nrun = nr;
    if (ncl) *ncl = nc;
    if ((runs && nr > cap) || ((rows || coef) && nc > cap)) { set_error("cap too small"); return NOPCS_ENOMEM; }
    if (runs)
        for (int r = 0; r < nr; ++r) { runs[2 * r] = P.runs[r].x; runs[2 * r + 1] = P.runs[r].y; }
    if (rows)
        for (int q = 0; q < nc; ++q) rows[q] = P.cl_row[q];
    if (coef)
        for (int q = 0; q < nc; ++q) {
            const int e = P.cl_row[q];
            for (int t = 0; t < kTaps; ++t) {
                const int j = e - kNb + t;
                coef[(size_t)q * kTaps + t] =
                    (j < P.cl_j0[q] || j >= P.cl_j0[q] + P.cl_len[q]) ? 0.0 : P.cl_coef[(size_t)q * kTaps + (j - P.cl_j0[q])];
            }
        }
    return NOPCS_OK;
}

int nopcs_set_deriv_form(int32_t form) {
    if (form < 0 || form > 2) { set_error("derivative form must be 0 (by size), 1 (pencil) or 2 (line march)"); return NOPCS_EINVAL; }
    g_deriv_form.store(form);
    return NOPCS_OK;
}

int nopcs_derivative(const nopcs_grid *grid, int dir, int precision, const double *f, double *d1, double *d2,
                     void *hip_stream) {
    if (!check_grid(grid)) return NOPCS_EINVAL;
    if (dir < 0 || dir > 2) { set_error("dir must be 0, 1 or 2"); return NOPCS_EINVAL; }
    if (precision != NOPCS_FP64) { set_error("nopcs_derivative: only NOPCS_FP64 is implemented"); return NOPCS_EINVAL; }
    if (!f || (!d1 && !d2)) { set_error("f and at least one of d1, d2 must be non-NULL"); return NOPCS_EINVAL; }
    LinePlanDev pl[3];
    int rc = get_plans(grid, pl);
    if (rc != NOPCS_OK) return rc;
    const hipStream_t st = (hipStream_t)hip_stream;
    if (d1 && !d2) {
        // the first derivative alone: the line march along y or z where it is chosen
        D1Forms fm(grid, pl, st);
        if (fm.march[dir]) {
            NOPCS_HIP_CHECK(fm.alloc(grid, pl, dir));
            NOPCS_HIP_CHECK(timed(NOPCS_K_DERIV, st, [&] { return fm.launch(dir, f, d1, grid, pl); }));
            return NOPCS_OK;
        }
    }
    const SweepGeom g = sweep_geom(grid->n, dir);
    NOPCS_HIP_CHECK(timed(NOPCS_K_DERIV, st, [&] { return launch_deriv(dir, f, d1, d2, g, pl[dir], st); }));
    return NOPCS_OK;
}


size_t nopcs_vorticity_workspace_bytes(const nopcs_grid *grid) {
    if (!check_grid(grid)) return 0;
    return (size_t)19 * (size_t)field_stride(grid) * sizeof(double);
}

int nopcs_vorticity_budget(const nse_params *params, const nopcs_grid *grid, const double *Q, double *out, void *ws,
                           size_t ws_bytes, void *hip_stream) {
    if (!check_grid(grid) || !check_params(params)) return NOPCS_EINVAL;
    if (!Q || !out) { set_error("Q and out must be non-NULL"); return NOPCS_EINVAL; }
    const size_t need = nopcs_vorticity_workspace_bytes(grid);
    if (!ws || ws_bytes < need) {
        set_error("vorticity workspace too small: need " + std::to_string(need) + " bytes");
        return NOPCS_EINVAL;
    }
    if (((uintptr_t)ws & 255) != 0) { set_error("workspace must be 256-byte aligned"); return NOPCS_EINVAL; }
    LinePlanDev pl[3];
    int rc = get_plans(grid, pl);
    if (rc != NOPCS_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const long long N = (long long)field_elems(grid), S = field_stride(grid);
    double *P = static_cast<double *>(ws), *G = P + 4 * S;
    NOPCS_HIP_CHECK(timed(NOPCS_K_VORT, st, [&] { return launch_vort_prims(Q, N, S, params->gamma - 1.0, P, st); }));
    // gradients of u, v, w (from P), rho (field 0 of Q) and p' (P field 3)
    const double *src[5] = {P, P + S, P + 2 * S, Q, P + 3 * S};
    D1Forms fm(grid, pl, st);
    NOPCS_HIP_CHECK(fm.alloc(grid, pl));
    for (int a = 0; a < 5; ++a)
        for (int d = 0; d < 3; ++d) {
            double *dst = G + (3 * a + d) * S;
            NOPCS_HIP_CHECK(timed(NOPCS_K_DERIV, st, [&] { return fm.launch(d, src[a], dst, grid, pl); }));
        }
    NOPCS_HIP_CHECK(timed(NOPCS_K_VORT, st, [&] { return launch_vort_combine(Q, G, N, S, out, st); }));
    return NOPCS_OK;
}

int nopcs_disturbance_pressure(const nse_params *params, const nopcs_grid *grid, const double *Q, const double *Q0,
                               double *out, void *hip_stream) {
    if (!check_grid(grid) || !check_params(params)) return NOPCS_EINVAL;
    if (!Q || !Q0 || !out) { set_error("Q, Q0 and out must be non-NULL"); return NOPCS_EINVAL; }
    const long long N = (long long)field_elems(grid);
    NOPCS_HIP_CHECK(timed(NOPCS_K_VORT, (hipStream_t)hip_stream, [&] {
        return launch_disturbance_pressure(Q, Q0, N, params->gamma - 1.0, out, (hipStream_t)hip_stream);
    }));
    return NOPCS_OK;
}

int nopcs_line_spectrum(const double *f, int32_t n, int64_t stride, double *amp, void *hip_stream) {
    if (!f || !amp) { set_error("f and amp must be non-NULL"); return NOPCS_EINVAL; }
    if (n < 2 || n > 16384) { set_error("line length must be in [2, 16384]"); return NOPCS_EINVAL; }
    if (stride < 1) { set_error("stride must be >= 1"); return NOPCS_EINVAL; }
    NOPCS_HIP_CHECK(timed(NOPCS_K_VORT, (hipStream_t)hip_stream,
                          [&] { return launch_line_spectrum(f, n, stride, amp, (hipStream_t)hip_stream); }));
    return NOPCS_OK;
}

static int rhs_into(const NdConst &c, const nopcs_grid *grid, const LinePlanDev pl[3], const double *Q, double *R,
                    double *clo, bool c32, hipStream_t st) {
    double ih[3];
    for (int d = 0; d < 3; ++d) ih[d] = (double)(grid->n[d] - 1) / grid->len[d];
    NOPCS_HIP_CHECK(timed(NOPCS_K_VISCOUS, st, [&] { return launch_visc(Q, R, false, grid->n, ih, c, st); }));
    NseSweepArgs a{};
    a.Qin = Q;
    a.R = R;
    a.r32 = false;
    a.N3 = (long long)field_elems(grid);
    a.c = c;
    for (int d = 0; d < 3; ++d) {
        const int rc = conv_sweep(d, a, grid, pl[d], clo, c32, st);
        if (rc != NOPCS_OK) return rc;
    }
    return NOPCS_OK;
}

// Workspace of the D1-based viscous variant: the right-hand side's own
// workspace, then u, v, w, T, 12 gradients (later the 12 flux derivatives)
// and 12 flux components, each field padded as in the vorticity budget.
size_t nopcs_compact_viscous_workspace_bytes(const nopcs_grid *grid) {
    if (!check_grid(grid)) return 0;
    return nopcs_workspace_bytes(grid, NOPCS_FP64) + (size_t)28 * (size_t)field_stride(grid) * sizeof(double);
}

int nse_rhs_compact_viscous(const nse_params *params, const nopcs_grid *grid, const double *Q, double *R, void *ws,
                            size_t ws_bytes, void *hip_stream) {
    if (!check_grid(grid) || !check_params(params)) return NOPCS_EINVAL;
    if (!Q || !R) { set_error("Q and R must be non-NULL"); return NOPCS_EINVAL; }
    const size_t need = nopcs_compact_viscous_workspace_bytes(grid);
    if (!ws || ws_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return NOPCS_EINVAL;
    }
    if (((uintptr_t)ws & 255) != 0) { set_error("workspace must be 256-byte aligned"); return NOPCS_EINVAL; }
    LinePlanDev pl[3];
    int rc = get_plans(grid, pl);
    if (rc != NOPCS_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const NdConst c = make_nd(*params);
    double *clo = reinterpret_cast<double *>(static_cast<char *>(ws) + 3 * state_bytes(grid));
    double *X = reinterpret_cast<double *>(static_cast<char *>(ws) + nopcs_workspace_bytes(grid, NOPCS_FP64));
    rc = compact_visc_into(c, grid, pl, Q, R, X, st);
    if (rc != NOPCS_OK) return rc;
    NseSweepArgs a{};
    a.Qin = Q;
    a.R = R;
    a.r32 = false;
    a.N3 = (long long)field_elems(grid);
    a.c = c;
    for (int d = 0; d < 3; ++d) {
        rc = conv_sweep(d, a, grid, pl[d], clo, false, st);
        if (rc != NOPCS_OK) return rc;
    }
    return NOPCS_OK;
}

// checks of a caller-provided workspace
static bool check_ws(const nopcs_grid *grid, int precision, const void *ws, size_t ws_bytes) {
    const size_t need = nopcs_workspace_bytes(grid, precision);
    if (!ws || ws_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return false;
    }
    if (((uintptr_t)ws & 255) != 0) {
        set_error("workspace must be 256-byte aligned");
        return false;
    }
    return true;
}

int nse_rhs(const nse_params *params, const nopcs_grid *grid, int precision, const double *Q, double *R, void *ws,
            size_t ws_bytes, void *hip_stream) {
    if (!check_grid(grid) || !check_params(params)) return NOPCS_EINVAL;
    if (precision != NOPCS_FP64 && precision != NOPCS_MIXED) { set_error("unknown precision"); return NOPCS_EINVAL; }
    if (!Q || !R) { set_error("Q and R must be non-NULL"); return NOPCS_EINVAL; }
    if (!check_ws(grid, precision, ws, ws_bytes)) return NOPCS_EINVAL;
    LinePlanDev pl[3];
    int rc = get_plans(grid, pl);
    if (rc != NOPCS_OK) return rc;
    double *clo = reinterpret_cast<double *>(static_cast<char *>(ws) + 3 * state_bytes(grid));
    return rhs_into(make_nd(*params), grid, pl, Q, R, clo, precision == NOPCS_MIXED, (hipStream_t)hip_stream);
}

// ---------------------------------------------------------------------------
// nse_rhs without allocation: the closure array of the y and z line marches
// (the only workspace nse_rhs uses) lives in a static device array of fixed
// size instead of the caller's workspace.  Each device holds its own copy of
// the array at its own address, looked up once per device with
// hipGetSymbolAddress; host code never passes the array's name to a kernel.
// ---------------------------------------------------------------------------
static constexpr size_t kNoAllocScratchBytes = (size_t)NOPCS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device (null: not looked up yet)

// address of this device's `scratch`, looked up on the first call on the device
int scratch_address(void **out) {
    int dev = 0;
    NOPCS_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal out of range for the static scratch array");
        return NOPCS_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        NOPCS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress gave no address for the scratch array");
            return NOPCS_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NOPCS_OK;
}
}  // namespace

extern "C" int nse_rhs_noalloc(const nse_params *params, const nopcs_grid *grid, int precision, const double *Q,
                               double *R, void *hip_stream) {
    if (!check_grid(grid) || !check_params(params)) return NOPCS_EINVAL;
    if (precision != NOPCS_FP64 && precision != NOPCS_MIXED) { set_error("unknown precision"); return NOPCS_EINVAL; }
    if (!Q || !R) { set_error("Q and R must be non-NULL"); return NOPCS_EINVAL; }
    LinePlanDev pl[3];
    int rc = get_plans(grid, pl, /*lookup_only=*/true);
    if (rc != NOPCS_OK) return rc;
    // the closure array of the larger of the y and z sweeps (as in nse_rhs's workspace)
    size_t need = 0;
    for (int d = 1; d <= 2; ++d) need = std::max(need, march_closure_elems(grid->n, d, pl[d].ncl) * sizeof(double));
    if (need > kNoAllocScratchBytes) {
        set_error("nse_rhs_noalloc: this grid needs " + std::to_string(need) + " bytes of scratch, more than the " +
                  std::to_string(kNoAllocScratchBytes) + " of the static array");
        return NOPCS_EINVAL;
    }
    void *clo = nullptr;
    rc = scratch_address(&clo);
    if (rc != NOPCS_OK) return rc;
    // every closure value is written by the closure pass before the run march
    // reads it: nothing in the array needs clearing
    t_no_alloc = true;
    rc = rhs_into(make_nd(*params), grid, pl, Q, R, static_cast<double *>(clo), precision == NOPCS_MIXED,
                  (hipStream_t)hip_stream);
    t_no_alloc = false;
    return rc;
}

int rk_step(const nse_params *params, const nopcs_grid *grid, int precision, double *Q, double dt, int32_t nsteps,
            void *ws, size_t ws_bytes, void *hip_stream) {
    if (!check_grid(grid) || !check_params(params)) return NOPCS_EINVAL;
    if (precision != NOPCS_FP64 && precision != NOPCS_MIXED) { set_error("unknown precision"); return NOPCS_EINVAL; }
    if (!Q) { set_error("Q must be non-NULL"); return NOPCS_EINVAL; }
    if (((uintptr_t)Q & 15) != 0) { set_error("Q must be 16-byte aligned"); return NOPCS_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error("dt must be positive and finite"); return NOPCS_EINVAL; }
    if (nsteps < 0) { set_error("nsteps must be >= 0"); return NOPCS_EINVAL; }
    if (!check_ws(grid, precision, ws, ws_bytes)) return NOPCS_EINVAL;
    LinePlanDev pl[3];
    int rc = get_plans(grid, pl);
    if (rc != NOPCS_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if (nsteps == 0) return NOPCS_OK;
    if (!g_graphs.load()) {
        for (int step = 0; step < nsteps; ++step) {
            rc = launch_step(*params, grid, precision, Q, dt, ws, pl, st);
            if (rc != NOPCS_OK) return rc;
        }
        return NOPCS_OK;
    }
    return step_graph(*params, grid, precision, Q, dt, ws, pl, nsteps, st);
}

// Filter plans of a grid (the derivative's segments and pieces, the filter's
// closure rows and elimination tables).
static int get_filter_plans(const nopcs_grid *g, double af, LinePlanDev pl[3]) {
    for (int d = 0; d < 3; ++d) {
        const int rc = get_line_plan(g->n[d], g->nseg[d], piece_length(d, g->n[d]), g->len[d], &pl[d], false,
                                     OP_FILTER, af);
        if (rc != NOPCS_OK) return rc;
        if (4 + pl[d].ncl > sweep_known_rows_max(g->n[d])) {
            set_error("too many segments along direction " + std::to_string(d) + " for " +
                      std::to_string(g->n[d]) + " points");
            return NOPCS_EINVAL;
        }
    }
    return NOPCS_OK;
}

static bool check_filter_alpha(double af) {
    if (!(af > -0.5 && af < 0.5)) {
        set_error("filter coefficient must lie in (-0.5, 0.5)");
        return false;
    }
    return true;
}

// The 3D filter of a state in place: every field along x, then y, then z, then
// the wall conditions.
static int filter_state(const nse_params &params, const nopcs_grid *grid, const LinePlanDev pl[3], double *Q,
                        hipStream_t st) {
    const NdConst c = make_nd(params);
    const size_t N = field_elems(grid);
    for (int f = 0; f < 5; ++f)
        for (int d = 0; d < 3; ++d) {
            const SweepGeom g = sweep_geom(grid->n, d);
            double *q = Q + f * N;
            NOPCS_HIP_CHECK(timed(NOPCS_K_FILTER, st, [&] { return launch_filter(d, q, q, g, pl[d], st); }));
        }
    for (int d = 0; d < 3; ++d)
        NOPCS_HIP_CHECK(timed(NOPCS_K_WALL, st, [&] { return launch_bc(Q, grid->n, d, c, st); }));
    return NOPCS_OK;
}

int nopcs_filter(const nse_params *params, const nopcs_grid *grid, double alpha_f, double *Q, void *hip_stream) {
    if (!check_grid(grid) || !check_params(params) || !check_filter_alpha(alpha_f)) return NOPCS_EINVAL;
    if (!Q) { set_error("Q must be non-NULL"); return NOPCS_EINVAL; }
    LinePlanDev pl[3];
    const int rc = get_filter_plans(grid, alpha_f, pl);
    if (rc != NOPCS_OK) return rc;
    return filter_state(*params, grid, pl, Q, (hipStream_t)hip_stream);
}

int rk_step_filtered(const nse_params *params, const nopcs_grid *grid, int precision, double *Q, double dt,
                     int32_t nsteps, int32_t filter_every, double alpha_f, void *ws, size_t ws_bytes,
                     void *hip_stream) {
    if (!check_grid(grid) || !check_params(params) || !check_filter_alpha(alpha_f)) return NOPCS_EINVAL;
    if (filter_every < 0) { set_error("filter_every must be >= 0"); return NOPCS_EINVAL; }
    if (nsteps < 0) { set_error("nsteps must be >= 0"); return NOPCS_EINVAL; }
    LinePlanDev pl[3];
    int rc = get_filter_plans(grid, alpha_f, pl);
    if (rc != NOPCS_OK) return rc;
    int done = 0;
    while (done < nsteps) {
        const int chunk = filter_every > 0 ? std::min(nsteps - done, filter_every) : nsteps - done;
        rc = rk_step(params, grid, precision, Q, dt, chunk, ws, ws_bytes, hip_stream);
        if (rc != NOPCS_OK) return rc;
        done += chunk;
        if (filter_every > 0 && chunk == filter_every) {
            rc = filter_state(*params, grid, pl, Q, (hipStream_t)hip_stream);
            if (rc != NOPCS_OK) return rc;
        }
    }
    return NOPCS_OK;
}

int rk_step_compact_viscous(const nse_params *params, const nopcs_grid *grid, double *Q, double dt, int32_t nsteps,
                            void *ws, size_t ws_bytes, void *hip_stream) {
    if (!check_grid(grid) || !check_params(params)) return NOPCS_EINVAL;
    if (!Q) { set_error("Q must be non-NULL"); return NOPCS_EINVAL; }
    if (((uintptr_t)Q & 15) != 0) { set_error("Q must be 16-byte aligned"); return NOPCS_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error("dt must be positive and finite"); return NOPCS_EINVAL; }
    if (nsteps < 0) { set_error("nsteps must be >= 0"); return NOPCS_EINVAL; }
    const size_t need = nopcs_compact_viscous_workspace_bytes(grid);
    if (!ws || ws_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return NOPCS_EINVAL;
    }
    if (((uintptr_t)ws & 255) != 0) { set_error("workspace must be 256-byte aligned"); return NOPCS_EINVAL; }
    LinePlanDev pl[3];
    int rc = get_plans(grid, pl);
    if (rc != NOPCS_OK) return rc;
    double *cvx = reinterpret_cast<double *>(static_cast<char *>(ws) + nopcs_workspace_bytes(grid, NOPCS_FP64));
    for (int step = 0; step < nsteps; ++step) {
        rc = launch_step(*params, grid, NOPCS_FP64, Q, dt, ws, pl, (hipStream_t)hip_stream, cvx);
        if (rc != NOPCS_OK) return rc;
    }
    return NOPCS_OK;
}

// How a batch of boxes is stepped (nopcs_set_batch_mode):
//   0 merged:   one launch per kernel and configuration over all boxes
//               (batch.hpp), captured as a graph;
//   1 branches: one graph branch per box, each box's launches as rk_step makes
//               them (the device overlaps the branches);
//   2 direct:   the launches of mode 0 issued on the stream, without a graph;
//   3 hybrid:   a branch of its own for every box whose stage kernels fill the
//               device alone (at least kOwnBranchPoints points), the others
//               merged in one more branch (the default).
// Merged launches run phase by phase, so every box of a merged launch waits
// for the largest at each of the step's phase boundaries; branches let boxes
// advance independently but cost a launch per kernel and box.  Many small
// boxes favour merging, a few large ones branches.
enum { BATCH_MERGED = 0, BATCH_BRANCHES = 1, BATCH_DIRECT = 2, BATCH_HYBRID = 3 };
static std::atomic<int> g_batch_mode{BATCH_HYBRID};
constexpr long long kOwnBranchPoints = 1LL << 21;   // 128^3

// The batched RK4 step of a set of boxes.  Boxes that share launches have
// their launches collected by phase (launch_step with a collector); each
// (phase, kernel) becomes one launch over a device table of the boxes'
// arguments.  The step is captured once as a graph -- one branch per group of
// boxes, forked from the capture stream and joined back -- cached per batch
// (mode, boxes, states, workspaces, dt, parameters, precision, piece lengths)
// and replayed nsteps times.
static int batch_step(const nse_params &params, int nbox, const nopcs_box *boxes, int precision, double dt,
                      const LinePlanDev (*pl)[3], int nsteps, hipStream_t st, int mode) {
    int dev = 0;
    NOPCS_HIP_CHECK(hipGetDevice(&dev));
    std::string key = "batch";
    put_bytes(key, mode);
    put_bytes(key, dev);
    put_bytes(key, params);
    put_bytes(key, precision);
    put_bytes(key, dt);
    for (int b = 0; b < nbox; ++b) {
        put_grid(key, boxes[b].grid);
        put_bytes(key, boxes[b].Q);
        put_bytes(key, boxes[b].ws);
        put_bytes(key, boxes[b].dt);
        for (int d = 0; d < 3; ++d) put_bytes(key, piece_length(d, boxes[b].grid.n[d]));
        put_bytes(key, visc_z_chunk(boxes[b].grid.n));
    }
    std::lock_guard<std::mutex> lk(g_gmu);
    auto it = g_graph_cache.find(key);
    if (it != g_graph_cache.end()) return replay(it->second, nsteps, st);
    evict_if_full();
    auto dt_of = [&](int b) { return boxes[b].dt > 0.0 ? boxes[b].dt : dt; };
    // groups: boxes with a branch of their own, and the boxes that share launches
    std::vector<int> own, merged;
    for (int b = 0; b < nbox; ++b) {
        const long long pts = (long long)boxes[b].grid.n[0] * boxes[b].grid.n[1] * boxes[b].grid.n[2];
        const bool alone = mode == BATCH_BRANCHES || (mode == BATCH_HYBRID && pts >= kOwnBranchPoints);
        (alone ? own : merged).push_back(b);
    }
    if (merged.size() == 1) {   // one box needs no table: its own launches
        own.push_back(merged[0]);
        merged.clear();
    }
    GraphEntry e;
    BatchCollector col;
    if (!merged.empty()) {
        for (int b : merged) {
            const int rc = launch_step(params, &boxes[b].grid, precision, boxes[b].Q, dt_of(b), boxes[b].ws, pl[b],
                                       nullptr, nullptr, &col);
            if (rc != NOPCS_OK) return rc;
        }
        // one device buffer holds every table, each 256-byte aligned
        size_t bytes = 0;
        for (auto &ph : col.phases)
            for (BatchLaunch &L : ph.second) {
                L.dev_off = bytes;
                bytes = (bytes + L.items.size() + 255) & ~(size_t)255;
            }
        std::vector<unsigned char> host(bytes, 0);
        for (auto &ph : col.phases)
            for (BatchLaunch &L : ph.second) std::memcpy(host.data() + L.dev_off, L.items.data(), L.items.size());
        NOPCS_HIP_CHECK(hipMalloc(&e.tables, bytes));
        if (hipMemcpy(e.tables, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(e.tables);
            set_error("upload of the batch tables failed");
            return NOPCS_EDEVICE;
        }
    }
    auto launch_merged = [&](hipStream_t s) -> hipError_t {
        for (auto &ph : col.phases)
            for (BatchLaunch &L : ph.second) {
                const hipError_t he = L.launch(static_cast<char *>(e.tables) + L.dev_off, L.ntab, L.total, L.blk, s);
                if (he != hipSuccess) return he;
            }
        return hipSuccess;
    };
    if (mode == BATCH_DIRECT) {   // every box merged (own is empty: nbox >= 2) or the lone box's launches
        if (merged.empty()) {
            for (int step = 0; step < nsteps; ++step) {
                const int rc = launch_step(params, &boxes[0].grid, precision, boxes[0].Q, dt_of(0), boxes[0].ws, pl[0],
                                           st);
                if (rc != NOPCS_OK) return rc;
            }
            return NOPCS_OK;
        }
        for (auto &ph : col.phases)
            for (BatchLaunch &L : ph.second) {
                e.launches.push_back(L);
                e.launches.back().items.clear();
            }
        if (hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipFree(e.tables);
            set_error("hipEventCreateWithFlags failed");
            return NOPCS_EDEVICE;
        }
        return replay(g_graph_cache[key] = e, nsteps, st);
    }
    auto fail = [&](int rc, hipError_t he) {
        if (e.graph) (void)hipGraphDestroy(e.graph);
        if (e.tables) (void)hipFree(e.tables);
        if (rc != NOPCS_OK) return rc;
        set_error(std::string("batch graph capture failed: ") + hipGetErrorString(he));
        return (int)NOPCS_EDEVICE;
    };
    hipStream_t &cs = g_capture_stream[dev];
    if (!cs) {
        const hipError_t r = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (r != hipSuccess) return fail(NOPCS_OK, r);
    }
    // branch streams and fork/join events of this device (kept until nopcs_release_plans)
    const int ngroups = (int)own.size() + (merged.empty() ? 0 : 1);
    std::vector<hipStream_t> &bs = g_branch_streams[dev];
    std::vector<hipEvent_t> &ev = g_branch_events[dev];
    while ((int)bs.size() < ngroups) {
        hipStream_t s = nullptr;
        const hipError_t r = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (r != hipSuccess) return fail(NOPCS_OK, r);
        bs.push_back(s);
    }
    while ((int)ev.size() < ngroups + 1) {
        hipEvent_t x = nullptr;
        const hipError_t r = hipEventCreateWithFlags(&x, hipEventDisableTiming);
        if (r != hipSuccess) return fail(NOPCS_OK, r);
        ev.push_back(x);
    }
    hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) return fail(NOPCS_OK, he);
    t_capturing = true;
    int rc = NOPCS_OK;
    if (ngroups == 1 && !merged.empty()) {
        he = launch_merged(cs);
    } else {
        he = hipEventRecord(ev[ngroups], cs);
        for (int gi = 0; gi < ngroups && rc == NOPCS_OK && he == hipSuccess; ++gi) {
            he = hipStreamWaitEvent(bs[gi], ev[ngroups], 0);
            if (he != hipSuccess) break;
            if (gi < (int)own.size()) {
                const int b = own[gi];
                rc = launch_step(params, &boxes[b].grid, precision, boxes[b].Q, dt_of(b), boxes[b].ws, pl[b], bs[gi]);
                if (rc != NOPCS_OK) break;
            } else {
                he = launch_merged(bs[gi]);
                if (he != hipSuccess) break;
            }
            he = hipEventRecord(ev[gi], bs[gi]);
            if (he == hipSuccess) he = hipStreamWaitEvent(cs, ev[gi], 0);
        }
    }
    t_capturing = false;
    const hipError_t ec = hipStreamEndCapture(cs, &e.graph);
    if (rc != NOPCS_OK || he != hipSuccess || ec != hipSuccess) return fail(rc, he != hipSuccess ? he : ec);
    void *tables = e.tables;
    const int ri = instantiate(e);
    if (ri != NOPCS_OK) {
        if (tables) (void)hipFree(tables);
        return ri;
    }
    return replay(g_graph_cache[key] = e, nsteps, st);
}

int nopcs_set_batch_mode(int32_t mode) {
    if (mode < BATCH_MERGED || mode > BATCH_HYBRID) { set_error("batch mode must be 0, 1, 2 or 3"); return NOPCS_EINVAL; }
    g_batch_mode.store(mode);
    return NOPCS_OK;
}

int rk_step_batch(const nse_params *params, int32_t nbox, const nopcs_box *boxes, int precision, double dt,
                  int32_t nsteps, void *hip_stream) {
    if (!check_params(params)) return NOPCS_EINVAL;
    if (nbox < 1 || nbox > NOPCS_MAX_BATCH) {
        set_error("nbox must be in [1, " + std::to_string(NOPCS_MAX_BATCH) + "]");
        return NOPCS_EINVAL;
    }
    if (!boxes) { set_error("boxes is NULL"); return NOPCS_EINVAL; }
    if (precision != NOPCS_FP64 && precision != NOPCS_MIXED) { set_error("unknown precision"); return NOPCS_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error("dt must be positive and finite"); return NOPCS_EINVAL; }
    if (nsteps < 0) { set_error("nsteps must be >= 0"); return NOPCS_EINVAL; }
    for (int b = 0; b < nbox; ++b) {
        const nopcs_box &x = boxes[b];
        if (!check_grid(&x.grid)) return NOPCS_EINVAL;
        if (!x.Q || ((uintptr_t)x.Q & 15) != 0) {
            set_error("box " + std::to_string(b) + ": Q must be non-NULL and 16-byte aligned");
            return NOPCS_EINVAL;
        }
        if (!check_ws(&x.grid, precision, x.ws, x.ws_bytes)) return NOPCS_EINVAL;
        if (!(x.dt >= 0.0) || !std::isfinite(x.dt)) {
            set_error("box " + std::to_string(b) + ": dt must be finite and >= 0 (0: the call's dt)");
            return NOPCS_EINVAL;
        }
        for (int c = 0; c < b; ++c)
            if (boxes[c].Q == x.Q || boxes[c].ws == x.ws) {
                set_error("boxes " + std::to_string(c) + " and " + std::to_string(b) + " share a state or workspace");
                return NOPCS_EINVAL;
            }
    }
    std::vector<LinePlanDev> plv((size_t)nbox * 3);
    LinePlanDev(*pl)[3] = reinterpret_cast<LinePlanDev(*)[3]>(plv.data());
    for (int b = 0; b < nbox; ++b) {
        const int rc = get_plans(&boxes[b].grid, pl[b]);
        if (rc != NOPCS_OK) return rc;
    }
    if (nsteps == 0) return NOPCS_OK;
    return batch_step(*params, nbox, boxes, precision, dt, pl, nsteps, (hipStream_t)hip_stream, g_batch_mode.load());
}

int nopcs_autotune(const nse_params *params, const nopcs_grid *grid, int precision, const double *Q, void *ws,
                   size_t ws_bytes, void *hip_stream, int32_t piece_out[3]) {
    if (!check_grid(grid) || !check_params(params)) return NOPCS_EINVAL;
    if (precision != NOPCS_FP64 && precision != NOPCS_MIXED) { set_error("unknown precision"); return NOPCS_EINVAL; }
    if (!Q || !piece_out) { set_error("Q and piece_out must be non-NULL"); return NOPCS_EINVAL; }
    if (!check_ws(grid, precision, ws, ws_bytes)) return NOPCS_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t bytes = 5 * field_elems(grid) * sizeof(double);
    double *scratch = nullptr;
    NOPCS_HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&scratch), bytes));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = NOPCS_OK;
    const double dt = 1e-9;   // any admissible step: only the time of the launches matters
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipMemcpyAsync(scratch, Q, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        set_error("autotune: device setup failed");
        rc = NOPCS_EDEVICE;
    }
    // one step untimed (plans, caches), two timed; the copy keeps Q untouched
    auto time_it = [&](float *ms) -> int {
        int r = rk_step(params, grid, precision, scratch, dt, 1, ws, ws_bytes, hip_stream);
        if (r != NOPCS_OK) return r;
        if (hipEventRecord(e0, st) != hipSuccess) return NOPCS_EDEVICE;
        r = rk_step(params, grid, precision, scratch, dt, 2, ws, ws_bytes, hip_stream);
        if (r != NOPCS_OK) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return NOPCS_EDEVICE;
        return NOPCS_OK;
    };
    int best[3];
    for (int d = 0; d < 3; ++d) best[d] = g_piece_len[d].load();
    for (int d = 0; d < 3 && rc == NOPCS_OK; ++d) {
        const int n = grid->n[d];
        const std::vector<int> cand = n <= 64 ? std::vector<int>{0, 16, 32} : std::vector<int>{16, 24, 32};
        float best_ms = 0.0f;
        int best_len = best[d];
        bool any = false;
        for (int len : cand) {
            g_piece_len[d].store(len);
            if (nopcs_workspace_bytes(grid, precision) > ws_bytes) continue;   // closure array would not fit
            LinePlanDev pl[3];
            if (get_plans(grid, pl) != NOPCS_OK) continue;                    // too many known rows per line
            float ms = 0.0f;
            rc = time_it(&ms);
            if (rc != NOPCS_OK) break;
            if (!any || ms < best_ms) {
                best_ms = ms;
                best_len = len;
                any = true;
            }
        }
        g_piece_len[d].store(best_len);
        best[d] = best_len;
    }
    // then the z chunk of the viscous kernel (planes per block), with the pieces chosen
    const int chunk0 = visc_z_chunk_setting();
    int best_chunk = chunk0;
    if (rc == NOPCS_OK) {
        float best_ms = 0.0f;
        bool any = false;
        for (int zc : {16, 32, 64, 128}) {
            if (zc > grid->n[2] && zc != 16) continue;
            set_visc_z_chunk(zc);
            float ms = 0.0f;
            rc = time_it(&ms);
            if (rc != NOPCS_OK) break;
            if (!any || ms < best_ms) {
                best_ms = ms;
                best_chunk = zc;
                any = true;
            }
        }
        set_visc_z_chunk(best_chunk);
    }
    if (rc != NOPCS_OK) {
        for (int d = 0; d < 3; ++d) g_piece_len[d].store(best[d]);
        set_visc_z_chunk(chunk0);
    }
    for (int d = 0; d < 3; ++d) piece_out[d] = piece_length(d, grid->n[d]);
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    return rc;
}

int nopcs_set_visc_chunk(int32_t planes) {
    if (planes != 0 && (planes < 8 || planes > 1024)) {
        set_error("viscous z chunk must be 0 (default) or 8..1024 planes");
        return NOPCS_EINVAL;
    }
    set_visc_z_chunk(planes);
    return NOPCS_OK;
}

int32_t nopcs_visc_chunk(const nopcs_grid *grid) {
    if (!check_grid(grid)) return NOPCS_EINVAL;
    return visc_z_chunk(grid->n);
}

int nopcs_set_graphs(int32_t on) {
    g_graphs.store(on ? 1 : 0);
    return NOPCS_OK;
}

int nopcs_set_graph_cache_limit(int32_t n) {
    if (n < 1 || n > 4096) { set_error("graph cache limit must be in [1, 4096]"); return NOPCS_EINVAL; }
    std::lock_guard<std::mutex> lk(g_gmu);
    g_max_graphs.store(n);
    evict_if_full(0);
    return NOPCS_OK;
}

int nopcs_set_piece_length(int32_t dir, int32_t piece_len) {
    if (dir < 0 || dir > 2) { set_error("dir must be 0, 1 or 2"); return NOPCS_EINVAL; }
    if (piece_len < -1 || (piece_len > 0 && piece_len < 8)) {
        set_error("piece_len must be -1, 0 or >= 8");
        return NOPCS_EINVAL;
    }
    g_piece_len[dir] = piece_len;
    return NOPCS_OK;
}

int nopcs_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (on) {
        for (auto &r : g_recs) {
            (void)hipEventSynchronize(r.b);
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        g_recs.clear();
        for (int k = 0; k < NOPCS_K_COUNT; ++k) {
            g_total_ms[k] = 0.0;
            g_launches[k] = 0;
        }
    }
    g_timing = on != 0;
    return NOPCS_OK;
}

int nopcs_timing_read(int32_t kernel, double *total_ms, int64_t *launches) {
    if (kernel < 0 || kernel >= NOPCS_K_COUNT) { set_error("unknown kernel id"); return NOPCS_EINVAL; }
    std::lock_guard<std::mutex> lk(g_tmu);
    const int rc = drain_timing();
    if (rc != NOPCS_OK) return rc;
    if (total_ms) *total_ms = g_total_ms[kernel];
    if (launches) *launches = g_launches[kernel];
    return NOPCS_OK;
}

}  // extern "C"
