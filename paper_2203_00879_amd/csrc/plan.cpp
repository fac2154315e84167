// plan.cpp -- host construction of NOHAP line plans and their device copies.
//
// A line of n points (nodes on both walls) is cut into the user's segments
// (Section 3, Fig. 2) and, optionally, each segment into shorter pieces.  Every
// piece boundary contributes two closure rows (the last point of one piece and
// the first of the next) whose derivative is the truncated equivalent explicit
// sum with the row of the global C = A^-1 B (Eqs. CS:fpCf, CS:fpCf_i).  Rows
// 0, 1, n-2 and n-1 are explicit second-order wall rows.  The compact rows left
// between known rows form independent constant-coefficient tridiagonal runs.
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

namespace nopcs {

std::vector<int> even_segments(int n, int nseg) {
    std::vector<int> lo(nseg);
    const int base = n / nseg, rem = n % nseg;
    int s = 0;
    for (int k = 0; k < nseg; ++k) {
        lo[k] = s;
        s += base + (k < rem ? 1 : 0);
    }
    return lo;
}

// Column j of the global C = A^-1 B (h = 1) of operator op, in long double:
// solve A x = B e_j.
static void global_column(int n, int j, int op, double alpha_f, std::vector<long double> &x,
                          std::vector<long double> &work) {
    const long double a = op == OP_FILTER ? (long double)alpha_f : (long double)kAlpha;
    std::vector<long double> &rhs = x;
    std::fill(rhs.begin(), rhs.end(), 0.0L);
    auto put = [&](int row, long double v) {
        if (row >= 0 && row < n) rhs[row] += v;
    };
    // B e_j: entries B_{i,j} of every row i that touches column j
    if (op == OP_FILTER) {
        // wall rows 0, 1, n-2, n-1 are the identity (left unfiltered); interior
        // rows a0 f_i + a1/2 (f_{i+1} + f_{i-1}) + a2/2 (f_{i+2} + f_{i-2})
        const long double af = alpha_f;
        const long double a0 = 5.0L / 8.0L + 0.75L * af, a1h = 0.5L * (0.5L + af), a2h = 0.5L * (-0.125L + 0.25L * af);
        if (j <= 1 || j >= n - 2) put(j, 1.0L);
        for (int i = j - 2; i <= j + 2; ++i) {
            if (i < 2 || i > n - 3) continue;
            const int k = j - i < 0 ? i - j : j - i;
            put(i, k == 0 ? a0 : k == 1 ? a1h : a2h);
        }
    } else {
        const long double b1 = kB1, b2 = kB2;
        if (j <= 2) {  // row 0: (-3/2, 2, -1/2) on columns 0..2
            const long double w0[3] = {-1.5L, 2.0L, -0.5L};
            put(0, w0[j]);
        }
        if (j == 0) put(1, -0.5L);
        if (j == 2) put(1, 0.5L);
        for (int i = j - 2; i <= j + 2; ++i) {
            if (i < 2 || i > n - 3) continue;
            const int k = j - i;
            const long double v = k == -2 ? -b2 : k == -1 ? -b1 : k == 1 ? b1 : k == 2 ? b2 : 0.0L;
            put(i, v);
        }
        if (j == n - 3) put(n - 2, -0.5L);
        if (j == n - 1) put(n - 2, 0.5L);
        if (j >= n - 3) {  // row n-1: (1/2, -2, 3/2) on columns n-3..n-1
            const long double w1[3] = {0.5L, -2.0L, 1.5L};
            put(n - 1, w1[j - (n - 3)]);
        }
    }
    // rows 0, 1, n-2, n-1 are explicit: x equals rhs there.  Rows 2..n-3:
    // a x_{i-1} + x_i + a x_{i+1} = rhs_i with x_1 and x_{n-2} known.
    const int m = n - 4;
    if (m <= 0) return;
    long double *cp = work.data();
    long double *dp = work.data() + n;
    long double prev_c = 0.0L, prev_d = 0.0L;
    for (int k = 0; k < m; ++k) {
        const int i = 2 + k;
        long double r = rhs[i];
        if (k == 0) r -= a * rhs[1];
        if (k == m - 1) r -= a * rhs[n - 2];
        const long double s = (k > 0) ? a : 0.0L;
        const long double den = 1.0L - s * prev_c;
        dp[k] = (r - s * prev_d) / den;
        cp[k] = a / den;
        prev_c = cp[k];
        prev_d = dp[k];
    }
    x[2 + m - 1] = dp[m - 1];
    for (int k = m - 2; k >= 0; --k) x[2 + k] = dp[k] - cp[k] * x[2 + k + 1];
}

void build_march_tables(LinePlanHost &P);

std::vector<uint8_t> row_kinds(int n, int nseg, int sub_len) {
    const std::vector<int> seg_lo = even_segments(n, nseg);
    // piece starts: user segment starts plus even cuts inside each segment
    std::vector<int> starts;
    for (int s = 0; s < nseg; ++s) {
        const int a = seg_lo[s];
        const int e = (s + 1 < nseg) ? seg_lo[s + 1] - 1 : n - 1;
        const int len = e - a + 1;
        int pieces = 1;
        if (sub_len > 0) pieces = (len + sub_len - 1) / sub_len;
        while (pieces > 1 && len / pieces < 4) --pieces;
        const std::vector<int> sub = even_segments(len, pieces);
        for (int v : sub) starts.push_back(a + v);
    }
    std::vector<uint8_t> kind(n, ROW_COMPACT);
    for (int i : {0, 1, n - 2, n - 1}) kind[i] = ROW_WALL;
    for (size_t q = 1; q < starts.size(); ++q) {
        const int b = starts[q];
        for (int e : {b - 1, b})
            if (kind[e] == ROW_COMPACT) kind[e] = ROW_CLOSURE;
    }
    return kind;
}

bool build_line_plan(int n, int nseg, int sub_len, LinePlanHost &P, std::string &err, int op, double alpha_f) {
    if (n < 8) {
        err = "line length must be >= 8 (got " + std::to_string(n) + ")";
        return false;
    }
    if (nseg < 1 || n < 4 * nseg) {
        err = "segments must be >= 1 and each at least 4 points long (n=" + std::to_string(n) +
              ", nseg=" + std::to_string(nseg) + ")";
        return false;
    }
    if (op == OP_FILTER && !(alpha_f > -0.5 && alpha_f < 0.5)) {
        err = "filter coefficient must lie in (-0.5, 0.5) (diagonally dominant system)";
        return false;
    }
    P = LinePlanHost();
    P.op = op;
    P.alpha = op == OP_FILTER ? alpha_f : kAlpha;
    P.n = n;
    P.nseg = nseg;
    P.sub_len = sub_len;
    P.seg_lo = even_segments(n, nseg);
    P.row_kind = row_kinds(n, nseg, sub_len);
    int lo = 1;
    for (int i = 2; i <= n - 2; ++i) {
        if (P.row_kind[i] != ROW_COMPACT) {
            if (i - lo >= 2) P.runs.push_back(make_int2(lo, i));
            lo = i;
        }
    }
    // closure rows of the global C (long double column solves, rounded once)
    std::vector<int> rows;
    for (int i = 0; i < n; ++i)
        if (P.row_kind[i] == ROW_CLOSURE) rows.push_back(i);
    const int ncl = (int)rows.size();
    P.cl_row = rows;
    P.cl_j0.resize(ncl);
    P.cl_len.resize(ncl);
    P.cl_coef.assign((size_t)ncl * kTaps, 0.0);
    if (ncl > 0) {
        std::vector<long double> col(n), work(2 * (size_t)n);
        for (int j = 0; j < n; ++j) {
            bool needed = false;
            for (int e : rows)
                if (j >= e - kNb && j <= e + kNb) { needed = true; break; }
            if (!needed) continue;
            global_column(n, j, op, alpha_f, col, work);
            for (int q = 0; q < ncl; ++q) {
                const int e = rows[q];
                if (j < e - kNb || j > e + kNb) continue;
                const int j0 = e - kNb < 0 ? 0 : e - kNb;
                P.cl_coef[(size_t)q * kTaps + (j - j0)] = (double)col[e];
            }
        }
        for (int q = 0; q < ncl; ++q) {
            const int e = rows[q];
            const int j0 = e - kNb < 0 ? 0 : e - kNb;
            const int j1 = e + kNb > n - 1 ? n - 1 : e + kNb;
            P.cl_j0[q] = j0;
            P.cl_len[q] = j1 - j0 + 1;
        }
    }
    // known-row slots: 0..3 for rows 0, 1, n-2, n-1; 4 + q for closure q
    P.kslot.assign(n, (short)-1);
    P.kslot[0] = 0;
    P.kslot[1] = 1;
    P.kslot[n - 2] = 2;
    P.kslot[n - 1] = 3;
    for (int q = 0; q < ncl; ++q) P.kslot[rows[q]] = (short)(4 + q);
    for (const int2 &r : P.runs) P.run_slot.push_back(make_int2(P.kslot[r.x], P.kslot[r.y]));
    // elimination tables of a constant-coefficient run, indexed by the position
    // k = 1, 2, ... inside the run (Thomas algorithm, Section 3)
    P.den.assign(n + 1, 0.0);
    P.rden.assign(n + 1, 0.0);
    P.cp.assign(n + 1, 0.0);
    double cprev = 0.0;
    for (int k = 1; k <= n; ++k) {
        const double s = (k > 1) ? P.alpha : 0.0;
        const double den = 1.0 - s * cprev;
        P.den[k] = den;
        P.rden[k] = 1.0 / den;
        P.cp[k] = P.alpha / den;
        cprev = P.cp[k];
    }
    build_march_tables(P);
    return true;
}

// Tables of the line-march sweeps: which run makes the R update of each known
// row, a slot schedule for accumulating all closure sums in one pass along the
// line, and groups of consecutive runs.
void build_march_tables(LinePlanHost &P) {
    const int n = P.n, nrun = (int)P.runs.size(), ncl = (int)P.cl_row.size();
    P.max_m = 0;
    for (const int2 &r : P.runs) P.max_m = std::max(P.max_m, r.y - r.x - 1);
    // every known row is a bound of some run (segments and pieces have >= 4
    // points); the first run that touches it updates it, rows 0 and n-1 go with
    // the first and the last run
    P.run_own.assign(nrun, 0);
    std::vector<char> done(n, 0);
    for (int r = 0; r < nrun; ++r) {
        const int2 b = P.runs[r];
        if (!done[b.x]) { P.run_own[r] |= 1; done[b.x] = 1; }
        if (!done[b.y]) { P.run_own[r] |= 2; done[b.y] = 1; }
    }
    if (nrun > 0) {
        P.run_own[0] |= 4;
        P.run_own[nrun - 1] |= 8;
    }
    // closure slots: interval colouring of the tap windows in row order
    std::vector<int> slot_of(ncl, -1), slot_end(kMaxSlots, -1);
    int nslot = 0;
    bool fits = true;
    for (int q = 0; q < ncl && fits; ++q) {
        int s = 0;
        while (s < kMaxSlots && slot_end[s] >= P.cl_j0[q]) ++s;
        if (s == kMaxSlots) { fits = false; break; }
        slot_of[q] = s;
        slot_end[s] = P.cl_j0[q] + P.cl_len[q] - 1;
        nslot = std::max(nslot, s + 1);
    }
    P.k1_S = !fits ? 0 : (nslot <= 8 ? 8 : kMaxSlots);
    P.k1_rec.assign((size_t)n * std::max(P.k1_S, 1), -1);
    P.k1_w.assign((size_t)n * std::max(P.k1_S, 1), 0.0);
    std::vector<int> ev(3 * (size_t)n, 0);
    if (P.k1_S > 0) {
        for (int q = 0; q < ncl; ++q) {
            for (int t = 0; t < P.cl_len[q]; ++t) {
                const int j = P.cl_j0[q] + t;
                int rec = q | (t << 12);
                if (t == 0) rec |= kRecOpen;
                if (j == P.cl_row[q]) rec |= kRecRow;
                if (t == P.cl_len[q] - 1) rec |= kRecClose;
                P.k1_rec[(size_t)j * P.k1_S + slot_of[q]] = rec;
                const int m3[3] = {rec & kRecOpen, rec & kRecRow, rec & kRecClose};
                for (int x = 0; x < 3; ++x)
                    if (m3[x]) ev[3 * (size_t)j + x] |= 1 << slot_of[q];
                P.k1_w[(size_t)j * P.k1_S + slot_of[q]] = P.cl_coef[(size_t)q * kTaps + t];
            }
        }
    }
    P.k1_evrow.clear();
    P.k1_evmask.clear();
    for (int j = 0; j < n; ++j)
        if (ev[3 * (size_t)j] | ev[3 * (size_t)j + 1] | ev[3 * (size_t)j + 2]) {
            P.k1_evrow.push_back(j);
            for (int x = 0; x < 3; ++x) P.k1_evmask.push_back(ev[3 * (size_t)j + x]);
        }
    P.cl_wsum.assign(ncl, 0.0);
    for (int q = 0; q < ncl; ++q) {
        double w = 0.0;
        for (int t = 0; t < P.cl_len[q]; ++t) w += P.cl_coef[(size_t)q * kTaps + t];
        P.cl_wsum[q] = w;
    }
    // run groups of about kGroupRows rows and at most kGroupRuns runs
    P.grp.clear();
    int r0 = 0, rows = 0;
    for (int r = 0; r < nrun; ++r) {
        rows += P.runs[r].y - P.runs[r].x;
        if (rows >= kGroupRows || r + 1 - r0 == kGroupRuns || r == nrun - 1) {
            P.grp.push_back(make_int2(r0, r + 1));
            r0 = r + 1;
            rows = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Device cache
// ---------------------------------------------------------------------------
namespace {
struct PlanEntry {
    std::vector<void *> bufs;   // one buffer (tables packed), or one per table in the CPU build
    LinePlanDev dev{};
};
std::mutex g_mu;
std::map<std::tuple<int, int, int, int, uint64_t, int, uint64_t>, PlanEntry> g_plans;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

int get_line_plan(int n, int nseg, int sub_len, double len, LinePlanDev *out, bool lookup_only, int op,
                  double alpha_f) {
    int dev = 0;
    NOPCS_HIP_CHECK(hipGetDevice(&dev));
    uint64_t lbits, abits = 0;
    std::memcpy(&lbits, &len, sizeof lbits);
    if (op == OP_FILTER) std::memcpy(&abits, &alpha_f, sizeof abits);
    const auto key = std::make_tuple(dev, n, nseg, sub_len, lbits, op, abits);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.dev;
        return NOPCS_OK;
    }
    if (lookup_only) {
        set_error("no cached line plan for n=" + std::to_string(n) + ", nseg=" + std::to_string(nseg) +
                  " on this device (an earlier call with this grid builds it)");
        return NOPCS_EINVAL;
    }
    LinePlanHost P;
    std::string err;
    if (!build_line_plan(n, nseg, sub_len, P, err, op, alpha_f)) {
        set_error(err);
        return NOPCS_EINVAL;
    }
    const int nrun = (int)P.runs.size(), ncl = (int)P.cl_row.size();
    // pack everything into one device buffer
    size_t off = 0;
    const size_t o_runs = off; off = align256(off + sizeof(int2) * (nrun + 1));
    const size_t o_rslot = off; off = align256(off + sizeof(int2) * (nrun + 1));
    const size_t o_kslot = off; off = align256(off + sizeof(short) * (n + 1));
    const size_t o_row = off;  off = align256(off + sizeof(int) * (ncl + 1));
    const size_t o_j0 = off;   off = align256(off + sizeof(int) * (ncl + 1));
    const size_t o_len = off;  off = align256(off + sizeof(int) * (ncl + 1));
    const size_t o_coefA = off; off = align256(off + sizeof(double) * ((size_t)ncl * 128 + 2));
    const size_t o_den = off;  off = align256(off + sizeof(double) * (n + 1));
    const size_t o_cp = off;   off = align256(off + sizeof(double) * (n + 1));
    const size_t o_d32 = off;  off = align256(off + sizeof(float) * (n + 1));
    const size_t o_c32b = off; off = align256(off + sizeof(float) * (n + 1));
    const int ngrp = (int)P.grp.size();
    const size_t o_grp = off;  off = align256(off + sizeof(int2) * (ngrp + 1));
    const size_t o_own = off;  off = align256(off + sizeof(int) * (nrun + 1));
    const size_t o_rec = off;  off = align256(off + sizeof(int) * (P.k1_rec.size() + 1));
    const size_t o_wsum = off; off = align256(off + sizeof(double) * (ncl + 1));
    const size_t o_k1w = off;  off = align256(off + sizeof(double) * (P.k1_w.size() + 1));
    const size_t o_evr = off;  off = align256(off + sizeof(int) * (P.k1_evrow.size() + 1));
    const size_t o_evm = off;  off = align256(off + sizeof(int) * (P.k1_evmask.size() + 1));
    std::vector<unsigned char> host(off, 0);
    auto cpy = [&](size_t o, const void *src, size_t bytes) {
        if (bytes) std::memcpy(host.data() + o, src, bytes);
    };
    cpy(o_runs, P.runs.data(), sizeof(int2) * nrun);
    cpy(o_rslot, P.run_slot.data(), sizeof(int2) * nrun);
    cpy(o_kslot, P.kslot.data(), sizeof(short) * n);
    cpy(o_row, P.cl_row.data(), sizeof(int) * ncl);
    cpy(o_j0, P.cl_j0.data(), sizeof(int) * ncl);
    cpy(o_len, P.cl_len.data(), sizeof(int) * ncl);
    // closure taps on the four aligned 32-row blocks that hold the tap window
    // (a window of 97 rows starting anywhere in a block ends in the fourth)
    std::vector<double> coefA((size_t)ncl * 128, 0.0);
    for (int q = 0; q < ncl; ++q) {
        const int a0 = P.cl_j0[q] - 32 * (P.cl_j0[q] / 32);
        for (int t = 0; t < P.cl_len[q]; ++t) {
            const int a = a0 + t;
            coefA[((size_t)(a / 2) * ncl + q) * 2 + (a % 2)] = P.cl_coef[(size_t)q * kTaps + t];
        }
    }
    cpy(o_coefA, coefA.data(), sizeof(double) * coefA.size());
    cpy(o_den, P.rden.data(), sizeof(double) * (n + 1));
    cpy(o_cp, P.cp.data(), sizeof(double) * (n + 1));
    std::vector<float> d32(P.rden.begin(), P.rden.end()), cp32(P.cp.begin(), P.cp.end());
    cpy(o_d32, d32.data(), sizeof(float) * (n + 1));
    cpy(o_c32b, cp32.data(), sizeof(float) * (n + 1));
    cpy(o_grp, P.grp.data(), sizeof(int2) * ngrp);
    cpy(o_own, P.run_own.data(), sizeof(int) * nrun);
    cpy(o_rec, P.k1_rec.data(), sizeof(int) * P.k1_rec.size());
    cpy(o_wsum, P.cl_wsum.data(), sizeof(double) * ncl);
    cpy(o_k1w, P.k1_w.data(), sizeof(double) * P.k1_w.size());
    cpy(o_evr, P.k1_evrow.data(), sizeof(int) * P.k1_evrow.size());
    cpy(o_evm, P.k1_evmask.data(), sizeof(int) * P.k1_evmask.size());
    // each table's offset in the blob and the bytes the kernels may read
    const size_t tab_off[] = {o_runs, o_rslot, o_kslot, o_row, o_j0, o_len, o_coefA, o_den, o_cp, o_d32, o_c32b,
                              o_grp, o_own, o_rec, o_wsum, o_k1w, o_evr, o_evm};
    const size_t tab_len[] = {sizeof(int2) * nrun, sizeof(int2) * nrun, sizeof(short) * n, sizeof(int) * ncl,
                              sizeof(int) * ncl, sizeof(int) * ncl, sizeof(double) * coefA.size(),
                              sizeof(double) * (n + 1), sizeof(double) * (n + 1), sizeof(float) * (n + 1),
                              sizeof(float) * (n + 1), sizeof(int2) * ngrp, sizeof(int) * nrun,
                              sizeof(int) * P.k1_rec.size(), sizeof(double) * ncl, sizeof(double) * P.k1_w.size(),
                              sizeof(int) * P.k1_evrow.size(), sizeof(int) * P.k1_evmask.size()};
    constexpr int ntab = sizeof(tab_off) / sizeof(tab_off[0]);
    static_assert(ntab == sizeof(tab_len) / sizeof(tab_len[0]), "one length per table");
    std::vector<void *> bufs;
    unsigned char *tab[ntab];
#ifdef NOPCS_CPU_EMUL
    // CPU build of the kernels: every table in a guarded allocation of its own,
    // sized exactly, so that a read past the end of any one table faults
    for (int t = 0; t < ntab; ++t) {
        void *b1 = nullptr;
        if (hipMalloc(&b1, tab_len[t]) != hipSuccess) {
            for (void *b : bufs) (void)hipFree(b);
            set_error("hipMalloc of a line plan failed");
            return NOPCS_ENOMEM;
        }
        bufs.push_back(b1);
        std::memcpy(b1, host.data() + tab_off[t], tab_len[t]);
        tab[t] = static_cast<unsigned char *>(b1);
    }
#else
    // one device buffer holds every table
    void *buf = nullptr;
    if (hipMalloc(&buf, off) != hipSuccess) {
        set_error("hipMalloc of a line plan failed");
        return NOPCS_ENOMEM;
    }
    if (hipMemcpy(buf, host.data(), off, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(buf);
        set_error("hipMemcpy of a line plan failed");
        return NOPCS_EDEVICE;
    }
    bufs.push_back(buf);
    for (int t = 0; t < ntab; ++t) tab[t] = static_cast<unsigned char *>(buf) + tab_off[t];
#endif
    LinePlanDev d;
    d.op = op;
    d.alpha = P.alpha;
    d.fc = filter_coefs(op == OP_FILTER ? alpha_f : 0.0);
    d.n = n;
    d.nrun = nrun;
    d.ncl = ncl;
    d.ih = (double)(n - 1) / len;
    d.runs = reinterpret_cast<const int2 *>(tab[0]);
    d.run_slot = reinterpret_cast<const int2 *>(tab[1]);
    d.kslot = reinterpret_cast<const short *>(tab[2]);
    d.cl_row = reinterpret_cast<const int *>(tab[3]);
    d.cl_j0 = reinterpret_cast<const int *>(tab[4]);
    d.cl_len = reinterpret_cast<const int *>(tab[5]);
    d.cl_coefA = reinterpret_cast<const double *>(tab[6]);
    d.rden = reinterpret_cast<const double *>(tab[7]);
    d.cp = reinterpret_cast<const double *>(tab[8]);
    d.rden32 = reinterpret_cast<const float *>(tab[9]);
    d.cp32 = reinterpret_cast<const float *>(tab[10]);
    d.max_m = P.max_m;
    d.ngrp = ngrp;
    d.k1_S = P.k1_S;
    d.grp = reinterpret_cast<const int2 *>(tab[11]);
    d.run_own = reinterpret_cast<const int *>(tab[12]);
    d.k1_rec = reinterpret_cast<const int *>(tab[13]);
    d.cl_wsum = reinterpret_cast<const double *>(tab[14]);
    d.k1_w = reinterpret_cast<const double *>(tab[15]);
    d.k1_nev = (int)P.k1_evrow.size();
    d.k1_evrow = reinterpret_cast<const int *>(tab[16]);
    d.k1_evmask = reinterpret_cast<const int *>(tab[17]);
    PlanEntry e;
    e.bufs = bufs;
    e.dev = d;
    g_plans[key] = e;
    *out = d;
    return NOPCS_OK;
}

void release_line_plans() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::get<0>(it->first) == dev) {
            for (void *b : it->second.bufs) (void)hipFree(b);
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace nopcs
