// Host side of libsgweno: plans (grid enumeration, layout, tiling), solvers
// bound to caller memory, the time loop and the C entry points of sgweno.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "sgw_api_internal.h"

namespace {
thread_local char g_err[512] = "";
}

sgw_status sgw_fail(sgw_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

sgw_status sgw_hip_fail(hipError_t e, const char* what)
{
    return sgw_fail(SGW_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char* sgw_last_error(void) { return g_err; }

extern "C" const char* sgw_status_string(sgw_status s)
{
    switch (s) {
    case SGW_OK: return "ok";
    case SGW_ERR_INVALID_ARG: return "invalid argument";
    case SGW_ERR_UNSUPPORTED: return "unsupported";
    case SGW_ERR_OUT_OF_MEMORY: return "out of memory";
    case SGW_ERR_NONFINITE: return "non-finite wave speed or time step";
    case SGW_ERR_HIP: return "HIP error";
    case SGW_ERR_STATE: return "call out of order";
    default: return "unknown status";
    }
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

// ---------------------------------------------------------------- index set
// All l in Z_{>=0}^d with |l| = s, lexicographic in (l_1..l_d): the first
// component counts up from 0 and the rest are filled recursively.
static void compositions(int d, int s, int pos, int* cur, std::vector<std::array<int, 4>>& out)
{
    if (pos == d - 1) {
        cur[pos] = s;
        std::array<int, 4> a = {0, 0, 0, 0};
        for (int k = 0; k < d; k++) a[k] = cur[k];
        out.push_back(a);
        return;
    }
    for (int v = 0; v <= s; v++) {
        cur[pos] = v;
        compositions(d, s - v, pos + 1, cur, out);
    }
}

static int64_t binom(int n, int k)
{
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 0; i < k; i++) r = r * (n - i) / (i + 1);
    return r;
}

// ---------------------------------------------------------------- tiling

// The line sweep divides segment and line indices with the fast divisions of its descriptor:
// check each against plain division at the ends of its range (0, d - 1, d, the largest index)
// before any kernel relies on it.
static bool line_divisions_ok(const GridDev& g)
{
    auto ok = [](const FastDiv& f, uint32_t d, uint32_t xmax) {
        if (f.d != d || d == 0) return false;
        const uint32_t xs[] = {0u, d - 1, d, xmax, xmax > 0 ? xmax - 1 : 0};
        for (uint32_t x : xs) {
            if (x > xmax) continue;
            const uint32_t q = (uint32_t)((((uint64_t)x * f.m) >> 32) + x) >> f.s;
            if (q != x / d) return false;
        }
        return true;
    };
    uint32_t size = 1;
    for (int k = 0; k < g.d; k++) size *= (uint32_t)g.n[k];
    for (int k = 0; k < g.d; k++) {
        const uint32_t segs = (uint32_t)g.lsegl[k] * (uint32_t)g.ltrans[k];
        if (!ok(g.fd_n[k], (uint32_t)g.n[k], size) || !ok(g.fd_lsegl[k], (uint32_t)g.lsegl[k], segs) ||
            !ok(g.fd_ltrans[k], (uint32_t)g.ltrans[k], segs))
            return false;
    }
    return true;
}

static void fill_box_geometry(GridDev& g, int precision)
{
    (void)precision;
    int core = 1;
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        if (k >= g.d) {
            g.t[k] = 1;
            g.halo[k] = 0;
            g.ntile[k] = 1;
            continue;
        }
        g.halo[k] = (g.t[k] < g.n[k]) ? 3 : 0;
        g.ntile[k] = g.n[k] / g.t[k];
    }
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        g.CS[k] = core;
        core *= g.t[k];
    }
    g.core_total = core;
    // LDS: core rows of t_0 values at an odd stride RS (columns hit distinct banks), then a low
    // and a high slab per halo direction (direction 0: rows of 3; others: the core layout with
    // extent 3 in that direction)
    g.lines = core / g.t[0];
    {
        // rows hold t_0 values, or the t_0 + 1 interface fluxes of direction 1 with a halo
        const int i0 = g.t[0] + (g.halo[0] ? 1 : 0);
        g.RS = i0 + ((i0 % 2 == 0 && g.lines > 1) ? 1 : 0);
    }
    g.whole = 1;
    for (int k = 0; k < g.d; k++) g.whole &= (g.t[k] == g.n[k]) ? 1 : 0;
    {
        int ls = 1;
        for (int k = 0; k < SGW_MAX_DIM; k++) {
            g.LS[k] = ls;
            ls *= (k == 0) ? g.RS : g.t[k];
        }
    }
    int pad = g.RS * g.lines;
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        g.slab_lo[k] = g.slab_hi[k] = 0;
        g.slab_n[k] = 0;
        if (k < g.d && g.halo[k]) {
            g.slab_n[k] = 3 * (core / g.t[k]);
            const int lds = (k == 0) ? 3 * g.lines : 3 * g.RS * (g.lines / g.t[k]);
            g.slab_lo[k] = pad;
            pad += lds;
            g.slab_hi[k] = pad;
            pad += lds;
        }
    }
    g.pad_total = pad;
    g.fd_lines = make_fastdiv((uint32_t)g.lines);
    g.rline = (SGW_BLOCK % g.t[0] == 0) ? SGW_BLOCK / g.t[0] : 0;
    g.nbox = 1;
    for (int k = 0; k < g.d; k++) g.nbox *= g.ntile[k];
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        g.I[k] = g.t[k] + (g.halo[k] ? 1 : 0);
        g.flux_total[k] = (k < g.d) ? core / g.t[k] * g.I[k] : 0;
        const int SEG = sgw_seg(g.d);
        g.nseg[k] = (g.I[k] + SEG - 1) / SEG;
        g.seg_total[k] = (k < g.d) ? core / g.t[k] * g.nseg[k] : 0;
        g.fd_nseg[k] = make_fastdiv((uint32_t)g.nseg[k]);
        // segment s reads window positions s*SEG - hf - 2 .. s*SEG - hf + SEG + 2: interior (no
        // halo, no wrap) for 1 <= s <= (t - 3 - SEG + hf) / SEG
        g.nlines[k] = core / g.t[k];
        g.fd_lines_k[k] = make_fastdiv((uint32_t)g.nlines[k]);
        {
            const int hf = g.halo[k] ? 1 : 0;
            const int top = g.t[k] - 3 - SEG + hf;
            g.nint[k] = (k < g.d && top >= SEG) ? top / SEG : 0;
        }
        if (k == 0) {
            g.F0S = g.RS;
            g.flux_total[0] = g.F0S * g.lines; // direction 0 keeps its interface rows at the core row stride
        }
        g.fd_CS[k] = make_fastdiv((uint32_t)g.CS[k]);
        g.fd_t[k] = make_fastdiv((uint32_t)g.t[k]);
        g.fd_I[k] = make_fastdiv((uint32_t)g.I[k]);
        g.fd_CSt[k] = make_fastdiv((uint32_t)(g.CS[k] * g.t[k]));
        g.fd_n[k] = make_fastdiv((uint32_t)(k < g.d ? g.n[k] : 1));
    }
    int fm = 0;
    for (int k = 0; k < g.d; k++) fm = g.flux_total[k] > fm ? g.flux_total[k] : fm;
    g.sf_elems = (fm + 1) / 2 * 2;
    // 3D/4D boxes that do not span their grid keep the global offset of every core row and
    // halo-slab row in LDS
    int rt = 0;
    for (int k = 0; k < SGW_MAX_DIM; k++) g.rt_off[k] = 0;
    if (g.d >= 3 && !g.whole) {
        rt = g.lines;
        for (int k = 1; k < g.d; k++)
            if (g.halo[k]) {
                g.rt_off[k] = rt;
                rt += 2 * (g.slab_n[k] / g.t[0]);
            }
    }
    g.rt_total = rt;
    g.pad2_ = 0;
}

// Box search: every combination of divisors t_k | n_k with a core of at most
// `target` nodes that fits the LDS budget; the cost per core node weighs the
// staged values (halo included; narrow rows along the contiguous direction
// count extra) against the interface fluxes (each costs two WENO5
// reconstructions, ~25 times a staged load).
static void choose_box(GridDev& g, int precision, int target, size_t lds_cap)
{
    std::vector<int> divs[SGW_MAX_DIM];
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        if (k >= g.d) {
            divs[k].push_back(1);
            continue;
        }
        for (int v = 1; v <= g.n[k]; v++)
            if (g.n[k] % v == 0) divs[k].push_back(v);
    }
    const int64_t grid_nodes = (int64_t)g.n[0] * g.n[1] * g.n[2] * g.n[3];
    const int min_core = (int)(grid_nodes < SGW_BLOCK ? grid_nodes : SGW_BLOCK);
    const double rs = precision == SGW_FP64 ? 8.0 : 4.0;
    double best = 1e300;
    int bt[SGW_MAX_DIM] = {g.n[0], g.n[1], g.n[2], g.n[3]};
    for (int a : divs[0])
        for (int b : divs[1])
            for (int c : divs[2])
                for (int e : divs[3]) {
                    const int64_t core = (int64_t)a * b * c * e;
                    if (core > target || core > SGW_BLOCK * SGW_MAXR || core < min_core) continue;
                    g.t[0] = a;
                    g.t[1] = b;
                    g.t[2] = c;
                    g.t[3] = e;
                    fill_box_geometry(g, precision);
                    if (stage_lds_bytes(g, precision) > lds_cap) continue;
                    double flux = 0.0;
                    for (int k = 0; k < g.d; k++) flux += (double)g.flux_total[k];
                    const double row_bytes = g.t[0] * rs;
                    const double load = g.pad_total * (row_bytes < 64.0 ? 64.0 / row_bytes : 1.0);
                    const double cost = (load + 25.0 * flux) / (double)core + 2000.0 / (double)core;
                    if (cost < best - 1e-12) {
                        best = cost;
                        for (int k = 0; k < SGW_MAX_DIM; k++) bt[k] = g.t[k];
                    }
                }
    for (int k = 0; k < SGW_MAX_DIM; k++) g.t[k] = bt[k];
    fill_box_geometry(g, precision);
}

// Coarse extent staged per tile in direction k.
static int coarse_extent(int T, int m, int N)
{
    if (m == 0) return T;
    // centres spanned by the tile's nodes J0..J0+T-1 (J0 a multiple of T), the most over the
    // tile positions, plus two stencil nodes on either side
    // tile positions (J0 a multiple of T): with x = (J0 + R/2) mod R the nodes span
    // floor((x + T - 1) / R) + 1 centres; x takes every value R/2 + j gcd(T, R) mod R (N is a
    // multiple of T and R), the largest R - gcd(T, R), or R/2 when R divides T
    (void)N;
    const int R = 1 << m;
    int g = R;
    while (T % g) g >>= 1;
    const int x = (g == R) ? R / 2 : R - g;
    return (x + T - 1) / R + 1 + 4;
}

static int last_refined(const sgw_plan& p, int g)
{
    int kl = -1;
    for (int k = 0; k < p.pb.dim; k++)
        if (p.cfg.finest_level - p.levels[g][k] > 0) kl = k;
    return kl;
}

// LDS elements of the two buffers.  The staged coarse block goes to buffer A and the passes
// write B, A, B, ... in turn.  The old form gives both buffers the largest staged block or pass
// output.  In the line form the last refined direction's pass goes to registers (its output
// needs no buffer), a grid refined along direction 1 reads its coarse rows from global memory
// (no staged block), and each buffer takes the largest output that lands in it.
static void prolong_buffer_elems(const sgw_plan& p, const int* T, bool lines, size_t* a_elems, size_t* b_elems,
                                 size_t* rows_max)
{
    size_t amax = 0, bmax = 0, rows = 0;
    for (int g = 0; g < p.G; g++) {
        int c[SGW_MAX_DIM];
        for (int k = 0; k < p.pb.dim; k++) c[k] = coarse_extent(T[k], p.cfg.finest_level - p.levels[g][k], p.N);
        size_t load = 1;
        for (int k = 0; k < p.pb.dim; k++) load *= (size_t)c[k];
        const int kl = last_refined(p, g);
        const bool direct = lines && p.cfg.finest_level - p.levels[g][0] > 0 && kl > 0;
        if (!direct) {
            amax = load > amax ? load : amax;
            const size_t r = load / (size_t)c[0];
            rows = r > rows ? r : rows;
        }
        int j = 0;
        for (int k = 0; k < p.pb.dim; k++) {
            if (lines && k >= kl) break;
            if (p.cfg.finest_level - p.levels[g][k] == 0) continue;
            size_t sz = 1;
            for (int i = 0; i < p.pb.dim; i++) sz *= (size_t)(i <= k ? T[i] : c[i]);
            size_t& m = (j % 2 == 0) ? bmax : amax;
            m = sz > m ? sz : m;
            j++;
        }
    }
    if (!lines) amax = bmax = amax > bmax ? amax : bmax;
    *a_elems = (amax + 1) / 2 * 2;
    *b_elems = (bmax + 1) / 2 * 2;
    if (rows_max) *rows_max = lines ? rows : 0;
}

static size_t prolong_lds_bytes(const sgw_plan& p, const int* T, bool lines)
{
    const size_t rs = p.cfg.precision == SGW_FP64 ? 8 : 4;
    size_t a = 0, b = 0, rows = 0;
    prolong_buffer_elems(p, T, lines, &a, &b, &rows);
    return rs * (a + b) + (lines ? 4 * rows : 0);
}

// Interpolations and staged coarse values of one finest-grid tile T, summed
// over the grids.  Directions are refined in order 1..d, so the pass of
// direction k covers the tile in directions <= k and the coarse block (stencil
// halo included) in the directions after k: a small T early and a large T late
// keeps the halo work of the early passes small.
static void prolong_tile_work(const sgw_plan& p, const int* T, double* interp, double* load)
{
    const int d = p.pb.dim;
    *interp = 0.0;
    *load = 0.0;
    for (int g = 0; g < p.G; g++) {
        int c[SGW_MAX_DIM];
        for (int k = 0; k < d; k++) c[k] = coarse_extent(T[k], p.cfg.finest_level - p.levels[g][k], p.N);
        double l = 1.0;
        for (int k = 0; k < d; k++) l *= c[k];
        *load += l;
        for (int k = 0; k < d; k++) {
            if (p.cfg.finest_level - p.levels[g][k] == 0) continue;
            double out = 1.0;
            for (int j = 0; j < d; j++) out *= (j <= k) ? T[j] : c[j];
            *interp += out;
        }
    }
}

// Estimated VALU lane-operations of one tile in the line form: a lane per line, rounds of
// SGW_BLOCK lines, only the wavefronts that hold a line issue.  Per staged value ~16, per
// row offset ~12 per direction, per line ~12, per coarse centre ~30, per fine node ~16 (FP32)
// or ~22 (FP64: the division's Newton steps), per accumulated node 2, and a node-by-node
// final pass (~60 per node) for the grid whose last direction is not refined.
static double prolong_lines_cost(const sgw_plan& p, const int* T)
{
    const int d = p.pb.dim;
    const double pt = p.cfg.precision == SGW_FP64 ? 22.0 : 16.0;
    double cost = 0.0;
    for (int g = 0; g < p.G; g++) {
        int c[SGW_MAX_DIM], m[SGW_MAX_DIM];
        for (int k = 0; k < d; k++) {
            m[k] = p.cfg.finest_level - p.levels[g][k];
            c[k] = coarse_extent(T[k], m[k], p.N);
        }
        double load = 1.0;
        for (int k = 0; k < d; k++) load *= c[k];
        const double rows = load / c[0];
        const int kl = last_refined(p, g);
        if (m[0] > 0 && kl > 0)
            cost += std::ceil(rows / SGW_BLOCK) * SGW_BLOCK * (12.0 * (d - 1) + 2.0 * c[0]); // rows read directly
        else
            cost += std::ceil(load / SGW_BLOCK) * SGW_BLOCK * 16.0 +
                    std::ceil(rows / SGW_BLOCK) * SGW_BLOCK * 12.0 * (d - 1);
        for (int k = 0; k < d && k <= kl; k++) {
            if (m[k] == 0) continue;
            const int R = 1 << m[k];
            const double cen = (T[k] >= R ? (T[k] - 1) / R + 2 : 2);
            double inner = 1.0, outer = 1.0;
            for (int j = 0; j < k; j++) inner *= T[j];
            for (int j = k + 1; j < d; j++) outer *= c[j];
            const double per_line = 12.0 + 30.0 * cen + pt * T[k];
            if (k == d - 1) {
                cost += SGW_BLOCK * (per_line + 2.0 * T[k]);
            } else if (k == kl) {
                cost += SGW_BLOCK * 60.0 * T[d - 1];
            } else {
                const double lines = inner * outer;
                for (double done = 0.0; done < lines; done += SGW_BLOCK) {
                    const double act = std::min((double)SGW_BLOCK, lines - done);
                    cost += std::ceil(act / 64.0) * 64.0 * per_line;
                }
            }
        }
        cost += 2000.0; // barriers and set-up per grid and tile
    }
    return cost;
}

// Tile search.  3D/4D: the line form, tiles with prod_{k<d-1} T_k = SGW_BLOCK and at most 16
// nodes per line along the last direction, LDS within 64 KB, cost by prolong_lines_cost per
// finest node plus the FP64 write (more when tile rows along direction 1 are short), scaled up
// when fewer than 4 workgroups per compute unit fit in LDS.  Otherwise (1D/2D, a manual tile or
// no such tile): every combination of divisors T_k | N with at most 8 (2D) or 16 points per
// thread and two LDS buffers within 64 KB; the cost per finest node counts interpolations (~50
// operations each), staged coarse values (~10), a fixed cost per grid and tile (barriers, set-up:
// ~2000) and the FP64 write of the node, scaled the same way.
static void choose_fine_tile(sgw_plan& p)
{
    const int d = p.pb.dim;
    const size_t rs = p.cfg.precision == SGW_FP64 ? 8 : 4;
    int T[SGW_MAX_DIM] = {1, 1, 1, 1};
    bool manual = false;
    for (int k = 0; k < d; k++) {
        T[k] = p.cfg.fine_tile[k] > 0 ? p.cfg.fine_tile[k] : p.N;
        manual |= p.cfg.fine_tile[k] > 0;
    }
    std::vector<int> divs;
    for (int v = 1; v <= p.N; v++)
        if (p.N % v == 0) divs.push_back(v);
    const int nd = (int)divs.size();
    auto occupancy_slow = [](size_t lds) {
        const double occ = (double)(163840 / (lds ? lds : 1));
        return occ >= 4.0 ? 1.0 : 4.0 / occ;
    };
    bool lines = false;
    if (manual && d >= 3) {
        // a manual tile takes the line form when it has its shape
        int64_t inner = 1;
        for (int k = 0; k < d - 1; k++) inner *= T[k];
        lines = inner == SGW_BLOCK && T[d - 1] <= 16 && prolong_lds_bytes(p, T, true) <= 64 * 1024;
    }
    if (!manual && d >= 3) {
        double best = 1e300;
        int bt[SGW_MAX_DIM] = {1, 1, 1, 1};
        int idx[SGW_MAX_DIM] = {0, 0, 0, 0};
        for (;;) {
            int t[SGW_MAX_DIM] = {1, 1, 1, 1};
            int64_t inner = 1;
            for (int k = 0; k < d; k++) {
                t[k] = divs[idx[k]];
                if (k < d - 1) inner *= t[k];
            }
            if (inner == SGW_BLOCK && t[d - 1] <= 16) {
                const size_t lds = prolong_lds_bytes(p, t, true);
                if (lds <= 64 * 1024) {
                    const double pts = (double)inner * t[d - 1];
                    const double write = 40.0 * (t[0] >= 8 ? 1.0 : 8.0 / t[0]);
                    const double cost = occupancy_slow(lds) * (prolong_lines_cost(p, t) / pts + write);
                    if (cost < best - 1e-9) {
                        best = cost;
                        for (int k = 0; k < SGW_MAX_DIM; k++) bt[k] = t[k];
                    }
                }
            }
            int k = 0;
            while (k < d && ++idx[k] == nd) idx[k++] = 0;
            if (k == d) break;
        }
        if (best < 1e300) {
            lines = true;
            for (int k = 0; k < d; k++) T[k] = bt[k];
        }
    }
    if (!manual && !lines) {
        const int cap = d <= 2 ? SGW_BLOCK * 8 : SGW_BLOCK * 16;
        double best = 1e300;
        int bt[SGW_MAX_DIM] = {1, 1, 1, 1};
        int idx[SGW_MAX_DIM] = {0, 0, 0, 0};
        for (;;) {
            int t[SGW_MAX_DIM] = {1, 1, 1, 1};
            int64_t pts = 1;
            for (int k = 0; k < d; k++) {
                t[k] = divs[idx[k]];
                pts *= t[k];
            }
            const size_t lds = prolong_lds_bytes(p, t, false);
            if (pts <= cap && pts >= SGW_BLOCK / 4 && lds <= 64 * 1024) {
                double interp, load;
                prolong_tile_work(p, t, &interp, &load);
                // the tile's FP64 rows along direction 1 are written to HBM: rows shorter than
                // 8 values (64 bytes) waste most of each write transaction
                const double write = 40.0 * (t[0] >= 8 ? 1.0 : 8.0 / t[0]);
                const double cost =
                    occupancy_slow(lds) * ((50.0 * interp + 10.0 * load + 2000.0 * p.G) / (double)pts + write);
                if (cost < best - 1e-9) {
                    best = cost;
                    for (int k = 0; k < SGW_MAX_DIM; k++) bt[k] = t[k];
                }
            }
            int k = 0;
            while (k < d && ++idx[k] == nd) idx[k++] = 0;
            if (k == d) break;
        }
        if (best < 1e300)
            for (int k = 0; k < d; k++) T[k] = bt[k];
    }
    for (int k = 0; k < SGW_MAX_DIM; k++) p.fine_T[k] = k < d ? T[k] : 1;
    p.fine_lines = lines;
    prolong_buffer_elems(p, p.fine_T, lines, &p.pro_buf_elems, &p.pro_bufb_elems, &p.pro_rows_max);
    p.pro_lds = prolong_lds_bytes(p, p.fine_T, lines);
}

// ---------------------------------------------------------------- plans

extern "C" sgw_status sgw_plan_create(const sgw_problem* pb, const sgw_config* cfg, sgw_plan_t** out)
{
    if (!pb || !cfg || !out) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    const int d = pb->dim;
    if (d < 1 || d > SGW_MAX_DIM) return sgw_fail(SGW_ERR_INVALID_ARG, "dim %d outside 1..4", d);
    if (cfg->root_cells < 4) return sgw_fail(SGW_ERR_INVALID_ARG, "root_cells %d < 4", cfg->root_cells);
    if (cfg->finest_level < 0 || cfg->finest_level > 12)
        return sgw_fail(SGW_ERR_INVALID_ARG, "finest_level %d outside 0..12", cfg->finest_level);
    if (!(cfg->cfl > 0.0 && cfg->cfl <= 1.5)) return sgw_fail(SGW_ERR_INVALID_ARG, "cfl %g outside (0, 1.5]", cfg->cfl);
    if (!(cfg->eps_flux > 0.0) || !(cfg->eps_interp > 0.0))
        return sgw_fail(SGW_ERR_INVALID_ARG, "epsilon must be positive");
    if (pb->flux < 0 || pb->flux > 4) return sgw_fail(SGW_ERR_INVALID_ARG, "unknown flux %d", pb->flux);
    if (pb->ic < 0 || pb->ic > 3) return sgw_fail(SGW_ERR_INVALID_ARG, "unknown initial condition %d", pb->ic);
    if (pb->reserved0 != 0) return sgw_fail(SGW_ERR_INVALID_ARG, "reserved0 must be 0");
    int zmask = 0;
    for (int k = 0; k < d; k++) {
        if (pb->bc[k] != SGW_BC_PERIODIC && pb->bc[k] != SGW_BC_ZERO)
            return sgw_fail(SGW_ERR_INVALID_ARG, "unknown boundary condition %d in direction %d", pb->bc[k], k);
        if (pb->bc[k] == SGW_BC_ZERO) zmask |= 1 << k;
    }
    if (!(pb->relax_tau >= 0.0) || !std::isfinite(pb->relax_tau))
        return sgw_fail(SGW_ERR_INVALID_ARG, "relax_tau %g must be finite and >= 0", pb->relax_tau);
    const bool relax = pb->relax_tau > 0.0;
    if (relax && !(pb->relax_theta > 0.0 && std::isfinite(pb->relax_theta)))
        return sgw_fail(SGW_ERR_INVALID_ARG, "relax_theta %g must be finite and > 0", pb->relax_theta);
    const bool phase = pb->flux == SGW_FLUX_VLASOV_FIXED_E || pb->flux == SGW_FLUX_VLASOV_HARMONIC ||
                       pb->ic == SGW_IC_MAXWELL_COS || pb->ic == SGW_IC_VLASOV_BOLTZMANN || relax;
    if (phase && (d % 2)) return sgw_fail(SGW_ERR_INVALID_ARG, "phase-space problems need an even dim");
    const bool vm = pb->flux == SGW_FLUX_VLASOV_MAXWELL;
    if (vm != (pb->ic == SGW_IC_VLASOV_MAXWELL))
        return sgw_fail(SGW_ERR_INVALID_ARG, "the Vlasov-Maxwell flux and initial condition go together");
    if (vm && d != 3) return sgw_fail(SGW_ERR_INVALID_ARG, "the Vlasov-Maxwell system needs dim 3");
    if (vm && relax) return sgw_fail(SGW_ERR_INVALID_ARG, "relaxation is not part of the Vlasov-Maxwell system");
    if (vm && zmask) return sgw_fail(SGW_ERR_UNSUPPORTED, "the Vlasov-Maxwell system runs with periodic boundaries");
    if (pb->ic == SGW_IC_VLASOV_BOLTZMANN && d != 2 && d != 4)
        return sgw_fail(SGW_ERR_INVALID_ARG, "the Vlasov-Boltzmann initial condition needs dim 2 or 4");
    if (cfg->dt_mode != SGW_DT_CFL && cfg->dt_mode != SGW_DT_POW53)
        return sgw_fail(SGW_ERR_INVALID_ARG, "unknown dt_mode %d", cfg->dt_mode);
    if (cfg->prolong != SGW_PROLONG_WENO5 && cfg->prolong != SGW_PROLONG_LAGRANGE5)
        return sgw_fail(SGW_ERR_INVALID_ARG, "unknown prolongation %d", cfg->prolong);
    if (cfg->precision != SGW_FP64 && cfg->precision != SGW_FP32_SWEEP)
        return sgw_fail(SGW_ERR_INVALID_ARG, "unknown precision %d", cfg->precision);
    for (int k = 0; k < d; k++)
        if (!(pb->hi[k] > pb->lo[k])) return sgw_fail(SGW_ERR_INVALID_ARG, "empty domain in direction %d", k);
    const int64_t N = (int64_t)cfg->root_cells << cfg->finest_level;
    double fine_nodes = 1.0;
    for (int k = 0; k < d; k++) fine_nodes *= (double)N;
    if (N > (1 << 20) || fine_nodes > 1099511627776.0)
        return sgw_fail(SGW_ERR_INVALID_ARG, "finest grid too large (%lld per direction)", (long long)N);

    sgw_plan* p = new sgw_plan();
    p->pb = *pb;
    p->cfg = *cfg;
    p->N = (int)N;
    p->fine_nodes = 1;
    for (int k = 0; k < d; k++) p->fine_nodes *= N;
    // index set: q = 0..d-1, |l| = N_L - q, coefficient (-1)^q C(d-1, q)
    for (int q = 0; q < d; q++) {
        const int s = cfg->finest_level - q;
        if (s < 0) continue;
        std::vector<std::array<int, 4>> ls;
        int cur[4] = {0, 0, 0, 0};
        compositions(d, s, 0, cur, ls);
        for (auto& l : ls) {
            p->levels.push_back(l);
            p->coefs.push_back((int)(binom(d - 1, q) * ((q & 1) ? -1 : 1)));
        }
    }
    p->G = (int)p->levels.size();
    p->offsets.resize(p->G + 1);
    p->grids.resize(p->G);
    int64_t tot = 0;
    const size_t lds_cap = 64 * 1024;
    int target = 1024;
    if (cfg->blocks_per_cu < 0 || cfg->blocks_per_cu > 64)
        return sgw_fail(SGW_ERR_INVALID_ARG, "blocks_per_cu %d outside 0..64", cfg->blocks_per_cu);
    if (cfg->sweep_form < 0 || cfg->sweep_form > 2)
        return sgw_fail(SGW_ERR_INVALID_ARG, "sweep_form %d outside 0..2", cfg->sweep_form);
    if (cfg->box_target) {
        if (cfg->box_target < 64 || cfg->box_target > SGW_BLOCK * SGW_MAXR) {
            delete p;
            return sgw_fail(SGW_ERR_INVALID_ARG, "box_target %d outside 64..%d", cfg->box_target, SGW_BLOCK * SGW_MAXR);
        }
        target = cfg->box_target;
    }
    for (int g = 0; g < p->G; g++) {
        GridDev& gd = p->grids[g];
        std::memset(&gd, 0, sizeof(gd));
        gd.d = d;
        int64_t n = 1;
        for (int k = 0; k < SGW_MAX_DIM; k++) {
            gd.n[k] = k < d ? (cfg->root_cells << p->levels[g][k]) : 1;
            gd.stride[k] = (int32_t)n;
            n *= gd.n[k];
        }
        if (n > (1ll << 30)) {
            delete p;
            return sgw_fail(SGW_ERR_INVALID_ARG, "component grid too large");
        }
        p->offsets[g] = tot;
        tot += n;
        bool manual = false;
        for (int k = 0; k < d; k++) manual |= cfg->box[k] > 0;
        if (manual && (zmask || relax || vm)) {
            delete p;
            return sgw_fail(SGW_ERR_UNSUPPORTED, "manual stage boxes with a zero boundary, relaxation or fields");
        }
        if ((d == 4 || (d == 3 && cfg->sweep_form != 2) || zmask || relax || vm) && !manual) {
            // 3D and 4D (3D stage boxes on request), zero boundaries and relaxation: the line
            // sweep (no stage boxes); a work item is SGW_LWAVE segments of sgw_lseg() nodes,
            // enough items for the direction with the most segments
            gd.line_mode = 1;
            gd.zmask = zmask;
            int64_t most = 0;
            for (int k = 0; k < SGW_MAX_DIM; k++) gd.fd_n[k] = make_fastdiv((uint32_t)gd.n[k]);
            for (int k = 0; k < d; k++) {
                const int ls = sgw_lseg(cfg->precision == SGW_FP64);
                gd.lsegl[k] = (gd.n[k] + ls - 1) / ls;
                gd.ltrans[k] = (int32_t)(n / gd.n[k]);
                gd.fd_lsegl[k] = make_fastdiv((uint32_t)gd.lsegl[k]);
                gd.fd_ltrans[k] = make_fastdiv((uint32_t)gd.ltrans[k]);
                if ((gd.n[k] & (gd.n[k] - 1)) == 0) gd.pow2_mask |= 1 << k;
                const int64_t segs = (int64_t)gd.lsegl[k] * gd.ltrans[k];
                most = segs > most ? segs : most;
            }
            gd.nbox = (int32_t)((most + SGW_LWAVE - 1) / SGW_LWAVE);
            p->line_mode = true;
            if (!line_divisions_ok(gd)) {
                delete p;
                return sgw_fail(SGW_ERR_UNSUPPORTED, "line sweep index division fails for grid %d", g);
            }
            continue;
        }
        if (manual) {
            for (int k = 0; k < SGW_MAX_DIM; k++) {
                gd.t[k] = (k < d && cfg->box[k] > 0) ? (cfg->box[k] < gd.n[k] ? cfg->box[k] : gd.n[k])
                                                     : (k < d ? gd.n[k] : 1);
                if (k < d && gd.n[k] % gd.t[k]) {
                    delete p;
                    return sgw_fail(SGW_ERR_UNSUPPORTED, "box %d does not divide extent %d", gd.t[k], gd.n[k]);
                }
            }
            fill_box_geometry(gd, cfg->precision);
            if (gd.core_total > SGW_BLOCK * SGW_MAXR || stage_lds_bytes(gd, cfg->precision) > lds_cap) {
                delete p;
                return sgw_fail(SGW_ERR_UNSUPPORTED, "box too large for one workgroup");
            }
        } else {
            choose_box(gd, cfg->precision, target, lds_cap);
        }
        // the kernel keeps SGW_MAXR nodes per thread and sizes LDS from these numbers
        if (gd.core_total > SGW_BLOCK * SGW_MAXR || stage_lds_bytes(gd, cfg->precision) > lds_cap) {
            delete p;
            return sgw_fail(SGW_ERR_UNSUPPORTED, "no stage box fits one workgroup for grid %d", g);
        }
    }
    p->offsets[p->G] = tot;
    p->total_nodes = tot;
    // 3D and 4D line sweeps: directions 1 and 2 in one launch over whole (x_1, x_2) planes when every
    // grid's plane fits a work item (the Vlasov-Maxwell coefficients come from the fields in the line
    // sweep only)
    p->plane01 = p->line_mode && !vm && ((d == 4 && cfg->sweep_form != 1) || (d == 3 && cfg->sweep_form == 0));
    for (int g = 0; g < p->G && p->plane01; g++)
        p->plane01 = p->grids[g].line_mode && p->grids[g].n[0] * p->grids[g].n[1] <= SGW_PLANE_CAP;
    p->nplane_items = 0;
    if (p->plane01)
        for (int g = 0; g < p->G; g++) {
            GridDev& gd = p->grids[g];
            gd.plane_nodes = gd.n[0] * gd.n[1];
            gd.nplanes = gd.n[2] * gd.n[3];
            gd.ppi = SGW_PLANE_CAP / gd.plane_nodes;
            p->nplane_items += (gd.nplanes + gd.ppi - 1) / gd.ppi;
        }
    p->zmask = zmask;
    p->relax = relax;
    p->vm = vm;
    // velocity moments (the density of the relaxation source, the currents of the Vlasov-Maxwell
    // system): per grid, blocks of SGW_RHO_COLS x nodes times chunks of SGW_RHO_CHUNK velocity rows
    p->nrho_items = 0;
    p->nrho_final = 0;
    if (relax || vm)
        for (int g = 0; g < p->G; g++) {
            GridDev& gd = p->grids[g];
            const int m = vm ? 1 : d / 2; // x directions: the first d/2, or x_2 alone
            int64_t nx = 1, nv = 1;
            for (int k = 0; k < m; k++) nx *= gd.n[k];
            for (int k = m; k < d; k++) nv *= gd.n[k];
            gd.relax = relax ? 1 : 0;
            gd.vm = vm ? 1 : 0;
            gd.nmom = vm ? 2 : 1;
            gd.nxr = (int32_t)nx;
            gd.nvr = (int32_t)nv;
            gd.rho_cb = (int32_t)((nx + SGW_RHO_COLS - 1) / SGW_RHO_COLS);
            gd.rho_nchunk = (int32_t)((nv + SGW_RHO_CHUNK - 1) / SGW_RHO_CHUNK);
            p->nrho_items += (int64_t)gd.rho_cb * gd.rho_nchunk;
            p->nrho_final += gd.rho_cb;
        }
    // the box list holds the grids that are one box first (their three stages run in one
    // launch), then the boxes of the others, grid by grid
    p->nitems = 0;
    p->nitems_whole = 0;
    p->stage_lds = p->lds_whole = p->lds_boxed = 0;
    for (int pass = 0; pass < 2; pass++)
        for (int g = 0; g < p->G; g++) {
            const bool one = p->grids[g].nbox == 1 && !p->grids[g].line_mode;
            if (one != (pass == 0)) continue;
            p->grids[g].first_item = (int32_t)p->nitems;
            p->nitems += p->grids[g].nbox;
            if (one) p->nitems_whole = p->nitems;
            const size_t l = stage_lds_bytes(p->grids[g], cfg->precision);
            p->stage_lds = l > p->stage_lds ? l : p->stage_lds;
            size_t& m = one ? p->lds_whole : p->lds_boxed;
            m = l > m ? l : m;
        }
    for (int k = 0; k < d; k++)
        if (cfg->fine_tile[k] > 0 && N % cfg->fine_tile[k]) {
            delete p;
            return sgw_fail(SGW_ERR_UNSUPPORTED, "fine tile %d does not divide %lld", cfg->fine_tile[k], (long long)N);
        }
    choose_fine_tile(*p);
    {
        int pts = 1;
        for (int k = 0; k < d; k++) pts *= p->fine_T[k];
        if (pts > SGW_BLOCK * 16 || p->pro_lds > 64 * 1024) {
            delete p;
            return sgw_fail(SGW_ERR_UNSUPPORTED, "prolongation tile too large for one workgroup");
        }
    }
    // byte layout
    const uint64_t rs = cfg->precision == SGW_FP64 ? 8 : 4;
    p->copy_bytes = align256((uint64_t)tot * rs);
    // Vlasov-Maxwell: the fields of every grid (FP64, 3 n_1 values) follow the nodes in each copy
    p->fields_total = 0;
    p->fields_off = 0;
    if (vm) {
        p->fields_off = p->copy_bytes;
        for (int g = 0; g < p->G; g++) {
            p->grids[g].fld_bytes =
                (int64_t)p->fields_off + 8 * p->fields_total - (int64_t)p->offsets[g] * (int64_t)rs;
            p->fields_total += 3 * (int64_t)p->grids[g].n[0];
        }
        p->copy_bytes = align256(p->fields_off + 8 * (uint64_t)p->fields_total);
    }
    p->state_bytes = 3 * p->copy_bytes;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    p->off_grids = take(sizeof(GridDev) * p->G);
    p->off_req = take(sizeof(ReqDev));
    p->off_items = take(sizeof(WorkItem) * p->nitems);
    p->off_alpha = take(sizeof(unsigned long long) * 4 * p->G);
    p->coef_off.assign((size_t)p->G * SGW_MAX_DIM, 0);
    uint64_t coef_elems = 0;
    if (pb->flux == SGW_FLUX_VLASOV_FIXED_E || pb->flux == SGW_FLUX_VLASOV_HARMONIC) {
        const int m = d / 2;
        for (int g = 0; g < p->G; g++)
            for (int k = 0; k < d; k++) {
                p->coef_off[(size_t)g * SGW_MAX_DIM + k] = (int64_t)coef_elems;
                const int src = k < m ? m + k : k - m;
                coef_elems += (uint64_t)p->grids[g].n[src];
            }
    } else if (vm) {
        // x_2 direction only: the coefficient xi_2 by the xi_2 node; the xi directions take theirs
        // from the fields
        for (int g = 0; g < p->G; g++) {
            p->coef_off[(size_t)g * SGW_MAX_DIM] = (int64_t)coef_elems;
            coef_elems += (uint64_t)p->grids[g].n[2];
        }
    }
    p->off_coef = take(sizeof(double) * (coef_elems ? coef_elems : 1));
    p->off_coef_off = take(sizeof(int64_t) * p->coef_off.size());
    p->off_pro = take(sizeof(ProDev) * p->G);
    p->off_fine = take(sizeof(FineDev));
    // per-point prolongation coefficients, entries for R = 2, 4, ..., 2^N_L
    p->off_stab = take(8 * rs * (((uint64_t)2 << cfg->finest_level) - 1));
    p->off_partials = take(sizeof(double) * 2 * SGW_NPART);
    p->off_result = take(sizeof(double) * 2);
    uint64_t foot = 0;
    if (pb->flux == SGW_FLUX_VLASOV_FIXED_E) foot = sizeof(double) * 2 * (uint64_t)(d / 2) * N * N;
    p->off_foot = take(foot ? foot : 8);
    // relaxation: velocity factor tables, density, its partial sums, work items of both passes
    p->mu_off.assign((size_t)p->G * SGW_MAX_DIM, 0);
    uint64_t mu_elems = 0, rho_elems = 0, part_elems = 0;
    if (relax || vm)
        for (int g = 0; g < p->G; g++) {
            const GridDev& gd = p->grids[g];
            if (relax)
                for (int k = d / 2; k < d; k++) {
                    p->mu_off[(size_t)g * SGW_MAX_DIM + k] = (int64_t)mu_elems;
                    mu_elems += (uint64_t)gd.n[k];
                }
            rho_elems += (uint64_t)gd.nmom * gd.nxr;
            part_elems += (uint64_t)gd.nmom * gd.nxr * (uint64_t)gd.rho_nchunk;
        }
    p->off_mu = take(sizeof(double) * (mu_elems ? mu_elems : 1));
    p->off_rho = take(sizeof(double) * (rho_elems ? rho_elems : 1));
    p->off_rho_part = take(sizeof(double) * (part_elems ? part_elems : 1));
    p->off_rho_items = take(sizeof(RhoItem) * (p->nrho_items + p->nrho_final + 1));
    p->off_vm_alpha = take(sizeof(double) * 6 * (vm ? p->G : 1));
    p->off_plane_items = take(sizeof(WorkItem) * (p->nplane_items ? p->nplane_items : 1));
    p->scratch_bytes = off;
    *out = p;
    return SGW_OK;
}

extern "C" void sgw_plan_free(sgw_plan_t* p) { delete p; }

extern "C" sgw_status sgw_plan_footprint(const sgw_plan_t* p, uint64_t* state_bytes, uint64_t* scratch_bytes,
                                         uint64_t* fine_bytes)
{
    if (!p) return sgw_fail(SGW_ERR_INVALID_ARG, "null plan");
    if (state_bytes) *state_bytes = p->state_bytes;
    if (scratch_bytes) *scratch_bytes = p->scratch_bytes;
    if (fine_bytes) *fine_bytes = (uint64_t)p->fine_nodes * sizeof(double);
    return SGW_OK;
}

extern "C" sgw_status sgw_plan_info(const sgw_plan_t* p, int32_t* num_grids, int64_t* total_nodes,
                                    int64_t* fine_nodes)
{
    if (!p) return sgw_fail(SGW_ERR_INVALID_ARG, "null plan");
    if (num_grids) *num_grids = p->G;
    if (total_nodes) *total_nodes = p->total_nodes;
    if (fine_nodes) *fine_nodes = p->fine_nodes;
    return SGW_OK;
}

extern "C" sgw_status sgw_plan_grid(const sgw_plan_t* p, int32_t g, int32_t level[SGW_MAX_DIM],
                                    int32_t shape[SGW_MAX_DIM], int32_t* coef, int64_t* offset)
{
    if (!p) return sgw_fail(SGW_ERR_INVALID_ARG, "null plan");
    if (g < 0 || g >= p->G) return sgw_fail(SGW_ERR_INVALID_ARG, "grid %d outside 0..%d", g, p->G - 1);
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        if (level) level[k] = k < p->pb.dim ? p->levels[g][k] : 0;
        if (shape) shape[k] = p->grids[g].n[k];
    }
    if (coef) *coef = p->coefs[g];
    if (offset) *offset = p->offsets[g];
    return SGW_OK;
}

// Box extents chosen for grid g (for tests and the tuner).
extern "C" sgw_status sgw_plan_fine_tile(const sgw_plan_t* p, int32_t tile[SGW_MAX_DIM])
{
    if (!p || !tile) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    for (int k = 0; k < SGW_MAX_DIM; k++) tile[k] = p->fine_T[k];
    return SGW_OK;
}

extern "C" sgw_status sgw_plan_fine_tile_count(const sgw_plan_t* p, int64_t* count)
{
    if (!p || !count) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    int64_t n = 1;
    for (int k = 0; k < p->pb.dim; k++) n *= p->N / p->fine_T[k];
    *count = n;
    return SGW_OK;
}

extern "C" sgw_status sgw_plan_grid_box(const sgw_plan_t* p, int32_t g, int32_t box[SGW_MAX_DIM])
{
    if (!p || g < 0 || g >= p->G || !box) return sgw_fail(SGW_ERR_INVALID_ARG, "bad grid");
    for (int k = 0; k < SGW_MAX_DIM; k++) box[k] = p->grids[g].t[k];
    return SGW_OK;
}

// ---------------------------------------------------------------- solvers

#define HIPCHK(expr, what)                                 \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return sgw_hip_fail(e_, what); \
    } while (0)

extern "C" sgw_status sgw_solver_create(sgw_plan_t* p, void* state_dev, void* scratch_dev, void* hip_stream,
                                        sgw_solver_t** out)
{
    if (!p || !state_dev || !scratch_dev || !out) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if (((uintptr_t)state_dev & 255) || ((uintptr_t)scratch_dev & 255))
        return sgw_fail(SGW_ERR_INVALID_ARG, "device buffers must be 256-byte aligned");
    *out = nullptr;
    sgw_solver* s = new sgw_solver();
    s->plan = p;
    s->state = (unsigned char*)state_dev;
    s->scratch = (unsigned char*)scratch_dev;
    s->stream = (hipStream_t)hip_stream;
    const int d = p->pb.dim;
    const uint64_t rs = p->cfg.precision == SGW_FP64 ? 8 : 4;
    s->grids_d = (GridDev*)(s->scratch + p->off_grids);
    s->req_d = (ReqDev*)(s->scratch + p->off_req);
    s->items_d = (WorkItem*)(s->scratch + p->off_items);
    s->alpha_d = (unsigned long long*)(s->scratch + p->off_alpha);
    s->coef_d = (double*)(s->scratch + p->off_coef);
    s->coef_off_d = (int64_t*)(s->scratch + p->off_coef_off);
    s->pro_d = (ProDev*)(s->scratch + p->off_pro);
    s->fine_d = (FineDev*)(s->scratch + p->off_fine);
    s->partials_d = (double*)(s->scratch + p->off_partials);
    s->result_d = (double*)(s->scratch + p->off_result);
    s->foot_d = (double*)(s->scratch + p->off_foot);
    s->rho_items_d = (RhoItem*)(s->scratch + p->off_rho_items);
    s->plane_items_d = (WorkItem*)(s->scratch + p->off_plane_items);

    const bool dyn = p->pb.flux == SGW_FLUX_BURGERS;
    const int N = p->N;
    // grid descriptors
    s->grids_h = p->grids;
    for (int g = 0; g < p->G; g++) {
        GridDev& gd = s->grids_h[g];
        const uint64_t eoff = (uint64_t)p->offsets[g] * rs;
        gd.u = s->state + eoff;
        gd.a = s->state + p->copy_bytes + eoff;
        gd.b = s->state + 2 * p->copy_bytes + eoff;
        gd.alpha = s->alpha_d + 4 * g;
        gd.req = s->req_d;
        gd.flux = p->pb.flux;
        gd.dyn_alpha = dyn ? 1 : 0;
        gd.linear = p->cfg.linear_weights ? 1 : 0;
        gd.eps = p->cfg.eps_flux;
        for (int k = 0; k < SGW_MAX_DIM; k++) {
            gd.coef[k] = nullptr;
            gd.coef_src[k] = -1;
            gd.lin_c[k] = 0.0;
            gd.alpha_c[k] = 0.0;
            if (k >= d) continue;
            gd.lo[k] = p->pb.lo[k];
            gd.h[k] = (p->pb.hi[k] - p->pb.lo[k]) / gd.n[k];
            gd.inv_h[k] = 1.0 / gd.h[k];
            if (p->pb.flux == SGW_FLUX_ADVECTION) {
                gd.lin_c[k] = p->pb.flux_params[k];
                gd.alpha_c[k] = std::fabs(p->pb.flux_params[k]);
            } else if (p->pb.flux == SGW_FLUX_VLASOV_FIXED_E || p->pb.flux == SGW_FLUX_VLASOV_HARMONIC) {
                const int m = d / 2;
                gd.coef_src[k] = k < m ? m + k : k - m;
                gd.coef[k] = s->coef_d + p->coef_off[(size_t)g * SGW_MAX_DIM + k];
            } else if (p->vm && k == 0) {
                gd.coef_src[0] = 2;
                gd.coef[0] = s->coef_d + p->coef_off[(size_t)g * SGW_MAX_DIM];
            }
        }
        if (p->vm) gd.vm_alpha = (double*)(s->scratch + p->off_vm_alpha) + 6 * g;
    }
    // velocity moments (relaxation: the velocity factors and the density; Vlasov-Maxwell: the
    // currents), their partial sums per grid, work items
    std::vector<double> mu_h;
    std::vector<RhoItem> rho_items_h;
    if (p->relax || p->vm) {
        const double th = p->pb.relax_theta;
        const double norm1 = p->relax ? 1.0 / std::sqrt(2.0 * M_PI * th) : 0.0;
        double* mu_base = (double*)(s->scratch + p->off_mu);
        double* rho_base = (double*)(s->scratch + p->off_rho);
        double* part_base = (double*)(s->scratch + p->off_rho_part);
        int64_t rho_off = 0, part_off = 0;
        for (int g = 0; g < p->G; g++) {
            GridDev& gd = s->grids_h[g];
            gd.inv_tau = p->relax ? 1.0 / p->pb.relax_tau : 0.0;
            gd.hv = 1.0;
            for (int k = p->vm ? 1 : d / 2; k < d; k++) {
                gd.hv *= gd.h[k];
                if (!p->relax) continue;
                const int64_t o = p->mu_off[(size_t)g * SGW_MAX_DIM + k];
                gd.mu[k] = mu_base + o;
                if ((int64_t)mu_h.size() < o + gd.n[k]) mu_h.resize((size_t)(o + gd.n[k]));
                for (int j = 0; j < gd.n[k]; j++) {
                    const double v = gd.lo[k] + j * gd.h[k];
                    mu_h[(size_t)(o + j)] = std::exp(-v * v / (2.0 * th)) * norm1;
                }
            }
            gd.rho = rho_base + rho_off;
            gd.rho_part = part_base + part_off;
            rho_off += (int64_t)gd.nmom * gd.nxr;
            part_off += (int64_t)gd.nmom * gd.nxr * gd.rho_nchunk;
            for (int c = 0; c < gd.rho_nchunk; c++)
                for (int b = 0; b < gd.rho_cb; b++) rho_items_h.push_back(RhoItem{s->grids_d + g, b, c});
        }
        // second pass: one item per (grid, column block), after the first pass's
        for (int g = 0; g < p->G; g++)
            for (int b = 0; b < s->grids_h[g].rho_cb; b++) rho_items_h.push_back(RhoItem{s->grids_d + g, b, 0});
    }
    // time-step record
    std::memset(&s->req_h, 0, sizeof(ReqDev));
    s->req_h.cfl = p->cfg.cfl;
    s->req_h.d = d;
    s->req_h.dt_mode = p->cfg.dt_mode;
    s->req_h.grids = s->grids_d;
    s->req_h.alpha = s->alpha_d;
    s->req_h.ngrids = p->G;
    s->req_h.dyn_alpha = dyn ? 1 : 0;
    s->req_h.active = 1;
    s->req_h.vm = p->vm ? 1 : 0;
    double hmin = INFINITY;
    for (int k = 0; k < d; k++) {
        s->req_h.hfin[k] = (p->pb.hi[k] - p->pb.lo[k]) / N;
        hmin = s->req_h.hfin[k] < hmin ? s->req_h.hfin[k] : hmin;
    }
    s->req_h.dt_pow53 = std::pow(hmin, 5.0 / 3.0);
    // plane work list (4D): ppi consecutive planes per item, grid by grid
    s->plane_first.assign(p->G + 1, 0);
    std::vector<WorkItem> plane_items_h;
    for (int g = 0; g < p->G; g++) {
        s->plane_first[g] = (int)plane_items_h.size();
        if (!p->plane01) continue;
        const GridDev& gd = p->grids[g];
        for (int b = 0; b < (gd.nplanes + gd.ppi - 1) / gd.ppi; b++) plane_items_h.push_back(WorkItem{s->grids_d + g, b, 0});
    }
    s->plane_first[p->G] = (int)plane_items_h.size();
    // work list: boxes of every grid, grid by grid
    s->items_h.resize(p->nitems);
    for (int g = 0; g < p->G; g++)
        for (int b = 0; b < p->grids[g].nbox; b++) {
            WorkItem& it = s->items_h[p->grids[g].first_item + b];
            it.g = s->grids_d + g;
            it.box = b;
            it.pad = 0;
        }
    // prolongation descriptors
    s->pro_h.resize(p->G);
    for (int g = 0; g < p->G; g++) {
        ProDev& pd = s->pro_h[g];
        std::memset(&pd, 0, sizeof(pd));
        pd.u = s->grids_h[g].u;
        pd.coef = p->coefs[g];
        int load = 1;
        for (int k = 0; k < SGW_MAX_DIM; k++) {
            pd.n[k] = s->grids_h[g].n[k];
            pd.stride[k] = s->grids_h[g].stride[k];
            if (k < d) {
                pd.m[k] = p->cfg.finest_level - p->levels[g][k];
                pd.c[k] = coarse_extent(p->fine_T[k], pd.m[k], p->N);
            } else {
                pd.m[k] = 0;
                pd.c[k] = 1;
            }
            load *= pd.c[k];
            pd.fd_c[k] = make_fastdiv((uint32_t)pd.c[k]);
            pd.fd_n[k] = make_fastdiv((uint32_t)pd.n[k]);
        }
        pd.load_total = load;
        pd.rows = load / pd.c[0];
        pd.klast = last_refined(*p, g);
        for (int k = 0; k < SGW_MAX_DIM; k++) {
            int o = 1;
            for (int j = k + 1; j < SGW_MAX_DIM; j++) o *= pd.c[j];
            pd.outer[k] = o;
        }
    }
    std::memset(&s->fine_h, 0, sizeof(FineDev));
    s->fine_h.d = d;
    s->fine_h.N = N;
    s->fine_h.G = p->G;
    s->fine_h.lagrange = p->cfg.prolong == SGW_PROLONG_LAGRANGE5;
    s->fine_h.eps = p->cfg.eps_interp;
    s->fine_h.zmask = p->zmask;
    s->fine_h.pad0 = (int32_t)p->pro_buf_elems;
    s->fine_h.pad1 = (int32_t)p->pro_bufb_elems;
    int pts = 1;
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        s->fine_h.T[k] = p->fine_T[k];
        s->fine_h.ntile[k] = k < d ? N / p->fine_T[k] : 1;
        s->fine_h.inner[k] = pts;
        s->fine_h.fd_T[k] = make_fastdiv((uint32_t)p->fine_T[k]);
        s->fine_h.fd_inner[k] = make_fastdiv((uint32_t)pts);
        pts *= p->fine_T[k];
    }
    s->fine_h.tile_points = pts;
    s->fine_h.lines = p->fine_lines ? 1 : 0;
    s->fine_h.rows_max = (int32_t)p->pro_rows_max;
    s->fine_h.stab = s->scratch + p->off_stab;
    // per-point coefficient table: entry (R - 2) + q of R = 2^m holds s = (q - R/2)/R, s/2, s^2/2
    // and the linear weights C_r(s) = ((s-1)(s-2)/12, (4-s^2)/6, (s+1)(s+2)/12) of eq. (lwlag)
    std::vector<double> stab_h((size_t)8 * (((size_t)2 << p->cfg.finest_level) - 1), 0.0);
    for (int m = 1; m <= p->cfg.finest_level; m++) {
        const int R = 1 << m;
        for (int q = 0; q < R; q++) {
            const double sv = (double)(q - R / 2) / (double)R;
            double* e = &stab_h[(size_t)8 * (R - 2 + q)];
            e[0] = 0.5 * sv;
            e[1] = 0.5 * sv * sv;
            e[2] = (sv - 1.0) * (sv - 2.0) / 12.0;
            e[3] = (4.0 - sv * sv) / 6.0;
            e[4] = (sv + 1.0) * (sv + 2.0) / 12.0;
        }
    }
    if (p->cfg.precision == SGW_FP64) {
        s->stab_h.resize(sizeof(double) * stab_h.size());
        std::memcpy(s->stab_h.data(), stab_h.data(), s->stab_h.size());
    } else {
        std::vector<float> f(stab_h.begin(), stab_h.end());
        s->stab_h.resize(sizeof(float) * f.size());
        std::memcpy(s->stab_h.data(), f.data(), s->stab_h.size());
    }

    hipStream_t st = s->stream;
    sgw_status rc = SGW_OK;
    auto cp = [&](void* dst, const void* src, size_t n) {
        if (rc != SGW_OK || n == 0) return;
        hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) rc = sgw_hip_fail(e, "upload descriptors");
    };
    cp(s->grids_d, s->grids_h.data(), sizeof(GridDev) * p->G);
    cp(s->req_d, &s->req_h, sizeof(ReqDev));
    cp(s->items_d, s->items_h.data(), sizeof(WorkItem) * p->nitems);
    cp(s->coef_off_d, p->coef_off.data(), sizeof(int64_t) * p->coef_off.size());
    cp(s->pro_d, s->pro_h.data(), sizeof(ProDev) * p->G);
    cp(s->fine_d, &s->fine_h, sizeof(FineDev));
    cp(s->scratch + p->off_stab, s->stab_h.data(), s->stab_h.size());
    if (p->relax) cp(s->scratch + p->off_mu, mu_h.data(), sizeof(double) * mu_h.size());
    if (p->relax || p->vm) cp(s->rho_items_d, rho_items_h.data(), sizeof(RhoItem) * rho_items_h.size());
    if (p->plane01) cp(s->plane_items_d, plane_items_h.data(), sizeof(WorkItem) * plane_items_h.size());
    if (rc == SGW_OK && (p->pb.flux == SGW_FLUX_VLASOV_FIXED_E || p->pb.flux == SGW_FLUX_VLASOV_HARMONIC || p->vm)) {
        hipError_t e = launch_coef_init(s->grids_d, s->grids_h.data(), p->G, s->coef_d, s->coef_off_d, &p->pb, st);
        if (e != hipSuccess) rc = sgw_hip_fail(e, "coefficient tables");
        // the host mirrors the constant wave speeds to plan the number of steps
        std::vector<GridDev> back(p->G);
        if (rc == SGW_OK) {
            e = hipMemcpyAsync(back.data(), s->grids_d, sizeof(GridDev) * p->G, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = sgw_hip_fail(e, "read back wave speeds");
        }
        if (rc == SGW_OK)
            for (int g = 0; g < p->G; g++)
                for (int k = 0; k < SGW_MAX_DIM; k++) s->grids_h[g].alpha_c[k] = back[g].alpha_c[k];
    }
    if (rc == SGW_OK) {
        hipError_t e = hipHostMalloc((void**)&s->req_pinned, sizeof(ReqDev), hipHostMallocDefault);
        if (e != hipSuccess) rc = sgw_hip_fail(e, "pinned host record");
    }
    if (rc == SGW_OK) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = sgw_hip_fail(e, "solver set-up");
    }
    if (rc != SGW_OK) {
        sgw_solver_free(s);
        return rc;
    }
    s->grid = p->lds_boxed ? stage_grid(p->cfg.precision, p->pb.dim, p->lds_boxed, p->cfg.blocks_per_cu) : 1;
    s->grid_whole = p->lds_whole ? stage_grid(p->cfg.precision, p->pb.dim, p->lds_whole, p->cfg.blocks_per_cu, true) : 1;
    *out = s;
    return SGW_OK;
}

static void destroy_graph(sgw_solver* s)
{
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    s->graph_exec = nullptr;
    s->graph = nullptr;
    s->cap_stream = nullptr;
}

extern "C" void sgw_solver_free(sgw_solver_t* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    destroy_graph(s);
    if (s->req_pinned) (void)hipHostFree(s->req_pinned);
    delete s;
}

extern "C" sgw_status sgw_solver_set_stream(sgw_solver_t* s, void* hip_stream)
{
    if (!s) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver");
    if (s->batch_slot >= 0) return sgw_fail(SGW_ERR_STATE, "solver is in a batch");
    s->stream = (hipStream_t)hip_stream;
    return SGW_OK;
}

extern "C" sgw_status sgw_restrict_initial(sgw_solver_t* s)
{
    if (!s) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver");
    const sgw_plan* p = s->plan;
    HIPCHK(launch_fill_u64(s->alpha_d, 4 * (int64_t)p->G, 0ull, s->stream), "clear wave speeds");
    HIPCHK(launch_restrict(s->grids_d, s->grids_h.data(), p->G, p->cfg.precision, &p->pb, s->stream), "restrict");
    if (p->vm)
        HIPCHK(launch_vm_fields(s->grids_d, p->G, -1, p->cfg.precision, p->pb.ic_params[1], p->pb.ic_params[5],
                                p->cfg.linear_weights, s->stream),
               "initial fields");
    HIPCHK(launch_req_reset(s->req_d, s->stream), "reset time");
    s->restricted = true;
    s->t_host = 0.0;
    return SGW_OK;
}

extern "C" sgw_status sgw_set_grid(sgw_solver_t* s, int32_t g, const void* src_dev)
{
    if (!s || !src_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    const sgw_plan* p = s->plan;
    if (g < 0 || g >= p->G) return sgw_fail(SGW_ERR_INVALID_ARG, "grid %d outside 0..%d", g, p->G - 1);
    if (s->batch_slot >= 0) return sgw_fail(SGW_ERR_STATE, "solver is in a batch");
    const GridDev& gd = s->grids_h[g];
    int64_t n = 1;
    for (int k = 0; k < gd.d; k++) n *= gd.n[k];
    const size_t rs = p->cfg.precision == SGW_FP64 ? 8 : 4;
    HIPCHK(hipMemcpyAsync(gd.u, src_dev, (size_t)n * rs, hipMemcpyDeviceToDevice, s->stream), "copy grid values");
    HIPCHK(launch_fill_u64(s->alpha_d + 4 * g, 4, 0ull, s->stream), "clear wave speeds");
    if (gd.dyn_alpha) HIPCHK(launch_grid_absmax(s->grids_d + g, n, p->cfg.precision, s->stream), "wave speed");
    HIPCHK(launch_req_reset(s->req_d, s->stream), "reset time");
    s->restricted = true;
    s->t_host = 0.0;
    return SGW_OK;
}

static uint64_t snap_alpha_off(const sgw_plan* p) { return align256(p->copy_bytes); }
static uint64_t snap_req_off(const sgw_plan* p) { return snap_alpha_off(p) + align256(sizeof(unsigned long long) * 4 * p->G); }

extern "C" uint64_t sgw_snapshot_bytes(const sgw_solver_t* s)
{
    if (!s) return 0;
    return snap_req_off(s->plan) + align256(sizeof(ReqDev));
}

extern "C" sgw_status sgw_snapshot(sgw_solver_t* s, void* dst_dev)
{
    if (!s || !dst_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if (!s->restricted) return sgw_fail(SGW_ERR_STATE, "snapshot before restrict");
    // a batch advances the solver on the batch stream: a copy on the solver stream could tear
    if (s->batch_slot >= 0) return sgw_fail(SGW_ERR_STATE, "solver is in a batch");
    const sgw_plan* p = s->plan;
    unsigned char* d = (unsigned char*)dst_dev;
    HIPCHK(hipMemcpyAsync(d, s->state, p->copy_bytes, hipMemcpyDeviceToDevice, s->stream), "snapshot state");
    HIPCHK(hipMemcpyAsync(d + snap_alpha_off(p), s->alpha_d, sizeof(unsigned long long) * 4 * p->G,
                          hipMemcpyDeviceToDevice, s->stream),
           "snapshot wave speeds");
    HIPCHK(hipMemcpyAsync(d + snap_req_off(p), s->req_d, sizeof(ReqDev), hipMemcpyDeviceToDevice, s->stream),
           "snapshot time");
    return SGW_OK;
}

extern "C" sgw_status sgw_restore(sgw_solver_t* s, const void* src_dev)
{
    if (!s || !src_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if (s->batch_slot >= 0) return sgw_fail(SGW_ERR_STATE, "solver is in a batch");
    const sgw_plan* p = s->plan;
    const unsigned char* d = (const unsigned char*)src_dev;
    HIPCHK(hipMemcpyAsync(s->state, d, p->copy_bytes, hipMemcpyDeviceToDevice, s->stream), "restore state");
    HIPCHK(hipMemcpyAsync(s->alpha_d, d + snap_alpha_off(p), sizeof(unsigned long long) * 4 * p->G,
                          hipMemcpyDeviceToDevice, s->stream),
           "restore wave speeds");
    HIPCHK(launch_req_restore(s->req_d, (const ReqDev*)(d + snap_req_off(p)), s->stream), "restore time");
    s->restricted = true;
    return SGW_OK;
}

static sgw_status read_req(sgw_solver* s)
{
    HIPCHK(hipMemcpyAsync(s->req_pinned, s->req_d, sizeof(ReqDev), hipMemcpyDeviceToHost, s->stream), "read time");
    HIPCHK(hipStreamSynchronize(s->stream), "synchronise");
    s->t_host = s->req_pinned->t;
    return SGW_OK;
}

// Launch the work of one time step (dt + three stages) on stream st.
static hipError_t enqueue_step(sgw_solver* s, int mode, hipStream_t st)
{
    const sgw_plan* p = s->plan;
    hipError_t e = launch_dt_one(s->req_d, st);
    if (e != hipSuccess) return e;
    // relaxation: rho(x) of each stage's input, before the stage's line sweeps; Vlasov-Maxwell: the
    // currents of the stage input, then the stage's field update (it writes the next stage's fields
    // and speeds, which the sweeps of this stage do not read)
    const int nrho = (p->relax || p->vm) ? (int)p->nrho_items : 0;
    auto moments = [&](int stage) {
        hipError_t r = hipSuccess;
        if (nrho) r = launch_rho(s->rho_items_d, nrho, (int)p->nrho_final, stage, p->cfg.precision, st);
        if (r == hipSuccess && p->vm)
            r = launch_vm_fields(s->grids_d, p->G, stage, p->cfg.precision, 0.0, 0.0, p->cfg.linear_weights, st);
        return r;
    };
    const int first_dir = p->plane01 ? 2 : 0;
    if (mode == SGW_RUN_PLAIN) {
        for (int stage = 0; stage < 3; stage++) {
            e = moments(stage);
            if (e != hipSuccess) return e;
            for (int g = 0; g < p->G; g++) {
                if (p->plane01) {
                    e = launch_planes(s->plane_items_d + s->plane_first[g], s->plane_first[g + 1] - s->plane_first[g],
                                      stage, p->cfg.precision, st);
                    if (e != hipSuccess) return e;
                }
                e = launch_stage(s->items_d + p->grids[g].first_item, p->grids[g].nbox, stage, p->cfg.precision,
                                 p->pb.dim, stage_lds_bytes(p->grids[g], p->cfg.precision), 0, st,
                                 p->grids[g].line_mode != 0, first_dir);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    }
    // grids that are one box: all three stages in one launch; the others stage by stage
    const int nw = (int)p->nitems_whole, nbx = (int)(p->nitems - p->nitems_whole);
    if (nw) {
        e = launch_stage(s->items_d, nw, SGW_STAGE_FUSED, p->cfg.precision, p->pb.dim, p->lds_whole, s->grid_whole, st);
        if (e != hipSuccess) return e;
    }
    for (int stage = 0; stage < 3 && nbx; stage++) {
        e = moments(stage);
        if (e != hipSuccess) return e;
        if (p->plane01) {
            e = launch_planes(s->plane_items_d, (int)p->nplane_items, stage, p->cfg.precision, st);
            if (e != hipSuccess) return e;
        }
        e = launch_stage(s->items_d + nw, nbx, stage, p->cfg.precision, p->pb.dim, p->lds_boxed, s->grid, st,
                         p->line_mode, first_dir);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" sgw_status sgw_solver_launch_stage(sgw_solver_t* s, int32_t stage, int32_t part, int32_t reps)
{
    if (!s) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver");
    if (stage < 0 || stage > 2 || reps < 0) return sgw_fail(SGW_ERR_INVALID_ARG, "stage %d or reps %d", stage, reps);
    if (!s->restricted) return sgw_fail(SGW_ERR_STATE, "launch before restrict");
    const sgw_plan* p = s->plan;
    const int d = p->pb.dim;
    if (part < 0 || part > 1 + d || (part == 1 && !p->plane01) || (part >= 2 && !p->line_mode))
        return sgw_fail(SGW_ERR_INVALID_ARG, "part %d is not a part of this plan's stage", part);
    // reopen the solve so that every launch does its work
    HIPCHK(launch_req_set_final(s->req_d, INFINITY, s->stream), "reopen");
    const int nw = (int)p->nitems_whole, nbx = (int)(p->nitems - p->nitems_whole);
    for (int r = 0; r < reps; r++) {
        hipError_t e = hipSuccess;
        if (part == 0) {
            if (p->relax || p->vm) e = launch_rho(s->rho_items_d, (int)p->nrho_items, (int)p->nrho_final, stage,
                                                  p->cfg.precision, s->stream);
            if (e == hipSuccess && p->vm)
                e = launch_vm_fields(s->grids_d, p->G, stage, p->cfg.precision, 0.0, 0.0, p->cfg.linear_weights,
                                     s->stream);
            if (e == hipSuccess && p->plane01)
                e = launch_planes(s->plane_items_d, (int)p->nplane_items, stage, p->cfg.precision, s->stream);
            if (e == hipSuccess && nw)
                e = launch_stage(s->items_d, nw, SGW_STAGE_FUSED, p->cfg.precision, d, p->lds_whole, s->grid_whole,
                                 s->stream);
            if (e == hipSuccess && nbx)
                e = launch_stage(s->items_d + nw, nbx, stage, p->cfg.precision, d, p->lds_boxed, s->grid, s->stream,
                                 p->line_mode, p->plane01 ? 2 : 0);
        } else if (part == 1) {
            e = launch_planes(s->plane_items_d, (int)p->nplane_items, stage, p->cfg.precision, s->stream);
        } else {
            e = launch_stage(s->items_d + nw, nbx, stage, p->cfg.precision, d, p->lds_boxed, s->grid, s->stream, true,
                             part - 2, part - 2);
        }
        if (e != hipSuccess) return sgw_hip_fail(e, "measured stage launch");
    }
    return SGW_OK;
}

static sgw_status build_graph(sgw_solver* s, int steps_per_graph)
{
    destroy_graph(s);
    HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking), "capture stream");
    HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t e = hipSuccess;
    for (int i = 0; i < steps_per_graph && e == hipSuccess; i++) e = enqueue_step(s, SGW_RUN_FUSED, s->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
    if (e != hipSuccess) return sgw_hip_fail(e, "capture step");
    if (e2 != hipSuccess) return sgw_hip_fail(e2, "end capture");
    s->graph = g;
    HIPCHK(hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0), "instantiate graph");
    s->graph_steps = steps_per_graph;
    return SGW_OK;
}

// Number of steps the shared-dt loop takes from t to T when every wave speed is
// constant (the same arithmetic the device performs).
static int64_t planned_steps(const sgw_solver* s, double t, double T)
{
    const sgw_plan* p = s->plan;
    const ReqDev& r = s->req_h;
    double dt;
    if (r.dt_mode == SGW_DT_POW53) {
        dt = r.dt_pow53;
    } else {
        double denom = 0.0;
        for (int k = 0; k < r.d; k++) {
            double A = 0.0;
            for (int g = 0; g < p->G; g++) {
                double a;
                if (r.dyn_alpha) {
                    // bound of max|u0| for a sine initial condition; only an estimate
                    a = std::fabs(p->pb.ic_params[0]) + std::fabs(p->pb.ic_params[1]);
                } else {
                    a = s->grids_h[g].alpha_c[k];
                }
                A = a > A ? a : A;
            }
            denom += A / r.hfin[k];
        }
        dt = denom > 0.0 ? r.cfl / denom : T - t;
    }
    int64_t n = 0;
    const double tol = 1e-12 * (T > 1.0 ? T : 1.0);
    while (T - t > tol && n < 10000000) {
        double d = dt > T - t ? T - t : dt;
        t += d;
        n++;
    }
    return n;
}

extern "C" sgw_status sgw_advance(sgw_solver_t* s, double t_final, int32_t mode)
{
    if (!s) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver");
    if (!s->restricted) return sgw_fail(SGW_ERR_STATE, "advance before restrict");
    if (mode < SGW_RUN_PLAIN || mode > SGW_RUN_GRAPH) return sgw_fail(SGW_ERR_INVALID_ARG, "unknown mode %d", mode);
    if (!(t_final >= 0.0) || !std::isfinite(t_final)) return sgw_fail(SGW_ERR_INVALID_ARG, "bad final time");
    HIPCHK(launch_req_set_final(s->req_d, t_final, s->stream), "set final time");
    sgw_status rc = read_req(s);
    if (rc != SGW_OK) return rc;
    if (s->req_pinned->nonfinite) return sgw_fail(SGW_ERR_NONFINITE, "non-finite wave speed");
    int64_t todo = planned_steps(s, s->t_host, t_final);
    if (mode == SGW_RUN_GRAPH && !s->graph_exec) {
        rc = build_graph(s, 4);
        if (rc != SGW_OK) return rc;
    }
    int64_t launched = 0;
    for (;;) {
        if (launched > 10000000) return sgw_fail(SGW_ERR_STATE, "more than 1e7 steps without reaching t_final");
        launched += todo;
        if (mode == SGW_RUN_GRAPH) {
            for (int64_t i = 0; i < todo; i += s->graph_steps)
                HIPCHK(hipGraphLaunch(s->graph_exec, s->stream), "graph launch");
        } else {
            for (int64_t i = 0; i < todo; i++) HIPCHK(enqueue_step(s, mode, s->stream), "step");
        }
        rc = read_req(s);
        if (rc != SGW_OK) return rc;
        if (s->req_pinned->nonfinite) return sgw_fail(SGW_ERR_NONFINITE, "non-finite wave speed or time step");
        if (s->req_pinned->done) break;
        // state-dependent speeds: the steps the last dt would take to t_final (at least 4), then
        // look again; steps past the end return at once
        todo = 4;
        const double dtl = s->req_pinned->dt, rem = t_final - s->req_pinned->t;
        if (dtl > 0.0 && rem > 0.0 && rem / dtl < 1e6) {
            const int64_t est = (int64_t)(0.9 * rem / dtl);
            todo = est > todo ? est : todo;
        }
    }
    return SGW_OK;
}

static int64_t fine_tiles(const sgw_solver* s);

extern "C" sgw_status sgw_prolongate_combine_tiles(sgw_solver_t* s, double* out_dev, int64_t first_tile,
                                                   int64_t num_tiles)
{
    if (!s || !out_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if (!s->restricted) return sgw_fail(SGW_ERR_STATE, "prolongate before restrict");
    const int64_t nt = fine_tiles(s);
    if (first_tile < 0 || num_tiles < 0 || first_tile > nt || num_tiles > nt - first_tile)
        return sgw_fail(SGW_ERR_INVALID_ARG, "tiles %lld + %lld outside 0..%lld", (long long)first_tile,
                        (long long)num_tiles, (long long)nt);
    if (nt > 0x7fffffff) return sgw_fail(SGW_ERR_UNSUPPORTED, "too many tiles");
    const sgw_plan* p = s->plan;
    HIPCHK(launch_prolong(s->pro_d, s->fine_d, s->fine_h, p->cfg.precision, p->pro_lds, out_dev, (int)first_tile,
                          (int)num_tiles, s->stream),
           "prolongate");
    return SGW_OK;
}

extern "C" sgw_status sgw_prolongate_combine(sgw_solver_t* s, double* out_dev)
{
    if (!s || !out_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    return sgw_prolongate_combine_tiles(s, out_dev, 0, fine_tiles(s));
}

extern "C" sgw_status sgw_exact(sgw_solver_t* s, double t, double* out_dev)
{
    if (!s || !out_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    const sgw_plan* p = s->plan;
    if (p->pb.flux == SGW_FLUX_BURGERS && p->pb.ic != SGW_IC_SINE)
        return sgw_fail(SGW_ERR_UNSUPPORTED, "Burgers exact solution needs a sine initial condition");
    if (p->pb.flux == SGW_FLUX_VLASOV_FIXED_E && p->pb.ic != SGW_IC_MAXWELL_COS)
        return sgw_fail(SGW_ERR_UNSUPPORTED, "Vlasov exact solution needs the Maxwellian initial condition");
    if (p->pb.flux == SGW_FLUX_VLASOV_HARMONIC || p->pb.ic == SGW_IC_VLASOV_BOLTZMANN || p->relax || p->zmask)
        return sgw_fail(SGW_ERR_UNSUPPORTED, "no closed-form solution for the Vlasov-Boltzmann model");
    if (p->vm) return sgw_fail(SGW_ERR_UNSUPPORTED, "no closed-form solution for the Vlasov-Maxwell system");
    ExactDev e;
    std::memset(&e, 0, sizeof(e));
    e.d = p->pb.dim;
    e.flux = p->pb.flux;
    e.ic = p->pb.ic;
    e.N = p->N;
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        e.lo[k] = p->pb.lo[k];
        e.h[k] = k < e.d ? (p->pb.hi[k] - p->pb.lo[k]) / p->N : 0.0;
        e.fp[k] = p->pb.flux_params[k];
    }
    for (int i = 0; i < 8; i++) e.ip[i] = p->pb.ic_params[i];
    e.t = t;
    HIPCHK(launch_exact(e, out_dev, s->foot_d, s->stream), "exact solution");
    return SGW_OK;
}

extern "C" sgw_status sgw_fields_combine(sgw_solver_t* s, double* out_dev)
{
    if (!s || !out_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    const sgw_plan* p = s->plan;
    if (!p->vm) return sgw_fail(SGW_ERR_INVALID_ARG, "the plan carries no fields");
    if (!s->restricted) return sgw_fail(SGW_ERR_STATE, "fields before restrict");
    HIPCHK(launch_fields_combine(s->grids_d, s->pro_d, s->fine_h, s->fine_d, out_dev, s->stream), "fields combine");
    return SGW_OK;
}

extern "C" sgw_status sgw_plan_fields(const sgw_plan_t* p, uint64_t* offset_bytes, int64_t* count)
{
    if (!p) return sgw_fail(SGW_ERR_INVALID_ARG, "null plan");
    if (offset_bytes) *offset_bytes = p->fields_off;
    if (count) *count = p->fields_total;
    return SGW_OK;
}

extern "C" sgw_status sgw_entropies(sgw_solver_t* s, const double* f, double* result_host)
{
    if (!s || !f || !result_host) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    const sgw_plan* p = s->plan;
    const int d = p->pb.dim;
    const double th = p->pb.relax_theta;
    if (d % 2) return sgw_fail(SGW_ERR_INVALID_ARG, "entropies need an even dim (x and v)");
    if (!(th > 0.0) || !std::isfinite(th)) return sgw_fail(SGW_ERR_INVALID_ARG, "relax_theta %g must be > 0", th);
    // int_x exp(-|x|^2/(2 theta)) dx over the x domain: a product of erf differences
    double zx = 1.0;
    for (int k = 0; k < d / 2; k++)
        zx *= std::sqrt(0.5 * M_PI * th) *
              (std::erf(p->pb.hi[k] / std::sqrt(2.0 * th)) - std::erf(p->pb.lo[k] / std::sqrt(2.0 * th)));
    HIPCHK(launch_entropies(s->fine_h, p->pb.lo, p->pb.hi, th, zx, f, s->partials_d, s->result_d, s->stream),
           "entropies");
    HIPCHK(hipMemcpyAsync(result_host, s->result_d, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream),
           "read entropies");
    HIPCHK(hipStreamSynchronize(s->stream), "synchronise");
    return SGW_OK;
}

extern "C" sgw_status sgw_norms(sgw_solver_t* s, const double* a, const double* b, double* result_host)
{
    if (!s || !a || !b || !result_host) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    HIPCHK(launch_norms(a, b, s->plan->fine_nodes, s->partials_d, s->result_d, s->stream), "norms");
    HIPCHK(hipMemcpyAsync(result_host, s->result_d, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream),
           "read norms");
    HIPCHK(hipStreamSynchronize(s->stream), "synchronise");
    return SGW_OK;
}

extern "C" sgw_status sgw_query(sgw_solver_t* s, double* t, int64_t* steps)
{
    if (!s) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver");
    sgw_status rc = read_req(s);
    if (rc != SGW_OK) return rc;
    if (t) *t = s->req_pinned->t;
    if (steps) *steps = s->req_pinned->steps;
    if (s->req_pinned->nonfinite) return sgw_fail(SGW_ERR_NONFINITE, "non-finite wave speed or time step");
    return SGW_OK;
}

extern "C" sgw_status sgw_norms_async(sgw_solver_t* s, const double* a, const double* b, double* result_dev)
{
    if (!s || !a || !b || !result_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    HIPCHK(launch_norms(a, b, s->plan->fine_nodes, s->partials_d, result_dev, s->stream), "norms");
    return SGW_OK;
}

static int64_t fine_tiles(const sgw_solver* s)
{
    int64_t t = 1;
    for (int k = 0; k < s->fine_h.d; k++) t *= s->fine_h.ntile[k];
    return t;
}

extern "C" uint64_t sgw_prolongate_many_scratch_bytes(sgw_solver_t* const* solvers, int32_t n)
{
    if (!solvers || n <= 0) return 0;
    return align256((uint64_t)n * sizeof(ProItem));
}

// `later` waits (an event, no host wait) for the work already enqueued on `earlier`.
static hipError_t stream_wait(hipStream_t later, hipStream_t earlier)
{
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    e = hipEventRecord(ev, earlier);
    if (e == hipSuccess) e = hipStreamWaitEvent(later, ev, 0);
    // an event may be destroyed once the wait is enqueued
    (void)hipEventDestroy(ev);
    return e;
}

// A many-solve call on stream st and the solvers' own streams: before the call st waits for
// each distinct solver stream that differs from it (after = false); after the call each such
// stream waits for st (after = true), so the solver's later calls follow the launch.
static hipError_t order_solver_streams(hipStream_t st, sgw_solver_t* const* solvers, int n, bool after)
{
    std::vector<hipStream_t> done;
    for (int i = 0; i < n; i++) {
        hipStream_t ss = solvers[i]->stream;
        if (ss == st || std::find(done.begin(), done.end(), ss) != done.end()) continue;
        const hipError_t e = after ? stream_wait(ss, st) : stream_wait(st, ss);
        if (e != hipSuccess) return e;
        done.push_back(ss);
    }
    return hipSuccess;
}

extern "C" sgw_status sgw_prolongate_combine_many(sgw_solver_t* const* solvers, double* const* outs, int32_t n,
                                                  void* scratch_dev, uint64_t scratch_bytes, void* hip_stream)
{
    if (!solvers || !outs || n <= 0 || !scratch_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if ((uintptr_t)scratch_dev & 255) return sgw_fail(SGW_ERR_INVALID_ARG, "scratch must be 256-byte aligned");
    const int d = solvers[0] ? solvers[0]->plan->pb.dim : 0;
    const int prec = solvers[0] ? solvers[0]->plan->cfg.precision : 0;
    if (n > 65535) return sgw_fail(SGW_ERR_INVALID_ARG, "at most 65535 solves per call, %d given", n);
    size_t lds = 0;
    int64_t max_tiles = 0;
    for (int i = 0; i < n; i++) {
        sgw_solver* s = solvers[i];
        if (!s || !outs[i]) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver or output %d", i);
        if (!s->restricted) return sgw_fail(SGW_ERR_STATE, "prolongate before restrict (solver %d)", i);
        if (s->plan->pb.dim != d || s->plan->cfg.precision != prec)
            return sgw_fail(SGW_ERR_INVALID_ARG, "solvers of one call must share dimension and precision");
        const size_t l = s->plan->pro_lds;
        lds = l > lds ? l : lds;
        const int64_t t = fine_tiles(s);
        max_tiles = t > max_tiles ? t : max_tiles;
    }
    if ((uint64_t)n * sizeof(ProItem) > scratch_bytes)
        return sgw_fail(SGW_ERR_OUT_OF_MEMORY, "scratch of %llu bytes, %llu needed", (unsigned long long)scratch_bytes,
                        (unsigned long long)((uint64_t)n * sizeof(ProItem)));
    if (max_tiles > 0x7fffffff) return sgw_fail(SGW_ERR_UNSUPPORTED, "too many tiles");
    Staging stg((size_t)n * sizeof(ProItem));
    HIPCHK(stg.err, "staging buffer");
    ProItem* items = (ProItem*)stg.host;
    for (int i = 0; i < n; i++)
        items[i] = ProItem{solvers[i]->pro_d, solvers[i]->fine_d, outs[i], (int32_t)fine_tiles(solvers[i]), 0};
    hipStream_t st = (hipStream_t)hip_stream;
    // the tiles read each solve's state after the work enqueued on its own stream
    HIPCHK(order_solver_streams(st, solvers, n, false), "order after solver streams");
    HIPCHK(stg.upload(0, scratch_dev, (size_t)n * sizeof(ProItem), st), "upload solve list");
    HIPCHK(launch_prolong_many((const ProItem*)scratch_dev, n, (int)max_tiles, d, prec, lds, st), "prolongate many");
    HIPCHK(order_solver_streams(st, solvers, n, true), "order solver streams after the launch");
    return SGW_OK;
}

// ---------------------------------------------------------------- restriction and norms of many solves

static const int64_t RESTRICT_CHUNK = 8 * SGW_BLOCK;

static int64_t restrict_chunks(const sgw_solver* s)
{
    int64_t c = 0;
    for (const GridDev& g : s->grids_h) {
        int64_t n = 1;
        for (int k = 0; k < g.d; k++) n *= g.n[k];
        c += (n + RESTRICT_CHUNK - 1) / RESTRICT_CHUNK;
    }
    return c;
}

extern "C" uint64_t sgw_restrict_many_scratch_bytes(sgw_solver_t* const* solvers, int32_t n)
{
    if (!solvers || n <= 0) return 0;
    int64_t chunks = 0;
    for (int i = 0; i < n; i++)
        if (solvers[i]) chunks += restrict_chunks(solvers[i]);
    return align256((uint64_t)n * sizeof(ResetItem)) + align256((uint64_t)chunks * sizeof(RestrictItem));
}

extern "C" sgw_status sgw_restrict_initial_many(sgw_solver_t* const* solvers, int32_t n, void* scratch_dev,
                                                uint64_t scratch_bytes, void* hip_stream)
{
    if (!solvers || n <= 0 || !scratch_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if ((uintptr_t)scratch_dev & 255) return sgw_fail(SGW_ERR_INVALID_ARG, "scratch must be 256-byte aligned");
    const int prec = solvers[0] ? solvers[0]->plan->cfg.precision : 0;
    for (int i = 0; i < n; i++) {
        if (!solvers[i]) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver %d", i);
        if (solvers[i]->plan->cfg.precision != prec)
            return sgw_fail(SGW_ERR_INVALID_ARG, "solvers of one call must share their precision");
        if (solvers[i]->plan->vm)
            return sgw_fail(SGW_ERR_UNSUPPORTED, "Vlasov-Maxwell solvers restrict alone (sgw_restrict_initial)");
    }
    const uint64_t need = sgw_restrict_many_scratch_bytes(solvers, n);
    if (need > scratch_bytes)
        return sgw_fail(SGW_ERR_OUT_OF_MEMORY, "scratch of %llu bytes, %llu needed", (unsigned long long)scratch_bytes,
                        (unsigned long long)need);
    const uint64_t off_items = align256((uint64_t)n * sizeof(ResetItem));
    const int64_t nchunks = (int64_t)((need - off_items) / sizeof(RestrictItem));
    if (nchunks > 0x7fffffff) return sgw_fail(SGW_ERR_UNSUPPORTED, "too many restriction chunks");
    Staging stg(need);
    HIPCHK(stg.err, "staging buffer");
    ResetItem* resets = (ResetItem*)stg.host;
    RestrictItem* items = (RestrictItem*)(stg.host + off_items);
    int64_t c = 0;
    for (int i = 0; i < n; i++) {
        sgw_solver* s = solvers[i];
        resets[i] = ResetItem{s->alpha_d, s->req_d, 4 * s->plan->G, 0};
        for (int g = 0; g < s->plan->G; g++) {
            const GridDev& gd = s->grids_h[g];
            int64_t total = 1;
            for (int k = 0; k < gd.d; k++) total *= gd.n[k];
            for (int64_t st = 0; st < total; st += RESTRICT_CHUNK) {
                RestrictItem& it = items[c++];
                it.g = s->grids_d + g;
                it.start = st;
                it.count = (int32_t)(total - st < RESTRICT_CHUNK ? total - st : RESTRICT_CHUNK);
                it.ic = s->plan->pb.ic;
                for (int q = 0; q < 8; q++) it.ip[q] = s->plan->pb.ic_params[q];
            }
        }
    }
    hipStream_t st = (hipStream_t)hip_stream;
    // earlier work of each solve on its own stream may still read its state
    HIPCHK(order_solver_streams(st, solvers, n, false), "order after solver streams");
    HIPCHK(stg.upload(0, scratch_dev, need, st), "upload restriction list");
    const unsigned char* base = (const unsigned char*)scratch_dev;
    HIPCHK(launch_restrict_many((const ResetItem*)base, n, (const RestrictItem*)(base + off_items), (int)c, prec, st),
           "restrict many");
    HIPCHK(order_solver_streams(st, solvers, n, true), "order solver streams after the launch");
    for (int i = 0; i < n; i++) {
        solvers[i]->restricted = true;
        solvers[i]->t_host = 0.0;
    }
    return SGW_OK;
}

static int norms_many_max_parts(sgw_solver_t* const* solvers, int32_t n)
{
    int mp = 1;
    for (int i = 0; i < n; i++)
        if (solvers[i]) {
            const int p = norms_parts(solvers[i]->plan->fine_nodes);
            mp = p > mp ? p : mp;
        }
    return mp;
}

extern "C" uint64_t sgw_norms_many_scratch_bytes(sgw_solver_t* const* solvers, int32_t n)
{
    if (!solvers || n <= 0) return 0;
    const int mp = norms_many_max_parts(solvers, n);
    return align256((uint64_t)n * sizeof(NormItem)) + align256((uint64_t)n * 2 * mp * sizeof(double));
}

extern "C" sgw_status sgw_norms_many(sgw_solver_t* const* solvers, const double* const* a, const double* const* b,
                                     int32_t n, double* result_dev, void* scratch_dev, uint64_t scratch_bytes,
                                     void* hip_stream)
{
    if (!solvers || !a || !b || n <= 0 || !result_dev || !scratch_dev)
        return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if (n > 65535) return sgw_fail(SGW_ERR_INVALID_ARG, "at most 65535 pairs per call, %d given", n);
    if ((uintptr_t)scratch_dev & 255) return sgw_fail(SGW_ERR_INVALID_ARG, "scratch must be 256-byte aligned");
    for (int i = 0; i < n; i++)
        if (!solvers[i] || !a[i] || !b[i]) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver or array %d", i);
    const uint64_t need = sgw_norms_many_scratch_bytes(solvers, n);
    if (need > scratch_bytes)
        return sgw_fail(SGW_ERR_OUT_OF_MEMORY, "scratch of %llu bytes, %llu needed", (unsigned long long)scratch_bytes,
                        (unsigned long long)need);
    const int mp = norms_many_max_parts(solvers, n);
    Staging stg(sizeof(NormItem) * (size_t)n);
    HIPCHK(stg.err, "staging buffer");
    NormItem* items = (NormItem*)stg.host;
    for (int i = 0; i < n; i++) {
        const int64_t cnt = solvers[i]->plan->fine_nodes;
        items[i] = NormItem{a[i], b[i], cnt, result_dev + 2 * (size_t)i, norms_parts(cnt), 0};
    }
    hipStream_t st = (hipStream_t)hip_stream;
    HIPCHK(order_solver_streams(st, solvers, n, false), "order after solver streams");
    unsigned char* base = (unsigned char*)scratch_dev;
    HIPCHK(stg.upload(0, base, sizeof(NormItem) * (size_t)n, st), "upload norm list");
    HIPCHK(launch_norms_many((const NormItem*)base, n, mp, (double*)(base + align256((uint64_t)n * sizeof(NormItem))),
                             st),
           "norms many");
    return SGW_OK;
}
