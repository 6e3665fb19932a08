// Internal definitions of libsgweno shared by its host and device sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sgweno.h"
#include "sgweno_measure.h"

#define SGW_BLOCK 256     // threads per workgroup of every kernel (4 wave64)
#define SGW_MAXR 8        // nodes per thread in the stage kernel: box core <= SGW_BLOCK * SGW_MAXR
#define SGW_NPART 1024    // most workgroups of the first norm pass (their count depends on n only)
#define SGW_STAGE_FUSED 3 // stage index of the launch that runs all three stages of whole-grid boxes
#define SGW_SEG 4         // interfaces per thread of the flux sweep (sliding window), d <= 3

// Interfaces per thread of the flux sweep of a d-dimensional grid.  4D boxes are short
// (4 or 8 nodes) in most directions, so 4 + 1 interfaces fill one segment of 5.  A box that
// spans its grid has t = n >= 4 nodes, which keeps every window position of the periodic
// wrap within two subtractions of t for both lengths.
__host__ __device__ constexpr int sgw_seg(int d) { return d == 4 ? 5 : SGW_SEG; }

// Division by a run-time constant d >= 1 for numerators below 2^31:
// q = (umulhi(x, m) + x) >> s with s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, s, pad;
};

static inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) s++;
    f.s = s;
    f.m = (uint32_t)((((1ull << s) - d) << 32) / d + 1);
    f.pad = 0;
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, FastDiv f)
{
    return (__umulhi(x, f.m) + x) >> f.s;
}

__device__ __forceinline__ uint32_t fdiv_ms(uint32_t x, uint32_t m, uint32_t s)
{
    return (__umulhi(x, m) + x) >> s;
}

// the same through a descriptor field of any address space
#define FDIV(x, f) fdiv_ms((uint32_t)(x), (f).m, (f).s)

struct ReqDev;

// max that keeps a NaN (a NaN wave speed must reach the time-step check)
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Max over the workgroup, then one atomic max on the bit pattern (non-negative
// doubles order like their unsigned bit patterns; NaN sorts above everything).
__device__ __forceinline__ void block_atomic_max(double v, unsigned long long* dst, double* red)
{
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < SGW_BLOCK / 64; w++) m = nanmax(m, red[w]);
        atomicMax(dst, (unsigned long long)__double_as_longlong(m));
    }
}

// One component grid as seen by the stage kernel.  Box = the tile one
// workgroup updates; t[k] divides n[k]; a box that does not span its grid in
// direction k carries 3 halo nodes on each side in that direction.  LDS holds
// the core box (row-major, strides CS) followed, for every such direction, by
// a low and a high slab: the core box with extent 3 in direction k.
struct alignas(64) GridDev {
    void* u;                         // u^n (also the output of stage 3)
    void* a;                         // output of stage 1
    void* b;                         // output of stage 2
    unsigned long long* alpha;       // [4]: slots 0..2 hold max|u| bits of the input of stage s
    ReqDev* req;                     // the solve this grid belongs to
    const double* coef[SGW_MAX_DIM]; // linear flux coefficient per node of direction coef_src[k]
    int32_t d, flux, dyn_alpha, linear;
    int32_t nbox, pad_total, core_total, first_item;
    int32_t n[SGW_MAX_DIM];
    int32_t stride[SGW_MAX_DIM];
    int32_t t[SGW_MAX_DIM];
    int32_t halo[SGW_MAX_DIM];       // 3 or 0
    int32_t ntile[SGW_MAX_DIM];
    int32_t slab_lo[SGW_MAX_DIM];    // LDS offset of the low / high halo slab of direction k
    int32_t slab_hi[SGW_MAX_DIM];
    int32_t CS[SGW_MAX_DIM];         // core strides
    int32_t I[SGW_MAX_DIM];          // interfaces per line in the box: t + (halo ? 1 : 0)
    int32_t flux_total[SGW_MAX_DIM]; // interfaces in the box per direction
    int32_t coef_src[SGW_MAX_DIM];   // direction whose node index selects the coefficient, -1: constant
    int32_t nseg[SGW_MAX_DIM];       // segments of sgw_seg(d) interfaces per line
    int32_t seg_total[SGW_MAX_DIM];  // work items of the segment loop: lines * nseg[k]
    int32_t LS[SGW_MAX_DIM];         // LDS strides of the core box (row stride RS)
    int32_t slab_n[SGW_MAX_DIM];     // values per halo slab (3 core / t_k)
    int32_t RS, lines, F0S, whole;   // LDS row stride of core and direction-1 fluxes (odd: conflict-free
                                     // columns), rows (core / t_0), F0S = RS, box = grid
    int32_t sf_elems, rline;         // elements of one interface-flux buffer (two alternate in LDS);
                                     // SGW_BLOCK / t_0 when t_0 divides SGW_BLOCK, else 0
    int32_t nlines[SGW_MAX_DIM];     // lines of the box along direction k: core / t_k
    int32_t rt_off[SGW_MAX_DIM];     // 3D/4D: offset of the slab-row table of direction k in the row tables
    int32_t rt_total, pad2_;         // 3D/4D: ints of the row tables (core rows, then slab rows)
    int32_t nint[SGW_MAX_DIM];       // interior segments per line (window inside the core, no wrap)
    FastDiv fd_lines;
    FastDiv fd_lines_k[SGW_MAX_DIM];
    FastDiv fd_nseg[SGW_MAX_DIM];
    FastDiv fd_CS[SGW_MAX_DIM];
    FastDiv fd_t[SGW_MAX_DIM];
    FastDiv fd_I[SGW_MAX_DIM];
    FastDiv fd_CSt[SGW_MAX_DIM];     // CS[k] * t[k]
    FastDiv fd_n[SGW_MAX_DIM];
    double lo[SGW_MAX_DIM];
    double h[SGW_MAX_DIM];
    double inv_h[SGW_MAX_DIM];
    double lin_c[SGW_MAX_DIM];       // constant coefficient of a linear flux (advection)
    double alpha_c[SGW_MAX_DIM];     // constant LF speed max|f_k'| (advection, Vlasov)
    double eps;
    // line sweep (4D grids): one launch per direction k, a lane per segment of sgw_lseg() nodes
    // of a grid line along k, SGW_LWAVE segments per work item
    int32_t line_mode;
    int32_t pow2_mask;               // bit k: n[k] is a power of two (periodic wrap by a mask)
    int32_t lsegl[SGW_MAX_DIM];      // segments per line along k: ceil(n[k] / sgw_lseg(precision))
    int32_t ltrans[SGW_MAX_DIM];     // lines along k: prod_{j != k} n[j]
    FastDiv fd_lsegl[SGW_MAX_DIM];
    FastDiv fd_ltrans[SGW_MAX_DIM];
    // zero boundary and the relaxation source of the Vlasov-Boltzmann model (line sweep only)
    int32_t zmask;                   // bit k: every value beyond either end of direction k is 0
    int32_t relax;                   // 1: the last direction adds (mu_inf(v) rho(x) - u) / tau
    int32_t nxr, nvr;                // x nodes (prod of the x extents) and velocity nodes
    int32_t rho_cb, rho_nchunk;      // moment launch: blocks of SGW_RHO_COLS x nodes, chunks of rows
    const double* mu[SGW_MAX_DIM];   // velocity direction k: exp(-v^2/(2 theta)) / sqrt(2 pi theta) per node
    double* rho;                     // nmom x nxr: the velocity moments of the current stage input
    double* rho_part;                // nmom x rho_nchunk x nxr partial sums
    double inv_tau, hv;              // 1 / tau and the velocity cell volume
    // Vlasov-Maxwell (d = 3: x_2, xi_1, xi_2): the grid's fields B_3, E_1, E_2 at its n[0] x_2 nodes,
    // FP64, fld_bytes past the grid's first node in each state copy
    int32_t vm, nmom;                // nmom: moments of the moment launch (1: rho; 2: j_1, j_2)
    int64_t fld_bytes;
    double* vm_alpha;                // [3 stages][2]: LF speeds of xi_1, xi_2 of each stage's fields
    // 4D plane launch: directions 1 and 2 of a stage over whole (x_1, x_2) planes in LDS, ppi
    // consecutive planes (n[0] n[1] nodes each, contiguous) per work item
    int32_t ppi, nplanes, plane_nodes, pad3_;
};

// nodes of one plane-launch work item (its planes staged in LDS, with their flux sums)
#ifndef SGW_PLANE_CAP
#define SGW_PLANE_CAP 2048
#endif

// density launch: SGW_RHO_COLS x nodes per workgroup, SGW_BLOCK / SGW_RHO_COLS row lanes,
// SGW_RHO_RPT rows per lane and chunk
#define SGW_RHO_COLS 64
#define SGW_RHO_RPT 16
#define SGW_RHO_CHUNK (SGW_RHO_RPT * (SGW_BLOCK / SGW_RHO_COLS))

// One (grid, block of x nodes, chunk of velocity rows) of the density's first pass, or one (grid,
// block of x nodes) of its second (chunk unused).
struct RhoItem {
    const GridDev* g;
    int32_t cb, chunk;
};

// nodes per segment of the line sweep: 4 in FP64 (fewer registers, more resident waves: 4 % faster
// on the 4D Vlasov march than 8), 8 in FP32
#ifndef SGW_LSEG64
#define SGW_LSEG64 4
#endif
#ifndef SGW_LSEG32
#define SGW_LSEG32 8
#endif
__host__ __device__ constexpr int sgw_lseg(bool fp64) { return fp64 ? SGW_LSEG64 : SGW_LSEG32; }
#define SGW_LWAVE 64  // segments (lanes) per work item of the line sweep: one wavefront

// Per-solve time-stepping record, written only by the device after set-up.
struct alignas(64) ReqDev {
    double t, T, dt, cfl, dt_pow53;
    double hfin[SGW_MAX_DIM];
    int64_t steps;
    const GridDev* grids;
    const unsigned long long* alpha; // the solve's wave-speed slots, 4 per grid (slot 0: max |u^n|)
    int32_t ngrids, d, dt_mode, done;
    int32_t nonfinite, dyn_alpha, active, vm; // vm: speeds of the xi directions from the fields
};

struct WorkItem {
    const GridDev* g;
    int32_t box;
    int32_t pad;
};

// One component grid as seen by the prolongation-combination kernel.
struct alignas(64) ProDev {
    const void* u;
    int32_t coef;
    int32_t load_total;              // prod c[k]
    int32_t m[SGW_MAX_DIM];          // refinement exponent N_L - l_k
    int32_t n[SGW_MAX_DIM];
    int32_t stride[SGW_MAX_DIM];
    int32_t c[SGW_MAX_DIM];          // coarse extent loaded per tile (T when m = 0)
    int32_t outer[SGW_MAX_DIM];      // prod_{j>k} c[j]
    FastDiv fd_c[SGW_MAX_DIM];
    FastDiv fd_n[SGW_MAX_DIM];
    int32_t klast;                   // last refined direction (-1: none)
    int32_t rows;                    // prod_{k>0} c[k]: rows of the coarse block along direction 1
};

struct alignas(64) FineDev {
    int32_t d, N, G, lagrange;
    int32_t T[SGW_MAX_DIM];
    int32_t ntile[SGW_MAX_DIM];
    int32_t inner[SGW_MAX_DIM];      // prod_{j<k} T[j]
    int32_t tile_points, pad0, pad1; // pad0, pad1: LDS elements of prolongation buffers A, B
    int32_t zmask;                   // bit k: coarse values beyond either end of direction k are 0
    FastDiv fd_T[SGW_MAX_DIM];
    FastDiv fd_inner[SGW_MAX_DIM];
    double eps;
    // 3D/4D tiles with prod_{k<d-1} T_k = SGW_BLOCK run the line form of the passes (lines = 1):
    // one lane per line, the stencil work shared by the fine points of a coarse interval, the
    // per-point coefficients read from stab (STab entries of the solver's precision, the
    // entries of R = 2^m from index R - 2 on), the last pass accumulated in registers
    const void* stab;
    int32_t lines, rows_max;         // rows_max: LDS row-offset table entries (line form)
};

// Per-point coefficients of WENO5 prolongation: fine offset q = 0..R-1 inside a coarse
// interval of R fine nodes, s = (q - R/2) / R; P_r(s) = c + h G_r + hs K_r with h = s / 2,
// hs = s^2 / 2, and the linear weights C_r(s) of eq. (lwlag).
template <typename Real>
struct alignas(8 * sizeof(Real)) STab {
    Real h, hs, c0, c1, c2, pad0, pad1, pad2;
};

// One (solve, finest-grid tile) of a batched prolongation launch.
// One solve of a prolongation over many solves: workgroup (x, y) takes finest-grid
// tile x of solve y (x < ntiles).
struct ProItem {
    const ProDev* pro;
    const FineDev* fine;
    double* out;
    int32_t ntiles, pad;
};

// One chunk of one component grid in a restriction over many solves.
struct RestrictItem {
    const GridDev* g;
    int64_t start;                   // first node of the chunk
    int32_t count;                   // nodes in the chunk
    int32_t ic;
    double ip[8];
};

// One solve's wave-speed slots and time-step record, cleared before its restriction.
struct ResetItem {
    unsigned long long* alpha;
    ReqDev* req;
    int32_t nalpha, pad;
};

// One (computed, reference) pair of a norms launch over many solves.
struct NormItem {
    const double* a;
    const double* b;
    int64_t n;
    double* result;                  // L1, Linf
    int32_t parts, pad;              // first-pass workgroups of this pair
};

// Problem constants the exact-solution kernels need.
struct ExactDev {
    int32_t d, flux, ic, N;
    double lo[SGW_MAX_DIM], h[SGW_MAX_DIM];
    double fp[SGW_MAX_DIM];
    double ip[8];
    double t;
    const double* foot;              // Vlasov: (X0, V0) per (x node, v node) pair and x direction
};

// ---------------------------------------------------------------- kernel launchers (kernels_*.hip)
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_coef_init(GridDev* grids_dev, const GridDev* grids_host, int G, double* coef_base,
                            const int64_t* coef_off_host, const sgw_problem* pb, hipStream_t s);
// rho(x) of the stage input of every relaxation grid: first-pass items[0..npartial), then
// second-pass items[npartial..npartial + nfinal), one workgroup each
hipError_t launch_rho(const RhoItem* items, int npartial, int nfinal, int stage, int precision, hipStream_t s);
// H_2 and H_log of a finest-grid solution: partial sums in partials, the two values in result
// Vlasov-Maxwell fields of every grid: stage 0..2 update from the stage's currents (one workgroup
// per grid), or (stage < 0) the initial fields B_3 = b sin(k0 x_2), E = 0 in u^n
hipError_t launch_vm_fields(const GridDev* grids_dev, int G, int stage, int precision, double b, double k0,
                            int eps_linear, hipStream_t s);
// the fields of u^n combined on the finest x_2 grid (3 N values)
hipError_t launch_fields_combine(const GridDev* grids_dev, const ProDev* pro_dev, const FineDev& fine_host,
                                 const FineDev* fine_dev, double* out, hipStream_t s);
hipError_t launch_entropies(const FineDev& f, const double* lo, const double* hi, double theta, double zx,
                            const double* fsol, double* partials, double* result, hipStream_t s);
hipError_t launch_restrict(const GridDev* grids_dev, const GridDev* grids_host, int G, int precision,
                           const sgw_problem* pb, hipStream_t s);
hipError_t launch_req_reset(ReqDev* r, hipStream_t s);
hipError_t launch_req_set_final(ReqDev* r, double T, hipStream_t s);
hipError_t launch_grid_absmax(GridDev* g_dev, int64_t n, int precision, hipStream_t s);
hipError_t launch_req_restore(ReqDev* dst, const ReqDev* src, hipStream_t s);
hipError_t launch_req_set_final_many(ReqDev* const* reqs, const double* tf, int n, hipStream_t s);
hipError_t launch_restrict_many(const ResetItem* resets, int nresets, const RestrictItem* items, int nitems,
                                int precision, hipStream_t s);
hipError_t launch_dt(ReqDev* const* reqs, int nreq, hipStream_t s);
hipError_t launch_dt_one(ReqDev* req, hipStream_t s);
// stage kernel of dimension dim over items[0..nitems); grid_cap caps the persistent grid.
// stage SGW_STAGE_FUSED: the three stages of whole-grid boxes in one launch.  lines: the
// items are line-sweep items (4D), one launch per direction.
hipError_t launch_stage(const WorkItem* items, int nitems, int stage, int precision, int dim, size_t lds_bytes,
                        int grid_cap, hipStream_t s, bool lines = false, int first_dir = 0, int last_dir = 3);
// 4D: directions 1 and 2 of stage `stage` over the plane work items[0..nitems)
hipError_t launch_planes(const WorkItem* items, int nitems, int stage, int precision, hipStream_t s);
// the same over items[range_dev[0] .. + range_dev[1]) read on the device (batches, graphs)
hipError_t launch_stage_range(const WorkItem* items, const int* range_dev, int blocks, int stage, int precision,
                              int dim, size_t lds_bytes, hipStream_t s, bool lines = false);
hipError_t launch_gather_done(ReqDev* const* reqs, int nreq, int* flags, hipStream_t s);
size_t stage_lds_bytes(const GridDev& g, int precision);
int stage_occupancy(int precision, int dim, size_t lds_bytes, bool fused = false);
// persistent grid: blocks per CU x CUs
int stage_grid(int precision, int dim, size_t lds_bytes, int blocks_per_cu, bool fused = false);
// finest-grid tiles first_tile .. first_tile + num_tiles - 1 (tile index: direction 1 fastest)
hipError_t launch_prolong(const ProDev* pro_dev, const FineDev* fine_dev, const FineDev& fine_host,
                          int precision, size_t lds_bytes, double* out, int first_tile, int num_tiles,
                          hipStream_t s);
// items: one per solve (n <= 65535); max_tiles: the largest ntiles
hipError_t launch_prolong_many(const ProItem* items, int nitems, int max_tiles, int d, int precision,
                               size_t lds_bytes, hipStream_t s);
hipError_t launch_exact(const ExactDev& e, double* out, double* foot_scratch, hipStream_t s);
hipError_t launch_norms(const double* a, const double* b, int64_t n, double* partials, double* result,
                        hipStream_t s);
int norms_parts(int64_t n);
hipError_t launch_norms_many(const NormItem* items, int n, int max_parts, double* partials, hipStream_t s);
