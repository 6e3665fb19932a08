// Per-step kernels of libsgweno around the stage kernel: initial restriction
// (one solve or many), the Vlasov coefficient tables and constant LF speeds,
// time-step records, the shared time step and the completion flags.
#include "sgw_internal.h"

namespace {

// ---------------------------------------------------------------- set-up kernels

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Coefficient tables of the fixed-field Vlasov flux and the constant LF speeds:
// f_{x_k} = v_k u (coefficient indexed by the v_k node), f_{v_k} = E_k(x_k) u with
// E_k = amp sin(kE x_k), or E_k = -x_k (harmonic: the field of the Vlasov-Boltzmann model); for
// the Vlasov-Maxwell system only direction x_2, whose coefficient is xi_2 (the xi directions take
// theirs from the fields).  One workgroup per (grid, direction); the max over the table is the LF
// speed.
__global__ void coef_init_kernel(GridDev* grids, double* coef_base, const int64_t* coef_off, double amp, double kE,
                                 int harmonic)
{
    __shared__ double red[SGW_BLOCK / 64];
    GridDev* g = grids + blockIdx.x;
    const int k = blockIdx.y;
    if (k >= g->d || g->coef_src[k] < 0) return;
    const int m = g->d / 2;
    const int src = g->coef_src[k];
    double* tab = coef_base + coef_off[blockIdx.x * SGW_MAX_DIM + k];
    const int n = g->n[src];
    double amax = 0.0;
    for (int j = threadIdx.x; j < n; j += SGW_BLOCK) {
        const double x = g->lo[src] + j * g->h[src];
        const double c = (k < m) ? x : harmonic ? -x : amp * sin(kE * x);
        tab[j] = c;
        amax = fmax(amax, fabs(c));
    }
    amax = wave_max(amax);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = red[0];
        for (int w = 1; w < SGW_BLOCK / 64; w++) mm = fmax(mm, red[w]);
        g->alpha_c[k] = mm;
    }
}

struct RestrictArgs {
    int32_t ic, precision;
    double ip[8];
};

// Alg. Step 1: the initial condition at node idx (row-major, direction 1
// fastest) of grid g, whose coordinates are x_j = lo + j h.
__device__ __forceinline__ double ic_value(const GridDev* g, int64_t idx, int ic, const double* ip)
{
    uint32_t r = (uint32_t)idx;
    double x[SGW_MAX_DIM] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < g->d; k++) {
        const uint32_t q = FDIV(r, g->fd_n[k]);
        const int j = (int)(r - q * (uint32_t)g->n[k]);
        r = q;
        x[k] = g->lo[k] + j * g->h[k];
    }
    if (ic == SGW_IC_SINE) {
        double s = 0.0;
        for (int k = 0; k < g->d; k++) s += x[k];
        return ip[0] + ip[1] * sin(ip[2] * s + ip[3]);
    }
    if (ic == SGW_IC_VLASOV_MAXWELL) {
        // Sec. 3.4, Example 6: two drifting Maxwellians in xi_1 times a Maxwellian in xi_2,
        // ip = (beta, b, delta, v01, v02, k0)
        const double be = ip[0], de = ip[2];
        const double a = x[1] - ip[3], c = x[1] + ip[4];
        return exp(-x[2] * x[2] / be) * (de * exp(-a * a / be) + (1.0 - de) * exp(-c * c / be)) / (M_PI * be);
    }
    const int m = g->d / 2;
    if (ic == SGW_IC_VLASOV_BOLTZMANN) {
        // Sec. 3.4, Example 5: sin(x_1^2/2)^2 [cos(x_2^2/2)^2] exp(-(|x|^2 + |v|^2)/2) / s
        double shape = 1.0, r2 = 0.0;
        for (int k = 0; k < m; k++) {
            const double q = (k == 0) ? sin(0.5 * x[k] * x[k]) : cos(0.5 * x[k] * x[k]);
            shape *= q * q;
        }
        for (int k = 0; k < g->d; k++) r2 += x[k] * x[k];
        return ip[0] * shape * exp(-0.5 * r2);
    }
    double v2 = 0.0, pert = 1.0, norm = 1.0;
    for (int k = 0; k < m; k++) {
        v2 += x[m + k] * x[m + k];
        pert *= cos(ip[1] * x[k] + ip[2 + k]);
        norm *= 2.0 * M_PI;
    }
    return exp(-0.5 * v2) / sqrt(norm) * (1.0 + ip[0] * pert);
}

template <typename Real>
__global__ void restrict_kernel(const GridDev* grids, RestrictArgs a)
{
    __shared__ double red[SGW_BLOCK / 64];
    const GridDev* g = grids + blockIdx.y;
    int64_t total = 1;
    for (int k = 0; k < g->d; k++) total *= g->n[k];
    Real* u = (Real*)g->u;
    double amax = 0.0;
    for (int64_t idx = blockIdx.x * (int64_t)SGW_BLOCK + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * SGW_BLOCK) {
        const Real vr = (Real)ic_value(g, idx, a.ic, a.ip);
        u[idx] = vr;
        amax = nanmax(amax, fabs((double)vr));
    }
    if (g->dyn_alpha) block_atomic_max(amax, g->alpha + 0, red);
}

// Restriction of many solves in one launch: one workgroup per chunk of a grid.
template <typename Real>
__global__ void restrict_many_kernel(const RestrictItem* items)
{
    __shared__ double red[SGW_BLOCK / 64];
    const RestrictItem* it = items + blockIdx.x;
    const GridDev* g = it->g;
    Real* u = (Real*)g->u;
    double amax = 0.0;
    for (int i = threadIdx.x; i < it->count; i += SGW_BLOCK) {
        const int64_t idx = it->start + i;
        const Real vr = (Real)ic_value(g, idx, it->ic, it->ip);
        u[idx] = vr;
        amax = nanmax(amax, fabs((double)vr));
    }
    if (g->dyn_alpha) block_atomic_max(amax, g->alpha + 0, red);
}

__device__ __forceinline__ void req_reset(ReqDev* r)
{
    r->t = 0.0;
    r->steps = 0;
    r->done = 0;
    r->nonfinite = 0;
    r->dt = 0.0;
}

// Before a restriction of many solves: clear each solve's wave-speed slots and
// rewind its time-step record (one workgroup per solve).
__global__ void reset_many_kernel(const ResetItem* items)
{
    const ResetItem* it = items + blockIdx.x;
    for (int i = threadIdx.x; i < it->nalpha; i += blockDim.x) it->alpha[i] = 0ull;
    if (threadIdx.x == 0) req_reset(it->req);
}

__global__ void req_reset_kernel(ReqDev* r) { req_reset(r); }

__global__ void req_set_final_kernel(ReqDev* r, double T)
{
    r->T = T;
    r->done = r->nonfinite ? 1 : 0;
}

// Final times of newly admitted batch slots; a NaN entry leaves its slot alone.
__global__ void req_set_final_many_kernel(ReqDev* const* reqs, const double* tf, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ReqDev* r = reqs[i];
    const double T = tf[i];
    if (!r || T != T) return;
    r->T = T;
    r->done = r->nonfinite ? 1 : 0;
}

// Largest |E_1 + xi_2 B_3| and |E_2 - xi_1 B_3| over the x_2 nodes i = first, first + step, ...
// of one Vlasov-Maxwell grid's fields fld (B_3, E_1, E_2) and the end nodes of the other velocity
// direction (for fixed fields the rounded expression is monotone in xi, so its largest magnitude
// over all nodes sits at an end node).
__device__ void vm_field_speeds(const GridDev* g, const double* fld, int first, int step, double* a1, double* a2)
{
#pragma clang fp contract(off)
    const int n0 = g->n[0];
    const double x1lo = g->lo[1], x1hi = g->lo[1] + (g->n[1] - 1) * g->h[1];
    const double x2lo = g->lo[2], x2hi = g->lo[2] + (g->n[2] - 1) * g->h[2];
    double m1 = 0.0, m2 = 0.0;
    for (int i = first; i < n0; i += step) {
        const double B = fld[i], E1 = fld[n0 + i], E2 = fld[2 * n0 + i];
        const double p1 = x2lo * B, q1 = x2hi * B, p2 = x1lo * B, q2 = x1hi * B;
        m1 = nanmax(m1, nanmax(fabs(E1 + p1), fabs(E1 + q1)));
        m2 = nanmax(m2, nanmax(fabs(E2 - p2), fabs(E2 - q2)));
    }
    *a1 = m1;
    *a2 = m2;
}

// The shared time step (Sec. 3): dt = cfl / sum_k (A_k / h_k^fine), A_k the
// largest LF speed over all component grids of the solve at u^n, clipped so the
// last step lands on T.  One wavefront per solve: lanes over grids, then a
// wave-wide max (exact, so the result does not depend on the order).
__device__ void dt_wave(ReqDev* r)
{
    const int lane = threadIdx.x & 63;
    // The record is read once through the constant address space (scalar loads, several in
    // flight together, instead of one dependent vector load per field).  This kernel writes
    // the record only after the last read.
    typedef const __attribute__((address_space(4))) ReqDev* ReqC;
    const ReqC rc = (ReqC)r;
    const int active = rc->active, done = rc->done, dt_mode = rc->dt_mode, dyn = rc->dyn_alpha;
    const int ngrids = rc->ngrids, d = rc->d;
    const double t = rc->t, T = rc->T, cfl = rc->cfl, dt_pow53 = rc->dt_pow53;
    const int64_t steps = rc->steps;
    const unsigned long long* alpha = rc->alpha;
    const GridDev* grids = rc->grids;
    double hfin[SGW_MAX_DIM];
#pragma unroll
    for (int k = 0; k < SGW_MAX_DIM; k++) hfin[k] = rc->hfin[k];
    if (!active || done) {
        if (lane == 0) r->dt = 0.0;
        return;
    }
    const double rem = T - t;
    const double tol = 1e-12 * (T > 1.0 ? T : 1.0);
    if (!(rem > tol)) {
        if (lane == 0) {
            r->done = 1;
            r->dt = 0.0;
        }
        return;
    }
    double dt;
    if (dt_mode == SGW_DT_POW53 && !rc->vm) {
        dt = dt_pow53;
    } else {
        double denom = 0.0;
        if (rc->vm) {
            // Vlasov-Maxwell: x_2 at its constant speed; xi_1, xi_2 at the maxima over each grid's
            // nodes of |E_1 + xi_2 B_3| and |E_2 - xi_1 B_3| of u^n's fields, attained at the end
            // nodes of the other velocity direction (the rounded expression is monotone in it);
            // each grid's pair goes to its stage-0 speed slots
            double A0 = 0.0, A1 = 0.0, A2 = 0.0;
            for (int g = lane; g < ngrids; g += 64) A0 = nanmax(A0, grids[g].alpha_c[0]);
            for (int g = 0; g < ngrids; g++) {
                const GridDev* G = grids + g;
                double a1, a2;
                vm_field_speeds(G, (const double*)((const char*)G->u + G->fld_bytes), lane, 64, &a1, &a2);
                a1 = wave_max(a1);
                a2 = wave_max(a2);
                if (lane == 0) {
                    G->vm_alpha[0] = a1;
                    G->vm_alpha[1] = a2;
                }
                A1 = nanmax(A1, a1);
                A2 = nanmax(A2, a2);
            }
            A0 = wave_max(A0);
            denom = dt_mode == SGW_DT_POW53 ? 0.0 : A0 / hfin[0] + A1 / hfin[1] + A2 / hfin[2];
        } else if (dyn) {
            // every grid of a solve has the same flux: one maximum of the state-dependent
            // speeds serves all directions
            double A = 0.0;
            for (int g = lane; g < ngrids; g += 64) A = nanmax(A, __longlong_as_double((long long)alpha[4 * g]));
            A = wave_max(A);
            for (int k = 0; k < d; k++) denom += A / hfin[k];
        } else {
            for (int k = 0; k < d; k++) {
                double A = 0.0;
                for (int g = lane; g < ngrids; g += 64) A = nanmax(A, grids[g].alpha_c[k]);
                A = wave_max(A);
                denom += A / hfin[k];
            }
        }
        if (denom != denom || denom > 1.7e308) {
            if (lane == 0) {
                r->nonfinite = 1;
                r->done = 1;
                r->dt = 0.0;
            }
            return;
        }
        dt = dt_mode == SGW_DT_POW53 ? dt_pow53 : denom > 0.0 ? cfl / denom : rem;
    }
    if (dt > rem) dt = rem;
    if (lane == 0) {
        r->dt = dt;
        r->t = t + dt;
        r->steps = steps + 1;
    }
}

__global__ void __launch_bounds__(64) dt_kernel(ReqDev* const* reqs, int nreq)
{
    const int i = blockIdx.x;
    if (i < nreq && reqs[i]) dt_wave(reqs[i]);
}

__global__ void __launch_bounds__(64) dt_one_kernel(ReqDev* r) { dt_wave(r); }

__global__ void gather_done_kernel(ReqDev* const* reqs, int nreq, int* flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nreq) flags[i] = reqs[i] ? (reqs[i]->done ? 1 : 0) | (reqs[i]->nonfinite ? 2 : 0) : 0;
}


// Largest |u| over one grid into its wave-speed slot 0 (caller-set initial data).
template <typename Real>
__global__ void grid_absmax_kernel(GridDev* g)
{
    __shared__ double red[SGW_BLOCK / 64];
    int64_t total = 1;
    for (int k = 0; k < g->d; k++) total *= g->n[k];
    const Real* u = (const Real*)g->u;
    double amax = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)SGW_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * SGW_BLOCK)
        amax = nanmax(amax, fabs((double)u[i]));
    block_atomic_max(amax, g->alpha + 0, red);
}

// The time fields of a snapshot record (t, steps, dt, completion flags) into a solve's record.
__global__ void req_restore_kernel(ReqDev* dst, const ReqDev* src)
{
    dst->t = src->t;
    dst->steps = src->steps;
    dst->dt = src->dt;
    dst->done = src->done;
    dst->nonfinite = src->nonfinite;
}

} // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int blocks = (int)((n + SGW_BLOCK - 1) / SGW_BLOCK);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks), dim3(SGW_BLOCK), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_coef_init(GridDev* grids_dev, const GridDev* grids_host, int G, double* coef_base,
                            const int64_t* coef_off_dev, const sgw_problem* pb, hipStream_t s)
{
    (void)grids_host;
    if (G <= 0) return hipSuccess;
    hipLaunchKernelGGL(coef_init_kernel, dim3(G, SGW_MAX_DIM), dim3(SGW_BLOCK), 0, s, grids_dev, coef_base,
                       coef_off_dev, pb->flux_params[0], pb->flux_params[1],
                       pb->flux == SGW_FLUX_VLASOV_HARMONIC ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_restrict(const GridDev* grids_dev, const GridDev* grids_host, int G, int precision,
                           const sgw_problem* pb, hipStream_t s)
{
    int64_t maxn = 1;
    for (int g = 0; g < G; g++) {
        int64_t n = 1;
        for (int k = 0; k < grids_host[g].d; k++) n *= grids_host[g].n[k];
        maxn = n > maxn ? n : maxn;
    }
    int bx = (int)((maxn + SGW_BLOCK - 1) / SGW_BLOCK);
    if (bx > 256) bx = 256;
    RestrictArgs a;
    a.ic = pb->ic;
    a.precision = precision;
    for (int i = 0; i < 8; i++) a.ip[i] = pb->ic_params[i];
    if (precision == SGW_FP64)
        hipLaunchKernelGGL(restrict_kernel<double>, dim3(bx, G), dim3(SGW_BLOCK), 0, s, grids_dev, a);
    else
        hipLaunchKernelGGL(restrict_kernel<float>, dim3(bx, G), dim3(SGW_BLOCK), 0, s, grids_dev, a);
    return hipGetLastError();
}

hipError_t launch_req_reset(ReqDev* r, hipStream_t s)
{
    hipLaunchKernelGGL(req_reset_kernel, dim3(1), dim3(1), 0, s, r);
    return hipGetLastError();
}

hipError_t launch_req_set_final(ReqDev* r, double T, hipStream_t s)
{
    hipLaunchKernelGGL(req_set_final_kernel, dim3(1), dim3(1), 0, s, r, T);
    return hipGetLastError();
}

hipError_t launch_req_set_final_many(ReqDev* const* reqs, const double* tf, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(req_set_final_many_kernel, dim3((n + SGW_BLOCK - 1) / SGW_BLOCK), dim3(SGW_BLOCK), 0, s, reqs,
                       tf, n);
    return hipGetLastError();
}

hipError_t launch_restrict_many(const ResetItem* resets, int nresets, const RestrictItem* items, int nitems,
                                int precision, hipStream_t s)
{
    if (nresets > 0) {
        hipLaunchKernelGGL(reset_many_kernel, dim3(nresets), dim3(64), 0, s, resets);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (nitems <= 0) return hipSuccess;
    if (precision == SGW_FP64)
        hipLaunchKernelGGL(restrict_many_kernel<double>, dim3(nitems), dim3(SGW_BLOCK), 0, s, items);
    else
        hipLaunchKernelGGL(restrict_many_kernel<float>, dim3(nitems), dim3(SGW_BLOCK), 0, s, items);
    return hipGetLastError();
}

hipError_t launch_dt(ReqDev* const* reqs, int nreq, hipStream_t s)
{
    if (nreq <= 0) return hipSuccess;
    hipLaunchKernelGGL(dt_kernel, dim3(nreq), dim3(64), 0, s, reqs, nreq);
    return hipGetLastError();
}

hipError_t launch_dt_one(ReqDev* req, hipStream_t s)
{
    hipLaunchKernelGGL(dt_one_kernel, dim3(1), dim3(64), 0, s, req);
    return hipGetLastError();
}

hipError_t launch_gather_done(ReqDev* const* reqs, int nreq, int* flags, hipStream_t s)
{
    if (nreq <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_done_kernel, dim3((nreq + 63) / 64), dim3(64), 0, s, reqs, nreq, flags);
    return hipGetLastError();
}

hipError_t launch_grid_absmax(GridDev* g_dev, int64_t n, int precision, hipStream_t s)
{
    int blocks = (int)((n + SGW_BLOCK - 1) / SGW_BLOCK);
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    if (precision == SGW_FP64)
        hipLaunchKernelGGL(grid_absmax_kernel<double>, dim3(blocks), dim3(SGW_BLOCK), 0, s, g_dev);
    else
        hipLaunchKernelGGL(grid_absmax_kernel<float>, dim3(blocks), dim3(SGW_BLOCK), 0, s, g_dev);
    return hipGetLastError();
}

hipError_t launch_req_restore(ReqDev* dst, const ReqDev* src, hipStream_t s)
{
    hipLaunchKernelGGL(req_restore_kernel, dim3(1), dim3(1), 0, s, dst, src);
    return hipGetLastError();
}
