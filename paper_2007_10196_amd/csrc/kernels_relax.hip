// Kernels of the kinetic models of Sec. 3.4 around the line sweep: the velocity moments of each
// Runge-Kutta stage's input (the density rho(x) = int f dv that the relaxation source
// (mu_inf(v) rho(x) - f) / tau of Example 5 reads; the currents j_q = int f xi_q dxi that drive the
// fields of Example 6), and the entropy functionals H_2 and H_log of a finest-grid solution.
#include <cmath>

#include "sgw_internal.h"

// descriptors are read through the constant address space (scalar loads)
#define SGW_CONST __attribute__((address_space(4)))
typedef const SGW_CONST GridDev* GridC;

namespace {

// The moments h_v * (sum over the velocity nodes of the grid of w f) of the stage input, with
// w = 1 (rho; nmom = 1) or w = xi_1, xi_2 (Vlasov-Maxwell, directions 2 and 3; nmom = 2), in two
// launches (the launch boundary orders the passes; no fences or counters).  The grid is an
// nvr x nxr matrix with the x nodes fastest.
//
// First pass: workgroup (grid, column block cb, chunk c) sums rows c * SGW_RHO_CHUNK ..
// + SGW_RHO_CHUNK of SGW_RHO_COLS columns: lane (col, r) takes rows r, r + L, r + 2L, ... (L row
// lanes) in FP64, the L row lanes are added in order through LDS and the block's sums go to
// rho_part[moment][c][x].
template <typename Real>
__global__ void __launch_bounds__(SGW_BLOCK) rho_partial_kernel(const RhoItem* __restrict__ items, int stage)
{
    constexpr int L = SGW_BLOCK / SGW_RHO_COLS;
    __shared__ double part[2][SGW_BLOCK];
    const SGW_CONST RhoItem* it = (const SGW_CONST RhoItem*)items + blockIdx.x;
    GridC g = (GridC)it->g;
    if (((const SGW_CONST ReqDev*)g->req)->done) return;
    const Real* __restrict__ in = (const Real*)(stage == 0 ? g->u : stage == 1 ? g->a : g->b);
    const int nx = g->nxr, nv = g->nvr, chunk = it->chunk, nch = g->rho_nchunk;
    const int col = threadIdx.x % SGW_RHO_COLS, lane = threadIdx.x / SGW_RHO_COLS;
    const int x = it->cb * SGW_RHO_COLS + col;
    const int r0 = chunk * SGW_RHO_CHUNK + lane;
    double sum = 0.0, sum2 = 0.0;
    if (g->nmom == 1) {
        if (x < nx) {
#pragma unroll
            for (int i = 0; i < SGW_RHO_RPT; i++) {
                const int r = r0 + i * L;
                if (r < nv) sum += (double)in[(int64_t)r * nx + x];
            }
        }
    } else if (x < nx) {
        // Vlasov-Maxwell: row r is velocity node (a, b) = (r mod n_2, r / n_2) of directions 2, 3
        const int n1 = g->n[1];
        for (int i = 0; i < SGW_RHO_RPT; i++) {
            const int r = r0 + i * L;
            if (r < nv) {
                const int bb = r / n1, a = r - bb * n1;
                const double f = (double)in[(int64_t)r * nx + x];
                sum = fma(f, g->lo[1] + a * g->h[1], sum);
                sum2 = fma(f, g->lo[2] + bb * g->h[2], sum2);
            }
        }
    }
    part[0][threadIdx.x] = sum;
    part[1][threadIdx.x] = sum2;
    __syncthreads();
    if (lane == 0 && x < nx)
        for (int m = 0; m < g->nmom; m++) {
            double s = part[m][col];
#pragma unroll
            for (int l = 1; l < L; l++) s += part[m][col + l * SGW_RHO_COLS];
            g->rho_part[((int64_t)m * nch + chunk) * nx + x] = s;
        }
}

// Second pass: workgroup (grid, column block cb) adds the chunks of its SGW_RHO_COLS columns:
// row lane l takes chunks l, l + L, ... in order, the lanes are added in order, the sum is
// scaled by h_v.  Every sum runs in a fixed order, so rho is bitwise repeatable.
__global__ void __launch_bounds__(SGW_BLOCK) rho_final_kernel(const RhoItem* __restrict__ items)
{
    constexpr int L = SGW_BLOCK / SGW_RHO_COLS;
    __shared__ double part[SGW_BLOCK];
    const SGW_CONST RhoItem* it = (const SGW_CONST RhoItem*)items + blockIdx.x;
    GridC g = (GridC)it->g;
    if (((const SGW_CONST ReqDev*)g->req)->done) return;
    const int nx = g->nxr, nch = g->rho_nchunk;
    const int col = threadIdx.x % SGW_RHO_COLS, lane = threadIdx.x / SGW_RHO_COLS;
    const int x = it->cb * SGW_RHO_COLS + col;
    for (int m = 0; m < g->nmom; m++) {
        const double* __restrict__ rp = g->rho_part + (int64_t)m * nch * nx;
        double sum = 0.0;
        if (x < nx)
            for (int c = lane; c < nch; c += L) sum += rp[(int64_t)c * nx + x];
        part[threadIdx.x] = sum;
        __syncthreads();
        if (lane == 0 && x < nx) {
            double s = part[col];
#pragma unroll
            for (int l = 1; l < L; l++) s += part[col + l * SGW_RHO_COLS];
            g->rho[(int64_t)m * nx + x] = s * g->hv;
        }
        __syncthreads();
    }
}

struct EntArgs {
    int32_t d, m;
    int64_t N, n;
    double lo[SGW_MAX_DIM], h[SGW_MAX_DIM];
    double inv_theta, mnorm;
};

// First pass: workgroup blk of `parts` sums H^2 M and H log(H) M (0 where H <= 0) over its
// strided share of the finest nodes, with M(x, v) = mnorm exp(-(|v|^2 + |x|^2) / (2 theta)),
// in a fixed tree order.
__global__ void __launch_bounds__(SGW_BLOCK) entropies_partial_kernel(EntArgs a, const double* __restrict__ f,
                                                                      double* partials)
{
    __shared__ double s2[SGW_BLOCK], sl[SGW_BLOCK];
    const int parts = gridDim.x;
    double q2 = 0.0, ql = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)SGW_BLOCK + threadIdx.x; i < a.n; i += (int64_t)parts * SGW_BLOCK) {
        int64_t r = i;
        double r2 = 0.0;
        for (int k = 0; k < a.d; k++) {
            const int64_t q = r / a.N;
            const double x = a.lo[k] + (double)(r - q * a.N) * a.h[k];
            r = q;
            r2 += x * x;
        }
        const double M = a.mnorm * exp(-0.5 * r2 * a.inv_theta);
        const double H = f[i] / M;
        q2 += H * H * M;
        if (H > 0.0) ql += H * log(H) * M;
    }
    s2[threadIdx.x] = q2;
    sl[threadIdx.x] = ql;
    __syncthreads();
    for (int w = SGW_BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s2[threadIdx.x] += s2[threadIdx.x + w];
            sl[threadIdx.x] += sl[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s2[0];
        partials[2 * blockIdx.x + 1] = sl[0];
    }
}

// Second pass: the np partials, zero-padded to SGW_NPART, in a fixed tree order, times the
// finest cell volume.
__global__ void __launch_bounds__(SGW_BLOCK) entropies_final_kernel(const double* partials, int np, double cell,
                                                                    double* result)
{
    __shared__ double s2[SGW_NPART], sl[SGW_NPART];
    for (int i = threadIdx.x; i < SGW_NPART; i += blockDim.x) {
        s2[i] = i < np ? partials[2 * i] : 0.0;
        sl[i] = i < np ? partials[2 * i + 1] : 0.0;
    }
    __syncthreads();
    for (int w = SGW_NPART / 2; w > 0; w >>= 1) {
        for (int i = threadIdx.x; i < w; i += blockDim.x) {
            s2[i] += s2[i + w];
            sl[i] += sl[i + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        result[0] = s2[0] * cell;
        result[1] = sl[0] * cell;
    }
}

} // namespace

hipError_t launch_rho(const RhoItem* items, int npartial, int nfinal, int stage, int precision, hipStream_t s)
{
    if (npartial <= 0) return hipSuccess;
    if (precision == SGW_FP64)
        hipLaunchKernelGGL(rho_partial_kernel<double>, dim3(npartial), dim3(SGW_BLOCK), 0, s, items, stage);
    else
        hipLaunchKernelGGL(rho_partial_kernel<float>, dim3(npartial), dim3(SGW_BLOCK), 0, s, items, stage);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(rho_final_kernel, dim3(nfinal), dim3(SGW_BLOCK), 0, s, items + npartial);
    return hipGetLastError();
}

hipError_t launch_entropies(const FineDev& f, const double* lo, const double* hi, double theta, double zx,
                            const double* fsol, double* partials, double* result, hipStream_t s)
{
    EntArgs a;
    a.d = f.d;
    a.m = f.d / 2;
    a.N = f.N;
    a.n = 1;
    double cell = 1.0;
    for (int k = 0; k < SGW_MAX_DIM; k++) {
        a.lo[k] = k < f.d ? lo[k] : 0.0;
        a.h[k] = k < f.d ? (hi[k] - lo[k]) / f.N : 0.0;
        if (k < f.d) {
            a.n *= f.N;
            cell *= a.h[k];
        }
    }
    a.inv_theta = 1.0 / theta;
    a.mnorm = 1.0 / (std::pow(2.0 * M_PI * theta, 0.5 * a.m) * zx);
    const int64_t pb = (a.n + SGW_BLOCK - 1) / SGW_BLOCK;
    const int parts = pb < 1 ? 1 : (pb > SGW_NPART ? SGW_NPART : (int)pb);
    hipLaunchKernelGGL(entropies_partial_kernel, dim3(parts), dim3(SGW_BLOCK), 0, s, a, fsol, partials);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(entropies_final_kernel, dim3(1), dim3(SGW_BLOCK), 0, s, partials, parts, cell, result);
    return hipGetLastError();
}
