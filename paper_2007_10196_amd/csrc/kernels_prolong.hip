// Prolongation + combination, exact solutions and error norms of libsgweno.
//
// Prolongation (Sec. 2.2.1): along each direction k with m = N_L - l_k > 0 the
// coarse line is refined by R = 2^m.  Fine node J falls in the half-open
// interval [x_{i-1/2}, x_{i+1/2}) of coarse node i = floor(J/R + 1/2) at offset
// s = J/R - i in [-1/2, 1/2); its value is the WENO5 interpolation of eqs.
// (lwlag), (eqnlnwe), (si), (nlweno) from u_{i-2..i+2}: the three quadratic
// interpolants P_r on the substencils, the positive linear weights C_r(s), the
// smoothness indicators beta_r, nonlinear weights C_r/(eps+beta_r)^2
// normalised.  Directions are refined in increasing order.  The combination
// (eq. genformusgc) adds c_g P U_g in FP64, grids in plan order.
//
// Layout: one workgroup owns a tile of the finest grid.  For each component
// grid it stages the coarse block the tile depends on in LDS, refines it
// direction by direction between two LDS buffers, and adds the result to FP64
// accumulators in registers; the tile is written once at the end.
#include "sgw_internal.h"

#define SGW_MAXRP 16 // finest-grid points per thread: tile <= SGW_BLOCK * SGW_MAXRP

namespace {

// descriptors live in the constant address space for the duration of a launch
#define SGW_CONST __attribute__((address_space(4)))
typedef const SGW_CONST ProDev* ProC;
typedef const SGW_CONST FineDev* FineC;
#define M24(a, b) __mul24((a), (b))

__device__ __forceinline__ float rdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// a / b for b > 0: hardware reciprocal, one Newton step, one residual correction
__device__ __forceinline__ double rdiv(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    const double q = a * r;
    return fma(fma(-b, q, a), r, q);
}

// P_r written about x_i: P_r(s) = c + s g_r + s^2 k_r, where 2 g_r is the (one-sided or
// central) first difference of substencil r at x_i and 2 k_r its second difference; the
// integral of eq. (si) then equals g_r^2 + (13/3) k_r^2, the Jiang-Shu quadratic forms of
// eq. (2.7.2).  The code keeps G_r = 2 g_r and K_r = 2 k_r: P_r = c + (s/2)(G_r + s K_r),
// and eps + beta_r = (eps4 + G_r^2 + 13/3 K_r^2) / 4 with eps4 = 4 eps, a factor common
// to the three weights that their normalisation cancels.
template <typename Real>
__device__ __forceinline__ Real interp5(Real a, Real b, Real c, Real d, Real e, Real s, Real eps4, int lagrange)
{
    const Real G0 = a - Real(4) * b + Real(3) * c, K0 = a - Real(2) * b + c;
    const Real G1 = d - b, K1 = b - Real(2) * c + d;
    const Real G2 = Real(-3) * c + Real(4) * d - e, K2 = c - Real(2) * d + e;
    const Real h = Real(0.5) * s;
    const Real P0 = c + h * (G0 + s * K0);
    const Real P1 = c + h * (G1 + s * K1);
    const Real P2 = c + h * (G2 + s * K2);
    const Real C0 = (s - Real(1)) * (s - Real(2)) * Real(1.0 / 12.0);
    const Real C1 = (Real(4) - s * s) * Real(1.0 / 6.0);
    const Real C2 = (s + Real(1)) * (s + Real(2)) * Real(1.0 / 12.0);
    if (lagrange) return C0 * P0 + C1 * P1 + C2 * P2;
    Real e0 = eps4 + (G0 * G0 + Real(13.0 / 3.0) * K0 * K0);
    Real e1 = eps4 + (G1 * G1 + Real(13.0 / 3.0) * K1 * K1);
    Real e2 = eps4 + (G2 * G2 + Real(13.0 / 3.0) * K2 * K2);
    e0 *= e0;
    e1 *= e1;
    e2 *= e2;
    const Real w0 = C0 * (e1 * e2), w1 = C1 * (e0 * e2), w2 = C2 * (e0 * e1);
    return rdiv(w0 * P0 + w1 * P1 + w2 * P2, w0 + w1 + w2);
}

// ZB: the problem has a zero boundary (FineDev.zmask): coarse positions beyond either end of
// such a direction read 0 instead of wrapping.
template <typename Real, int D, bool ZB>
__device__ __forceinline__ void prolong_tile(ProC pro, FineC F, double* __restrict__ out, int tile)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    int J0[D];
    {
        int r = tile;
        for (int k = 0; k < D; k++) {
            const int q = r / F->ntile[k];
            J0[k] = (r - q * F->ntile[k]) * F->T[k];
            r = q;
        }
    }
    const int tile_points = F->tile_points;
    const Real eps4 = (Real)(4.0 * F->eps);
    const int lagrange = F->lagrange;
    double acc[SGW_MAXRP];
#pragma unroll
    for (int r = 0; r < SGW_MAXRP; r++) acc[r] = 0.0;
    Real* bufA = (Real*)smem;
    Real* bufB = bufA + F->pad0; // pad0 holds the per-buffer element count (even)

    for (int gidx = 0; gidx < F->G; gidx++) {
        ProC p = pro + gidx;
        const Real* __restrict__ u = (const Real*)p->u;
        int cl[D];
#pragma unroll
        for (int k = 0; k < D; k++) {
            const int m = p->m[k];
            cl[k] = (m == 0) ? J0[k] : (((2 * J0[k] + (1 << m)) >> (m + 1)) - 2);
        }
        // ---- coarse block this tile depends on (periodic wrap, or 0 beyond a zero boundary)
        for (int e = tid; e < p->load_total; e += SGW_BLOCK) {
            uint32_t r = (uint32_t)e;
            int gi = 0;
            bool zero = false;
#pragma unroll
            for (int k = 0; k < D; k++) {
                const uint32_t q = FDIV(r, p->fd_c[k]);
                const int c = (int)(r - q * (uint32_t)p->c[k]);
                r = q;
                // periodic wrap: cl + c + 2n is >= 0, its remainder by n by the fast division
                const uint32_t xw = (uint32_t)(cl[k] + c + 2 * p->n[k]);
                const int x = (int)(xw - FDIV(xw, p->fd_n[k]) * (uint32_t)p->n[k]);
                gi += x * p->stride[k];
                if (ZB && ((F->zmask >> k) & 1)) zero |= (cl[k] + c < 0) || (cl[k] + c >= p->n[k]);
            }
            bufA[e] = zero ? Real(0) : u[gi];
        }
        __syncthreads();
        Real* src = bufA;
        Real* dst = bufB;
#pragma unroll
        for (int k = 0; k < D; k++) {
            const int m = p->m[k];
            if (m == 0) continue;
            const int Tk = F->T[k];
            const int ck = p->c[k];
            const int inner = F->inner[k];
            const int total = inner * Tk * p->outer[k];
            const int R = 1 << m;
            const Real invR = Real(1) / Real(R);
            for (int o = tid; o < total; o += SGW_BLOCK) {
                // LDS indices stay below 2^24: 24-bit multiplies and 32-bit offsets
                const uint32_t r1 = FDIV((uint32_t)o, F->fd_inner[k]);
                const int a = o - M24((int)r1, inner);
                const uint32_t bq = FDIV(r1, F->fd_T[k]);
                const int jl = (int)r1 - M24((int)bq, Tk);
                const int J = J0[k] + jl;
                const int i = (2 * J + R) >> (m + 1);
                const Real s = (Real)(J - i * R) * invR;
                const int li = i - cl[k];
                const uint32_t base = (uint32_t)(a + M24(inner, (li - 2) + M24(ck, (int)bq)));
                const uint32_t st = (uint32_t)inner;
                dst[o] = interp5<Real>(src[base], src[base + st], src[base + 2 * st], src[base + 3 * st],
                                       src[base + 4 * st], s, eps4, lagrange);
            }
            __syncthreads();
            Real* t = src;
            src = dst;
            dst = t;
        }
        const double cg = (double)p->coef;
#pragma unroll
        for (int r = 0; r < SGW_MAXRP; r++) {
            const int e = tid + r * SGW_BLOCK;
            if (e < tile_points) acc[r] += cg * (double)src[e];
        }
        __syncthreads();
    }
    // ---- write the tile
#pragma unroll
    for (int r = 0; r < SGW_MAXRP; r++) {
        const int e = tid + r * SGW_BLOCK;
        if (e < tile_points) {
            uint32_t rr = (uint32_t)e;
            int64_t gi = 0, st = 1;
#pragma unroll
            for (int k = 0; k < D; k++) {
                const uint32_t q = FDIV(rr, F->fd_T[k]);
                const int c = (int)(rr - q * (uint32_t)F->T[k]);
                rr = q;
                gi += (int64_t)(J0[k] + c) * st;
                st *= F->N;
            }
            out[gi] = acc[r];
        }
    }
}

// ---------------------------------------------------------------- line form (3D, 4D)
//
// The same interpolation, organised so that the work depending only on a coarse stencil is
// done once for the R fine nodes it serves.  One lane refines one line of a pass: for each
// coarse centre i on the line it forms the differences G_r, K_r of the three substencils, the
// squared weight denominators e_r = (eps4 + G_r^2 + 13/3 K_r^2)^2 and the products
// E_r = e_r' e_r'' (the common factor of eq. (nlweno) after clearing denominators), and the
// centre's A_r = E_r c, B_r = E_r G_r, D_r = E_r K_r.  Each fine node at offset s then costs
// E_r P_r(s) = A_r + h B_r + hs D_r, the sums num = sum C_r E_r P_r and den = sum C_r E_r and
// one division, with h, hs and C_r(s) read from a table whose index is the same for every
// lane (scalar loads).  A node at s = 0 takes the centre's value: every P_r(0) = u_i.

// Sliding state of the stencil along a line: for centre i it holds u_i, u_{i+1}, u_{i+2},
// the first differences D1(i) = u_i - u_{i-1}, D1(i+1), the second differences
// K_r = D2(i-1+r), D2(j) = u_{j-1} - 2 u_j + u_{j+1}, and kk_r = eps4 + 13/3 K_r^2.  Moving to
// centre i+1 takes one new value and one new difference of each order.
template <typename Real>
struct Slide {
    Real c, d, e, D1a, D1b, K0, K1, K2, kk0, kk1, kk2;
};

template <typename Real, bool LAG>
__device__ __forceinline__ void slide_init(Slide<Real>& w, Real a, Real b, Real c, Real d, Real e, Real eps4)
{
#pragma clang fp contract(off)
    w.c = c, w.d = d, w.e = e;
    w.D1a = c - b;
    w.D1b = d - c;
    w.K0 = fma(Real(-2), b, a) + c;
    w.K1 = fma(Real(-2), c, b) + d;
    w.K2 = fma(Real(-2), d, c) + e;
    if (!LAG) {
        w.kk0 = fma(Real(13.0 / 3.0) * w.K0, w.K0, eps4);
        w.kk1 = fma(Real(13.0 / 3.0) * w.K1, w.K1, eps4);
        w.kk2 = fma(Real(13.0 / 3.0) * w.K2, w.K2, eps4);
    }
}

template <typename Real, bool LAG>
__device__ __forceinline__ void slide_next(Slide<Real>& w, Real f, Real eps4)
{
#pragma clang fp contract(off)
    w.D1a = w.D1b;
    w.D1b = w.e - w.d;
    w.K0 = w.K1;
    w.K1 = w.K2;
    w.K2 = fma(Real(-2), w.e, w.d) + f;
    if (!LAG) {
        w.kk0 = w.kk1;
        w.kk1 = w.kk2;
        w.kk2 = fma(Real(13.0 / 3.0) * w.K2, w.K2, eps4);
    }
    w.c = w.d, w.d = w.e, w.e = f;
}

// What the fine nodes of one centre share: with G_r the first-derivative differences of the
// substencils (G0 = K0 + 2 D1(i), G1 = D1(i) + D1(i+1), G2 = 2 D1(i+1) - K2), the squared
// weight denominators e_r = (kk_r + G_r^2)^2, E_r = e_r' e_r'' and A_r = E_r u_i, B_r = E_r G_r,
// D_r = E_r K_r (Lagrange: E_r = 1).
template <typename Real>
struct Centre {
    Real c, A0, A1, A2, B0, B1, B2, D0, D1, D2, E0, E1, E2;
};

template <typename Real, bool LAG>
__device__ __forceinline__ void centre_setup(Centre<Real>& z, const Slide<Real>& w)
{
#pragma clang fp contract(off)
    const Real G0 = fma(Real(2), w.D1a, w.K0), G1 = w.D1a + w.D1b, G2 = fma(Real(2), w.D1b, -w.K2);
    z.c = w.c;
    if (LAG) {
        z.A0 = z.A1 = z.A2 = w.c;
        z.B0 = G0, z.B1 = G1, z.B2 = G2;
        z.D0 = w.K0, z.D1 = w.K1, z.D2 = w.K2;
        z.E0 = z.E1 = z.E2 = Real(1);
        return;
    }
    Real e0 = fma(G0, G0, w.kk0), e1 = fma(G1, G1, w.kk1), e2 = fma(G2, G2, w.kk2);
    e0 *= e0;
    e1 *= e1;
    e2 *= e2;
    z.E0 = e1 * e2;
    z.E1 = e0 * e2;
    z.E2 = e0 * e1;
    z.A0 = z.E0 * w.c, z.A1 = z.E1 * w.c, z.A2 = z.E2 * w.c;
    z.B0 = z.E0 * G0, z.B1 = z.E1 * G1, z.B2 = z.E2 * G2;
    z.D0 = z.E0 * w.K0, z.D1 = z.E1 * w.K1, z.D2 = z.E2 * w.K2;
}

template <typename Real, bool LAG>
__device__ __forceinline__ Real centre_value(const Centre<Real>& z, const SGW_CONST STab<Real>& t, int copy)
{
#pragma clang fp contract(off)
    if (copy) return z.c;
    const Real Q0 = fma(t.hs, z.D0, fma(t.h, z.B0, z.A0));
    const Real Q1 = fma(t.hs, z.D1, fma(t.h, z.B1, z.A1));
    const Real Q2 = fma(t.hs, z.D2, fma(t.h, z.B2, z.A2));
    const Real num = fma(t.c2, Q2, fma(t.c1, Q1, t.c0 * Q0));
    if (LAG) return num;
    return rdiv(num, fma(t.c2, z.E2, fma(t.c1, z.E1, t.c0 * z.E0)));
}

// Each refinement loop below runs in a lambda of its own that takes the centre by value: the
// same arithmetic as the loop written inline (bitwise equal results), which the compiler
// schedules about 6 % faster for the FP64 4D launch.
template <typename Real, int D, bool LAG, bool ZB>
__device__ __forceinline__ void prolong_tile_lines(ProC pro, FineC F, double* __restrict__ out, int tile)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    int J0[D];
    {
        int r = tile;
        for (int k = 0; k < D; k++) {
            const int q = r / F->ntile[k];
            J0[k] = (r - q * F->ntile[k]) * F->T[k];
            r = q;
        }
    }
    const Real eps4 = (Real)(4.0 * F->eps);
    const int lagrange = LAG ? 1 : 0;
    const int Tlast = F->T[D - 1];
    typedef const SGW_CONST STab<Real>* TabC;
    const TabC stab = (TabC)F->stab;
    double acc[SGW_MAXRP];
#pragma unroll
    for (int r = 0; r < SGW_MAXRP; r++) acc[r] = 0.0;
    Real* bufA = (Real*)smem;
    Real* bufB = bufA + F->pad0;
    int* rowoff = (int*)(bufB + F->pad1);

    for (int gidx = 0; gidx < F->G; gidx++) {
        ProC p = pro + gidx;
        const Real* __restrict__ u = (const Real*)p->u;
        int cl[D];
#pragma unroll
        for (int k = 0; k < D; k++) {
            const int m = p->m[k];
            cl[k] = (m == 0) ? J0[k] : (((2 * J0[k] + (1 << m)) >> (m + 1)) - 2);
        }
        const int kl = p->klast;
        // element offset of row r of the coarse block (its position along directions 2..d,
        // periodic wrap: cl + c + 2n >= 0 takes its remainder by n with the fast division);
        // -1 for a row beyond either end of a zero-boundary direction (all its values are 0)
        const int zm = ZB ? F->zmask : 0;
        auto row_offset = [&](int r) {
            uint32_t rr = (uint32_t)r;
            int gi = 0;
            bool zero = false;
#pragma unroll
            for (int k = 1; k < D; k++) {
                const uint32_t q = FDIV(rr, p->fd_c[k]);
                const int c = (int)(rr - q * (uint32_t)p->c[k]);
                rr = q;
                const uint32_t xw = (uint32_t)(cl[k] + c + 2 * p->n[k]);
                gi += (int)(xw - FDIV(xw, p->fd_n[k]) * (uint32_t)p->n[k]) * p->stride[k];
                if (ZB && ((zm >> k) & 1)) zero |= (cl[k] + c < 0) || (cl[k] + c >= p->n[k]);
            }
            return zero ? -1 : gi;
        };
        // wrapped position along direction 1 of coarse index cl_1 + l: the same for every lane;
        // -1 beyond either end of a zero boundary
        const int c0 = p->c[0], n0 = p->n[0];
        auto wrap0 = [&](int l) {
            if (ZB && (zm & 1) && (cl[0] + l < 0 || cl[0] + l >= n0)) return -1;
            const uint32_t xw = (uint32_t)(cl[0] + l + 2 * n0);
            return (int)(xw - FDIV(xw, p->fd_n[0]) * (uint32_t)n0);
        };
        // a grid refined along direction 1 reads its coarse rows from global memory in the first
        // pass; the others stage the coarse block in LDS first
        const bool direct = p->m[0] > 0 && kl > 0;
        Real* src = bufA;
        Real* dst = bufB;
        if (!direct) {
            const int rows = p->rows;
            for (int r = tid; r < rows; r += SGW_BLOCK) rowoff[r] = row_offset(r);
            __syncthreads();
            for (int e = tid; e < p->load_total; e += SGW_BLOCK) {
                const uint32_t row = FDIV((uint32_t)e, p->fd_c[0]);
                const int x0 = e - (int)row * c0;
                const uint32_t xw = (uint32_t)(cl[0] + x0 + 2 * n0);
                const int x = (int)(xw - FDIV(xw, p->fd_n[0]) * (uint32_t)n0);
                if (ZB) {
                    const int ro = rowoff[row];
                    const bool out0 = (zm & 1) && (cl[0] + x0 < 0 || cl[0] + x0 >= n0);
                    bufA[e] = (ro < 0 || out0) ? Real(0) : u[ro + x];
                } else {
                    bufA[e] = u[rowoff[row] + x];
                }
            }
            __syncthreads();
        } else {
            // ---- first pass from global memory: lane L refines coarse row L along direction 1
            const int m = p->m[0];
            const int T0 = F->T[0], lines = p->rows;
            const int R = 1 << m, half = R >> 1, Jk = J0[0];
            const int ifirst = (2 * Jk + R) >> (m + 1);
            const TabC tb = stab + (R - 2);
            for (int L = tid; L < lines; L += SGW_BLOCK) {
                const int ro = row_offset(L);
                const Real* __restrict__ up = u + (ro < 0 ? 0 : ro);
                // coarse value l of the row (0 beyond a zero boundary)
                auto val = [&](int l) {
                    if (!ZB) return up[wrap0(l)];
                    const int x = wrap0(l);
                    return (ro < 0 || x < 0) ? Real(0) : up[x];
                };
                Real* dp = bufB + L * T0;
                Slide<Real> w;
                slide_init<Real, LAG>(w, val(0), val(1), val(2), val(3), val(4), eps4);
                auto run = [&](auto z) {
                    int li = 5;
                    centre_setup<Real, LAG>(z, w);
                    int next = ifirst * R + half - Jk;
#pragma unroll 2
                    for (int t = 0; t < T0; t++) {
                        if (t == next) {
                            slide_next<Real, LAG>(w, val(li), eps4);
                            li++;
                            centre_setup<Real, LAG>(z, w);
                            next += R;
                        }
                        const int q = (Jk + t + half) & (R - 1);
                        dp[t] = centre_value<Real, LAG>(z, tb[q], q == half);
                    }
                };
                run(Centre<Real>());
            }
            __syncthreads();
            src = bufB;
            dst = bufA;
        }
        // ---- passes before the last refined direction: one lane per line, into LDS
#pragma unroll
        for (int k = 0; k < D - 1; k++) {
            const int m = p->m[k];
            if (m == 0 || k >= kl || (k == 0 && direct)) continue;
            const int Tk = F->T[k], ck = p->c[k], inner = F->inner[k];
            const int lines = inner * p->outer[k];
            const int R = 1 << m, half = R >> 1, Jk = J0[k];
            const int ifirst = (2 * Jk + R) >> (m + 1);
            const TabC tb = stab + (R - 2);
            for (int L = tid; L < lines; L += SGW_BLOCK) {
                const int b = (int)FDIV((uint32_t)L, F->fd_inner[k]);
                const int a = L - b * inner;
                const Real* sp = src + a + inner * (ck * b);
                Real* dp = dst + a + inner * (Tk * b);
                Slide<Real> w;
                slide_init<Real, LAG>(w, sp[0], sp[inner], sp[2 * inner], sp[3 * inner], sp[4 * inner], eps4);
                auto run = [&](auto z) {
                    const Real* nx = sp + 5 * inner;
                    centre_setup<Real, LAG>(z, w);
                    int next = ifirst * R + half - Jk; // first node of the next centre
#pragma unroll 4
                    for (int t = 0; t < Tk; t++) {
                        if (t == next) {
                            slide_next<Real, LAG>(w, *nx, eps4);
                            nx += inner;
                            centre_setup<Real, LAG>(z, w);
                            next += R;
                        }
                        const int q = (Jk + t + half) & (R - 1);
                        dp[t * inner] = centre_value<Real, LAG>(z, tb[q], q == half);
                    }
                };
                run(Centre<Real>());
            }
            __syncthreads();
            Real* sw = src;
            src = dst;
            dst = sw;
        }
        const double cg = (double)p->coef;
        if (kl == D - 1) {
            // ---- last direction: the tile has SGW_BLOCK lines along it, lane tid takes line tid
            // and adds its nodes straight into its accumulators (node tid + SGW_BLOCK t)
            const int m = p->m[D - 1];
            const int R = 1 << m, half = R >> 1, Jk = J0[D - 1];
            const int ifirst = (2 * Jk + R) >> (m + 1);
            const TabC tb = stab + (R - 2);
            const Real* sp = src + tid;
            Slide<Real> w;
            slide_init<Real, LAG>(w, sp[0], sp[SGW_BLOCK], sp[2 * SGW_BLOCK], sp[3 * SGW_BLOCK], sp[4 * SGW_BLOCK],
                                  eps4);
            auto run = [&](auto z) {
                const Real* nx = sp + 5 * SGW_BLOCK;
                centre_setup<Real, LAG>(z, w);
                int next = ifirst * R + half - Jk;
#pragma unroll
                for (int t = 0; t < SGW_MAXRP; t++) {
                    if (t < Tlast) {
                        if (t == next) {
                            slide_next<Real, LAG>(w, *nx, eps4);
                            nx += SGW_BLOCK;
                            centre_setup<Real, LAG>(z, w);
                            next += R;
                        }
                        const int q = (Jk + t + half) & (R - 1);
                        acc[t] = fma(cg, (double)centre_value<Real, LAG>(z, tb[q], q == half), acc[t]);
                    }
                }
            };
            run(Centre<Real>());
        } else if (kl >= 0) {
            // ---- the grid whose last direction is not refined: its last pass (direction kl,
            // every later direction at tile extent) node by node, lane tid taking node
            // (a, t) of each of the Tlast slices
            int Jk = J0[0], clk = cl[0];
#pragma unroll
            for (int k = 1; k < D; k++)
                if (k == kl) Jk = J0[k], clk = cl[k];
            const int m = p->m[kl];
            const int R = 1 << m;
            const int inner = F->inner[kl], ck = p->c[kl];
            const int t = (int)FDIV((uint32_t)tid, F->fd_inner[kl]);
            const int a = tid - t * inner;
            const int J = Jk + t;
            const int i = (2 * J + R) >> (m + 1);
            const Real sv = (Real)(J - i * R) * (Real(1) / Real(R));
            const Real* sp = src + a + inner * (i - clk - 2);
            const int slice = inner * ck;
#pragma unroll
            for (int bq = 0; bq < SGW_MAXRP; bq++) {
                if (bq < Tlast) {
                    const Real* q = sp + bq * slice;
                    acc[bq] = fma(cg, (double)interp5<Real>(q[0], q[inner], q[2 * inner], q[3 * inner], q[4 * inner],
                                                            sv, eps4, lagrange),
                                  acc[bq]);
                }
            }
        } else {
            // ---- no direction refined: the coarse block is the tile
#pragma unroll
            for (int r = 0; r < SGW_MAXRP; r++)
                if (r < Tlast) acc[r] = fma(cg, (double)src[tid + r * SGW_BLOCK], acc[r]);
        }
        __syncthreads();
    }
    // ---- write the tile: node tid + SGW_BLOCK t of the tile lies at offset t along the last
    // direction
    int64_t gi = 0, st = 1;
    {
        uint32_t rr = (uint32_t)tid;
#pragma unroll
        for (int k = 0; k < D - 1; k++) {
            const uint32_t q = FDIV(rr, F->fd_T[k]);
            const int c = (int)(rr - q * (uint32_t)F->T[k]);
            rr = q;
            gi += (int64_t)(J0[k] + c) * st;
            st *= F->N;
        }
        gi += (int64_t)J0[D - 1] * st;
    }
#pragma unroll
    for (int r = 0; r < SGW_MAXRP; r++)
        if (r < Tlast) out[gi + (int64_t)r * st] = acc[r];
}

template <typename Real, int D>
__device__ __forceinline__ void prolong_any(ProC pro, FineC F, double* out, int tile)
{
    if constexpr (D >= 3) {
        if (F->lines) {
            if (F->zmask) {
                if (F->lagrange)
                    prolong_tile_lines<Real, D, true, true>(pro, F, out, tile);
                else
                    prolong_tile_lines<Real, D, false, true>(pro, F, out, tile);
            } else {
                if (F->lagrange)
                    prolong_tile_lines<Real, D, true, false>(pro, F, out, tile);
                else
                    prolong_tile_lines<Real, D, false, false>(pro, F, out, tile);
            }
            return;
        }
    }
    if (F->zmask)
        prolong_tile<Real, D, true>(pro, F, out, tile);
    else
        prolong_tile<Real, D, false>(pro, F, out, tile);
}

template <typename Real, int D>
__global__ void __launch_bounds__(SGW_BLOCK) prolong_kernel(const ProDev* pro, const FineDev* fine, double* out,
                                                            int first_tile)
{
    // XCD-aware order: workgroups go to the 8 XCDs in turn, so XCD x takes the contiguous tile
    // range [x n/8, (x+1) n/8) of the launch's tiles first_tile .. first_tile + n - 1 and
    // neighbouring tiles share its L2 (coarse blocks, partly written output lines)
    int b = blockIdx.x;
    const int nt = gridDim.x;
    if ((nt & 7) == 0) b = (b & 7) * (nt >> 3) + (b >> 3);
    prolong_any<Real, D>((ProC)pro, (FineC)fine, out, first_tile + b);
}

// one workgroup per (solve, tile) over many solves of one dimension and precision
template <typename Real, int D>
__global__ void __launch_bounds__(SGW_BLOCK) prolong_many_kernel(const ProItem* items)
{
    const SGW_CONST ProItem* it = (const SGW_CONST ProItem*)items + blockIdx.y;
    if ((int)blockIdx.x >= it->ntiles) return;
    int b = blockIdx.x;
    const int nt = gridDim.x;
    if ((nt & 7) == 0 && it->ntiles == nt) b = (b & 7) * (nt >> 3) + (b >> 3);
    prolong_any<Real, D>((ProC)it->pro, (FineC)it->fine, it->out, b);
}

// ---------------------------------------------------------------- exact solutions

__device__ double u0_sine(const ExactDev& e, const double* x)
{
    double s = 0.0;
    for (int k = 0; k < e.d; k++) s += x[k];
    return e.ip[0] + e.ip[1] * sin(e.ip[2] * s + e.ip[3]);
}

__device__ double f0_maxwell(const ExactDev& e, const double* x)
{
    const int m = e.d / 2;
    double v2 = 0.0, pert = 1.0, norm = 1.0;
    for (int k = 0; k < m; k++) {
        v2 += x[m + k] * x[m + k];
        pert *= cos(e.ip[1] * x[k] + e.ip[2 + k]);
        norm *= 2.0 * M_PI;
    }
    return exp(-0.5 * v2) / sqrt(norm) * (1.0 + e.ip[0] * pert);
}

// Vlasov characteristics x' = v, v' = amp sin(kE x), integrated back from t to 0
// with classical RK4 for every (x node, v node) pair of each x direction.
__global__ void vlasov_foot_kernel(ExactDev e, double* foot)
{
    const int N = e.N;
    const int m = e.d / 2;
    const int64_t total = (int64_t)m * N * N;
    const double amp = e.fp[0], kE = e.fp[1];
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int jx = (int)(idx % N);
        const int jv = (int)((idx / N) % N);
        const int k = (int)(idx / ((int64_t)N * N));
        double X = e.lo[k] + jx * e.h[k];
        double V = e.lo[m + k] + jv * e.h[m + k];
        const int nsteps = (int)ceil(e.t / 1e-3);
        if (nsteps >= 1) {
            const double h = -e.t / nsteps;
            for (int s = 0; s < nsteps; s++) {
                const double k1x = V, k1v = amp * sin(kE * X);
                const double k2x = V + 0.5 * h * k1v, k2v = amp * sin(kE * (X + 0.5 * h * k1x));
                const double k3x = V + 0.5 * h * k2v, k3v = amp * sin(kE * (X + 0.5 * h * k2x));
                const double k4x = V + h * k3v, k4v = amp * sin(kE * (X + h * k3x));
                X += h / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
                V += h / 6.0 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
            }
        }
        foot[2 * idx] = X;
        foot[2 * idx + 1] = V;
    }
}

__global__ void exact_kernel(ExactDev e, double* out)
{
    const int N = e.N;
    int64_t total = 1;
    for (int k = 0; k < e.d; k++) total *= N;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int j[SGW_MAX_DIM] = {0, 0, 0, 0};
        double x[SGW_MAX_DIM] = {0.0, 0.0, 0.0, 0.0};
        int64_t r = idx;
        for (int k = 0; k < e.d; k++) {
            j[k] = (int)(r % N);
            r /= N;
            x[k] = e.lo[k] + j[k] * e.h[k];
        }
        double v;
        if (e.flux == SGW_FLUX_ADVECTION) {
            for (int k = 0; k < e.d; k++) x[k] -= e.fp[k] * e.t;
            v = (e.ic == SGW_IC_SINE) ? u0_sine(e, x) : f0_maxwell(e, x);
        } else if (e.flux == SGW_FLUX_BURGERS) {
            // u = w(xi), xi = sum x_k, w = g(xi - d w t): Newton's method from w = g(xi)
            double xi = 0.0;
            for (int k = 0; k < e.d; k++) xi += x[k];
            const double c0 = e.ip[0], A = e.ip[1], kap = e.ip[2], ph = e.ip[3], dd = e.d;
            double w = c0 + A * sin(kap * xi + ph);
            for (int it = 0; it < 100; it++) {
                const double arg = kap * (xi - dd * w * e.t) + ph;
                const double Fv = w - c0 - A * sin(arg);
                const double dF = 1.0 + A * cos(arg) * kap * dd * e.t;
                const double dw = Fv / dF;
                w -= dw;
                if (fabs(dw) < 1e-16 * (1.0 + fabs(w))) break;
            }
            v = w;
        } else {
            const int m = e.d / 2;
            double y[SGW_MAX_DIM] = {0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < m; k++) {
                const int64_t p = ((int64_t)k * N + j[m + k]) * N + j[k];
                y[k] = e.foot[2 * p];
                y[m + k] = e.foot[2 * p + 1];
            }
            v = f0_maxwell(e, y);
        }
        out[idx] = v;
    }
}

// ---------------------------------------------------------------- norms (fixed order)

// First pass: workgroup blk of `parts` reduces its strided share of |a - b|
// (sum and NaN-keeping max) in a fixed tree order.
__device__ void norms_partial_block(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                    int parts, int blk, double* out2)
{
    __shared__ double ss[SGW_BLOCK], sm[SGW_BLOCK];
    double s = 0.0, mx = 0.0;
    for (int64_t i = blk * (int64_t)SGW_BLOCK + threadIdx.x; i < n; i += (int64_t)parts * SGW_BLOCK) {
        const double d = fabs(a[i] - b[i]);
        s += d;
        mx = (d > mx || d != d) ? d : mx;
    }
    ss[threadIdx.x] = s;
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int w = SGW_BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            ss[threadIdx.x] += ss[threadIdx.x + w];
            const double o = sm[threadIdx.x + w];
            sm[threadIdx.x] = (o > sm[threadIdx.x] || o != o) ? o : sm[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = ss[0];
        out2[1] = sm[0];
    }
}

// Second pass: the np partials, zero-padded to SGW_NPART, in a fixed tree order.
__device__ void norms_final_block(const double* partials, int np, int64_t n, double* result)
{
    __shared__ double ss[SGW_NPART], sm[SGW_NPART];
    for (int i = threadIdx.x; i < SGW_NPART; i += blockDim.x) {
        ss[i] = i < np ? partials[2 * i] : 0.0;
        sm[i] = i < np ? partials[2 * i + 1] : 0.0;
    }
    __syncthreads();
    for (int w = SGW_NPART / 2; w > 0; w >>= 1) {
        for (int i = threadIdx.x; i < w; i += blockDim.x) {
            ss[i] += ss[i + w];
            const double o = sm[i + w];
            sm[i] = (o > sm[i] || o != o) ? o : sm[i];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        result[0] = n > 0 ? ss[0] / (double)n : 0.0;
        result[1] = sm[0];
    }
}

__global__ void norms_partial_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                     double* partials)
{
    norms_partial_block(a, b, n, gridDim.x, blockIdx.x, partials + 2 * blockIdx.x);
}

__global__ void norms_final_kernel(const double* partials, int np, int64_t n, double* result)
{
    norms_final_block(partials, np, n, result);
}

// Many pairs in one launch: blockIdx.y is the pair, the same per-pair order as above.
__global__ void norms_partial_many_kernel(const NormItem* items, double* partials, int stride)
{
    const NormItem* it = items + blockIdx.y;
    if ((int)blockIdx.x >= it->parts) return;
    norms_partial_block(it->a, it->b, it->n, it->parts, blockIdx.x,
                        partials + (size_t)blockIdx.y * stride + 2 * blockIdx.x);
}

__global__ void norms_final_many_kernel(const NormItem* items, const double* partials, int stride)
{
    const NormItem* it = items + blockIdx.x;
    norms_final_block(partials + (size_t)blockIdx.x * stride, it->parts, it->n, it->result);
}

// ---------------------------------------------------------------- Vlasov-Maxwell fields

// Thread (q, J): field q (B_3, E_1, E_2) at finest x_2 node J, the combination over the grids in
// plan order of c_g times the grid's field at J, prolongated along x_2 as in Sec. 2.2.1 (node J
// refines coarse node i = floor(J/R + 1/2) at offset s = J/R - i, periodic stencil i-2..i+2).
__global__ void fields_combine_kernel(const GridDev* grids, const ProDev* pro, const FineDev* fine, double* out)
{
    const int N = fine->N, G = fine->G;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * N) return;
    const int q = e / N, J = e - q * N;
    const double eps4 = 4.0 * fine->eps;
    const int lagrange = fine->lagrange;
    double acc = 0.0;
    for (int g = 0; g < G; g++) {
        const GridDev* gd = grids + g;
        const int n0 = gd->n[0], m = pro[g].m[0];
        const double* f = (const double*)((const char*)gd->u + gd->fld_bytes) + q * n0;
        double v;
        if (m == 0) {
            v = f[J];
        } else {
            const int R = 1 << m;
            const int i = (2 * J + R) >> (m + 1);
            const double sv = (double)(J - i * R) / (double)R;
            double st[5];
            for (int t = 0; t < 5; t++) {
                int p = i - 2 + t;
                p += p < 0 ? n0 : 0;
                p -= p >= n0 ? n0 : 0;
                st[t] = f[p];
            }
            v = interp5<double>(st[0], st[1], st[2], st[3], st[4], sv, eps4, lagrange);
        }
        acc = fma((double)pro[g].coef, v, acc);
    }
    out[e] = acc;
}

} // namespace

hipError_t launch_fields_combine(const GridDev* grids_dev, const ProDev* pro_dev, const FineDev& fine_host,
                                 const FineDev* fine_dev, double* out, hipStream_t s)
{
    const int n = 3 * fine_host.N;
    hipLaunchKernelGGL(fields_combine_kernel, dim3((n + SGW_BLOCK - 1) / SGW_BLOCK), dim3(SGW_BLOCK), 0, s, grids_dev,
                       pro_dev, fine_dev, out);
    return hipGetLastError();
}

hipError_t launch_prolong(const ProDev* pro_dev, const FineDev* fine_dev, const FineDev& fh, int precision,
                          size_t lds_bytes, double* out, int first_tile, int num_tiles, hipStream_t s)
{
    if (num_tiles <= 0) return hipSuccess;
#define SGW_PRO(R, DD)                                                                                       \
    hipLaunchKernelGGL((prolong_kernel<R, DD>), dim3(num_tiles), dim3(SGW_BLOCK), lds_bytes, s, pro_dev, fine_dev, \
                       out, first_tile)
    if (precision == SGW_FP64) {
        switch (fh.d) {
        case 1: SGW_PRO(double, 1); break;
        case 2: SGW_PRO(double, 2); break;
        case 3: SGW_PRO(double, 3); break;
        default: SGW_PRO(double, 4); break;
        }
    } else {
        switch (fh.d) {
        case 1: SGW_PRO(float, 1); break;
        case 2: SGW_PRO(float, 2); break;
        case 3: SGW_PRO(float, 3); break;
        default: SGW_PRO(float, 4); break;
        }
    }
#undef SGW_PRO
    return hipGetLastError();
}

hipError_t launch_prolong_many(const ProItem* items, int nitems, int max_tiles, int d, int precision,
                               size_t lds_bytes, hipStream_t s)
{
    if (nitems <= 0 || max_tiles <= 0) return hipSuccess;
#define SGW_PROM(R, DD) \
    hipLaunchKernelGGL((prolong_many_kernel<R, DD>), dim3(max_tiles, nitems), dim3(SGW_BLOCK), lds_bytes, s, items)
    if (precision == SGW_FP64) {
        switch (d) {
        case 1: SGW_PROM(double, 1); break;
        case 2: SGW_PROM(double, 2); break;
        case 3: SGW_PROM(double, 3); break;
        default: SGW_PROM(double, 4); break;
        }
    } else {
        switch (d) {
        case 1: SGW_PROM(float, 1); break;
        case 2: SGW_PROM(float, 2); break;
        case 3: SGW_PROM(float, 3); break;
        default: SGW_PROM(float, 4); break;
        }
    }
#undef SGW_PROM
    return hipGetLastError();
}

hipError_t launch_exact(const ExactDev& e, double* out, double* foot_scratch, hipStream_t s)
{
    ExactDev ee = e;
    if (e.flux == SGW_FLUX_VLASOV_FIXED_E) {
        ee.foot = foot_scratch;
        hipLaunchKernelGGL(vlasov_foot_kernel, dim3(256), dim3(SGW_BLOCK), 0, s, ee, foot_scratch);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(exact_kernel, dim3(2048), dim3(SGW_BLOCK), 0, s, ee, out);
    return hipGetLastError();
}

int norms_parts(int64_t n)
{
    const int64_t p = (n + SGW_BLOCK - 1) / SGW_BLOCK;
    return p < 1 ? 1 : (p > SGW_NPART ? SGW_NPART : (int)p);
}

hipError_t launch_norms(const double* a, const double* b, int64_t n, double* partials, double* result, hipStream_t s)
{
    const int parts = norms_parts(n);
    hipLaunchKernelGGL(norms_partial_kernel, dim3(parts), dim3(SGW_BLOCK), 0, s, a, b, n, partials);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(SGW_BLOCK), 0, s, partials, parts, n, result);
    return hipGetLastError();
}

hipError_t launch_norms_many(const NormItem* items, int n, int max_parts, double* partials, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(norms_partial_many_kernel, dim3(max_parts, n), dim3(SGW_BLOCK), 0, s, items, partials,
                       2 * max_parts);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(norms_final_many_kernel, dim3(n), dim3(SGW_BLOCK), 0, s, items, partials, 2 * max_parts);
    return hipGetLastError();
}
