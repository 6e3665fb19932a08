// The fused WENO5-LF + TVD-RK3 stage kernel of libsgweno (the time-marching hot
// loop); the kernels around it (restriction, time step, flags) are in
// kernels_step.hip.
//
// The stage kernel follows Sec. 2.1 of the paper: for every direction k the
// flux f_k is split by the global Lax-Friedrichs rule (eq. LFflux) into
// f^+ = (f + alpha u)/2 and f^- = (f - alpha u)/2, the interface flux at
// x_{i+1/2} is the WENO5 reconstruction of f^+ from (i-2..i+2) plus the mirror
// reconstruction of f^- from (i+3..i-1) (eqs. 2.7, 2.7.1, 2.6, 2.7.2), and the
// operator is the conservative difference of eq. (2.9), summed over k.  The
// TVD-RK3 (Shu-Osher) stage combination is applied in the same pass; a box that
// is its whole grid runs all three stages in one launch.
//
// Layout: one workgroup owns a box of one component grid.  The box and a
// 3-node halo in every direction where the box does not span the grid are
// staged in LDS (periodic wrap of the halo applied while loading; within a box
// that spans its grid the wrap is resolved on the LDS indices), one direction at
// a time the interface fluxes of the box go to one of two alternating LDS
// arrays, and each thread accumulates the flux differences of its nodes in
// registers.  Launches are persistent: a workgroup takes a contiguous range of a
// box list that covers many grids of many solves.
#include "sgw_internal.h"

// Only the explicit fma calls fuse: with contraction left to the compiler, a product that
// feeds an addition could fuse in one kernel instantiation and not in another, and the
// fused and split kernels would round differently.
#pragma clang fp contract(off)

namespace {

// descriptors live in the constant address space for the duration of a launch
#define SGW_CONST __attribute__((address_space(4)))
typedef const SGW_CONST GridDev* GridC;
// LDS indices stay below 2^16: the full-rate 24-bit multiply is exact for them
#define M24(a, b) __mul24((a), (b))

// c + num / den: one reciprocal and an fma in FP32; in FP64 the hardware
// reciprocal, one Newton step and a residual correction of the quotient (den > 0)
__device__ __forceinline__ float wsum(float c, float num, float den) { return fmaf(num, __builtin_amdgcn_rcpf(den), c); }
__device__ __forceinline__ double wsum(double c, double num, double den)
{
    double r = __builtin_amdgcn_rcp(den);
    r = fma(fma(-den, r, 1.0), r, r);
    double q = num * r;
    q = fma(fma(-den, q, num), r, q);
    return c + q;
}

// max(m, |x|) for m >= 0 that keeps a NaN: the bit patterns of non-negative floats
// order as unsigned integers, with every NaN above infinity
__device__ __forceinline__ float absmax(float m, float x)
{
    return __uint_as_float(max(__float_as_uint(m), __float_as_uint(x) & 0x7fffffffu));
}
__device__ __forceinline__ double absmax(double m, double x)
{
    const double a = fabs(x);
    return (a > m || a != a) ? a : m;
}

// WENO5 flux (eqs. 2.7, 2.7.1, 2.6, 2.7.2) of the positive-wind big stencil
// (a..e) = (f_{i-2} .. f_{i+2}), written in differences so that neighbouring
// interfaces share them: c = f_i, D0..D3 = b-a, c-b, d-c, e-d.  The candidate
// values are q_r - c = (5 D1 - 2 D0)/6, (D1 + 2 D2)/6, (4 D2 - D3)/6 and the
// smoothness indicators beta_r = 13/12 s_r^2 + 1/4 g_r^2 with the second
// differences s_r = a-2b+c, b-2c+d, c-2d+e and g_r = 3 D1 - D0, D1 + D2, D3 - 3 D2.
// The normalised weights are unchanged when eps and every beta_r are scaled by
// the same factor, so 4 (eps + beta_r) = T_r + g_r^2 with
// T_r = 13/3 s_r^2 + 4 eps is used (T_r belongs to a second difference, which
// three neighbouring interfaces share), and the weights d_r/(...)^2 are
// normalised with one division (numerator and denominator times the product of
// the three squares).  R_r = d_r (q_r - c).
template <typename Real, bool LINEAR>
__device__ __forceinline__ Real weno5s(Real c, Real D0, Real D1, Real D2, Real D3, Real T0, Real T1, Real T2)
{
    // every multiply-add is an explicit fma: a flux then rounds the same wherever it sits in a
    // window, so results do not depend on the box decomposition
    const Real d2 = Real(1.2 / 6.0) * D2;
    const Real R0 = fma(Real(0.5 / 6.0), D1, Real(-0.2 / 6.0) * D0);
    const Real R1 = fma(Real(0.6 / 6.0), D1, d2);
    const Real R2 = fma(Real(-0.3 / 6.0), D3, d2);
    if (LINEAR) return c + ((R0 + R1) + R2);
    const Real g0 = fma(Real(3), D1, -D0), g1 = D1 + D2, g2 = fma(Real(-3), D2, D3);
    Real e0 = fma(g0, g0, T0);
    Real e1 = fma(g1, g1, T1);
    Real e2 = fma(g2, g2, T2);
    e0 *= e0;
    e1 *= e1;
    e2 *= e2;
    const Real P12 = e1 * e2, P02 = e0 * e2, P01 = e0 * e1;
    const Real num = fma(R2, P01, fma(R1, P02, R0 * P12));
    const Real den = fma(Real(0.3), P01, fma(Real(0.6), P02, Real(0.1) * P12));
    return wsum(c, num, den);
}

// NI consecutive interface fluxes F_{i+1/2}, i = i0..i0+NI-1, from the NI+5 split values
// f^+-_{i0-2} .. f^+-_{i0+NI+2} of one line (eq. LFflux): the positive-wind reconstruction of
// f^+ on i-2..i+2 plus the mirrored one of f^- on i+3..i-1.  A split part flagged identically zero
// contributes exactly zero and is skipped.  epsT = 4 eps.  LINEAR: the linear weights d_r.
template <typename Real, int NI, bool LINEAR>
__device__ __forceinline__ void split_fluxes(const Real* pv, const Real* mv, bool plus, bool minus, Real epsT,
                                             Real* F)
{
    if (plus) {
        Real dp[NI + 4], tp[NI + 4];
#pragma unroll
        for (int q = 0; q < NI + 4; q++) dp[q] = pv[q + 1] - pv[q];
        tp[0] = Real(0);
#pragma unroll
        for (int q = 1; q < NI + 4; q++) {
            const Real sp = dp[q] - dp[q - 1];
            tp[q] = fma(Real(13.0 / 3.0) * sp, sp, epsT);
        }
#pragma unroll
        for (int s = 0; s < NI; s++)
            F[s] = weno5s<Real, LINEAR>(pv[s + 2], dp[s], dp[s + 1], dp[s + 2], dp[s + 3], tp[s + 1], tp[s + 2],
                                        tp[s + 3]);
    } else {
#pragma unroll
        for (int s = 0; s < NI; s++) F[s] = Real(0);
    }
    if (minus) {
        Real dm[NI + 4], tm[NI + 4];
#pragma unroll
        for (int q = 0; q < NI + 4; q++) dm[q] = mv[q + 1] - mv[q];
        tm[0] = Real(0);
#pragma unroll
        for (int q = 1; q < NI + 4; q++) {
            const Real sm = dm[q] - dm[q - 1];
            tm[q] = fma(Real(13.0 / 3.0) * sm, sm, epsT);
        }
#pragma unroll
        for (int s = 0; s < NI; s++)
            F[s] += weno5s<Real, LINEAR>(mv[s + 3], -dm[s + 4], -dm[s + 3], -dm[s + 2], -dm[s + 1], tm[s + 4],
                                         tm[s + 3], tm[s + 2]);
    }
}

// The same from the NI+5 values u_{i0-2} .. u_{i0+NI+2} of one line: LF split f^+- (eq.
// LFflux) of Burgers' flux or of a linear flux c u (f^+- = cp u, cm u with cp, cm = (c +- alpha)/2;
// a part with cp or cm = 0 is skipped).
template <typename Real, int NI, bool LINEAR>
__device__ __forceinline__ void window_fluxes(const Real* v, bool burgers, Real cp, Real cm, Real alpha, Real epsT,
                                              Real* F)
{
    // the flux type and the wind sides are uniform: branch once per window, not per value
    Real pv[NI + 5], mv[NI + 5];
    if (burgers) {
        const Real ha = Real(0.5) * alpha;
#pragma unroll
        for (int q = 0; q < NI + 5; q++) {
            // f^+ = (u^2/2 + alpha u)/2 = u (u/4 + alpha/2), f^- = f^+ - alpha u
            pv[q] = v[q] * fma(Real(0.25), v[q], ha);
            mv[q] = fma(-alpha, v[q], pv[q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < NI + 5; q++) {
            pv[q] = cp * v[q];
            mv[q] = cm * v[q];
        }
    }
    split_fluxes<Real, NI, LINEAR>(pv, mv, burgers || cp != Real(0), burgers || cm != Real(0), epsT, F);
}

// One RK stage of one box (FUSED = false), or all three stages of a box that is its
// whole grid (FUSED = true): the stage results stay in LDS, u^n is read once and u^{n+1}
// written once, and the wave speed of each stage input is a workgroup maximum.  red holds
// one double per wavefront.
// ROWS: t_1 divides the block size, so a thread's nodes share one column and step through
// the rows by a fixed count (one variant per case, chosen once per box).
template <typename Real, int D, bool FUSED, bool ROWS>
__device__ __forceinline__ void stage_box(GridC g, int box, int stage, Real* su, Real* sf, double* red)
{
    constexpr int SEG = sgw_seg(D);
    int tid = threadIdx.x;
    const double dt = ((const SGW_CONST ReqDev*)g->req)->dt;
    const Real dtr = (Real)dt;

    int o[D];
    {
        int r = box;
        for (int k = 0; k < D; k++) {
            const int q = r / g->ntile[k];
            o[k] = (r - q * g->ntile[k]) * g->t[k];
            r = q;
        }
    }
    const Real* __restrict__ in = (const Real*)(FUSED || stage == 0 ? g->u : stage == 1 ? g->a : g->b);
    Real* __restrict__ out = (Real*)(FUSED || stage == 2 ? g->u : stage == 0 ? g->a : g->b);
    const Real* __restrict__ u0 = (const Real*)g->u;

    // the wave-speed slot the next stage reads is cleared by the stage before it
    if (!FUSED && g->dyn_alpha && box == 0 && tid == 0) g->alpha[(stage + 2) % 3] = 0ull;

    const int core_total = g->core_total;
    const int t0 = g->t[0];
    const int RS = g->RS;         // LDS row stride of the core box (odd: conflict-free columns)
    const bool whole = g->whole;  // the box is the whole grid: global index = core index

    // This thread's nodes are e = tid + r * SGW_BLOCK (row-major in the box): row `line` of
    // t_0 values and column c0.  When t_0 divides the block size all of them share the column
    // and the row advances by rline per r.
    const int rline = g->rline;
    uint32_t l00 = FDIV((uint32_t)tid, g->fd_t[0]);
    int c00 = tid - M24((int)l00, t0);
    auto node_rc = [&](int r, int& line, int& c0) {
        if (ROWS) {
            line = (int)l00 + r * rline;
            c0 = c00;
        } else {
            const int e = tid + r * SGW_BLOCK;
            const uint32_t q = FDIV((uint32_t)e, g->fd_t[0]);
            line = (int)q;
            c0 = e - M24((int)q, t0);
        }
    };
    // 3D/4D: global offsets of the box rows (and of the halo slab rows) go to an LDS table
    // once per box, so a staged value costs one table read instead of a division per direction
    int* __restrict__ rt = (int*)(sf + 2 * g->sf_elems);
    if constexpr (D >= 3) {
        if (!whole) {
            for (int ln = tid; ln < g->lines; ln += SGW_BLOCK) {
                uint32_t r = (uint32_t)ln;
                int gi = o[0];
#pragma unroll
                for (int j = 1; j < D; j++) {
                    const uint32_t q = FDIV(r, g->fd_t[j]);
                    gi += (o[j] + (int)(r - q * (uint32_t)g->t[j])) * g->stride[j];
                    r = q;
                }
                rt[ln] = gi;
            }
#pragma unroll
            for (int k = 1; k < D; k++) {
                if (!g->halo[k]) continue;
                const int nr = g->slab_n[k] / t0; // slab rows per side
                for (int e = tid; e < 2 * nr; e += SGW_BLOCK) {
                    const int side = e >= nr ? 1 : 0;
                    uint32_t r = (uint32_t)(e - side * nr);
                    int gi = o[0];
#pragma unroll
                    for (int j = 1; j < D; j++) {
                        int x;
                        if (j == k) {
                            const uint32_t q = r / 3u;
                            const int c = (int)(r - 3u * q);
                            r = q;
                            x = side ? o[j] + g->t[j] + c : o[j] - 3 + c;
                            x += (x < 0) ? g->n[j] : 0;
                            x -= (x >= g->n[j]) ? g->n[j] : 0;
                        } else {
                            const uint32_t q = FDIV(r, g->fd_t[j]);
                            x = o[j] + (int)(r - q * (uint32_t)g->t[j]);
                            r = q;
                        }
                        gi += x * g->stride[j];
                    }
                    rt[g->rt_off[k] + e] = gi;
                }
            }
            __syncthreads();
        }
    }
    auto node_gi = [&](int r, int line, int c0) -> int {
        if (whole) return tid + r * SGW_BLOCK;
        if constexpr (D == 1) return o[0] + c0;
        else if constexpr (D == 2) return (o[0] + c0) + (o[1] + line) * g->stride[1];
        else return rt[line] + c0;
    };

    // ---- core box -> LDS
#pragma unroll
    for (int r = 0; r < SGW_MAXR; r++) {
        if (tid + r * SGW_BLOCK < core_total) {
            int line, c0;
            node_rc(r, line, c0);
            su[c0 + M24(RS, line)] = in[node_gi(r, line, c0)];
        }
    }
    // ---- halo slabs: the core box with extent 3 in direction k, periodic wrap on the global index
#pragma unroll
    for (int k = 0; k < D; k++) {
        if (!g->halo[k]) continue;
        if constexpr (D >= 3) {
            // rows of the slab from the tables: direction 1 slabs are 3 values at each core row,
            // the others rows of t_1 values
            const int sn = g->slab_n[k];
            for (int e = tid; e < 2 * sn; e += SGW_BLOCK) {
                const int side = e >= sn ? 1 : 0;
                const int r = e - side * sn;
                int gi, li;
                if (k == 0) {
                    const int ln = (int)((uint32_t)r / 3u);
                    const int c = r - 3 * ln;
                    int x = side ? o[0] + t0 + c : o[0] - 3 + c;
                    x += (x < 0) ? g->n[0] : 0;
                    x -= (x >= g->n[0]) ? g->n[0] : 0;
                    gi = rt[ln] - o[0] + x;
                    li = r;
                } else {
                    const int rho = (int)FDIV((uint32_t)r, g->fd_t[0]);
                    const int c0 = r - M24(rho, t0);
                    gi = rt[g->rt_off[k] + side * (sn / t0) + rho] + c0;
                    li = c0 + M24(RS, rho);
                }
                su[(side ? g->slab_hi[k] : g->slab_lo[k]) + li] = in[gi];
            }
            continue;
        }
        const int sn = g->slab_n[k];
        const int w0 = k == 0 ? 3 : RS;
        for (int e = tid; e < 2 * sn; e += SGW_BLOCK) {
            const int side = e >= sn ? 1 : 0;
            uint32_t r = (uint32_t)(e - side * sn);
            int gi = 0, li = 0, mul = 1;
#pragma unroll
            for (int j = 0; j < D; j++) {
                int c, x;
                if (j == k) {
                    const uint32_t q = r / 3u;
                    c = (int)(r - 3u * q);
                    r = q;
                    x = side ? o[j] + g->t[j] + c : o[j] - 3 + c;
                } else {
                    const uint32_t q = FDIV(r, g->fd_t[j]);
                    c = (int)(r - q * (uint32_t)g->t[j]);
                    r = q;
                    x = o[j] + c;
                }
                x += (x < 0) ? g->n[j] : 0;
                x -= (x >= g->n[j]) ? g->n[j] : 0;
                gi += x * g->stride[j];
                li += c * mul;
                mul *= (j == 0) ? w0 : (j == k ? 3 : g->t[j]);
            }
            su[(side ? g->slab_hi[k] : g->slab_lo[k]) + li] = in[gi];
        }
    }
    __syncthreads();

    const Real epsT = (Real)(g->eps * 4.0);
    const int linear = g->linear;
    const bool burgers = g->flux == SGW_FLUX_BURGERS;
    Real dyn_alpha = Real(0);
    if (g->dyn_alpha) dyn_alpha = (Real)__longlong_as_double((long long)g->alpha[FUSED ? 0 : stage]);
    // the fused launch keeps the split stages' invariant between steps: slot 0 holds
    // max |u^n|, slots 1 and 2 are zero
    if (FUSED && g->dyn_alpha && tid == 0) {
        g->alpha[1] = 0ull;
        g->alpha[2] = 0ull;
    }

    const int s_first = FUSED ? 0 : stage, s_last = FUSED ? 2 : stage;
#pragma unroll 1
    for (int s = s_first; s <= s_last; s++) {
    if (FUSED) {
        // the node indices are recomputed in every stage rather than kept live across the
        // three (an empty asm hides their invariance from the compiler)
        asm volatile("" : "+v"(tid), "+v"(l00), "+v"(c00));
    }
    Real acc[SGW_MAXR];
#pragma unroll
    for (int r = 0; r < SGW_MAXR; r++) acc[r] = Real(0);

#pragma unroll
    for (int k = 0; k < D; k++) {
        const int hf = g->halo[k] ? 1 : 0;
        const int tk = g->t[k];
        const bool pow2 = (tk & (tk - 1)) == 0;
        const int CSk = g->CS[k];
        const int LSk = (k == 0) ? 1 : g->LS[k];
        const int Ik = g->I[k];
        const int slo = g->slab_lo[k], shi = g->slab_hi[k];
        const Real alpha = g->dyn_alpha ? dyn_alpha : (Real)g->alpha_c[k];
        const double* __restrict__ ctab = g->coef[k];
        const int csrc = g->coef_src[k];
        const Real cconst = (Real)g->lin_c[k];
        // directions alternate between two flux buffers: one barrier per direction
        Real* __restrict__ sfk = (k & 1) ? sf + g->sf_elems : sf;
        // ---- interface fluxes F_{i+1/2} of the box in direction k -> sf.  Each thread takes
        //      SEG consecutive interfaces of one line from a window of SEG + 5 values;
        //      consecutive lanes take neighbouring lines (stride 1, or RS for direction 1).
        const int stot = g->seg_total[k];
        const int Lk = g->nlines[k];
        const int nint = g->nint[k];
        const int int_total = M24(Lk, nint);
        const bool seg_exact = Ik % SEG == 0;
        for (int w = tid; w < stot; w += SGW_BLOCK) {
            // interior segments (window inside the core, no wrap) first, then the edge ones;
            // consecutive lanes take neighbouring lines of the same segment
            const bool interior = w < int_total;
            // the contiguous fast path for whole wavefronts of interior segments only, so that no
            // wavefront runs both paths
            const bool fast = w < (int_total & ~63);
            const int wl = interior ? w : w - int_total;
            const uint32_t sq = FDIV((uint32_t)wl, g->fd_lines_k[k]);
            const int line = wl - M24((int)sq, Lk);
            const int seg = interior ? 1 + (int)sq : (sq == 0 ? 0 : (int)sq + nint);
            int base_core, base_slab, lbase, fbase, fstride;
            if (k == 0) {
                base_core = M24(line, RS);
                base_slab = M24(line, 3);
                lbase = M24(line, t0);
                fbase = M24(line, RS);
                fstride = 1;
            } else {
                const uint32_t outer = FDIV((uint32_t)line, g->fd_CS[k]);
                const int inner = line - M24((int)outer, CSk);
                int inner_lds = inner;
                if (k >= 2) inner_lds += M24(RS - t0, (int)FDIV((uint32_t)inner, g->fd_t[0]));
                base_core = inner_lds + M24((int)outer, LSk * tk);
                base_slab = inner_lds + M24((int)outer, 3 * LSk);
                lbase = inner + M24((int)outer, CSk * tk);
                fbase = inner + M24((int)outer, CSk * Ik);
                fstride = CSk;
            }
            const int i0 = seg * SEG - hf; // first interface: x_{i0+1/2}
            Real v[SEG + 5];
            if (fast) {
                const int a0 = base_core + M24(i0 - 2, LSk);
#pragma unroll
                for (int q = 0; q < SEG + 5; q++) v[q] = su[a0 + (k == 0 ? q : M24(q, LSk))];
            } else if (hf) {
                // window position p < 0 lies in the low slab, p >= t in the high one: pick the
                // base by selects (no divergent branches), then add p times the line stride
                const int blo = slo + base_slab + 3 * LSk, bhi = shi + base_slab - tk * LSk;
#pragma unroll
                for (int q = 0; q < SEG + 5; q++) {
                    int p = i0 + q - 2;
                    p = p > tk + 2 ? tk + 2 : p; // past the last interface: valid data, result unused
                    const int bs = p < 0 ? blo : base_core;
                    v[q] = su[(p >= tk ? bhi : bs) + M24(p, LSk)];
                }
            } else if (pow2) {
                // the box spans the grid and t is a power of two: the periodic wrap is a mask
                // (window positions run from -2 up, two's complement wraps them)
#pragma unroll
                for (int q = 0; q < SEG + 5; q++) {
                    const int p = (i0 + q - 2) & (tk - 1);
                    v[q] = su[base_core + (k == 0 ? p : M24(p, LSk))];
                }
            } else {
#pragma unroll
                for (int q = 0; q < SEG + 5; q++) {
                    int p = i0 + q - 2;
                    p += (p < 0) ? tk : 0;
                    p -= (p >= tk) ? tk : 0;
                    p -= (p >= tk) ? tk : 0;
                    v[q] = su[base_core + M24(p, LSk)];
                }
            }
            Real cp = Real(0), cm = Real(0);
            if (!burgers) {
                // f_k = c u along the line (advection, Vlasov): f^+- = (c +- alpha)/2 u
                Real c = cconst;
                if (csrc >= 0) {
                    const uint32_t q = FDIV((uint32_t)lbase, g->fd_CS[csrc]);
                    c = (Real)ctab[o[csrc] + (int)(q - FDIV(q, g->fd_t[csrc]) * (uint32_t)g->t[csrc])];
                }
                cp = Real(0.5) * (c + alpha);
                cm = Real(0.5) * (c - alpha);
            }
            Real F[SEG];
            // the weight type is uniform over the launch's grids: one branch per window
            if (linear)
                window_fluxes<Real, SEG, true>(v, burgers, cp, cm, alpha, epsT, F);
            else
                window_fluxes<Real, SEG, false>(v, burgers, cp, cm, alpha, epsT, F);
            Real* __restrict__ fp = sfk + fbase + M24(seg * SEG, fstride);
            if (seg_exact) {
                // the segments tile the interfaces of the line: no store to skip
#pragma unroll
                for (int s = 0; s < SEG; s++) fp[k == 0 ? s : M24(s, fstride)] = F[s];
            } else {
#pragma unroll
                for (int s = 0; s < SEG; s++) {
                    const int ip = seg * SEG + s; // i + hf
                    if (interior || ip < Ik) fp[k == 0 ? s : M24(s, fstride)] = F[s];
                }
            }
        }
        __syncthreads();
        // ---- flux differences of eq. (2.9) for the nodes this thread owns
        const Real ih = (Real)g->inv_h[k];
        // ROWS: a thread's nodes share one column, so along direction 0 the lower interface
        // sits at the same offset from the upper one in every row
        const int fhi0 = c00 + hf + M24((int)l00, RS);
        const int dlo0 = (hf || c00 > 0) ? -1 : t0 - 1;
        int fstep0 = M24(rline, RS);
        // kept opaque: otherwise the row offsets are refactored into a full 32-bit multiply per row
        asm volatile("" : "+s"(fstep0));
#pragma unroll
        for (int r = 0; r < SGW_MAXR; r++) {
            const int e = tid + r * SGW_BLOCK;
            if (e < core_total) {
                int fhi, flo;
                if (k == 0 && ROWS) {
                    fhi = fhi0 + r * fstep0;
                    flo = fhi + dlo0;
                } else if (k == 0) {
                    // interface rows share the core row stride RS
                    int line, c0;
                    node_rc(r, line, c0);
                    fhi = c0 + hf + M24(line, RS);
                    flo = (hf || c0 > 0) ? fhi - 1 : fhi + t0 - 1;
                } else {
                    int hi = 0, lo = e;
                    if (k < D - 1) {
                        hi = (int)FDIV((uint32_t)e, g->fd_CSt[k]);
                        lo = e - M24(hi, (int)g->fd_CSt[k].d);
                    }
                    fhi = lo + hf * CSk + M24(hi, CSk * Ik);
                    flo = (hf || lo >= CSk) ? fhi - CSk : fhi + (tk - 1) * CSk;
                }
                acc[r] = fma(sfk[flo] - sfk[fhi], ih, acc[r]);
            }
        }
    }

    // ---- TVD-RK3 stage: u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1)); u = 1/3 u + 2/3 (u2 + dt L(u2))
    Real amax = Real(0);
#pragma unroll
    for (int r = 0; r < SGW_MAXR; r++) {
        if (tid + r * SGW_BLOCK < core_total) {
            int line, c0;
            node_rc(r, line, c0);
            const int gi = node_gi(r, line, c0);
            const int li = c0 + M24(RS, line);
            const Real val = fma(dtr, acc[r], su[li]);
            Real res;
            if (s == 0) res = val;
            else if (s == 1) res = fma(Real(0.75), u0[gi], Real(0.25) * val);
            else res = fma(Real(1.0 / 3.0), u0[gi], Real(2.0 / 3.0) * val);
            // the fused launch keeps the first two stage results in LDS (each thread
            // rewrites its own nodes; every flux read of this stage is behind a barrier)
            if (FUSED && s < 2)
                su[li] = res;
            else
                out[gi] = res;
            amax = absmax(amax, res);
        }
    }
    if (!FUSED) {
        // one atomic max per wavefront on the bit pattern (order-free, no barrier)
        if (g->dyn_alpha) {
            const double m = wave_max((double)amax);
            if ((tid & 63) == 0) atomicMax(g->alpha + (stage + 1) % 3, (unsigned long long)__double_as_longlong(m));
        }
    } else if (g->dyn_alpha) {
        // the box is the grid: the wave speed of the next stage is the workgroup maximum
        // (the same value the split stages reach with atomics)
        const double m = wave_max((double)amax);
        if ((tid & 63) == 0) red[tid >> 6] = m;
        __syncthreads();
        double mall = red[0];
#pragma unroll
        for (int w = 1; w < SGW_BLOCK / 64; w++) mall = nanmax(mall, red[w]);
        // the same in every lane: keep it in scalar registers
        const long long mb = __double_as_longlong(mall);
        mall = __longlong_as_double(
            (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(mb >> 32)) << 32) |
                        (unsigned)__builtin_amdgcn_readfirstlane((int)mb)));
        if (s < 2)
            dyn_alpha = (Real)mall;
        else if (tid == 0)
            g->alpha[0] = (unsigned long long)__double_as_longlong(mall);
    } else if (s < 2) {
        __syncthreads();
    }
    }
}

// One kernel per precision and dimension, so each gets its own registers and code size;
// FUSED: the three RK stages of whole-grid boxes in one launch.
template <typename Real, int D, bool FUSED>
__global__ void __launch_bounds__(SGW_BLOCK) stage_kernel(const WorkItem* __restrict__ items, int nitems,
                                                          const int* __restrict__ range_dev, int stage)
{
    // a batch keeps its box list ranges (offset, count) in device memory, so a captured
    // graph stays valid as solves come and go
    if (range_dev) {
        items += range_dev[0];
        nitems = range_dev[1];
    }
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[SGW_BLOCK / 64];
    // XCD-aware order: consecutive workgroup ids land on different XCDs, so hand
    // each XCD a contiguous run of boxes (neighbouring boxes share halo lines in L2).
    // Each workgroup takes a contiguous range of floor or ceil(nitems / nb) boxes,
    // so every XCD and every CU gets the same share.
    const int nb = gridDim.x;
    int bid = blockIdx.x;
    if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
    const int w_end = (int)(((uint64_t)(bid + 1) * (uint32_t)nitems) / (uint32_t)nb);
    for (int w = (int)(((uint64_t)bid * (uint32_t)nitems) / (uint32_t)nb); w < w_end; w++) {
        // descriptors are read-only during the launch: read them through the constant
        // address space so the compiler keeps them in scalar registers
        const SGW_CONST WorkItem* it = (const SGW_CONST WorkItem*)items + w;
        GridC g = (GridC)it->g;
        const int ibox = it->box;
        if (((const SGW_CONST ReqDev*)g->req)->done) continue;
        const size_t su_elems = (size_t)g->pad_total;
        Real* su = (Real*)smem;
        Real* sf = su + ((su_elems + 1) & ~(size_t)1);
        if (g->rline)
            stage_box<Real, D, FUSED, true>(g, ibox, stage, su, sf, red);
        else
            stage_box<Real, D, FUSED, false>(g, ibox, stage, su, sf, red);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- line sweep (4D; zero boundary, relaxation)
//
// The same stage with one launch per direction k and no halo: a lane takes a segment of
// sgw_lseg() nodes of one grid line along k, reads the 6 more values its interface fluxes
// need (periodic wrap along the line, or 0 beyond a zero boundary) straight from memory,
// forms their fluxes with window_fluxes (the box kernel's arithmetic, so the same
// bits) and adds (F_{i-1/2} - F_{i+1/2}) / h_k of its nodes to the sum of the earlier
// directions.  That partial sum waits in a state copy the stage does not read: the stage
// output for stages 1 and 2, the stage-1 buffer in stage 3.  The last direction adds the
// relaxation source (mu_inf(v) rho(x) - u) / tau of the Vlasov-Boltzmann model (Sec. 3.4,
// Example 5) where the grid has one, applies the Runge-Kutta combination, writes the stage
// output and reduces the next wave speed.
template <typename Real, int D, int k, bool LIN, bool ZB>
__device__ __forceinline__ void line_segment(GridC g, int blk, int stage, Real alpha, Real& amax)
{
    constexpr int SGW_LS = sgw_lseg(sizeof(Real) == 8);
    const int lane = threadIdx.x;
    const int n = g->n[k], segl = g->lsegl[k], trans = g->ltrans[k];
    const int sid = blk * SGW_LWAVE + lane;
    if (sid >= segl * trans) return;
    int q, t;
    if constexpr (k == 0) {
        // the segments of one row on neighbouring lanes: each lane streams its piece of the row
        const uint32_t a = FDIV((uint32_t)sid, g->fd_lsegl[0]);
        t = (int)a;
        q = sid - (int)a * segl;
    } else {
        // neighbouring lines (direction 1 fastest) on neighbouring lanes: coalesced
        const uint32_t a = FDIV((uint32_t)sid, g->fd_ltrans[k]);
        q = (int)a;
        t = sid - (int)a * trans;
    }
    // the line's position: t over the directions other than k, direction 1 fastest
    const int csrc = g->coef_src[k];
    constexpr bool last = k == D - 1;
    const bool relax = last && g->relax;
    int base = 0, xc = 0, ix = 0;
    int xj[D]; // the line's node index along each other direction
    double muf = 1.0;
    {
        uint32_t r = (uint32_t)t;
#pragma unroll
        for (int j = 0; j < D; j++) {
            xj[j] = 0;
            if (j == k) continue;
            const uint32_t qq = FDIV(r, g->fd_n[j]);
            const int x = (int)(r - qq * (uint32_t)g->n[j]);
            r = qq;
            xj[j] = x;
            base += x * g->stride[j];
            if (j == csrc) xc = x;
            if (relax) {
                // the x directions come first, so the x part of the offset is the x-node index
                if (2 * j < D) ix += x * g->stride[j];
                else muf *= g->mu[j][x];
            }
        }
    }
    const int stride = g->stride[k];
    const int i0 = q * SGW_LS;
    const Real* __restrict__ in = (const Real*)(stage == 0 ? g->u : stage == 1 ? g->a : g->b);
    Real v[SGW_LS + 6]; // u_{i0-3} .. u_{i0+SGW_LS+2}
    if (ZB && ((g->zmask >> k) & 1)) {
        // zero boundary: nothing wraps, positions beyond either end read 0
#pragma unroll
        for (int c = 0; c < SGW_LS + 6; c++) {
            const int p = i0 - 3 + c;
            v[c] = (p >= 0 && p < n) ? in[base + p * stride] : Real(0);
        }
    } else if ((g->pow2_mask >> k) & 1) {
#pragma unroll
        for (int c = 0; c < SGW_LS + 6; c++) v[c] = in[base + ((i0 - 3 + c) & (n - 1)) * stride];
    } else {
        // n >= 4: positions -3 .. n + 9 need at most one addition or three subtractions
#pragma unroll
        for (int c = 0; c < SGW_LS + 6; c++) {
            int p = i0 - 3 + c;
            p += p < 0 ? n : 0;
            p -= p >= n ? n : 0;
            p -= p >= n ? n : 0;
            p -= p >= n ? n : 0;
            v[c] = in[base + p * stride];
        }
    }
    // the sum of the earlier directions and (last direction, stages 2 and 3) u^n of the
    // segment's nodes are loaded with the window, so their latency overlaps it
    Real* __restrict__ part = (Real*)(stage == 1 ? g->b : g->a);
    const Real* __restrict__ u0 = (const Real*)g->u;
    Real pin[SGW_LS], un[SGW_LS];
#pragma unroll
    for (int i = 0; i < SGW_LS; i++) {
        const bool in_line = i0 + i < n;
        const int gi = base + (i0 + i) * stride;
        pin[i] = (k > 0 && in_line) ? part[gi] : Real(0);
        un[i] = (last && stage > 0 && in_line) ? u0[gi] : Real(0);
    }
    const bool burgers = g->flux == SGW_FLUX_BURGERS;
    Real cp = Real(0), cm = Real(0);
    if (!burgers) {
        // f_k = c u along the line (advection, Vlasov): f^+- = (c +- alpha)/2 u
        Real c = (Real)g->lin_c[k];
        if (csrc >= 0) c = (Real)g->coef[k][xc];
        if constexpr (D == 3 && k > 0) {
            if (g->vm) {
                // Vlasov-Maxwell: the Lorentz force of this stage's fields at the line's x_2 node,
                // E_1 + xi_2 B_3 (direction xi_1) or E_2 - xi_1 B_3 (direction xi_2)
                const double* fld = (const double*)((const char*)in + g->fld_bytes);
                const int n0 = g->n[0], i2 = xj[0];
                const double B = fld[i2];
                if (k == 1) {
                    const double xi2 = g->lo[2] + xj[2] * g->h[2];
                    c = (Real)(fld[n0 + i2] + xi2 * B);
                } else {
                    const double xi1 = g->lo[1] + xj[1] * g->h[1];
                    c = (Real)(fld[2 * n0 + i2] - xi1 * B);
                }
            }
        }
        cp = Real(0.5) * (c + alpha);
        cm = Real(0.5) * (c - alpha);
    }
    Real F[SGW_LS + 1]; // F_{i0-1/2} .. F_{i0+SGW_LS-1/2}
    window_fluxes<Real, SGW_LS + 1, LIN>(v, burgers, cp, cm, alpha, (Real)(g->eps * 4.0), F);
    const Real ih = (Real)g->inv_h[k];
    if constexpr (!last) {
#pragma unroll
        for (int i = 0; i < SGW_LS; i++)
            if (i0 + i < n) part[base + (i0 + i) * stride] = fma(F[i] - F[i + 1], ih, pin[i]);
        return;
    }
    // ---- last direction: TVD-RK3 stage u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1));
    //      u = 1/3 u + 2/3 (u2 + dt L(u2))
    const Real dtr = (Real)((const SGW_CONST ReqDev*)g->req)->dt;
    Real* __restrict__ out = (Real*)(stage == 0 ? g->a : stage == 1 ? g->b : g->u);
    Real rmu = Real(0), itau = Real(0);
    const double* __restrict__ muk = g->mu[k];
    if (relax) {
        // rho(x) of this stage's input times the velocity factors of the other directions
        rmu = (Real)(muf * g->rho[ix]);
        itau = (Real)g->inv_tau;
    }
#pragma unroll
    for (int i = 0; i < SGW_LS; i++)
        if (i0 + i < n) {
            Real acc = fma(F[i] - F[i + 1], ih, pin[i]);
            if (relax) acc = fma(fma(rmu, (Real)muk[i0 + i], -v[i + 3]), itau, acc);
            const Real val = fma(dtr, acc, v[i + 3]);
            Real res;
            if (stage == 0) res = val;
            else if (stage == 1) res = fma(Real(0.75), un[i], Real(0.25) * val);
            else res = fma(Real(1.0 / 3.0), un[i], Real(2.0 / 3.0) * val);
            out[base + (i0 + i) * stride] = res;
            amax = absmax(amax, res);
        }
}

// One wavefront per workgroup, persistent over a contiguous range of the work items
// (grid, block of SGW_LWAVE segments).
template <typename Real, int D, int k>
__global__ void __launch_bounds__(SGW_LWAVE) line_kernel(const WorkItem* __restrict__ items, int nitems,
                                                         const int* __restrict__ range_dev, int stage)
{
    if (range_dev) {
        items += range_dev[0];
        nitems = range_dev[1];
    }
    // XCD-aware order, as in the box kernel: neighbouring items (neighbouring lines of one
    // grid) on one XCD share its L2
    const int nb = gridDim.x;
    int bid = blockIdx.x;
    if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
    const int w_end = (int)(((uint64_t)(bid + 1) * (uint32_t)nitems) / (uint32_t)nb);
    for (int w = (int)(((uint64_t)bid * (uint32_t)nitems) / (uint32_t)nb); w < w_end; w++) {
        const SGW_CONST WorkItem* it = (const SGW_CONST WorkItem*)items + w;
        GridC g = (GridC)it->g;
        if (((const SGW_CONST ReqDev*)g->req)->done) continue;
        // the wave-speed slot the next stage reads is cleared by the stage before it
        if (k == 0 && g->dyn_alpha && it->box == 0 && threadIdx.x == 0) g->alpha[(stage + 2) % 3] = 0ull;
        Real alpha = g->dyn_alpha ? (Real)__longlong_as_double((long long)g->alpha[stage]) : (Real)g->alpha_c[k];
        // Vlasov-Maxwell: the xi directions' speeds of this stage's fields
        if (D == 3 && k > 0 && g->vm) alpha = (Real)g->vm_alpha[2 * stage + k - 1];
        Real amax = Real(0);
        if (g->zmask) {
            if (g->linear)
                line_segment<Real, D, k, true, true>(g, it->box, stage, alpha, amax);
            else
                line_segment<Real, D, k, false, true>(g, it->box, stage, alpha, amax);
        } else {
            if (g->linear)
                line_segment<Real, D, k, true, false>(g, it->box, stage, alpha, amax);
            else
                line_segment<Real, D, k, false, false>(g, it->box, stage, alpha, amax);
        }
        if (k == D - 1 && g->dyn_alpha) {
            // one atomic max per wavefront on the bit pattern (order-free)
            const double m = wave_max((double)amax);
            if (threadIdx.x == 0) atomicMax(g->alpha + (stage + 1) % 3, (unsigned long long)__double_as_longlong(m));
        }
    }
}

// ---------------------------------------------------------------- 4D: directions 1 and 2 in one launch
//
// segments of SGW_PSEG nodes: a work item of SGW_PLANE_CAP nodes gives every thread one segment
// per direction (a flux depends only on its window's values, so the segment length does not change
// the bits; 4-node segments over 1024-node items measured 8 % slower on the 4D Vlasov solve)
#ifndef SGW_PSEG
#define SGW_PSEG 8  // the plane launch keeps 8-node segments in both precisions
#endif
//
// A work item is ppi consecutive (x_1, x_2) planes of one 4D grid (contiguous in memory, at most
// SGW_PLANE_CAP nodes).  The workgroup stages them in LDS, forms the direction-1 flux differences of
// every node (segments of SGW_PSEG nodes along the rows, the line sweep's windows and arithmetic),
// adds the direction-2 differences (segments along the columns, neighbouring threads on neighbouring
// columns) and writes the sum to the stage's partial-sum copy, where the line sweeps of directions
// 3 and 4 continue.  The two sums are formed in the line sweep's order, so the stage gives the
// same bits as four line launches, and it reads the stage input once instead of twice and skips one
// round trip of the partial sum.

// index of direction csrc of a node at (x_1, x_2) of plane p of grid g
__device__ __forceinline__ int plane_coord(GridC g, int csrc, int x0, int x1, int plane)
{
    if (csrc == 0) return x0;
    if (csrc == 1) return x1;
    const int n2 = g->n[2];
    const int x3 = plane / n2;
    return csrc == 2 ? plane - x3 * n2 : x3;
}

template <typename Real, bool LIN, bool ZB>
__device__ __forceinline__ void plane_item(GridC g, int item, int stage, Real alpha0, Real alpha1, Real* V, Real* A)
{
    const int tid = threadIdx.x;
    const int n0 = g->n[0], n1 = g->n[1], pn = g->plane_nodes;
    const int p0 = item * g->ppi;
    const int np = min(g->ppi, g->nplanes - p0);
    const int N = np * pn;
    const int64_t base = (int64_t)p0 * pn;
    const Real* __restrict__ in = (const Real*)(stage == 0 ? g->u : stage == 1 ? g->a : g->b) + base;
    Real* __restrict__ part = (Real*)(stage == 1 ? g->b : g->a) + base;
    // LDS rows of n0 values at the odd stride RS = n0 + 1: threads on neighbouring rows (direction 1)
    // and on neighbouring columns (direction 2) hit distinct banks
    const int RS = n0 + 1;
#pragma unroll 8
    for (int e = tid; e < N; e += SGW_BLOCK) {
        const int row = (int)FDIV((uint32_t)e, g->fd_n[0]);
        V[row * RS + (e - row * n0)] = in[e];
    }
    __syncthreads();
    const bool burgers = g->flux == SGW_FLUX_BURGERS;
    const Real epsT = (Real)(g->eps * 4.0);
    // ---- direction 1: neighbouring threads on neighbouring rows
    {
        const int nseg = (n0 + SGW_PSEG - 1) / SGW_PSEG, rows = np * n1, csrc = g->coef_src[0];
        const Real ih = (Real)g->inv_h[0];
        const bool zero = ZB && (g->zmask & 1);
#pragma unroll 2
        for (int sgi = tid; sgi < rows * nseg; sgi += SGW_BLOCK) {
            const int q = sgi / rows, row = sgi - q * rows;
            const int i0 = q * SGW_PSEG;
            const Real* vr = V + row * RS;
            Real v[SGW_PSEG + 6];
#pragma unroll
            for (int c = 0; c < SGW_PSEG + 6; c++) {
                int p = i0 - 3 + c;
                if (zero) {
                    v[c] = (p >= 0 && p < n0) ? vr[p] : Real(0);
                } else {
                    p += p < 0 ? n0 : 0;
                    p -= p >= n0 ? n0 : 0;
                    p -= p >= n0 ? n0 : 0;
                    p -= p >= n0 ? n0 : 0;
                    v[c] = vr[p];
                }
            }
            Real cp = Real(0), cm = Real(0);
            if (!burgers) {
                Real c = (Real)g->lin_c[0];
                if (csrc >= 0) {
                    const int pl = row / n1;
                    c = (Real)g->coef[0][plane_coord(g, csrc, 0, row - pl * n1, p0 + pl)];
                }
                cp = Real(0.5) * (c + alpha0);
                cm = Real(0.5) * (c - alpha0);
            }
            Real F[SGW_PSEG + 1];
            window_fluxes<Real, SGW_PSEG + 1, LIN>(v, burgers, cp, cm, alpha0, epsT, F);
#pragma unroll
            for (int i = 0; i < SGW_PSEG; i++)
                if (i0 + i < n0) A[row * RS + i0 + i] = fma(F[i] - F[i + 1], ih, Real(0));
        }
    }
    __syncthreads();
    // ---- direction 2: neighbouring threads on neighbouring columns
    {
        const int nseg = (n1 + SGW_PSEG - 1) / SGW_PSEG, cols = np * n0, csrc = g->coef_src[1];
        const Real ih = (Real)g->inv_h[1];
        const bool zero = ZB && ((g->zmask >> 1) & 1);
#pragma unroll 2
        for (int sgi = tid; sgi < cols * nseg; sgi += SGW_BLOCK) {
            const int q = sgi / cols, col = sgi - q * cols;
            const int pl = col / n0, x0 = col - pl * n0;
            const int i0 = q * SGW_PSEG;
            const Real* vc = V + pl * n1 * RS + x0;
            Real v[SGW_PSEG + 6];
#pragma unroll
            for (int c = 0; c < SGW_PSEG + 6; c++) {
                int p = i0 - 3 + c;
                if (zero) {
                    v[c] = (p >= 0 && p < n1) ? vc[p * RS] : Real(0);
                } else {
                    p += p < 0 ? n1 : 0;
                    p -= p >= n1 ? n1 : 0;
                    p -= p >= n1 ? n1 : 0;
                    p -= p >= n1 ? n1 : 0;
                    v[c] = vc[p * RS];
                }
            }
            Real cp = Real(0), cm = Real(0);
            if (!burgers) {
                Real c = (Real)g->lin_c[1];
                if (csrc >= 0) c = (Real)g->coef[1][plane_coord(g, csrc, x0, 0, p0 + pl)];
                cp = Real(0.5) * (c + alpha1);
                cm = Real(0.5) * (c - alpha1);
            }
            Real F[SGW_PSEG + 1];
            window_fluxes<Real, SGW_PSEG + 1, LIN>(v, burgers, cp, cm, alpha1, epsT, F);
            Real* a = A + pl * n1 * RS + x0;
#pragma unroll
            for (int i = 0; i < SGW_PSEG; i++)
                if (i0 + i < n1) a[(i0 + i) * RS] = fma(F[i] - F[i + 1], ih, a[(i0 + i) * RS]);
        }
    }
    __syncthreads();
#pragma unroll 8
    for (int e = tid; e < N; e += SGW_BLOCK) {
        const int row = (int)FDIV((uint32_t)e, g->fd_n[0]);
        part[e] = A[row * RS + (e - row * n0)];
    }
    __syncthreads();
}

template <typename Real>
__global__ void __launch_bounds__(SGW_BLOCK) plane_kernel(const WorkItem* __restrict__ items, int nitems, int stage)
{
    // rows of n0 values at stride n0 + 1: at most SGW_PLANE_CAP + SGW_PLANE_CAP / 4 entries (n0 >= 4)
    __shared__ Real V[SGW_PLANE_CAP + SGW_PLANE_CAP / 4];
    __shared__ Real A[SGW_PLANE_CAP + SGW_PLANE_CAP / 4];
    // XCD-aware order, as in the other persistent launches
    const int nb = gridDim.x;
    int bid = blockIdx.x;
    if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
    const int w_end = (int)(((uint64_t)(bid + 1) * (uint32_t)nitems) / (uint32_t)nb);
    for (int w = (int)(((uint64_t)bid * (uint32_t)nitems) / (uint32_t)nb); w < w_end; w++) {
        const SGW_CONST WorkItem* it = (const SGW_CONST WorkItem*)items + w;
        GridC g = (GridC)it->g;
        if (((const SGW_CONST ReqDev*)g->req)->done) continue;
        // the wave-speed slot the next stage reads is cleared by the stage before it
        if (g->dyn_alpha && it->box == 0 && threadIdx.x == 0) g->alpha[(stage + 2) % 3] = 0ull;
        Real a0, a1;
        if (g->dyn_alpha) {
            a0 = a1 = (Real)__longlong_as_double((long long)g->alpha[stage]);
        } else {
            a0 = (Real)g->alpha_c[0];
            a1 = (Real)g->alpha_c[1];
        }
        if (g->zmask) {
            if (g->linear) plane_item<Real, true, true>(g, it->box, stage, a0, a1, V, A);
            else plane_item<Real, false, true>(g, it->box, stage, a0, a1, V, A);
        } else {
            if (g->linear) plane_item<Real, true, false>(g, it->box, stage, a0, a1, V, A);
            else plane_item<Real, false, false>(g, it->box, stage, a0, a1, V, A);
        }
    }
}

template <typename Real>
hipError_t launch_lines(const WorkItem* items, int nitems, const int* range_dev, int blocks, int stage, int dim,
                        hipStream_t s, int first_dir, int last_dir = 3)
{
#define SGW_LINE(DD, K)                                                                                        \
    if (K >= first_dir && K <= last_dir) {                                                                      \
        hipLaunchKernelGGL((line_kernel<Real, DD, K>), dim3(blocks), dim3(SGW_LWAVE), 0, s, items, nitems,      \
                           range_dev, stage);                                                                   \
        const hipError_t e_ = hipGetLastError();                                                                \
        if (e_ != hipSuccess) return e_;                                                                        \
    }
    switch (dim) {
    case 1: SGW_LINE(1, 0) break;
    case 2: SGW_LINE(2, 0) SGW_LINE(2, 1) break;
    case 3: SGW_LINE(3, 0) SGW_LINE(3, 1) SGW_LINE(3, 2) break;
    case 4: SGW_LINE(4, 0) SGW_LINE(4, 1) SGW_LINE(4, 2) SGW_LINE(4, 3) break;
    default: return hipErrorInvalidValue;
    }
#undef SGW_LINE
    return hipSuccess;
}

// ---------------------------------------------------------------- Vlasov-Maxwell fields
//
// One workgroup per component grid.  stage < 0: the initial fields of u^n, B_3 = b sin(k0 x_2),
// E_1 = E_2 = 0.  stage s = 0..2: the Runge-Kutta stage s of the field equations B_3' = dE_1/dx_2,
// E_1' = dB_3/dx_2 - j_1, E_2' = -j_2 (Sec. 3.4, Example 6), discretised like eq. (2.9): WENO5
// with global LF splitting of F(B_3, E_1) = (-E_1, -B_3) at alpha = 1, each component on its own,
// the currents of the stage input from the moment pass.  The output is the next stage's fields
// (u^{n+1}'s after stage 2), whose xi-direction LF speeds go to the next stage's slots.
template <bool LIN>
__device__ void vm_fields_grid(const GridDev* g, int stage, double b, double k0, double* red)
{
    const int n = g->n[0];
    const double h = g->h[0];
    double* f0 = (double*)((char*)g->u + g->fld_bytes);
    if (stage < 0) {
        for (int i = threadIdx.x; i < n; i += SGW_BLOCK) {
            f0[i] = b * sin(k0 * (g->lo[0] + i * g->h[0]));
            f0[n + i] = 0.0;
            f0[2 * n + i] = 0.0;
        }
        return;
    }
    const double* fin = (const double*)((const char*)(stage == 0 ? g->u : stage == 1 ? g->a : g->b) + g->fld_bytes);
    double* out = (double*)((char*)(stage == 0 ? g->a : stage == 1 ? g->b : g->u) + g->fld_bytes);
    const double dt = ((const ReqDev*)g->req)->dt;
    const double* j1 = g->rho;
    const double* j2 = g->rho + g->nxr;
    const double epsT = 4.0 * g->eps;
    const double x1lo = g->lo[1], x1hi = g->lo[1] + (g->n[1] - 1) * g->h[1];
    const double x2lo = g->lo[2], x2hi = g->lo[2] + (g->n[2] - 1) * g->h[2];
    double m1 = 0.0, m2 = 0.0;
    for (int i = threadIdx.x; i < n; i += SGW_BLOCK) {
        // split values at i-3 .. i+3 (periodic), then the interface fluxes at i-1/2 and i+1/2
        double pB[7], mB[7], pE[7], mE[7];
#pragma unroll
        for (int q = 0; q < 7; q++) {
            int p = i - 3 + q;
            p += p < 0 ? n : 0;
            p -= p >= n ? n : 0;
            const double B = fin[p], E = fin[n + p];
            pB[q] = 0.5 * (-E + B);
            mB[q] = 0.5 * (-E - B);
            pE[q] = 0.5 * (-B + E);
            mE[q] = 0.5 * (-B - E);
        }
        double FB[2], FE[2];
        split_fluxes<double, 2, LIN>(pB, mB, true, true, epsT, FB);
        split_fluxes<double, 2, LIN>(pE, mE, true, true, epsT, FE);
        const double LB = -(FB[1] - FB[0]) / h;
        const double LE1 = -(FE[1] - FE[0]) / h - j1[i];
        const double LE2 = -j2[i];
        const double w[3] = {LB, LE1, LE2};
        double v[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const double y = fin[q * n + i] + dt * w[q];
            if (stage == 0) v[q] = y;
            else if (stage == 1) v[q] = 0.75 * f0[q * n + i] + 0.25 * y;
            else v[q] = f0[q * n + i] / 3.0 + 2.0 / 3.0 * y;
        }
        // stage 2 writes u^n's fields in place: this thread read them above
#pragma unroll
        for (int q = 0; q < 3; q++) out[q * n + i] = v[q];
        const double p1 = x2lo * v[0], q1 = x2hi * v[0], p2 = x1lo * v[0], q2 = x1hi * v[0];
        m1 = nanmax(m1, nanmax(fabs(v[1] + p1), fabs(v[1] + q1)));
        m2 = nanmax(m2, nanmax(fabs(v[2] - p2), fabs(v[2] - q2)));
    }
    if (stage == 2) return; // the time-step kernel takes u^{n+1}'s speeds
    m1 = wave_max(m1);
    m2 = wave_max(m2);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[2 * wave] = m1;
        red[2 * wave + 1] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a1 = red[0], a2 = red[1];
        for (int w2 = 1; w2 < SGW_BLOCK / 64; w2++) {
            a1 = nanmax(a1, red[2 * w2]);
            a2 = nanmax(a2, red[2 * w2 + 1]);
        }
        g->vm_alpha[2 * (stage + 1)] = a1;
        g->vm_alpha[2 * (stage + 1) + 1] = a2;
    }
}

__global__ void __launch_bounds__(SGW_BLOCK) vm_fields_kernel(const GridDev* grids, int stage, double b, double k0,
                                                              int linear)
{
    __shared__ double red[2 * (SGW_BLOCK / 64)];
    const GridDev* g = grids + blockIdx.x;
    if (stage >= 0 && ((const ReqDev*)g->req)->done) return;
    if (linear)
        vm_fields_grid<true>(g, stage, b, k0, red);
    else
        vm_fields_grid<false>(g, stage, b, k0, red);
}

template <typename Real, int D, bool FUSED>
int occupancy_d(size_t lds_bytes)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage_kernel<Real, D, FUSED>, SGW_BLOCK, lds_bytes) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

template <typename Real, bool FUSED>
int occupancy_r(int dim, size_t lds_bytes)
{
    switch (dim) {
    case 1: return occupancy_d<Real, 1, FUSED>(lds_bytes);
    case 2: return occupancy_d<Real, 2, FUSED>(lds_bytes);
    case 3: return occupancy_d<Real, 3, FUSED>(lds_bytes);
    default: return occupancy_d<Real, 4, FUSED>(lds_bytes);
    }
}

template <typename Real, int D, bool FUSED>
hipError_t launch_d(const WorkItem* items, int nitems, const int* range_dev, int blocks, int stage, size_t lds,
                    hipStream_t s)
{
    hipLaunchKernelGGL((stage_kernel<Real, D, FUSED>), dim3(blocks), dim3(SGW_BLOCK), lds, s, items, nitems,
                       range_dev, stage);
    return hipGetLastError();
}

template <typename Real, bool FUSED>
hipError_t launch_f(int dim, const WorkItem* items, int nitems, const int* range_dev, int blocks, int stage,
                    size_t lds, hipStream_t s)
{
    switch (dim) {
    case 1: return launch_d<Real, 1, FUSED>(items, nitems, range_dev, blocks, stage, lds, s);
    case 2: return launch_d<Real, 2, FUSED>(items, nitems, range_dev, blocks, stage, lds, s);
    case 3: return launch_d<Real, 3, FUSED>(items, nitems, range_dev, blocks, stage, lds, s);
    default: return launch_d<Real, 4, FUSED>(items, nitems, range_dev, blocks, stage, lds, s);
    }
}

template <typename Real>
hipError_t launch_r(int dim, const WorkItem* items, int nitems, const int* range_dev, int blocks, int stage,
                    size_t lds, hipStream_t s)
{
    if (stage == SGW_STAGE_FUSED) return launch_f<Real, true>(dim, items, nitems, range_dev, blocks, stage, lds, s);
    return launch_f<Real, false>(dim, items, nitems, range_dev, blocks, stage, lds, s);
}

} // namespace

// ---------------------------------------------------------------- launchers

size_t stage_lds_bytes(const GridDev& g, int precision)
{
    if (g.line_mode) return 16; // the line sweep uses no LDS; a nominal size keeps its launches in the lists
    const size_t rs = precision == SGW_FP64 ? 8 : 4;
    int fmax_ = 0;
    for (int k = 0; k < g.d; k++) fmax_ = g.flux_total[k] > fmax_ ? g.flux_total[k] : fmax_;
    // staged values, two flux buffers, then (3D/4D) the row tables of 32-bit offsets
    return rs * (((size_t)g.pad_total + 1) / 2 * 2 + 2 * (((size_t)fmax_ + 1) / 2 * 2)) + 4 * (size_t)g.rt_total;
}

int device_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
        n = 256;
    return n;
}

int stage_grid(int precision, int dim, size_t lds_bytes, int blocks_per_cu, bool fused)
{
    int occ = stage_occupancy(precision, dim, lds_bytes, fused);
    if (blocks_per_cu > 0 && blocks_per_cu < occ) occ = blocks_per_cu;
    return occ * device_cus();
}

int stage_occupancy(int precision, int dim, size_t lds_bytes, bool fused)
{
    if (fused)
        return precision == SGW_FP64 ? occupancy_r<double, true>(dim, lds_bytes)
                                     : occupancy_r<float, true>(dim, lds_bytes);
    return precision == SGW_FP64 ? occupancy_r<double, false>(dim, lds_bytes) : occupancy_r<float, false>(dim, lds_bytes);
}

// persistent one-wavefront workgroups of the line sweep: 16 per compute unit
#ifndef SGW_LINE_WAVES_PER_CU
#define SGW_LINE_WAVES_PER_CU 24
#endif
int line_grid() { return SGW_LINE_WAVES_PER_CU * device_cus(); }

hipError_t launch_stage(const WorkItem* items, int nitems, int stage, int precision, int dim, size_t lds_bytes,
                        int grid_cap, hipStream_t s, bool lines, int first_dir, int last_dir)
{
    if (nitems <= 0) return hipSuccess;
    if (lines) {
        int blocks = nitems < line_grid() ? nitems : line_grid();
        if (precision == SGW_FP64)
            return launch_lines<double>(items, nitems, nullptr, blocks, stage, dim, s, first_dir, last_dir);
        return launch_lines<float>(items, nitems, nullptr, blocks, stage, dim, s, first_dir, last_dir);
    }
    int blocks = nitems;
    if (grid_cap > 0 && blocks > grid_cap) blocks = grid_cap;
    if (precision == SGW_FP64) return launch_r<double>(dim, items, nitems, nullptr, blocks, stage, lds_bytes, s);
    return launch_r<float>(dim, items, nitems, nullptr, blocks, stage, lds_bytes, s);
}

// persistent plane launch: the resident workgroups of the kernel (LDS-limited) on every CU
hipError_t launch_planes(const WorkItem* items, int nitems, int stage, int precision, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    static int occ[2] = {0, 0};
    const int pi = precision == SGW_FP64 ? 0 : 1;
    if (!occ[pi]) {
        int nb = 0;
        hipError_t e = precision == SGW_FP64
                           ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, plane_kernel<double>, SGW_BLOCK, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, plane_kernel<float>, SGW_BLOCK, 0);
        occ[pi] = (e == hipSuccess && nb > 0) ? nb : 1;
    }
    int blocks = occ[pi] * device_cus();
    blocks = nitems < blocks ? nitems : blocks;
    if (precision == SGW_FP64)
        hipLaunchKernelGGL(plane_kernel<double>, dim3(blocks), dim3(SGW_BLOCK), 0, s, items, nitems, stage);
    else
        hipLaunchKernelGGL(plane_kernel<float>, dim3(blocks), dim3(SGW_BLOCK), 0, s, items, nitems, stage);
    return hipGetLastError();
}

hipError_t launch_vm_fields(const GridDev* grids_dev, int G, int stage, int precision, double b, double k0,
                            int linear, hipStream_t s)
{
    (void)precision;
    if (G <= 0) return hipSuccess;
    hipLaunchKernelGGL(vm_fields_kernel, dim3(G), dim3(SGW_BLOCK), 0, s, grids_dev, stage, b, k0, linear);
    return hipGetLastError();
}

hipError_t launch_stage_range(const WorkItem* items, const int* range_dev, int blocks, int stage, int precision,
                              int dim, size_t lds_bytes, hipStream_t s, bool lines)
{
    if (lines) {
        if (precision == SGW_FP64) return launch_lines<double>(items, 0, range_dev, line_grid(), stage, dim, s, 0);
        return launch_lines<float>(items, 0, range_dev, line_grid(), stage, dim, s, 0);
    }
    if (precision == SGW_FP64) return launch_r<double>(dim, items, 0, range_dev, blocks, stage, lds_bytes, s);
    return launch_r<float>(dim, items, 0, range_dev, blocks, stage, lds_bytes, s);
}
