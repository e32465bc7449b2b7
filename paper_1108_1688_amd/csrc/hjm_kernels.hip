// HIP kernels (gfx950) of the Douglas-ADI step for the single-factor HJM model
// with stochastic volatility.  FP64 throughout; no MFMA (nothing here is a
// dense contraction: the step is a stencil plus tridiagonal recurrences and is
// bound by memory traffic and latency).
//
// One Douglas step (section 5.1 of the paper, theta = 1/2, operators at
// t_{n+1/2}) is three launches:
//   k_xr  explicit predictor D0 = dt (A0+A1+A2+A3) U^n (eq. (discreta) with
//         the centred stencils of eq. (esquema)) fused with the r sweep
//         (I - theta dt A1) D1 = D0 along the contiguous r lines;
//   k_v   (I - theta dt A2) D2 = D1 along v (stride nr), in place in D;
//   k_yu  (I - theta dt A3) D3 = D2 along y (stride nr*nv), fused with
//         U^{n+1} = U^n + D3.
// Dirichlet nodes carry identity rows and D0 = g(t_{n+1}) - g(t_n).
//
// Coefficients.  Every operator coefficient is affine in a couple of per-line
// quantities (v_j and c = f_t + kappa f + y_k for r; q = lambda^2 r^{2 gamma}
// v for y), so the host tabulates per node the few numbers that turn each one
// into one or two FMAs (see the table layouts in hjm_internal.h).  Outflow
// faces (one-sided rows of section 7.3) and Dirichlet rows are just other
// table entries: the kernels have no face branches.
//
// Line solves.  The rows of a line are split into S segments of at most ROWS
// rows held in the registers of S threads.  Outflow faces put one entry
// beyond the band in rows 0 and n-1; those unknowns are eliminated from rows 1
// and n-2 first and recovered last.  No pivoting: diagonals are >= 1 and the
// pivots are checked (> 0) into the health flag.  Two ways of combining the
// segments:
//   chain  the Thomas recurrence in row order, segment s starting once segment
//          s-1 has handed over (c', d') of its last row (LDS, one barrier per
//          stage); the elimination order of a sequential solve, accurate for
//          any of this problem's lines.  Used for y (advection only, Courant
//          numbers up to ~1e4 in the far field) and v.
//   spike  every segment eliminates at once, carrying the coupling to its
//          neighbours as spikes; a per-line reduced system of the segments'
//          end rows is then solved and each segment back-substitutes.  Fully
//          parallel but only as accurate as the rows are diagonally dominant,
//          so the host selects it for the r lines only when the cell Courant
//          number theta dt |b| / (2 h) stays below 0.4 on every r row.
// The v-line matrix depends on j alone, so its LU factors are built once per
// solve on the host and every v line runs a division-free chained recurrence.
// All per-row loops are fully unrolled and branch-free (rows outside a
// segment's range are masked with selects), so table reads and loads are free
// to be scheduled ahead of the serial recurrences.
//
// Work is described by (solve, tile) tasks so that one launch can cover many
// independent solves of different shapes (batched mode); a null task list
// means one solve whose tile index is the workgroup index.

#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

#include "hjm_internal.h"

namespace hjm {
namespace {

typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(3))) double ldouble;

__device__ __forceinline__ gdouble* gp(double* p) { return (gdouble*)p; }
__device__ __forceinline__ gcdouble* gp(const double* p) { return (gcdouble*)p; }

// The coefficient tables are written by the host before a solve starts and
// only read by kernels: reading them through the constant address space lets
// wave-uniform reads go through scalar loads (which the kernels' own stores
// to the grid arrays cannot alias).
typedef __attribute__((address_space(4))) const double kcdouble;
__device__ __forceinline__ kcdouble* kp(const double* p) { return (kcdouble*)(uintptr_t)p; }

__device__ __forceinline__ double dirichlet_value(const SolveDesc& s, gcdouble* stn, double r, double y)
{
    // p(t,T) = A exp(-G r - H y): bond reconstruction formula (section 3.1)
    // with the time-only factor A = P(0,T)/P(0,t) exp(G f(0,t)) and H = G^2/2
    // taken from the step table.
    double pT = stn[ST_AT] * exp(-stn[ST_GT] * r - stn[ST_HT] * y);
    if (s.kind == KIND_BOND) return pT;
    double pM = stn[ST_AM] * exp(-stn[ST_GM] * r - stn[ST_HM] * y);
    double lin = pT - s.accrual * pM;
    if (s.kind == KIND_CAPLET) return lin > 0.0 ? lin : 0.0;
    if (s.kind == KIND_FLOORLET) return -lin > 0.0 ? -lin : 0.0;
    return lin;
}

// 1/x for the positive pivots of the line solves: the hardware estimate
// refined by two Newton-Raphson steps r <- r + r (1 - x r) (each doubles the
// number of correct bits), a few ulps from the correctly rounded quotient at
// half the instructions of the IEEE division sequence.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ void raise_flag(const SolveDesc& s)
{
    // vector store of a constant; concurrent writers store the same value
    *(__attribute__((address_space(1))) volatile int32_t*)s.flag = 1;
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) in turn, by
// workgroup index mod 8.  Give each XCD a contiguous range of tiles instead,
// so that tiles that read each other's halo lines run on the same L2 (a
// bijection on [0, n): the tail beyond a multiple of 8 keeps its index).
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int per = n >> 3;
    if (b >= per * 8) return b;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int pow2_ceil(int n)
{
    int t = 1;
    while (t < n) t <<= 1;
    return t;
}

// ---------------------------------------------------------------------------
// Segments.
// ---------------------------------------------------------------------------
template <int ROWS>
struct Seg {
    double d[ROWS];   // right-hand side -> d' -> solution
    double cp[ROWS];  // super-diagonal, then modified super-diagonal c'
    int p, len, n, seg, S, lo, hi;
    double b0, c0, e0, d0;  // row 0 (first segment)
    double al, bl, el, dl;  // row n-1 (last segment)
};

template <int ROWS>
__device__ __forceinline__ void seg_init(Seg<ROWS>& g, int n, int S, int seg)
{
    g.n = n;
    g.S = S;
    g.seg = seg;
    g.p = (seg * n) / S;
    g.len = ((seg + 1) * n) / S - g.p;
    g.lo = 0;
    g.hi = g.len - 1;
}

// Boundary-row eliminations of the first / last segment (row(m, A, B, C, E)
// gives row m).  Returns the modified rows 1 and n-2 in (b1m, c1m), (a2m, b2m).
template <int ROWS, class RowFn>
__device__ __forceinline__ bool seg_ends(Seg<ROWS>& g, const RowFn& row, double& b1m, double& c1m, double& a2m,
                                         double& b2m)
{
    bool ok = true;
    if (g.seg == 0) {
        // eliminate x0 (row 0: b0 x0 + c0 x1 + e0 x2 = d0) from row 1
        double A, B, C, E;
        row(0, A, B, C, E);
        g.b0 = B; g.c0 = C; g.e0 = E; g.d0 = g.d[0];
        double A1, B1, C1, E1;
        row(1, A1, B1, C1, E1);
        const double f = A1 / B;
        b1m = B1 - f * C;
        c1m = C1 - f * E;
        g.d[1] = g.d[1] - f * g.d[0];
        g.lo = 1;
        ok = ok && (B > 0.0);
    }
    if (g.seg == g.S - 1) {
        // eliminate x_{n-1} (row n-1: e x_{n-3} + a x_{n-2} + b x_{n-1}) from row n-2
        double A, B, C, E;
        row(g.n - 1, A, B, C, E);
        g.al = A; g.bl = B; g.el = E;
        double dl = 0.0;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) dl = (mm == g.len - 1) ? g.d[mm] : dl;
        g.dl = dl;
        double A2, B2, C2, E2;
        row(g.n - 2, A2, B2, C2, E2);
        const double f = C2 / B;
        a2m = A2 - f * E;
        b2m = B2 - f * A;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) g.d[mm] = (mm == g.len - 2) ? g.d[mm] - f * dl : g.d[mm];
        g.hi = g.len - 2;
        ok = ok && (B > 0.0);
    }
    return ok;
}

// Recover x0 and x_{n-1} from their own rows once the interior is solved.
template <int ROWS>
__device__ __forceinline__ void seg_finish(Seg<ROWS>& g)
{
    if (g.seg == 0) g.d[0] = (g.d0 - g.c0 * g.d[1] - g.e0 * g.d[2]) / g.b0;
    if (g.seg == g.S - 1) {
        double x3 = 0.0, x2 = 0.0;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            x3 = (mm == g.len - 3) ? g.d[mm] : x3;
            x2 = (mm == g.len - 2) ? g.d[mm] : x2;
        }
        const double xl = (g.dl - g.el * x3 - g.al * x2) / g.bl;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) g.d[mm] = (mm == g.len - 1) ? xl : g.d[mm];
    }
}

// Chained Thomas on coefficients already in registers: ca (sub-diagonal), cb
// (diagonal) and g.cp (super-diagonal) for rows lo..hi of the segment.  Every
// thread of the workgroup calls it (barriers inside when S > 1); xch is the
// line's two-double hand-over slot in LDS.
template <int ROWS>
__device__ __forceinline__ bool chain_core(Seg<ROWS>& g, const double (&ca)[ROWS], const double (&cb)[ROWS],
                                           bool work, ldouble* xch)
{
    bool ok = true;
    for (int stage = 0; stage < g.S; ++stage) {
        if (work && g.seg == stage) {
            double cprev = 0.0, dprev = 0.0;
            if (stage > 0) { cprev = xch[0]; dprev = xch[1]; }
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) {
                const bool act = mm >= g.lo && mm <= g.hi;
                const double den = cb[mm] - ca[mm] * cprev;
                const double inv = 1.0 / den;
                const double cn = g.cp[mm] * inv;
                const double dn = (g.d[mm] - ca[mm] * dprev) * inv;
                ok = ok && (!act || den > 0.0);
                cprev = act ? cn : cprev;
                dprev = act ? dn : dprev;
                g.cp[mm] = act ? cn : 0.0;
                g.d[mm] = act ? dn : g.d[mm];
            }
            xch[0] = cprev;
            xch[1] = dprev;
        }
        if (g.S > 1) __syncthreads();
    }
    for (int stage = g.S - 1; stage >= 0; --stage) {
        if (work && g.seg == stage) {
            double x = (stage < g.S - 1) ? xch[0] : 0.0;
#pragma unroll
            for (int mm = ROWS - 1; mm >= 0; --mm) {
                const bool act = mm >= g.lo && mm <= g.hi;
                const double xn = g.d[mm] - g.cp[mm] * x;
                x = act ? xn : x;
                g.d[mm] = act ? xn : g.d[mm];
            }
            xch[0] = x;
            seg_finish(g);
        }
        if (g.S > 1) __syncthreads();
    }
    return ok;
}

// ---------------------------------------------------------------------------
// r rows.  LDS table rt6 holds P, Q, ALO, ADI, AUP, RR (each nr long) for the
// interior rows of the solve; the face rows are read from the full table.
// ---------------------------------------------------------------------------
struct RowRFull {  // any row, from the global table (face rows only)
    gcdouble* rt;
    int nr;
    double v, c, tdt;
    __device__ __forceinline__ void operator()(int i, double& A, double& B, double& C, double& E) const
    {
        const double e = rt[RT_P * nr + i] * c + rt[RT_Q * nr + i];
        const double olo = rt[RT_MLO * nr + i] * e + rt[RT_ALO * nr + i] * v;
        const double odi = rt[RT_MDI * nr + i] * e + rt[RT_ADI * nr + i] * v - rt[RT_RR * nr + i];
        const double oup = rt[RT_MUP * nr + i] * e + rt[RT_AUP * nr + i] * v;
        const double oex = rt[RT_MEX * nr + i] * e;
        A = -tdt * olo;
        B = 1.0 - tdt * odi;
        C = -tdt * oup;
        E = -tdt * oex;
    }
};

// interior r row i of (I - theta dt A1) from the LDS table
__device__ __forceinline__ void row_r_interior(const ldouble* rt6, int nr, int i, double v, double c, double tdt,
                                               double& A, double& B, double& C)
{
    const double e = rt6[i] * c + rt6[nr + i];
    A = -tdt * (rt6[2 * nr + i] * v - e);
    B = 1.0 - tdt * (rt6[3 * nr + i] * v - rt6[5 * nr + i]);
    C = -tdt * (rt6[4 * nr + i] * v + e);
}

// Spike (partition) solve of r lines.  Every thread calls it; red is the
// line's S * kRed scratch in LDS.  After the local elimination each segment
// leaves in red[seg] the first/last effective rows of its three local
// solutions y (right-hand side), v (unit coupling to the previous segment)
// and w (to the next): x = y - X_L v - X_R w.  One thread per line solves
// the reduced system of the segments' end unknowns; every segment then
// back-substitutes.
template <int ROWS>
__device__ __forceinline__ void spike_solve_r(Seg<ROWS>& g, const RowRFull& full, const ldouble* rt6, bool work,
                                              ldouble* red, const SolveDesc& s)
{
    double vp[ROWS];
    double b1m = 1.0, c1m = 0.0, a2m = 0.0, b2m = 1.0;
    bool ok = true;
    const bool first = g.seg == 0;
    const bool last = g.seg == g.S - 1;
    const int nr = g.n;
    ldouble* slot = red + g.seg * kRed;
    if (work) {
        ok = seg_ends(g, full, b1m, c1m, a2m, b2m);
        double cprev = 0.0, yprev = 0.0, vprev = 0.0;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            const int i = min(g.p + mm, nr - 2);
            double A, B, C;
            row_r_interior(rt6, nr, i, full.v, full.c, full.tdt, A, B, C);
            if (first && mm == 1) { A = 0.0; B = b1m; C = c1m; }
            if (last && mm == g.len - 2) { A = a2m; B = b2m; C = 0.0; }
            const bool act = mm >= g.lo && mm <= g.hi;
            const bool top = mm == g.lo;
            const double den = top ? B : B - A * cprev;
            const double inv = 1.0 / den;
            const double yv = (top ? g.d[mm] : g.d[mm] - A * yprev) * inv;
            const double vv = (top ? A : -A * vprev) * inv;
            const double cn = C * inv;
            ok = ok && (!act || den > 0.0);
            cprev = act ? cn : cprev;
            yprev = act ? yv : yprev;
            vprev = act ? vv : vprev;
            g.cp[mm] = act ? cn : 0.0;
            g.d[mm] = act ? yv : g.d[mm];
            vp[mm] = act ? vv : 0.0;
        }
        if (g.S > 1) {
            double yL = 0.0, vL = 0.0, wL = 0.0;
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) {
                const bool h = mm == g.hi;
                yL = h ? g.d[mm] : yL;
                vL = h ? vp[mm] : vL;
                wL = h ? g.cp[mm] : wL;
            }
            double y = yL, v = vL, w = wL;
#pragma unroll
            for (int mm = ROWS - 1; mm >= 0; --mm) {
                const bool act = mm >= g.lo && mm < g.hi;
                const double yn = g.d[mm] - g.cp[mm] * y;
                const double vn = vp[mm] - g.cp[mm] * v;
                const double wn = -g.cp[mm] * w;
                y = act ? yn : y;
                v = act ? vn : v;
                w = act ? wn : w;
            }
            slot[0] = y; slot[1] = v; slot[2] = w;
            slot[3] = yL; slot[4] = vL; slot[5] = wL;
        }
    }
    double XL = 0.0, XR = 0.0;
    if (g.S > 1) {
        __syncthreads();
        if (work && first) {
            // F_s = yF - vF L_{s-1} - wF F_{s+1};  L_s = yL - vL L_{s-1} - wL F_{s+1}
            // forward: L_s = alp + bet F_{s+1}, F_s = gam + del F_{s+1}
            double alp = 0.0, bet = 0.0;
            for (int q = 0; q < g.S; ++q) {
                ldouble* r = red + q * kRed;
                const double yF = r[0], vF = r[1], wF = r[2], yL = r[3], vL = r[4], wL = r[5];
                double gam, del, a, b;
                if (q == 0) {
                    gam = yF; del = -wF; a = yL; b = -wL;
                } else {
                    const double den = 1.0 + vF * bet;
                    ok = ok && (den > 0.0);
                    const double inv = 1.0 / den;
                    gam = (yF - vF * alp) * inv;
                    del = -wF * inv;
                    a = yL - vL * alp - vL * bet * gam;
                    b = -vL * bet * del - wL;
                }
                r[0] = gam; r[1] = del; r[2] = a; r[3] = b;
                alp = a;
                bet = b;
            }
            double Fnext = 0.0;
            for (int q = g.S - 1; q >= 0; --q) {
                ldouble* r = red + q * kRed;
                const double F = r[0] + r[1] * Fnext;
                const double Lq = r[2] + r[3] * Fnext;
                r[6] = Fnext;  // X_R of segment q
                r[5] = Lq;
                Fnext = F;
            }
            for (int q = g.S - 1; q >= 1; --q) red[q * kRed + 7] = red[(q - 1) * kRed + 5];
            red[7] = 0.0;
        }
        __syncthreads();
        if (work) { XL = slot[7]; XR = slot[6]; }
    }
    if (work) {
        double x = 0.0;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            const double xn = g.d[mm] - XL * vp[mm] - XR * g.cp[mm];
            x = (mm == g.hi) ? xn : x;
        }
#pragma unroll
        for (int mm = ROWS - 1; mm >= 0; --mm) {
            const bool h = mm == g.hi;
            const bool act = mm >= g.lo && mm < g.hi;
            const double xn = g.d[mm] - XL * vp[mm] - g.cp[mm] * x;
            x = act ? xn : x;
            g.d[mm] = (act || h) ? x : g.d[mm];
        }
        seg_finish(g);
        if (!ok) raise_flag(s);
    }
}

// Chained solve of r lines (fallback when the rows are not diagonally dominant).
template <int ROWS>
__device__ __forceinline__ void chain_solve_r(Seg<ROWS>& g, const RowRFull& full, const ldouble* rt6, bool work,
                                              ldouble* xch, const SolveDesc& s)
{
    double ca[ROWS], cb[ROWS];
    double b1m = 1.0, c1m = 0.0, a2m = 0.0, b2m = 1.0;
    bool ok = true;
    if (work) {
        ok = seg_ends(g, full, b1m, c1m, a2m, b2m);
        const bool first = g.seg == 0;
        const bool last = g.seg == g.S - 1;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            const int i = min(g.p + mm, g.n - 2);
            double A, B, C;
            row_r_interior(rt6, g.n, i, full.v, full.c, full.tdt, A, B, C);
            if (first && mm == 1) { A = 0.0; B = b1m; C = c1m; }
            if (last && mm == g.len - 2) { A = a2m; B = b2m; C = 0.0; }
            const bool act = mm >= g.lo && mm <= g.hi;
            ca[mm] = act ? A : 0.0;
            cb[mm] = act ? B : 1.0;
            g.cp[mm] = act ? C : 0.0;
        }
    }
    ok = chain_core(g, ca, cb, work, xch) && ok;
    if (work && !ok) raise_flag(s);
}

// per-line constants of the explicit phase, kLC doubles per line in LDS
enum { LC_V = 0, LC_C, LC_O0, LC_O1, LC_O2, LC_O3, LC_O4, LC_VX, LC_PV, LC_K, LC_W0, LC_W1, LC_W2, LC_W3, LC_W4,
       LC_Y, kLC };

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
// Gauss-Legendre rule of kSoftQ points on [-1, 1]: the roots of P_n by
// Newton's method from cos(pi (q + 3/4) / (n + 1/2)), weights
// 2 / ((1 - x^2) P_n'(x)^2).
// One root per call: the workgroup's first kSoftQ threads each find one.
constexpr int kSoftQ = 16;
__device__ void gauss_legendre_root(int q, ldouble* x, ldouble* w)
{
    double z = cos(3.14159265358979323846 * (q + 0.75) / (kSoftQ + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= kSoftQ; ++m) {
            const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / (double)m;
            p0 = p1;
            p1 = p2;
        }
        dp = kSoftQ * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (fabs(dz) < 1e-16) break;
    }
    x[q] = z;
    w[q] = 2.0 / ((1.0 - z * z) * dp * dp);
}

// The terminal data averaged over [rlo, rhi] x [ylo, yhi] (section 7.2).  At
// t = T, Delta p(T, T_M; r, y) = c e^{-G r - G^2 y / 2} with c = Delta A_M
// (the step table's bond factor at t = T) and G = G(T_M - T); for each y the
// r-integral of the payoff is closed form on either side of the kink
// r* = ln(c e^{-G^2 y / 2}) / G, and the y-average takes kSoftQ points.
__device__ double payoff_cell(const SolveDesc& s, gcdouble* st0, const ldouble* x, const ldouble* w, double rlo,
                              double rhi, double ylo, double yhi)
{
    if (s.kind == KIND_BOND) return 1.0;
    const double G = st0[ST_GM];
    const double c = s.accrual * st0[ST_AM];
    const double ym = 0.5 * (ylo + yhi), hy = 0.5 * (yhi - ylo);
    double sum = 0.0;
    for (int q = 0; q < kSoftQ; ++q) {
        const double y = ym + hy * x[q];
        const double cy = c * exp(-0.5 * G * G * y);
        const double rs = log(cy) / G;
        double a = rlo, b = rhi, sign = 1.0;
        if (s.kind == KIND_CAPLET) a = fmax(a, rs);
        else if (s.kind == KIND_FLOORLET) { b = fmin(b, rs); sign = -1.0; }
        // e^{-G a} (1 - e^{-G (b - a)}) / G through expm1: no cancellation on short elements
        const double I = b > a ? sign * ((b - a) + cy * exp(-G * a) * expm1(-G * (b - a)) / G) : 0.0;
        sum += w[q] * I;
    }
    return 0.5 * sum / (rhi - rlo);
}

// Terminal data U = payoff at t = T, pointwise or (soften) averaged over the
// node's control element, centred on it in the mesh coordinates
// ([z(x - h/2), z(x + h/2)] in r and y, from the tables): at every
// non-Dirichlet node (soften 1) or where the payoff's kink crosses the element
// (soften 2).  Thread = one (i, k) column, written to every j (lanes are
// consecutive i: each store is contiguous).
__global__ __launch_bounds__(kBlock) void k_terminal(const SolveDesc* __restrict__ descs)
{
    const SolveDesc& s = descs[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) *(__attribute__((address_space(1))) volatile int32_t*)s.flag = 0;
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    gcdouble* r = gp(s.rt) + RT_R * nr;
    gcdouble* y = gp(s.yt) + YT_Y * ny;
    gcdouble* st0 = gp(s.st);
    gdouble* U = gp(s.U);
    // the Gauss-Legendre rule, once per workgroup (s.soften is uniform here)
    __shared__ double gl[2 * kSoftQ];
    ldouble* gx = (ldouble*)gl;
    ldouble* gw = gx + kSoftQ;
    if (s.soften) {
        if (threadIdx.x < kSoftQ) gauss_legendre_root(threadIdx.x, gx, gw);
        __syncthreads();
    }
    const size_t sy = (size_t)nr * nv;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < (int64_t)nr * ny;
         p += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(p % nr);
        const int k = (int)(p / nr);
        const bool dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir) || (k == ny - 1 && s.y_hi_dir);
        double u = dirichlet_value(s, st0, r[i], y[k]);
        if (s.soften && !dir) {
            gcdouble* rt = gp(s.rt);
            gcdouble* yt = gp(s.yt);
            const double rlo = rt[RT_ELO * nr + i], rhi = rt[RT_EHI * nr + i];
            const double ylo = yt[YT_ELO * ny + k], yhi = yt[YT_EHI * ny + k];
            bool take = s.soften == 1;
            if (s.soften == 2 && (s.kind == KIND_CAPLET || s.kind == KIND_FLOORLET)) {
                // the kink r*(y) = ln(c e^{-G^2 y / 2}) / G falls with y
                const double G = st0[ST_GM], c = s.accrual * st0[ST_AM];
                const double top = (log(c) - 0.5 * G * G * ylo) / G, bot = (log(c) - 0.5 * G * G * yhi) / G;
                take = top >= rlo && bot <= rhi;
            }
            if (take) u = payoff_cell(s, st0, gx, gw, rlo, rhi, ylo, yhi);
        }
        gdouble* col = U + (size_t)k * sy + i;
        for (int j = 0; j < nv; ++j) col[(size_t)j * nr] = u;
    }
}

// Explicit predictor + r sweep.  Tile = L consecutive r lines (q = k nv + j)
// with two halo lines on each side, each row stored as [0 0 u_0 .. u_{nr-1} 0 0]
// (pitch >= nr + 4).  LDS: U tile (L+4) x pitch, r solve table 6 x nr,
// per-line constants L x kLC, line-solve scratch.  In the explicit phase
// thread t owns columns t % tpl (+ tpl c) of lines t / tpl + lpp m.
template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_xr(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks,
                                               int step)
{
    extern __shared__ double lds_raw[];
    ldouble* lds = (ldouble*)lds_raw;
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    if (step >= s.n_steps) return;  // whole workgroup: uniform
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int L = s.r_L, S = s.r_S, pitch = s.r_pitch;
    const int nlines = nv * ny;
    const int q0 = tk.y * L;
    const int nl = min(L, nlines - q0);
    const int t = threadIdx.x;
    ldouble* ut = lds;
    ldouble* rt6 = ut + (size_t)(L + 4) * pitch;
    ldouble* lcon = rt6 + 6 * nr;
    ldouble* red = lcon + (size_t)L * kLC;
    gcdouble* U = gp(s.U);
    gdouble* D = gp(s.D);
    gcdouble* rt = gp(s.rt);
    gcdouble* stn = gp(s.st) + kStepStride * step;
    gcdouble* stn1 = stn + kStepStride;
    const double phi = stn[ST_PHI];
    const int tpl = min(kBlock, pow2_ceil(nr));
    const int lpp = kBlock / tpl;
    const int ci = t % tpl;
    const int lr = t / tpl;
    const int creps = (nr + tpl - 1) / tpl;
    const size_t sy = (size_t)nr * nv;

    // Phase A: r solve table, per-line constants and the U tile into LDS
    for (int i = t; i < nr; i += kBlock) {
        rt6[i] = rt[RT_P * nr + i];
        rt6[nr + i] = rt[RT_Q * nr + i];
        rt6[2 * nr + i] = rt[RT_ALO * nr + i];
        rt6[3 * nr + i] = rt[RT_ADI * nr + i];
        rt6[4 * nr + i] = rt[RT_AUP * nr + i];
        rt6[5 * nr + i] = rt[RT_RR * nr + i];
    }
    for (int l = t; l < nl; l += kBlock) {
        const int q = q0 + l;
        const int k = q / nv;
        const int j = q - k * nv;
        gcdouble* vt = gp(s.vt);
        gcdouble* yt = gp(s.yt);
        ldouble* c = lcon + l * kLC;
        const double v = vt[VT_V * nv + j];
        c[LC_V] = v;
        c[LC_C] = phi + yt[YT_Y * ny + k];
        for (int w = 0; w < 5; ++w) c[LC_O0 + w] = vt[(VT_O0 + w) * nv + j];
        c[LC_VX] = vt[VT_X * nv + j];
        c[LC_PV] = v * yt[YT_I * ny + k];
        c[LC_K] = yt[YT_K * ny + k];
        for (int w = 0; w < 5; ++w) c[LC_W0 + w] = yt[(YT_W0 + w) * ny + k];
        c[LC_Y] = yt[YT_Y * ny + k];
    }
    {
        // each thread loads its share of the tile into registers first, so
        // that all of its loads are in flight together
        const int nrows = nl + 4;
        double buf[ROWS + 8];
        int c = 0, lm = 0;
#pragma unroll
        for (int m = 0; m < ROWS + 8; ++m) {
            const int lt = lr + lpp * lm;
            const int i = ci + tpl * c;
            const int q = q0 - 2 + lt;
            buf[m] = (lt < nrows && i < nr && q >= 0 && q < nlines) ? U[(size_t)q * nr + i] : 0.0;
            if (++c == creps) { c = 0; ++lm; }
        }
        c = 0;
        lm = 0;
#pragma unroll
        for (int m = 0; m < ROWS + 8; ++m) {
            const int lt = lr + lpp * lm;
            const int i = ci + tpl * c;
            if (lt < nrows && i < nr) ut[lt * pitch + 2 + i] = buf[m];
            if (++c == creps) { c = 0; ++lm; }
        }
        for (int lt = lr; lt < nrows; lt += lpp)
            if (ci < 2) {
                ut[lt * pitch + ci] = 0.0;
                ut[lt * pitch + nr + 2 + ci] = 0.0;
            }
    }
    __syncthreads();

    // Phase B: explicit predictor, D0 kept in registers until the tile is free.
    // Thread t handles columns ci + tpl c (c < creps) of lines lr + lpp m.
    double dv[ROWS + 1];
    {
        double um[ROWS + 1], upv[ROWS + 1];
        // y neighbours first, all loads in flight together; on a y face the
        // missing neighbour is replaced by the node itself (weight zero)
        {
            int c = 0, lm = 0;
#pragma unroll
            for (int m = 0; m < ROWS + 1; ++m) {
                const int l = lr + lpp * lm;
                const int i = ci + tpl * c;
                um[m] = 0.0;
                upv[m] = 0.0;
                if (l < nl && i < nr) {
                    const int q = q0 + l;
                    const int k = q / nv;
                    const size_t gq = (size_t)q * nr + i;
                    um[m] = U[k > 0 ? gq - sy : gq];
                    upv[m] = U[k < ny - 1 ? gq + sy : gq];
                }
                if (++c == creps) { c = 0; ++lm; }
            }
        }
        int c = 0, lm = 0;
#pragma unroll
        for (int m = 0; m < ROWS + 1; ++m) {
            const int l = lr + lpp * lm;
            const int i = ci + tpl * c;
            dv[m] = 0.0;
            if (l < nl && i < nr) {
                const int q = q0 + l;
                const int k = q / nv;
                const ldouble* lc = lcon + l * kLC;
                const ldouble* u0 = ut + (l + 2) * pitch + 2 + i;
                const double u = u0[0];
                const double v = lc[LC_V];
                // A1 (r, with the reaction term): tabulated row, see hjm_internal.h
                const double e = rt[RT_P * nr + i] * lc[LC_C] + rt[RT_Q * nr + i];
                const double olo = rt[RT_MLO * nr + i] * e + rt[RT_ALO * nr + i] * v;
                const double odi = rt[RT_MDI * nr + i] * e + rt[RT_ADI * nr + i] * v - rt[RT_RR * nr + i];
                const double oup = rt[RT_MUP * nr + i] * e + rt[RT_AUP * nr + i] * v;
                const double oex = rt[RT_MEX * nr + i] * e;
                const double uex = i == 0 ? u0[2] : u0[-2];
                const double a1 = olo * u0[-1] + odi * u + oup * u0[1] + oex * uex;
                // A2 (v): offsets -2..+2 (the tile always holds them)
                const double a2 = lc[LC_O0] * u0[-2 * pitch] + lc[LC_O1] * u0[-pitch] + lc[LC_O2] * u +
                                  lc[LC_O3] * u0[pitch] + lc[LC_O4] * u0[2 * pitch];
                // A3 (y, advection): the k -+ 2 neighbours only on outflow y faces
                double ey = 0.0;
                if (k == 0) ey = lc[LC_W4] * U[(size_t)q * nr + i + 2 * sy];
                if (k == ny - 1 && !s.y_hi_dir) ey = lc[LC_W0] * U[(size_t)q * nr + i - 2 * sy];
                const double by = rt[RT_Y * nr + i] * lc[LC_PV] - lc[LC_K];
                const double a3 = by * (lc[LC_W1] * um[m] + lc[LC_W2] * u + lc[LC_W3] * upv[m] + ey);
                // A0 (mixed r-v), zero on the (r, v) faces through the tables
                const double cross = (u0[1 + pitch] - u0[1 - pitch]) - (u0[-1 + pitch] - u0[-1 - pitch]);
                const double a0 = rt[RT_X * nr + i] * lc[LC_VX] * cross;
                double val = s.dt * (((a1 + a2) + a3) + a0);
                if ((i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir) || (k == ny - 1 && s.y_hi_dir)) {
                    const double ri = rt[RT_R * nr + i], yk = lc[LC_Y];
                    val = dirichlet_value(s, stn1, ri, yk) - dirichlet_value(s, stn, ri, yk);
                }
                dv[m] = val;
            }
            if (++c == creps) { c = 0; ++lm; }
        }
    }
    __syncthreads();
    {
        int c = 0, lm = 0;
#pragma unroll
        for (int m = 0; m < ROWS + 1; ++m) {
            const int l = lr + lpp * lm;
            const int i = ci + tpl * c;
            if (l < nl && i < nr) ut[(l + 2) * pitch + 2 + i] = dv[m];
            if (++c == creps) { c = 0; ++lm; }
        }
    }
    __syncthreads();

    // Phase C: line solves (rows in registers)
    const int l = t % L;
    const int seg = t / L;
    const bool active = seg < S && l < nl;
    const int q = q0 + l;
    const int k = q / nv;
    const bool line_dir = (k == ny - 1) && s.y_hi_dir;
    const bool work = active && !line_dir;
    Seg<ROWS> g;
    seg_init(g, nr, S, seg < S ? seg : 0);
    ldouble* row_lds = ut + (l + 2) * pitch + 2 + g.p;
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) g.d[mm] = (work && mm < g.len) ? row_lds[mm] : 0.0;
    RowRFull full;
    full.rt = rt;
    full.nr = nr;
    full.v = active ? lcon[l * kLC + LC_V] : 0.0;
    full.c = active ? lcon[l * kLC + LC_C] : 0.0;
    full.tdt = s.tdt;
    if (s.r_mode == R_SPIKE) spike_solve_r(g, full, rt6, work, red + (size_t)l * S * kRed, s);
    else chain_solve_r(g, full, rt6, work, red + 2 * l, s);
    if (work) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) row_lds[mm] = g.d[mm];
    }
    __syncthreads();

    // Phase D: D1 back to global memory (the tile's lines are contiguous)
    gdouble* Dt = D + (size_t)q0 * nr;
    for (int ll = lr; ll < nl; ll += lpp)
        for (int i = ci; i < nr; i += tpl) Dt[(size_t)ll * nr + i] = ut[(ll + 2) * pitch + 2 + i];
}

// v sweep: shared factors of the v-line matrix, chained recurrence.
template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_v(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks)
{
    extern __shared__ double lds_raw[];
    ldouble* lds = (ldouble*)lds_raw;
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int L = s.v_L, S = s.v_S;
    const int t = threadIdx.x;
    ldouble* xch = lds;
    const int l = t % L;
    const int seg = t / L;
    const int q = tk.y * L + l;  // line (i, k), q = k*nr + i
    const bool active = seg < S && q < nr * ny;
    const int k = q / nr;
    const int i = q - k * nr;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir) || (k == ny - 1 && s.y_hi_dir);
    const bool work = active && !line_dir;  // identity lines keep D
    Seg<ROWS> g;
    seg_init(g, nv, S, seg < S ? seg : 0);
    gdouble* base = gp(s.D) + (size_t)k * nv * nr + i + (size_t)g.p * nr;
    // the segment's factors (same for every line) and its rows
    gcdouble* vf = gp(s.vf);
    double fa[ROWS], fi[ROWS];
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) {
        const int jj = min(g.p + mm, nv - 1);
        fa[mm] = vf[VF_A * nv + jj];
        fi[mm] = vf[VF_INV * nv + jj];
        g.cp[mm] = vf[VF_C * nv + jj];
        g.d[mm] = (work && mm < g.len) ? base[(size_t)mm * nr] : 0.0;
    }
    const bool first = g.seg == 0;
    const bool last = g.seg == S - 1;
    gcdouble* fs = vf + kVF * nv;
    if (work && first) {
        g.d0 = g.d[0];
        g.d[1] = g.d[1] - fs[VS_F1] * g.d[0];
        g.lo = 1;
    }
    if (work && last) {
        double dl = 0.0;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) dl = (mm == g.len - 1) ? g.d[mm] : dl;
        g.dl = dl;
        const double f2 = fs[VS_F2];
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) g.d[mm] = (mm == g.len - 2) ? g.d[mm] - f2 * dl : g.d[mm];
        g.hi = g.len - 2;
    }
    ldouble* x2 = xch + 2 * l;
    for (int stage = 0; stage < S; ++stage) {
        if (work && seg == stage) {
            double dprev = stage > 0 ? x2[1] : 0.0;
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) {
                const bool act = mm >= g.lo && mm <= g.hi;
                const double dn = (g.d[mm] - fa[mm] * dprev) * fi[mm];
                dprev = act ? dn : dprev;
                g.d[mm] = act ? dn : g.d[mm];
            }
            x2[1] = dprev;
        }
        if (S > 1) __syncthreads();
    }
    for (int stage = S - 1; stage >= 0; --stage) {
        if (work && seg == stage) {
            double x = stage < S - 1 ? x2[0] : 0.0;
#pragma unroll
            for (int mm = ROWS - 1; mm >= 0; --mm) {
                const bool act = mm >= g.lo && mm <= g.hi;
                const double xn = g.d[mm] - g.cp[mm] * x;
                x = act ? xn : x;
                g.d[mm] = act ? xn : g.d[mm];
            }
            x2[0] = x;
            if (first) g.d[0] = (g.d0 - fs[VS_C0] * g.d[1] - fs[VS_E0] * g.d[2]) / fs[VS_B0];
            if (last) {
                double x3 = 0.0, xn2 = 0.0;
#pragma unroll
                for (int mm = 0; mm < ROWS; ++mm) {
                    x3 = (mm == g.len - 3) ? g.d[mm] : x3;
                    xn2 = (mm == g.len - 2) ? g.d[mm] : xn2;
                }
                const double xl = (g.dl - fs[VS_EL] * x3 - fs[VS_AL] * xn2) / fs[VS_BL];
#pragma unroll
                for (int mm = 0; mm < ROWS; ++mm) g.d[mm] = (mm == g.len - 1) ? xl : g.d[mm];
            }
        }
        if (S > 1) __syncthreads();
    }
    if (work) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) base[(size_t)mm * nr] = g.d[mm];
    }
}

// y row k of (I - theta dt A3) on a line with q = lambda^2 r^{2 gamma} v
struct RowY {
    gcdouble* yt;
    int ny;
    double qv;
    __device__ __forceinline__ void operator()(int k, double& A, double& B, double& C, double& E) const
    {
        const double a = yt[YT_T1 * ny + k] * qv + yt[YT_T2 * ny + k];
        A = yt[YT_MA * ny + k] * a;
        B = 1.0 + yt[YT_MB * ny + k] * a;
        C = yt[YT_MC * ny + k] * a;
        E = yt[YT_ME * ny + k] * a;
    }
};

// y sweep + update: chained Thomas per line (i, j), then U += D3.
template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_yu(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks)
{
    extern __shared__ double lds_raw[];
    ldouble* lds = (ldouble*)lds_raw;
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int L = s.y_L, S = s.y_S;
    const int t = threadIdx.x;
    ldouble* xch = lds;
    const int l = t % L;
    const int seg = t / L;
    const int q = tk.y * L + l;  // line (i, j), q = j*nr + i
    const bool active = seg < S && q < nr * nv;
    const int j = q / nr;
    const int i = q - j * nr;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir);
    const bool work = active && !line_dir;
    Seg<ROWS> g;
    seg_init(g, ny, S, seg < S ? seg : 0);
    const size_t sy = (size_t)nr * nv;
    const size_t off = (size_t)q + (size_t)g.p * sy;
    gcdouble* D = gp(s.D);
    gdouble* U = gp(s.U);
    gcdouble* yt = gp(s.yt);
    double u[ROWS];
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) {
        const bool in = active && mm < g.len;
        g.d[mm] = in ? D[off + (size_t)mm * sy] : 0.0;
        u[mm] = in ? U[off + (size_t)mm * sy] : 0.0;
    }
    RowY row;
    row.yt = yt;
    row.ny = ny;
    row.qv = active ? gp(s.rt)[RT_Y * nr + i] * gp(s.vt)[VT_V * nv + j] : 0.0;
    double ca[ROWS], cb[ROWS];
    double b1m = 1.0, c1m = 0.0, a2m = 0.0, b2m = 1.0;
    bool ok = true;
    if (work) {
        ok = seg_ends(g, row, b1m, c1m, a2m, b2m);
        const bool first = g.seg == 0;
        const bool last = g.seg == S - 1;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            const int kk = min(g.p + mm, ny - 1);
            double A, B, C, E;
            row(kk, A, B, C, E);
            if (first && mm == 1) { A = 0.0; B = b1m; C = c1m; }
            if (last && mm == g.len - 2) { A = a2m; B = b2m; C = 0.0; }
            const bool act = mm >= g.lo && mm <= g.hi;
            ca[mm] = act ? A : 0.0;
            cb[mm] = act ? B : 1.0;
            g.cp[mm] = act ? C : 0.0;
        }
    }
    ok = chain_core(g, ca, cb, work, xch + 2 * l) && ok;
    if (work && !ok) raise_flag(s);
    if (active) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) U[off + (size_t)mm * sy] = u[mm] + g.d[mm];
    }
}

// ---------------------------------------------------------------------------
// Split path: explicit predictor and r sweep as two kernels.
// ---------------------------------------------------------------------------

// Wave-level barrier for data exchanged through LDS between the lanes of one
// wavefront (the lanes execute in lockstep; this orders the LDS accesses).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Neighbouring lanes' values by one DPP move per 32-bit half (wave_shr:1,
// wave_shl:1: lane l reads lane l - 1, resp. l + 1, across the whole wave):
// VALU moves, no LDS-pipe round trip.  Lane 0 (resp. 63) keeps its own
// value; the callers overwrite those lanes.
__device__ __forceinline__ double from_lane_below(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_lane_above(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// The value of the lane OFF below (row_shr) or above (row_shl) inside the
// calling lane's row of 16 lanes, one DPP move per 32-bit half; a lane whose
// source lies outside its row reads 0 (bound_ctrl; the callers select, so no
// copy of the lane's own value is needed first).
template <int OFF>
__device__ __forceinline__ double row_below(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x110 + OFF, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x110 + OFF, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
template <int OFF>
__device__ __forceinline__ double row_above(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x100 + OFF, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x100 + OFF, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// The spike method's reduced system for lines of S <= 16 segments, each
// segment in one lane (seg = lane mod S; a line's lanes lie inside one row of
// 16 lanes), by parallel scans across the line's lanes instead of one lane's
// serial sweep.  Segment s knows the first- and last-row values of its three
// local solutions: F_s = yF - vF L_{s-1} - wF F_{s+1}, L_s = yL - vL L_{s-1} -
// wL F_{s+1} (F, L: the segment's first and last unknowns).  Forward
// elimination gives L_s = alp_s + bet_s F_{s+1} and F_s = gam_s + del_s F_{s+1},
// with the pivot den_s = 1 + vF bet_{s-1}; with alp = a / z, bet = b / z
// (z_s = den_s z_{s-1}, z_{-1} = 1, a = b = 0) that recurrence is linear,
// (a, b, z)_s = M_s (a, b, z)_{s-1} with
//   M_s = [[-vL, yL vF - vL yF, yL], [0, vL wF - wL vF, -wL], [0, vF, 1]],
// so an inclusive scan of the products M_s ... M_0 (log2 S steps of row
// shifts) gives every (a, b, z)_s at once.  Then gam_s = (yF z_{s-1} -
// vF a_{s-1}) / z_s, del_s = -wF z_{s-1} / z_s, and the backward recurrence
// F_s = gam_s + del_s F_{s+1} (F_S = 0) is a suffix scan of affine maps.
// Returns the coupling values XL = L_{s-1} and XR = F_{s+1} of this lane's
// segment (0 at the line's ends); false after a non-positive pivot.
__device__ __forceinline__ bool reduced_scan(int seg, int S, double yF, double vF, double wF, double yL, double vL,
                                             double wL, double& XL, double& XR)
{
    // this segment's transfer matrix, [[x, r0, r1], [0, b00, b01], [0, b10, b11]]
    double x = -vL, r0 = yL * vF - vL * yF, r1 = yL, b00 = vL * wF - wL * vF, b01 = -wL, b10 = vF, b11 = 1.0;
    auto fwd = [&](auto off_c) {
        constexpr int OFF = decltype(off_c)::value;
        if (S <= OFF) return;  // wave-uniform
        const double qx = row_below<OFF>(x), q0 = row_below<OFF>(r0), q1 = row_below<OFF>(r1);
        const double c00 = row_below<OFF>(b00), c01 = row_below<OFF>(b01);
        const double c10 = row_below<OFF>(b10), c11 = row_below<OFF>(b11);
        if (seg >= OFF) {
            const double nr0 = x * q0 + r0 * c00 + r1 * c10;
            const double nr1 = x * q1 + r0 * c01 + r1 * c11;
            const double n00 = b00 * c00 + b01 * c10, n01 = b00 * c01 + b01 * c11;
            const double n10 = b10 * c00 + b11 * c10, n11 = b10 * c01 + b11 * c11;
            x = x * qx;
            r0 = nr0; r1 = nr1;
            b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
    };
    fwd(std::integral_constant<int, 1>());
    fwd(std::integral_constant<int, 2>());
    fwd(std::integral_constant<int, 4>());
    fwd(std::integral_constant<int, 8>());
    // (a, b, z) of this segment and of the previous one
    const double a = r1, b = b01, z = b11;
    double ap = row_below<1>(a), zp = row_below<1>(z);
    if (seg == 0) { ap = 0.0; zp = 1.0; }
    const bool ok = z > 0.0;
    const double iz = rcp_nr(z);
    double del = -wF * zp * iz;
    double gam = (yF * zp - vF * ap) * iz;
    const double alp = a * iz, bet = b * iz;
    // F_s = gam_s + del_s F_{s+1}: compose the affine maps toward the line's end
    auto bwd = [&](auto off_c) {
        constexpr int OFF = decltype(off_c)::value;
        if (S <= OFF) return;  // wave-uniform
        const double qd = row_above<OFF>(del), qg = row_above<OFF>(gam);
        if (seg + OFF < S) {
            gam = del * qg + gam;
            del = del * qd;
        }
    };
    bwd(std::integral_constant<int, 1>());
    bwd(std::integral_constant<int, 2>());
    bwd(std::integral_constant<int, 4>());
    bwd(std::integral_constant<int, 8>());
    const double F = gam;
    double Fn = row_above<1>(F);
    if (seg == S - 1) Fn = 0.0;
    const double L = alp + bet * Fn;
    double Lp = row_below<1>(L);
    if (seg == 0) Lp = 0.0;
    XL = Lp;
    XR = Fn;
    return ok;
}

// Explicit predictor D0 = dt (A1 + A2 + A3 + A0) U^n (eq. (discreta) with the
// centred stencils of eq. (esquema), one-sided rows on outflow faces), and the
// Dirichlet increment on Dirichlet nodes, at the J nodes (i, j0 + m, k),
// m < J, j0 + m < nv; put(m, value) receives each.  The caller's lanes are
// consecutive i (lane = threadIdx.x mod 64, whole waves), so every load of a
// wave is one contiguous row segment.  The loads are issued up front: the v
// window u(i, j0-2 .. j0+J+1) and the two y neighbours; the outflow extra
// entry (two nodes in) only on the r faces, where its weight is not zero.
// The neighbouring columns u(i -+ 1, j0-1 .. j0+J) are loaded too (SHFL
// false) or taken from the neighbouring lanes' v windows by DPP moves across
// the wave, the wave's edge lanes loading theirs (SHFL true: fewer loads and
// registers; measured faster inside the fused kernel, slower in the
// explicit kernel alone).  j0 must be wave-uniform (the v-table reads are
// scalar).
template <int J, bool SHFL, class Put>
__device__ __forceinline__ void explicit_nodes(const SolveDesc& s, int i, int k, int j0, int step, const Put& put)
{
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    gcdouble* U = gp(s.U);
    gcdouble* rt = gp(s.rt);
    kcdouble* vt = kp(s.vt);
    gcdouble* yt = gp(s.yt);
    gcdouble* stn = gp(s.st) + kStepStride * step;

    const size_t sl = (size_t)nr;       // stride of j
    const size_t sy = (size_t)nr * nv;  // stride of k
    gcdouble* col = U + (size_t)k * sy; // (k, j = 0, i = 0)
    const int im = max(i - 1, 0), ip = min(i + 1, nr - 1);
    // y stencil: two neighbours (offsets oa, ob) and the node itself
    const bool yhd = s.y_hi_dir && k == ny - 1;
    int oa = -1, ob = 1;
    if (k == 0) { oa = 1; ob = 2; }
    else if (k == ny - 1) { oa = -2; ob = -1; }
    if (yhd) { oa = 0; ob = 0; }
    gcdouble* cola = col + (ptrdiff_t)oa * (ptrdiff_t)sy;  // plane k + oa
    gcdouble* colb = col + (ptrdiff_t)ob * (ptrdiff_t)sy;
    const int dx = i == 0 ? 2 : (i == nr - 1 ? -2 : 0);
    auto jcl = [&](int jj) { return (size_t)min(max(jj, 0), nv - 1) * sl; };
    double cw[J + 4], lw[J + 2], rw[J + 2], ya[J], yb[J], ux[J];
#pragma unroll
    for (int m = 0; m < J + 4; ++m) cw[m] = col[jcl(j0 - 2 + m) + i];
#pragma unroll
    for (int m = 0; m < J; ++m) {
        ya[m] = cola[jcl(j0 + m) + i];
        yb[m] = colb[jcl(j0 + m) + i];
    }
    if (SHFL) {
        // the r faces clamp to the node itself
        const int lane = (int)(threadIdx.x & 63);
#pragma unroll
        for (int m = 0; m < J + 2; ++m) {
            const double lo = from_lane_below(cw[m + 1]);
            const double hi = from_lane_above(cw[m + 1]);
            lw[m] = i == 0 ? cw[m + 1] : lo;
            rw[m] = i == nr - 1 ? cw[m + 1] : hi;
        }
        if (lane == 0 && i > 0) {
#pragma unroll
            for (int m = 0; m < J + 2; ++m) lw[m] = col[jcl(j0 - 1 + m) + im];
        }
        if (lane == 63 && i < nr - 1) {
#pragma unroll
            for (int m = 0; m < J + 2; ++m) rw[m] = col[jcl(j0 - 1 + m) + ip];
        }
    } else {
#pragma unroll
        for (int m = 0; m < J + 2; ++m) {
            lw[m] = col[jcl(j0 - 1 + m) + im];
            rw[m] = col[jcl(j0 - 1 + m) + ip];
        }
    }
    if (dx != 0) {
        // outflow r face rows reach two nodes in
#pragma unroll
        for (int m = 0; m < J; ++m) ux[m] = col[jcl(j0 + m) + (size_t)(i + dx)];
    } else {
        // interior rows: the extra entry has weight zero
#pragma unroll
        for (int m = 0; m < J; ++m) ux[m] = cw[m + 2];
    }

    // per-column constants: A1 row pieces (affine in v), A3 coefficient, A0 factor
    const double c = stn[ST_PHI] + yt[YT_Y * ny + k];
    const double e = rt[RT_P * nr + i] * c + rt[RT_Q * nr + i];
    const double mlo = rt[RT_MLO * nr + i] * e, alo = rt[RT_ALO * nr + i];
    const double mdi = rt[RT_MDI * nr + i] * e - rt[RT_RR * nr + i], adi = rt[RT_ADI * nr + i];
    const double mup = rt[RT_MUP * nr + i] * e, aup = rt[RT_AUP * nr + i];
    const double mex = rt[RT_MEX * nr + i] * e;
    const double ryk = rt[RT_Y * nr + i] * yt[YT_I * ny + k];
    const double kyk = yt[YT_K * ny + k];
    const double rx = rt[RT_X * nr + i];
    // (entries chosen first, then loaded unconditionally: no load in a
    // branch, which would wait for every load before it)
    const double wa = yt[(k == 0 ? YT_W3 : (k == ny - 1 ? YT_W0 : YT_W1)) * ny + k];
    const double wb = yt[(k == 0 ? YT_W4 : (k == ny - 1 ? YT_W1 : YT_W3)) * ny + k];
    const double w2 = yt[YT_W2 * ny + k];
    // Dirichlet nodes: the increment does not depend on j
    gcdouble* gdn = gp(s.gd) + (size_t)step * (2 * ny + nr);
    const bool rlo = i == 0 && s.r_lo_dir, rhi = i == nr - 1 && s.r_hi_dir;
    const bool dir = rlo || rhi || yhd;
    const double gval = dir ? gdn[yhd ? 2 * ny + i : (rlo ? k : (rhi ? ny + k : 0))] : 0.0;
    const double dt = s.dt;
#pragma unroll
    for (int m = 0; m < J; ++m) {
        const int j = j0 + m;
        if (j >= nv) break;  // wave-uniform
        const double v = vt[VT_V * nv + j];
        const double olo = mlo + alo * v, odi = mdi + adi * v, oup = mup + aup * v;
        const double a1 = olo * lw[m + 1] + odi * cw[m + 2] + oup * rw[m + 1] + mex * ux[m];
        const double a2 = vt[VT_O0 * nv + j] * cw[m] + vt[VT_O1 * nv + j] * cw[m + 1] +
                          vt[VT_O2 * nv + j] * cw[m + 2] + vt[VT_O3 * nv + j] * cw[m + 3] +
                          vt[VT_O4 * nv + j] * cw[m + 4];
        const double by = ryk * v - kyk;
        const double a3 = by * (wa * ya[m] + w2 * cw[m + 2] + wb * yb[m]);
        const double cross = (rw[m + 2] - rw[m]) - (lw[m + 2] - lw[m]);
        const double a0 = rx * vt[VT_X * nv + j] * cross;
        const double val = dt * (((a1 + a2) + a3) + a0);
        put(m, dir ? gval : val);
    }
}

// The corrected start of the Craig-Sneyd family at the same J nodes, for
// the second sweep sequence of a step (the descriptor's D is the correction
// array):  E0 = dt A U + dt (a0 A0 + a1 (A1 + A2 + A3)) D3 + b D3 on
// non-Dirichlet nodes, with (a0, a1, b) = (sc_a0, sc_a1, sc_b) and D3 the
// first sequence's result; on Dirichlet nodes the increment g(t_{n+1}) -
// g(t_n) when b = 0 (the correction is relative to U^n) and 0 otherwise (HV:
// relative to U^n + D3, which already holds it).  The stencil of U, then the
// same stencil of D3, each over windows loaded as the predictor loads them.
template <int J, bool SHFL, class Put>
__device__ __forceinline__ void corrected_start(const SolveDesc& s, int i, int k, int j0, int step, const Put& put)
{
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    gcdouble* rt = gp(s.rt);
    kcdouble* vt = kp(s.vt);
    gcdouble* yt = gp(s.yt);
    gcdouble* stn = gp(s.st) + kStepStride * step;

    const size_t sl = (size_t)nr;       // stride of j
    const size_t sy = (size_t)nr * nv;  // stride of k
    const int im = max(i - 1, 0), ip = min(i + 1, nr - 1);
    // y stencil: two neighbours (offsets oa, ob) and the node itself
    const bool yhd = s.y_hi_dir && k == ny - 1;
    int oa = -1, ob = 1;
    if (k == 0) { oa = 1; ob = 2; }
    else if (k == ny - 1) { oa = -2; ob = -1; }
    if (yhd) { oa = 0; ob = 0; }
    const int dx = i == 0 ? 2 : (i == nr - 1 ? -2 : 0);
    auto jcl = [&](int jj) { return (size_t)min(max(jj, 0), nv - 1) * sl; };
    double cw[J + 4], lw[J + 2], rw[J + 2], ya[J], yb[J], ux[J];
    // the windows of field F around the J nodes
    auto load = [&](gcdouble* F) {
        gcdouble* col = F + (size_t)k * sy;                          // (k, j = 0, i = 0)
        gcdouble* cola = col + (ptrdiff_t)oa * (ptrdiff_t)sy;         // plane k + oa
        gcdouble* colb = col + (ptrdiff_t)ob * (ptrdiff_t)sy;
#pragma unroll
        for (int m = 0; m < J + 4; ++m) cw[m] = col[jcl(j0 - 2 + m) + i];
#pragma unroll
        for (int m = 0; m < J; ++m) {
            ya[m] = cola[jcl(j0 + m) + i];
            yb[m] = colb[jcl(j0 + m) + i];
        }
        if (SHFL) {
            // the r faces clamp to the node itself
            const int lane = (int)(threadIdx.x & 63);
#pragma unroll
            for (int m = 0; m < J + 2; ++m) {
                const double lo = from_lane_below(cw[m + 1]);
                const double hi = from_lane_above(cw[m + 1]);
                lw[m] = i == 0 ? cw[m + 1] : lo;
                rw[m] = i == nr - 1 ? cw[m + 1] : hi;
            }
            if (lane == 0 && i > 0) {
#pragma unroll
                for (int m = 0; m < J + 2; ++m) lw[m] = col[jcl(j0 - 1 + m) + im];
            }
            if (lane == 63 && i < nr - 1) {
#pragma unroll
                for (int m = 0; m < J + 2; ++m) rw[m] = col[jcl(j0 - 1 + m) + ip];
            }
        } else {
#pragma unroll
            for (int m = 0; m < J + 2; ++m) {
                lw[m] = col[jcl(j0 - 1 + m) + im];
                rw[m] = col[jcl(j0 - 1 + m) + ip];
            }
        }
        if (dx != 0) {
            // outflow r face rows reach two nodes in
#pragma unroll
            for (int m = 0; m < J; ++m) ux[m] = col[jcl(j0 + m) + (size_t)(i + dx)];
        } else {
            // interior rows: the extra entry has weight zero
#pragma unroll
            for (int m = 0; m < J; ++m) ux[m] = cw[m + 2];
        }
    };

    load(gp(s.U));
    // per-column constants: A1 row pieces (affine in v), A3 coefficient, A0 factor
    const double c = stn[ST_PHI] + yt[YT_Y * ny + k];
    const double e = rt[RT_P * nr + i] * c + rt[RT_Q * nr + i];
    const double mlo = rt[RT_MLO * nr + i] * e, alo = rt[RT_ALO * nr + i];
    const double mdi = rt[RT_MDI * nr + i] * e - rt[RT_RR * nr + i], adi = rt[RT_ADI * nr + i];
    const double mup = rt[RT_MUP * nr + i] * e, aup = rt[RT_AUP * nr + i];
    const double mex = rt[RT_MEX * nr + i] * e;
    const double ryk = rt[RT_Y * nr + i] * yt[YT_I * ny + k];
    const double kyk = yt[YT_K * ny + k];
    const double rx = rt[RT_X * nr + i];
    // (entries chosen first, then loaded unconditionally: no load in a
    // branch, which would wait for every load before it)
    const double wa = yt[(k == 0 ? YT_W3 : (k == ny - 1 ? YT_W0 : YT_W1)) * ny + k];
    const double wb = yt[(k == 0 ? YT_W4 : (k == ny - 1 ? YT_W1 : YT_W3)) * ny + k];
    const double w2 = yt[YT_W2 * ny + k];
    // (A1 + A2 + A3) and A0 of the loaded field at node j0 + m
    auto stencil = [&](int m, double& a123, double& a0) {
        const int j = j0 + m;
        const double v = vt[VT_V * nv + j];
        const double olo = mlo + alo * v, odi = mdi + adi * v, oup = mup + aup * v;
        const double a1 = olo * lw[m + 1] + odi * cw[m + 2] + oup * rw[m + 1] + mex * ux[m];
        const double a2 = vt[VT_O0 * nv + j] * cw[m] + vt[VT_O1 * nv + j] * cw[m + 1] +
                          vt[VT_O2 * nv + j] * cw[m + 2] + vt[VT_O3 * nv + j] * cw[m + 3] +
                          vt[VT_O4 * nv + j] * cw[m + 4];
        const double by = ryk * v - kyk;
        const double a3 = by * (wa * ya[m] + w2 * cw[m + 2] + wb * yb[m]);
        const double cross = (rw[m + 2] - rw[m]) - (lw[m + 2] - lw[m]);
        a123 = (a1 + a2) + a3;
        a0 = rx * vt[VT_X * nv + j] * cross;
    };
    // Dirichlet nodes: the increment does not depend on j
    gcdouble* gdn = gp(s.gd) + (size_t)step * (2 * ny + nr);
    const bool rlo = i == 0 && s.r_lo_dir, rhi = i == nr - 1 && s.r_hi_dir;
    const bool dir = rlo || rhi || yhd;
    const double gval = dir ? gdn[yhd ? 2 * ny + i : (rlo ? k : (rhi ? ny + k : 0))] : 0.0;
    const double dt = s.dt;
    {
        double su[J], s0[J];
#pragma unroll
        for (int m = 0; m < J; ++m) {
            if (j0 + m >= nv) break;
            stencil(m, su[m], s0[m]);
        }
        load(gp(s.D3));
        const double a0c = s.sc_a0, a1c = s.sc_a1, bc = s.sc_b;
        const double gdir = bc == 0.0 ? gval : 0.0;
#pragma unroll
        for (int m = 0; m < J; ++m) {
            if (j0 + m >= nv) break;
            double d123, d0;
            stencil(m, d123, d0);
            const double val = dt * ((su[m] + a1c * d123) + (s0[m] + a0c * d0)) + bc * cw[m + 2];
            put(m, dir ? gdir : val);
        }
    }
}

// Explicit predictor alone (split path), or the corrected start of the
// Craig-Sneyd family (STAGE2).  Thread = one (i, k) column and J consecutive
// v nodes.
template <int J, bool STAGE2>
__global__ __launch_bounds__(kBlock) void k_exp(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks,
                                                int step)
{
    const int bi = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int2 tk = tasks ? tasks[bi] : make_int2(0, bi);
    const SolveDesc& s = descs[tk.x];
    if (step >= s.n_steps) return;
    const int nr = s.nr;
    const int cb = tk.y % s.exp_cb;
    const int jc = tk.y / s.exp_cb;
    const int p = cb * kExpCols + (int)threadIdx.x;
    if (p >= nr * s.ny) return;  // no barriers below
    const int k = p / nr;
    const int i = p - k * nr;
    // j is the same on every lane: keep it (and the v-table reads) scalar
    const int j0 = __builtin_amdgcn_readfirstlane(jc * J);
    gdouble* dcol = gp(s.D) + (size_t)k * nr * s.nv + (size_t)j0 * nr + i;
    auto put = [&](int m, double x) { dcol[(size_t)m * nr] = x; };
    if constexpr (STAGE2)
        corrected_start<J, false>(s, i, k, j0, step, put);
    else
        explicit_nodes<J, false>(s, i, k, j0, step, put);
}

// The r-axis table entries of the two face rows (0 and nr - 1) that
// RowRFull reads, staged in LDS once per workgroup so that the spike solve's
// first and last lanes take them from there: kFace doubles, row 0 then row
// nr - 1, each in the order of kFaceRows.  Every thread calls it; the caller
// synchronises the workgroup before reading.
constexpr int kFaceRows[] = {RT_P, RT_Q, RT_MLO, RT_ALO, RT_MDI, RT_ADI, RT_RR, RT_MUP, RT_AUP, RT_MEX};
constexpr int kFaceN = 10;
constexpr int kFace = 2 * kFaceN;
// the rows above, four bits each (an immediate: no load of the index table)
constexpr uint64_t face_rows_packed()
{
    uint64_t p = 0;
    for (int c = 0; c < kFaceN; ++c) p |= (uint64_t)kFaceRows[c] << (4 * c);
    return p;
}
static_assert(RT_EHI < 16, "table rows fit four bits");
// Thread t < kFace's entry of the face rows (load_face) and its store into
// LDS (store_face), apart so that callers can issue the load early.
__device__ __forceinline__ double load_face(const SolveDesc& s)
{
    const int t = (int)threadIdx.x;
    if (t >= kFace) return 0.0;
    const int w = t / kFaceN;
    const int row = (int)((face_rows_packed() >> (4 * (t - w * kFaceN))) & 15u);
    return gp(s.rt)[(size_t)row * s.nr + (w ? s.nr - 1 : 0)];
}
__device__ __forceinline__ void store_face(ldouble* face, double x)
{
    const int t = (int)threadIdx.x;
    if (t < kFace) face[t] = x;
}
__device__ __forceinline__ void stage_face(const SolveDesc& s, ldouble* face)
{
    store_face(face, load_face(s));
}

// Face row w (0: row 0, 1: row nr - 1) of (I - theta dt A1) on a line with
// variance v and c = f_t + kappa f + y, from the staged entries (as RowRFull).
__device__ __forceinline__ void face_row(const ldouble* face, int w, double v, double c, double tdt, double& A,
                                         double& B, double& C, double& E)
{
    const ldouble* f = face + w * kFaceN;
    const double e = f[0] * c + f[1];
    const double olo = f[2] * e + f[3] * v;
    const double odi = f[4] * e + f[5] * v - f[6];
    const double oup = f[7] * e + f[8] * v;
    const double oex = f[9] * e;
    A = -tdt * olo;
    B = 1.0 - tdt * odi;
    C = -tdt * oup;
    E = -tdt * oex;
}

// The spike solve of one r line of nr = S * ROWS rows (S a power of two <=
// 64) by S consecutive lanes of a wavefront: this lane holds rows
// [seg ROWS, (seg + 1) ROWS) in d (right-hand side in, solution out).  tseg
// is the segment's block of the staged row table, my the lane's 8-double
// slot of LDS scratch (the line's lanes' slots are consecutive).  Each lane
// eliminates its rows (spikes v toward the previous segment, w toward the
// next), lane 0 of the line solves the reduced system of the segments' end
// unknowns, and every lane back-substitutes.  The outflow face rows (one
// entry beyond the band) are folded into rows 1 and n-2 first and recovered
// last.  Accurate when the rows are diagonally dominant (the host selects
// this path only then).  Returns false after a non-positive pivot.
template <int ROWS>
__device__ __forceinline__ bool spike_r_lane(const SolveDesc& s, const ldouble* tseg, const ldouble* face, ldouble* my,
                                             int seg, int S, double v, double c, double (&d)[ROWS])
{
    auto coef = [&](int mm, double& A, double& B, double& C) {
        const ldouble* tb = tseg + mm;
        const double e = tb[RF_P * ROWS] * c + tb[RF_Q * ROWS];
        A = tb[RF_ALO * ROWS] * v + e;
        B = tb[RF_ADI * ROWS] * v + tb[RF_B * ROWS];
        C = tb[RF_AUP * ROWS] * v - e;
    };
    const bool first = seg == 0;
    const bool last = seg == S - 1;
    bool ok = true;
    // face rows: fold row 0 into row 1 and row n-1 into row n-2
    double fb0 = 1.0, fc0 = 0.0, fe0 = 0.0, fd0 = 0.0, b1 = 0.0, c1 = 0.0, d1 = 0.0;
    double fal = 0.0, fbl = 1.0, fel = 0.0, fdl = 0.0, a2 = 0.0, b2 = 0.0, d2 = 0.0;
    if (first) {
        double A0, B0, C0, E0, A1, B1, C1;
        face_row(face, 0, v, c, s.tdt, A0, B0, C0, E0);
        coef(1, A1, B1, C1);
        const double f = A1 / B0;
        fb0 = B0; fc0 = C0; fe0 = E0; fd0 = d[0];
        b1 = B1 - f * C0;
        c1 = C1 - f * E0;
        d1 = d[1] - f * d[0];
        ok = ok && B0 > 0.0;
    }
    if (last) {
        double Al, Bl, Cl, El, A2, B2, C2;
        face_row(face, 1, v, c, s.tdt, Al, Bl, Cl, El);
        coef(ROWS - 2, A2, B2, C2);
        const double f = C2 / Bl;
        fal = Al; fbl = Bl; fel = El; fdl = d[ROWS - 1];
        a2 = A2 - f * El;
        b2 = B2 - f * Al;
        d2 = d[ROWS - 2] - f * d[ROWS - 1];
        ok = ok && Bl > 0.0;
    }
    if (first) { d[0] = 0.0; d[1] = d1; }
    if (last) { d[ROWS - 1] = 0.0; d[ROWS - 2] = d2; }

    // local elimination: y' (in d), v' (coupling to the previous segment), c'
    double vp[ROWS], cp[ROWS];
    double cprev = 0.0, yprev = 0.0, vprev = -1.0;
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) {
        double A, B, C;
        coef(mm, A, B, C);
        if (mm == 0) { A = first ? 0.0 : A; B = first ? 1.0 : B; C = first ? 0.0 : C; }
        if (mm == 1) { A = first ? 0.0 : A; B = first ? b1 : B; C = first ? c1 : C; }
        if (mm == ROWS - 2) { A = last ? a2 : A; B = last ? b2 : B; C = last ? 0.0 : C; }
        if (mm == ROWS - 1) { A = last ? 0.0 : A; B = last ? 1.0 : B; C = last ? 0.0 : C; }
        const double den = B - A * cprev;
        const double inv = rcp_nr(den);
        ok = ok && den > 0.0;
        cprev = C * inv;
        yprev = (d[mm] - A * yprev) * inv;
        vprev = -A * vprev * inv;
        cp[mm] = cprev;
        d[mm] = yprev;
        vp[mm] = vprev;
    }
    double XL = 0.0, XR = 0.0;
    if (S > 1) {
        // first-row values of the three local solutions
        double y = d[ROWS - 1], vv = vp[ROWS - 1], w = cp[ROWS - 1];
#pragma unroll
        for (int mm = ROWS - 2; mm >= 0; --mm) {
            y = d[mm] - cp[mm] * y;
            vv = vp[mm] - cp[mm] * vv;
            w = -cp[mm] * w;
        }
        if (S <= 16) {
            ok = reduced_scan(seg, S, y, vv, w, d[ROWS - 1], vp[ROWS - 1], cp[ROWS - 1], XL, XR) && ok;
        } else {
        my[0] = y; my[1] = vv; my[2] = w;
        my[3] = d[ROWS - 1]; my[4] = vp[ROWS - 1]; my[5] = cp[ROWS - 1];
        wave_sync();
        if (first) {
            // F_s = yF - vF L_{s-1} - wF F_{s+1};  L_s = yL - vL L_{s-1} - wL F_{s+1}
            // forward: L_s = alp + bet F_{s+1}, F_s = gam + del F_{s+1}
            double alp = 0.0, bet = 0.0;
#pragma unroll 4
            for (int qq = 0; qq < S; ++qq) {
                ldouble* r = my + qq * 8;
                const double yF = r[0], vF = r[1], wF = r[2], yL = r[3], vL = r[4], wL = r[5];
                const double den = 1.0 + vF * bet;
                ok = ok && den > 0.0;
                const double inv = rcp_nr(den);
                const double gam = (yF - vF * alp) * inv;
                const double del = -wF * inv;
                alp = yL - vL * alp - vL * bet * gam;
                bet = -vL * bet * del - wL;
                r[0] = gam; r[1] = del; r[2] = alp; r[3] = bet;
            }
            // backward: F_q and L_q from F_{q+1}; segment q+1 couples to L_q
            // on its left and segment q to F_{q+1} on its right
            double Fn = 0.0;
#pragma unroll 4
            for (int qq = S - 1; qq >= 0; --qq) {
                ldouble* r = my + qq * 8;
                const double F = r[0] + r[1] * Fn;
                const double L = r[2] + r[3] * Fn;
                r[6] = Fn;                        // X_R of segment q
                if (qq + 1 < S) r[8 + 7] = L;     // X_L of segment q+1
                Fn = F;
            }
            my[7] = 0.0;                          // X_L of segment 0
        }
        wave_sync();
        XL = my[7];
        XR = my[6];
        }
    }
    // back substitution with the coupling values
    double x = d[ROWS - 1] - XL * vp[ROWS - 1] - XR * cp[ROWS - 1];
    d[ROWS - 1] = x;
#pragma unroll
    for (int mm = ROWS - 2; mm >= 0; --mm) {
        x = (d[mm] - XL * vp[mm]) - cp[mm] * x;
        d[mm] = x;
    }
    if (first) d[0] = (fd0 - fc0 * d[1] - fe0 * d[2]) / fb0;
    if (last) d[ROWS - 1] = (fdl - fel * d[ROWS - 3] - fal * d[ROWS - 2]) / fbl;
    return ok;
}

// Stage the split-path r row table into LDS, one block per segment:
// [seg][kRF * ROWS + 1] (the odd pitch spreads the segments of a wave over
// the LDS banks).  The caller synchronises the workgroup before reading it.
// MAXIT > 0 bounds the thread's share (kRF nr <= MAXIT kBlock): its loads
// are then all issued before the first LDS write, one memory latency instead
// of one per element.
template <int ROWS, int MAXIT = 0>
__device__ __forceinline__ void stage_rf(const SolveDesc& s, ldouble* tab)
{
    if constexpr (MAXIT >= kRF) {
        if (s.nr == kBlock) {
            // one r node per thread: its kRF rows, no division by nr
            constexpr int TP = kRF * ROWS + 1;
            gcdouble* rf = gp(s.rf);
            const int i = (int)threadIdx.x;
            const int sg = i / ROWS;
            const int mm = i - sg * ROWS;
            double x[kRF];
#pragma unroll
            for (int c6 = 0; c6 < kRF; ++c6) x[c6] = rf[c6 * kBlock + i];
#pragma unroll
            for (int c6 = 0; c6 < kRF; ++c6) tab[sg * TP + c6 * ROWS + mm] = x[c6];
            return;
        }
    }
    if constexpr (MAXIT > 0) {
        constexpr int TP = kRF * ROWS + 1;
        const int n = kRF * s.nr;
        gcdouble* rf = gp(s.rf);
        double x[MAXIT];
#pragma unroll
        for (int q = 0; q < MAXIT; ++q) {
            const int idx = (int)threadIdx.x + q * kBlock;
            x[q] = idx < n ? rf[idx] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < MAXIT; ++q) {
            const int idx = (int)threadIdx.x + q * kBlock;
            if (idx < n) {
                const int c6 = idx / s.nr;
                const int i = idx - c6 * s.nr;
                const int sg = i / ROWS;
                tab[sg * TP + c6 * ROWS + (i - sg * ROWS)] = x[q];
            }
        }
        // a table longer than the bound (never for the callers' shapes) goes on below
    }
    constexpr int TP = kRF * ROWS + 1;
    const int nr = s.nr;
    gcdouble* rf = gp(s.rf);
    for (int idx = (int)threadIdx.x + MAXIT * kBlock; idx < kRF * nr; idx += kBlock) {
        const int c6 = idx / nr;
        const int i = idx - c6 * nr;
        const int sg = i / ROWS;
        const int mm = i - sg * ROWS;
        tab[sg * TP + c6 * ROWS + mm] = rf[idx];
    }
}

// r sweep (I - theta dt A1) D1 = D0 by the spike method (split path): lines
// of nr = S * ROWS rows, S a power of two <= 64, each solved by S consecutive
// lanes of a wavefront.
template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_rs(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks,
                                               int step)
{
    extern __shared__ double lds_raw[];
    ldouble* lds = (ldouble*)lds_raw;
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    if (step >= s.n_steps) return;  // whole workgroup: uniform
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int S = s.rs_S;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int seg = lane & (S - 1);
    const int nlines = nv * ny;
    const int q_raw = tk.y * s.rs_L + (t >> 6) * (64 >> s.rs_log2S) + (lane >> s.rs_log2S);
    const bool active = q_raw < nlines;
    const int q = active ? q_raw : nlines - 1;  // tail lanes repeat the last line, store nothing
    const int k = q / nv;
    const int j = q - k * nv;
    const bool store = active && !(s.y_hi_dir && k == ny - 1);
    // the line's rows first, so that their loads are in flight while the row
    // table is staged
    const double v = gp(s.vt)[VT_V * nv + j];
    const double c = gp(s.st)[kStepStride * step + ST_PHI] + gp(s.yt)[YT_Y * ny + k];
    gdouble* line = gp(s.D) + (size_t)q * nr + (size_t)seg * ROWS;
    double d[ROWS];
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) d[mm] = line[mm];
    constexpr int TP = kRF * ROWS + 1;
    ldouble* tab = lds;
    ldouble* red = lds + (size_t)TP * S;  // 8 doubles per thread
    ldouble* face = red + (size_t)kBlock * 8;
    stage_rf<ROWS>(s, tab);
    stage_face(s, face);
    __syncthreads();
    const bool ok = spike_r_lane<ROWS>(s, tab + seg * TP, face, red + t * 8, seg, S, v, c, d);
    if (store) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) line[mm] = d[mm];
    }
    if (store && !ok) raise_flag(s);
}

// A solve's grid as a raw buffer: a load names a per-lane byte offset
// (one VGPR, the same for every load of a thread) and a wave-uniform byte
// offset (an SGPR, formed by scalar arithmetic), so loads cost no vector
// address arithmetic.  The host keeps the grid under 4 GiB for this path.
struct GridBuf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ GridBuf(const double* base, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)bytes, 0x00020000))
    {
    }
    __device__ __forceinline__ double operator()(uint32_t voff, uint32_t soff) const
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
};

// Per-column constants of the explicit predictor at (i, plane k): the A1
// row pieces (affine in v), the A3 coefficient and weights, the A0 factor,
// and the Dirichlet increment of the column's Dirichlet nodes (as
// explicit_nodes forms them).
struct ExpColumn {
    double mlo, alo, mdi, adi, mup, aup, mex, ryk, kyk, rx, wa, wb, w2, gval, dt;
    double cy;  // c = f_t + kappa f + y of plane k (the r rows' shift)
    bool dir, yhd;
    int dx;  // outflow r face rows reach two nodes in (+2 at r_min, -2 at r_max)
    __device__ __forceinline__ ExpColumn(const SolveDesc& s, int i, int k, int step)
    {
        const int nr = s.nr, ny = s.ny;
        gcdouble* rt = gp(s.rt);
        // the plane's entries through the constant space: scalar loads where
        // k is the same on every lane
        kcdouble* yt = kp(s.yt);
        kcdouble* stn = kp(s.st) + kStepStride * step;
        const double c = stn[ST_PHI] + yt[YT_Y * ny + k];
        cy = c;
        const double e = rt[RT_P * nr + i] * c + rt[RT_Q * nr + i];
        mlo = rt[RT_MLO * nr + i] * e;
        alo = rt[RT_ALO * nr + i];
        mdi = rt[RT_MDI * nr + i] * e - rt[RT_RR * nr + i];
        adi = rt[RT_ADI * nr + i];
        mup = rt[RT_MUP * nr + i] * e;
        aup = rt[RT_AUP * nr + i];
        mex = rt[RT_MEX * nr + i] * e;
        ryk = rt[RT_Y * nr + i] * yt[YT_I * ny + k];
        kyk = yt[YT_K * ny + k];
        rx = rt[RT_X * nr + i];
        // the y weights of plane k's two neighbours (one-sided on the y
        // faces) and the Dirichlet increment: the entries are chosen first
        // and then loaded, every load unconditional, so that none of them
        // waits for the others (or for the grid loads before them)
        const int wra = k == 0 ? YT_W3 : (k == ny - 1 ? YT_W0 : YT_W1);
        const int wrb = k == 0 ? YT_W4 : (k == ny - 1 ? YT_W1 : YT_W3);
        wa = yt[wra * ny + k];
        wb = yt[wrb * ny + k];
        w2 = yt[YT_W2 * ny + k];
        yhd = s.y_hi_dir && k == ny - 1;
        gcdouble* gdn = gp(s.gd) + (size_t)step * (2 * ny + nr);
        const bool rlo = i == 0 && s.r_lo_dir, rhi = i == nr - 1 && s.r_hi_dir;
        dir = rlo || rhi || yhd;
        const double g = gdn[yhd ? 2 * ny + i : (rlo ? k : (rhi ? ny + k : 0))];
        gval = dir ? g : 0.0;
        dt = s.dt;
        dx = i == 0 ? 2 : (i == nr - 1 ? -2 : 0);
    }
};

// D0 at (i, j0 + m, k), m < J, j0 + m < nv, from the LDS window (wcol: this
// thread's column of the window, J + 2 rows at pitch nr holding v nodes
// j0 - 1 .. j0 + J; the neighbouring columns beside it; ulo, uhi: this
// column's v nodes j0 - 2 and j0 + J + 1, which only the v stencil of the
// thread's own column reads), the tile's
// v-table values in LDS (vtc: kVT rows of J, row r node m = vt[r][j0 + m];
// every lane reads the same address, a broadcast) and the y neighbours ya,
// yb (planes k + oa, k + ob): the arithmetic of explicit_nodes, so the same
// values.  Nothing here waits on a scalar load: the v-table values come
// from LDS, whose reads return in order.  Each window row is read once
// (its centre and its two neighbours) and kept in registers while the
// stencils of the next nodes need it; the scheduler is fenced every CH
// nodes, so that the registers hold a few rows, not the whole window.
template <int J>
__device__ __forceinline__ void window_nodes(const SolveDesc& s, const ldouble* wcol, const ldouble* vtc,
                                             const ExpColumn& q, const double (&ya)[J], const double (&yb)[J],
                                             double ulo, double uhi, int j0, double (&out)[J])
{
    const int nr = s.nr;
    constexpr int CH = 4;
    // window row w holds v node j0 - 1 + w (w = 0 .. J + 1), node m's centre
    // is row m + 1.  Rolled through registers: c0 .. c3 = u(i, j - 2 ..
    // j + 1), lm, rm and l0, r0 = u(i -+ 1) at j - 1 and j; node m reads row
    // m + 2's neighbours and row m + 3's centre (past the window: uhi).
    double c0 = ulo, c1 = wcol[0], c2 = wcol[nr], c3 = wcol[2 * nr];
    double lm = wcol[-1], rm = wcol[1], l0 = wcol[nr - 1], r0 = wcol[nr + 1];
#pragma unroll
    for (int m = 0; m < J; ++m) {
        if (m % CH == 0) __builtin_amdgcn_sched_barrier(0);
        // every node of the tile, also those past nv (in-bounds reads of the
        // clamped window rows; their results are never stored): no exit from
        // the unrolled loop
        const ldouble* w0 = wcol + (size_t)(m + 1) * nr;
        const double lwp = w0[nr - 1], rwp = w0[nr + 1];
        const double c4 = m + 3 > J + 1 ? uhi : wcol[(size_t)(m + 3) * nr];
        const double cw5[5] = {c0, c1, c2, c3, c4};  // u(i, j - 2 .. j + 2)
        // the outflow extra entry (dx = 0 inside, where it reads the node
        // itself under a zero weight): one read for every lane
        const double ux = w0[q.dx];
        const double v = vtc[VT_V * J + m];
        const double olo = q.mlo + q.alo * v, odi = q.mdi + q.adi * v, oup = q.mup + q.aup * v;
        const double a1 = olo * l0 + odi * cw5[2] + oup * r0 + q.mex * ux;
        const double a2 = vtc[VT_O0 * J + m] * cw5[0] + vtc[VT_O1 * J + m] * cw5[1] +
                          vtc[VT_O2 * J + m] * cw5[2] + vtc[VT_O3 * J + m] * cw5[3] +
                          vtc[VT_O4 * J + m] * cw5[4];
        const double by = q.ryk * v - q.kyk;
        const double a3 = by * (q.wa * ya[m] + q.w2 * cw5[2] + q.wb * yb[m]);
        const double cross = (rwp - rm) - (lwp - lm);
        const double a0 = q.rx * vtc[VT_X * J + m] * cross;
        double val = q.dt * (((a1 + a2) + a3) + a0);
        // formed on every lane and then selected: a branch around it for
        // the Dirichlet lanes would copy the live arrays at every join
        asm volatile("" : "+v"(val));
        out[m] = q.dir ? q.gval : val;
        c0 = c1; c1 = c2; c2 = c3; c3 = c4;
        lm = l0; rm = r0; l0 = lwp; r0 = rwp;
    }
}

// The window's guard doubles (two before it, two after its rows of P planes:
// finite, so that i -+ 1 and i -+ 2 stay inside; their weights are zero where
// they leave a row).
__device__ __forceinline__ void window_guards(ldouble* win, int P, int WR, int nr)
{
    const int t = (int)threadIdx.x;
    if (t < 2) {
        win[t - 2] = 0.0;
        win[(size_t)P * WR * nr + t] = 0.0;
    }
}

// Explicit predictor of the fused kernel from an LDS window.  Thread
// (i, plane kk) loads its column u(i, j0-2 .. j0+J+1) of plane k and its J y
// neighbours of planes k+oa, k+ob straight into registers, all at once (v
// rows past the faces clamp to the face row, scalar arithmetic); the columns'
// v nodes j0-1 .. j0+J go to the window win (per plane J + 2 rows of nr, row
// pitch nr); after a barrier every neighbour is an LDS read at a fixed offset
// from the thread's column (window_nodes).  out[m] receives D0 at (i, j0 + m, k) for
// j0 + m < nv.  UK: every wave lies inside one plane (nr a multiple of 64),
// so k, the y offsets and the y-table reads are wave-uniform.  stage() runs
// once the grid loads are issued (the caller's own staging into LDS).  Every
// thread of the workgroup calls it (one barrier inside).
template <int J, bool UK, class Stage>
__device__ __forceinline__ void explicit_window(const SolveDesc& s, ldouble* win, ldouble* vtc, ldouble* cpl, int P,
                                                int k0, int j0, int step, double (&out)[J], const Stage& stage)
{
    constexpr int WR = J + 4;   // the column's v nodes j0 - 2 .. j0 + J + 1
    constexpr int WL = J + 2;   // the window's rows: v nodes j0 - 1 .. j0 + J
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int t = (int)threadIdx.x;
    const int kk = t / nr;
    const int i = t - kk * nr;
    const bool act = kk < P && k0 + kk < ny;
    int k = min(k0 + kk, ny - 1);
    if (UK) k = __builtin_amdgcn_readfirstlane(k);
    const bool yhd = s.y_hi_dir && k == ny - 1;
    int oa = -1, ob = 1;
    if (k == 0) { oa = 1; ob = 2; }
    else if (k == ny - 1) { oa = -2; ob = -1; }
    if (yhd) { oa = 0; ob = 0; }
    const uint32_t sl = (uint32_t)nr * 8u;
    const uint32_t sy = (uint32_t)nv * sl;
    const GridBuf U(s.U, sy * (uint32_t)ny);
    // per-lane byte offsets: the column of plane k and of the two y neighbours
    const uint32_t vo = (uint32_t)(UK ? i : k * nr * nv + i) * 8u;
    const uint32_t po = UK ? (uint32_t)k * sy : 0u;
    const uint32_t voa = UK ? vo : vo + (uint32_t)(oa * (int)sy);
    const uint32_t vob = UK ? vo : vo + (uint32_t)(ob * (int)sy);
    const uint32_t poa = UK ? (uint32_t)(k + oa) * sy : 0u;
    const uint32_t pob = UK ? (uint32_t)(k + ob) * sy : 0u;
    auto row = [&](int j) { return (uint32_t)min(max(j, 0), nv - 1) * sl; };
    double cw[WR], ya[J], yb[J];
    if (act) {
#pragma unroll
        for (int m = 0; m < WR; ++m) cw[m] = U(vo, po + row(j0 - 2 + m));
#pragma unroll
        for (int m = 0; m < J; ++m) {
            ya[m] = U(voa, poa + row(j0 + m));
            yb[m] = U(vob, pob + row(j0 + m));
        }
    }
    // the tile's v-table values (kVT rows of J; v nodes past nv repeat the
    // last one, whose results are not stored) by vector loads, into LDS
    double vv = 0.0;
    if (t < kVT * J) {
        const int r = t / J;
        vv = gp(s.vt)[(size_t)r * nv + min(j0 + (t - r * J), nv - 1)];
    }
    const ExpColumn q(s, i, k, step);
    // the caller's staging (its loads queue behind the grid's and the
    // column constants')
    stage();
    ldouble* wcol = win + (size_t)kk * WL * nr + i;
    window_guards(win, P, WL, nr);
    if (t < kVT * J) vtc[t] = vv;
    if (i == 0 && kk < P) cpl[kk] = q.cy;  // each plane's c, for the r solve
    if (act) {
#pragma unroll
        for (int m = 0; m < WL; ++m) wcol[(size_t)m * nr] = cw[m + 1];
    }
    __syncthreads();
    if (!act) return;
    window_nodes<J>(s, wcol, vtc, q, ya, yb, cw[0], cw[WR - 1], j0, out);
}

// The r lines of a fused tile (P planes from k0 x kExrJ v nodes from j0,
// D0 in the tile: line (plane kk, node jj) at (kk kExrJ + jj) LP, segment g
// at g (ROWS + 1)) by the spike method, S = rs_S lanes per line, and D1 to
// memory.  The lanes of pass p reuse their own lines' part of the tile as the
// reduced-system scratch once every lane has read its rows (pass p's scratch
// is its first 8 kBlock doubles, inside its kBlock / S lines; the tile is
// sized to whole passes).  Every thread calls it, after a barrier that
// follows the tile's writes.
template <int ROWS, bool FOLD = false>
__device__ __forceinline__ void solve_tile(const SolveDesc& s, ldouble* tile, const ldouble* tab, const ldouble* face,
                                           const ldouble* vtc, const ldouble* cpl, int P, int k0, int j0, int step)
{
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int S = s.rs_S;
    const int log2S = s.rs_log2S;
    constexpr int SP = ROWS + 1;
    constexpr int TP = kRF * ROWS + 1;
    const int LP = S * SP;
    const int t = (int)threadIdx.x;
    const int L = P * kExrJ;
    for (int base = 0; base < L * S; base += kBlock) {  // uniform trip count
        const int u = base + t;
        const int ln = u >> log2S;
        const int seg = u & (S - 1);
        const int kk = ln / kExrJ;
        const int jj = ln - kk * kExrJ;
        const int k = min(k0 + kk, ny - 1);
        const int j = min(j0 + jj, nv - 1);
        const bool active = ln < L && k0 + kk < ny && j0 + jj < nv;
        double d[ROWS];
        const ldouble* src = tile + (size_t)min(ln, L - 1) * LP + seg * SP;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) d[mm] = src[mm];
        __syncthreads();  // every lane of the pass has read its rows: the scratch may overwrite them
        // Dirichlet y_max lines keep D0 (wave-uniform: a wave's lines share the plane)
        const bool ydir = s.y_hi_dir && k == ny - 1;
        bool ok = true;
        if (!ydir) {
            // the line's v and c from the explicit phase's LDS copies (the
            // v-table cache, one c per plane): no memory round trip here
            const double v = vtc[VT_V * kExrJ + jj];
            const double c = cpl[min(kk, P - 1)];
            ok = spike_r_lane<ROWS>(s, tab + seg * TP, face, tile + (size_t)base * SP + t * 8, seg, S, v, c, d);
        }
        if constexpr (FOLD) {
            // D1 back into the lane's own rows of the tile (no reduced-system
            // scratch in LDS for S <= 16, so no other lane reads them), for
            // the tile's v sweep
            ldouble* dst = tile + (size_t)min(ln, L - 1) * LP + seg * SP;
            if (active) {
#pragma unroll
                for (int mm = 0; mm < ROWS; ++mm) dst[mm] = d[mm];
            }
            if (active && !ok) raise_flag(s);
        } else if (active) {
            gdouble* line = gp(s.D) + ((size_t)k * nv + j) * nr + (size_t)seg * ROWS;
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) line[mm] = d[mm];
            if (!ok) raise_flag(s);
        }
        // the next pass reads only its own lines' rows, which this pass's
        // scratch does not reach: no barrier needed here
    }
}

// The v sweep folded into the fused kernel (Douglas, the v lines cut into
// segments of kExrJ = 16 rows, one per tile): the segmented solve of k_vs
// (hjm_internal.h, VG_*) run on the tile's segment from zero in both
// directions, by thread (i, plane), on D1 read back from the tile.  It
// stores the segment's local solution x0 (the face rows' own D1 at j = 0
// and nv - 1, which k_vfix recovers), the forward end value d'_end and the
// backward first value x0_first; k_vfix composes the segments of each
// (i, k) line and k_yc adds K_j d'_in + H_j x_in as it loads D2, K = the
// backward sweep of G.  Lines on Dirichlet faces keep D1 (end values 0).
template <int ROWS>
__device__ __forceinline__ void fold_v_tile(const SolveDesc& s, const ldouble* tile, int P, int k0, int j0)
{
    constexpr int J = kExrJ;
    constexpr int SP = ROWS + 1;
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int LP = s.rs_S * SP;  // the tile's line pitch
    const int t = (int)threadIdx.x;
    const int kk = t / nr;
    const int i = t - kk * nr;
    const int k = k0 + kk;
    if (kk >= P || k >= ny) return;
    const int g = i / ROWS;
    const ldouble* col = tile + (size_t)kk * J * LP + g * SP + (i - g * ROWS);
    const int Sv = s.vs_S;
    const int sv = j0 / J;
    const bool first = sv == 0, last = sv == Sv - 1;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir) || (k == ny - 1 && s.y_hi_dir);
    kcdouble* vg = kp(s.vg) + j0;
    kcdouble* fs = kp(s.vf) + kVF * nv;
    double d[J];
#pragma unroll
    for (int m = 0; m < J; ++m) d[m] = col[(size_t)m * LP];
    double lend = 0.0, x0f = 0.0;
    if (!line_dir) {
        const double d0 = d[0], dl = d[J - 1];
        if (first) d[1] = d[1] - fs[VS_F1] * d0;
        if (last) d[J - 2] = d[J - 2] - fs[VS_F2] * dl;
        double l = 0.0;
#pragma unroll
        for (int m = 0; m < J; ++m) {
            l = vg[VG_INV * nv + m] * d[m] + vg[VG_AL * nv + m] * l;
            d[m] = l;
        }
        lend = d[J - 1];
        double x = 0.0;
#pragma unroll
        for (int m = J - 1; m >= 0; --m) {
            x = d[m] - vg[VG_CP * nv + m] * x;
            d[m] = x;
        }
        x0f = d[0];
        if (first) d[0] = d0;
        if (last) d[J - 1] = dl;
    }
    // non-temporal: the y sweep reads D1 back two launches later, after
    // the hand-over kernel, so streaming it past the caches keeps them for
    // the window's halo reads (measured faster for both kernels)
    gdouble* line = gp(s.D) + ((size_t)k * nv + j0) * nr + i;
#pragma unroll
    for (int m = 0; m < J; ++m) __builtin_nontemporal_store(d[m], &line[(size_t)m * nr]);
    const size_t A = (size_t)nr * ny * Sv;
    const size_t e = ((size_t)k * Sv + sv) * nr + i;
    gdouble* ends = gp(s.yinv);
    ends[e] = lend;
    ends[A + e] = x0f;
}

// Explicit predictor (or, STAGE2, the corrected start of the Craig-Sneyd
// family) and r sweep in one kernel (nr <= 256, nr = S * ROWS as for k_rs,
// ROWS >= 8): the workgroup computes D0 on kExrJ consecutive v nodes of
// exr_P = exr_planes(nr, ROWS) whole y planes (thread = (i, plane)) into an LDS tile,
// then solves the tile's exr_P * kExrJ r lines with the spike method, S lanes
// per line, and writes D1.  D0 never goes to memory: 16 bytes per point less
// than the split pair.  Tile layout: line (plane kk, node jj) at
// (kk kExrJ + jj) S (ROWS + 1), its segment g at g (ROWS + 1) (the pad spreads
// a wave's segments over the banks).  The lanes of pass p reuse their own
// lines' part of the tile as the reduced-system scratch once every lane has
// read its rows (pass p's scratch is its first 8 kBlock doubles, inside its
// kBlock / S lines; the tile is sized to whole passes).  Three waves per SIMD
// (at most 168 VGPRs, no spills) measured faster than two.
// v nodes per explicit chunk of k_exr: 8; 4 for the corrected start, which
// holds the stencil of U while it loads the windows of D3
template <bool STAGE2>
constexpr int kExrChunk = STAGE2 ? 4 : 8;

template <int ROWS, bool STAGE2, bool WIN = false, bool FOLD = false>
__global__ __launch_bounds__(kBlock, 3) void k_exr(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks,
                                                int step)
{
    extern __shared__ double lds_raw[];
    ldouble* lds = (ldouble*)lds_raw;
    const int bi = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int2 tk = tasks ? tasks[bi] : make_int2(0, bi);
    const SolveDesc& s = descs[tk.x];
    if (step >= s.n_steps) return;  // whole workgroup: uniform
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int P = s.exr_P;
    const int S = s.rs_S;
    constexpr int SP = ROWS + 1;
    const int LP = S * SP;
    const int nvb = (nv + kExrJ - 1) / kExrJ;
    const int kb = tk.y / nvb;
    const int jb = tk.y - kb * nvb;
    const int k0 = kb * P;
    const int j0 = __builtin_amdgcn_readfirstlane(jb * kExrJ);
    const int t = threadIdx.x;
    ldouble* tile = lds;
    ldouble* tab = lds + s.exr_tab;  // after the tile, rounded up to whole passes
    // after the row table and the window variant's v-table cache
    ldouble* face = tab + (size_t)S * (kRF * ROWS + 1) + (size_t)kVT * kExrJ;
    // the row table and the face rows into LDS first (staged after the grid
    // loads, their waits held up the explicit phase: measured slower)
    auto stage_table = [&]() {};
    const double fv = load_face(s);  // issued with the row table's loads
    stage_rf<ROWS, (kRF * kExrMaxNr + kBlock - 1) / kBlock>(s, tab);
    store_face(face, fv);
    // the v-table cache after the row table, the planes' c after the face rows
    ldouble* vtc = tab + (size_t)S * (kRF * ROWS + 1);
    ldouble* cpl = face + kFace;
    if constexpr (WIN && !STAGE2) {
        // explicit phase from the LDS window (it shares the LDS of the tile,
        // which is written once every thread has finished reading it)
        double out[kExrJ];
        if (nr % 64 == 0)
            explicit_window<kExrJ, true>(s, tile + 2, vtc, cpl, P, k0, j0, step, out, stage_table);
        else
            explicit_window<kExrJ, false>(s, tile + 2, vtc, cpl, P, k0, j0, step, out, stage_table);
        const int kk = t / nr;
        const int i = t - kk * nr;
        __syncthreads();
        if (kk < P && k0 + kk < ny) {
            const int g = i / ROWS;
            ldouble* dst = tile + (size_t)kk * kExrJ * LP + g * SP + (i - g * ROWS);
#pragma unroll
            for (int m = 0; m < kExrJ; ++m)
                if (j0 + m < nv) dst[(size_t)m * LP] = out[m];
        }
    } else {
        // explicit phase: thread (i, plane kk); planes past ny do nothing
        const int kk = t / nr;
        const int i = t - kk * nr;
        const int k = k0 + kk;
        if (kk < P && k < ny) {
            const int g = i / ROWS;
            ldouble* dst = tile + (size_t)kk * kExrJ * LP + g * SP + (i - g * ROWS);
#pragma unroll 1
            for (int jc = 0; jc < kExrJ; jc += kExrChunk<STAGE2>) {
                auto put = [&](int m, double x) { dst[(size_t)(jc + m) * LP] = x; };
                if constexpr (STAGE2)
                    corrected_start<kExrChunk<STAGE2>, true>(s, i, k, j0 + jc, step, put);
                else
                    explicit_nodes<kExrChunk<STAGE2>, true>(s, i, k, j0 + jc, step, put);
            }
        }
    }
    __syncthreads();
    if constexpr (WIN && !STAGE2 && FOLD) {
        // D1 stays in the tile; after every line is solved, the tile's v sweep
        solve_tile<ROWS, true>(s, tile, tab, face, vtc, cpl, P, k0, j0, step);
        __syncthreads();
        fold_v_tile<ROWS>(s, tile, P, k0, j0);
    } else if constexpr (WIN && !STAGE2) {
        solve_tile<ROWS>(s, tile, tab, face, vtc, cpl, P, k0, j0, step);
    } else {
        // the same passes as solve_tile, written out here: inlined as one
        // function the per-lane-load variants keep fewer registers spilled
        const int log2S = s.rs_log2S;
        constexpr int TP = kRF * ROWS + 1;
        const double phi = gp(s.st)[kStepStride * step + ST_PHI];
        const int L = P * kExrJ;
        for (int base = 0; base < L * S; base += kBlock) {  // uniform trip count
            const int u = base + t;
            const int ln = u >> log2S;
            const int seg = u & (S - 1);
            const int kk = ln / kExrJ;
            const int jj = ln - kk * kExrJ;
            const int k = min(k0 + kk, ny - 1);
            const int j = min(j0 + jj, nv - 1);
            const bool active = ln < L && k0 + kk < ny && j0 + jj < nv;
            double d[ROWS];
            const ldouble* src = tile + (size_t)min(ln, L - 1) * LP + seg * SP;
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) d[mm] = src[mm];
            __syncthreads();  // every lane of the pass has read its rows: the scratch may overwrite them
            // Dirichlet y_max lines keep D0 (wave-uniform: a wave's lines share the plane)
            const bool ydir = s.y_hi_dir && k == ny - 1;
            bool ok = true;
            if (!ydir) {
                const double v = gp(s.vt)[VT_V * nv + j];
                const double c = phi + gp(s.yt)[YT_Y * ny + k];
                ok = spike_r_lane<ROWS>(s, tab + seg * TP, face, tile + (size_t)base * SP + t * 8, seg, S, v, c, d);
            }
            if (active) {
                gdouble* line = gp(s.D) + ((size_t)k * nv + j) * nr + (size_t)seg * ROWS;
#pragma unroll
                for (int mm = 0; mm < ROWS; ++mm) line[mm] = d[mm];
                if (!ok) raise_flag(s);
            }
        }
    }
}

// v sweep, segmented: the v-line matrix is the same on every line, so its
// factors and the segment products G, H are host constants (see VG_* in
// hjm_internal.h).  Workgroup = vs_S waves; wave w holds rows
// [w ROWS, (w+1) ROWS) of 64 consecutive lines (i, k) (lanes = consecutive i:
// every load and store is one contiguous row segment).  Each segment sweeps
// forward and backward from zero; the segment-end values cross the workgroup
// through LDS once per direction.
template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_vs(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks)
{
    extern __shared__ double lds_raw[];
    ldouble* lds = (ldouble*)lds_raw;
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int S = s.vs_S;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int seg = __builtin_amdgcn_readfirstlane(t >> 6);
    const bool in_seg = seg < S;
    const int nlines = nr * ny;
    const int q_raw = tk.y * 64 + lane;
    const bool active = q_raw < nlines;
    const int q = active ? q_raw : nlines - 1;
    const int k = q / nr;
    const int i = q - k * nr;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir) || (k == ny - 1 && s.y_hi_dir);
    const int sg = in_seg ? seg : 0;
    gdouble* base = gp(s.D) + ((size_t)k * nv + (size_t)sg * ROWS) * nr + i;
    gcdouble* vg = gp(s.vg) + sg * ROWS;
    gcdouble* fs = gp(s.vf) + kVF * nv;
    const bool first = sg == 0;
    const bool last = sg == S - 1;
    double d[ROWS];
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) d[mm] = base[(size_t)mm * nr];
    const double d0 = d[0], dl = d[ROWS - 1];
    if (first) d[1] = d[1] - fs[VS_F1] * d0;
    if (last) d[ROWS - 2] = d[ROWS - 2] - fs[VS_F2] * dl;
    double l = 0.0;
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) {
        l = vg[VG_INV * nv + mm] * d[mm] + vg[VG_AL * nv + mm] * l;
        d[mm] = l;
    }
    ldouble* lend = lds;
    ldouble* bfirst = lds + (size_t)4 * 64;
    if (in_seg) lend[seg * 64 + lane] = d[ROWS - 1];
    __syncthreads();
    double din = 0.0;
    for (int qq = 0; qq < sg; ++qq) din = lend[qq * 64 + lane] + gp(s.vg)[VG_G * nv + qq * ROWS + ROWS - 1] * din;
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) d[mm] = d[mm] + vg[VG_G * nv + mm] * din;
    double x = 0.0;
#pragma unroll
    for (int mm = ROWS - 1; mm >= 0; --mm) {
        x = d[mm] - vg[VG_CP * nv + mm] * x;
        d[mm] = x;
    }
    if (in_seg) bfirst[seg * 64 + lane] = d[0];
    __syncthreads();
    double xin = 0.0;
    for (int qq = S - 1; qq > sg; --qq) xin = bfirst[qq * 64 + lane] + gp(s.vg)[VG_H * nv + qq * ROWS] * xin;
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) d[mm] = d[mm] + vg[VG_H * nv + mm] * xin;
    if (first) d[0] = (d0 - fs[VS_C0] * d[1] - fs[VS_E0] * d[2]) / fs[VS_B0];
    if (last) d[ROWS - 1] = (dl - fs[VS_EL] * d[ROWS - 3] - fs[VS_AL] * d[ROWS - 2]) / fs[VS_BL];
    if (in_seg && active && !line_dir) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) base[(size_t)mm * nr] = d[mm];
    }
}

// D2 of a folded v sweep: the segment's local solution plus the hand-over
// terms (one expression, so that k_vfix and k_yc form the same value).
__device__ __forceinline__ double fold_v_value(double x0, double K, double din, double H, double xin)
{
    return fma(H, xin, fma(K, din, x0));
}

// The segment hand-over of the folded v sweep (fold_v_tile), one thread per
// v line (i, k), SV = vs_S segments (every solve of the launch has SV): the
// recurrences of k_vs across segments, d'_in(s) = d'_end(s - 1) + G_last(s -
// 1) d'_in(s - 1) from d'_in(0) = 0, and x_in(s) = x_first(s + 1) +
// H_first(s + 1) x_in(s + 1) from x_in(SV - 1) = 0, where the first value of
// segment s + 1's backward sweep is x0_first + K_first d'_in; then rows 0 and
// nv - 1 (outflow faces) from their own rows and the final values of rows 1,
// 2 and nv - 3, nv - 2, as k_vs forms them.  The hand-over values go to the
// solve's y-pivot array, which the folded solve does not otherwise use:
// [d'_end | x0_first | d'_in | x_in], each [k][segment][i].  Lines on
// Dirichlet faces keep D1 (zero hand-over).  Every load is issued before the
// recurrences (one memory round trip, not one per segment).
template <int SV>
__global__ __launch_bounds__(kBlock) void k_vfix(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks)
{
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int q = tk.y * kBlock + (int)threadIdx.x;
    if (q >= nr * ny) return;
    const int k = q / nr;
    const int i = q - k * nr;
    constexpr int J = kExrJ;
    const size_t A = (size_t)nr * ny * SV;
    const size_t e0 = (size_t)k * SV * nr + i;
    gdouble* ends = gp(s.yinv);
    gdouble* D = gp(s.D) + (size_t)k * nv * nr + i;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir) || (k == ny - 1 && s.y_hi_dir);
    gcdouble* vg = gp(s.vg);
    // the end values of segments 0 .. SV - 2 and the first values of
    // segments 1 .. SV - 1, and the local solutions of the rows the face rows
    // read
    double lend[SV], x0f[SV];
#pragma unroll
    for (int sv = 0; sv < SV; ++sv) {
        lend[sv] = sv < SV - 1 ? ends[e0 + (size_t)sv * nr] : 0.0;
        x0f[sv] = sv > 0 ? ends[A + e0 + (size_t)sv * nr] : 0.0;
    }
    const double u0 = D[0], u1 = D[nr], u2 = D[(size_t)2 * nr];
    const double ua = D[(size_t)(nv - 3) * nr], ub = D[(size_t)(nv - 2) * nr], ul = D[(size_t)(nv - 1) * nr];
    double din[SV], xin[SV];
    din[0] = 0.0;
#pragma unroll
    for (int sv = 1; sv < SV; ++sv) din[sv] = lend[sv - 1] + vg[VG_G * nv + sv * J - 1] * din[sv - 1];
    double x = 0.0;
#pragma unroll
    for (int sv = SV - 1; sv >= 0; --sv) {
        xin[sv] = x;
        if (sv > 0) {
            const double bf = fma(vg[VG_K * nv + sv * J], din[sv], x0f[sv]);
            x = bf + vg[VG_H * nv + sv * J] * x;
        }
    }
#pragma unroll
    for (int sv = 0; sv < SV; ++sv) {
        ends[2 * A + e0 + (size_t)sv * nr] = line_dir ? 0.0 : din[sv];
        ends[3 * A + e0 + (size_t)sv * nr] = line_dir ? 0.0 : xin[sv];
    }
    if (line_dir) return;
    gcdouble* fs = gp(s.vf) + kVF * nv;
    auto fin = [&](double u, int j, int sv) { return fold_v_value(u, vg[VG_K * nv + j], din[sv], vg[VG_H * nv + j], xin[sv]); };
    const double x1 = fin(u1, 1, 0), x2 = fin(u2, 2, 0);
    const double xa = fin(ua, nv - 3, SV - 1), xb = fin(ub, nv - 2, SV - 1);
    D[0] = (u0 - fs[VS_C0] * x1 - fs[VS_E0] * x2) / fs[VS_B0];
    D[(size_t)(nv - 1) * nr] = (ul - fs[VS_EL] * xa - fs[VS_AL] * xb) / fs[VS_BL];
}

// Reciprocal pivots 1 / den_k of every y line (i, j) of (I - theta dt A3),
// which do not change from step to step: the Thomas forward recurrence
// den_k = B_k - A_k c'_{k-1}, c'_k = C_k / den_k in row order (the quotient
// taken as C_k times the reciprocal, as the sweep does), with the outflow row
// 0 folded into row 1 and the last row into row n-2 exactly as in the
// per-step solve; rows 0 and n-1 are identity rows (1).  One thread per line,
// written once per solve; a non-positive pivot raises the health flag.
__global__ __launch_bounds__(kBlock) void k_ypiv(const SolveDesc* __restrict__ descs)
{
    const SolveDesc& s = descs[blockIdx.y];
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    if (s.yc_S == 0 || s.ypiv_skip) return;
    const int q = blockIdx.x * kBlock + threadIdx.x;  // q = j nr + i
    if (q >= nr * nv) return;
    const int j = q / nr;
    const int i = q - j * nr;
    const size_t sy = (size_t)nr * nv;
    gdouble* yinv = gp(s.yinv) + q;
    RowY row;
    row.yt = gp(s.yt);
    row.ny = ny;
    row.qv = gp(s.rt)[RT_Y * nr + i] * gp(s.vt)[VT_V * nv + j];
    double A0, B0, C0, E0, A1, B1, C1, E1, Al, Bl, Cl, El, A2, B2, C2, E2;
    row(0, A0, B0, C0, E0);
    row(1, A1, B1, C1, E1);
    row(ny - 1, Al, Bl, Cl, El);
    row(ny - 2, A2, B2, C2, E2);
    const double f1 = A1 / B0, f2 = C2 / Bl;
    bool ok = B0 > 0.0 && Bl > 0.0;
    double cprev = 0.0;
    yinv[0] = 1.0;
    for (int kk = 1; kk < ny - 1; ++kk) {
        double A, B, C, E;
        row(kk, A, B, C, E);
        if (kk == 1) { A = 0.0; B = B1 - f1 * C0; C = C1 - f1 * E0; }
        if (kk == ny - 2) { A = A2 - f2 * El; B = B2 - f2 * Al; C = 0.0; }
        const double den = B - A * cprev;
        ok = ok && den > 0.0;
        const double inv = rcp_nr(den);
        cprev = C * inv;
        yinv[(size_t)kk * sy] = inv;
    }
    yinv[(size_t)(ny - 1) * sy] = 1.0;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir);
    if (!ok && !line_dir) raise_flag(s);
}

// Exact rescaling by a power of two (no rounding): the minors recurrence is
// homogeneous, so a common factor of its two carried values changes no ratio.
__device__ __forceinline__ int pow2_exponent(double x)
{
    return __builtin_amdgcn_frexp_exp(x);
}

// y sweep + update: Thomas in row order, segments of ROWS rows chained
// through LDS (segment s runs once segment s-1 has handed over d' of its last
// row); the only serial work per row is one FMA forward and one backward.
// Then U^{n+1} = U^n + D3.  Workgroup = yc_S waves; wave w holds rows
// [w ROWS, (w+1) ROWS) of 64 consecutive lines (i, j), so row reads are
// contiguous and the y-table reads are wave-uniform.
//
// The reciprocal pivots 1 / den_k either come from the array k_ypiv wrote
// (MINORS false) or are formed here each step (MINORS true), which saves
// reading one grid-sized array per step.  Thomas's pivots are ratios of
// consecutive leading minors of the line matrix, den_k = th_k / th_{k-1}, and
// the minors obey the linear recurrence th_k = B_k th_{k-1} - A_k C_{k-1}
// th_{k-2} (th_{-1} = 1, th_{-2} = 0): no division on its chain.  Every
// segment first carries the basis (1, 0), (0, 1) of (th_{b-1}, th_{b-2})
// through its rows (a 2x2 transfer, in parallel over segments); segment s then
// composes the transfers of segments 0 .. s-1 into its own start values and
// replays its rows, 1 / den_k = th_{k-1} / th_k off the chain.  On these
// lines the off-diagonal product A_k C_{k-1} is negative except where the y
// drift changes sign (and small there), so the minors are sums of positive
// terms: as accurate as the pivots of the division recurrence.  Both carried
// values are rescaled by a power of two every 8 rows (exact), so the minors
// never overflow.
template <int ROWS, int MODE, bool MINORS, bool FOLD = false>
__global__ __launch_bounds__(64 * yc_max_segments(ROWS)) void k_yc(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks)
{
    extern __shared__ double lds_raw[];
    ldouble* lds = (ldouble*)lds_raw;
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int S = s.yc_S;
    const int t = threadIdx.x;
    const int l = t & 63;
    const int seg = __builtin_amdgcn_readfirstlane(t >> 6);
    const int q = tk.y * 64 + l;  // line (i, j), q = j nr + i
    const bool active = seg < S && q < nr * nv;
    const int qc = active ? q : 0;
    const int j = qc / nr;
    const int i = qc - j * nr;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir);
    const bool work = active && !line_dir;
    const int sg = seg < S ? seg : 0;
    const size_t sy = (size_t)nr * nv;
    const size_t off = (size_t)qc + (size_t)sg * ROWS * sy;
    gdouble* D = gp(s.D);
    gdouble* U = gp(s.U);
    kcdouble* yt = kp(s.yt);
    const bool first = sg == 0;
    const bool last = sg == S - 1;
    // inactive lanes read line 0 of segment 0 (in bounds; never stored), so
    // the loads need no branches.  C inv waits in LDS and U^n is read only at
    // the end, so that the chains hold just d and -A inv in registers and two
    // workgroups fit on a compute unit.
    double d[ROWS], al[ROWS], iv[ROWS];
    // D2 is read once (non-temporal: the next step rewrites it), which
    // leaves the caches to the hand-over values the segment's rows share
#pragma unroll
    for (int mm = 0; mm < ROWS; ++mm) {
        d[mm] = __builtin_nontemporal_load(&D[off + (size_t)mm * sy]);
        if constexpr (!MINORS) iv[mm] = gp(s.yinv)[off + (size_t)mm * sy];
    }
    if constexpr (FOLD) {
        // the folded v sweep's hand-over terms (k_vfix), as D2 is loaded
        const int Sv = s.vs_S;
        const int sv = j / kExrJ;
        const size_t A = (size_t)nr * ny * Sv;
        gcdouble* ho = gp(s.yinv) + 2 * A + (size_t)sv * nr + i;
        const double Kj = gp(s.vg)[VG_K * nv + j], Hj = gp(s.vg)[VG_H * nv + j];
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            const size_t e = (size_t)(sg * ROWS + mm) * Sv * nr;
            d[mm] = fold_v_value(d[mm], Kj, ho[e], Hj, ho[A + e]);
        }
    }
    // C inv goes to LDS (it is needed only by the backward chain), [row][lane]
    ldouble* cpl = lds + 128 + (size_t)sg * ROWS * 64 + l;
    const double qv = gp(s.rt)[RT_Y * nr + i] * gp(s.vt)[VT_V * nv + j];
    // the row entries from the tables; yq and the table pointer are passed
    // in, so that a pass that recomputes them (MINORS: the transfer, then
    // the replay) can hide the repeat from the compiler, which would
    // otherwise keep every row's entries live between the passes
    auto row_of = [&](kcdouble* ytab, double yq, int kk, double& A, double& B, double& C, double& E) {
        const double a = ytab[YT_T1 * ny + kk] * yq + ytab[YT_T2 * ny + kk];
        A = ytab[YT_MA * ny + kk] * a;
        B = 1.0 + ytab[YT_MB * ny + kk] * a;
        C = ytab[YT_MC * ny + kk] * a;
        E = ytab[YT_ME * ny + kk] * a;
    };
    auto row = [&](int kk, double& A, double& B, double& C, double& E) { row_of(yt, qv, kk, A, B, C, E); };
    double d0 = 0.0, B0 = 1.0, C0 = 0.0, E0 = 0.0, dl = 0.0, Al = 0.0, Bl = 1.0, El = 0.0;
    double c1m = 0.0, a2m = 0.0, b1m = 1.0, b2m = 1.0;
    if (first) {
        double A0, A1, B1, C1, E1;
        row(0, A0, B0, C0, E0);
        row(1, A1, B1, C1, E1);
        const double f = A1 / B0;
        c1m = C1 - f * E0;
        b1m = B1 - f * C0;
        d0 = d[0];
        if (work) d[1] = d[1] - f * d0;
    }
    if (last) {
        double Cl, A2, B2, C2, E2;
        row(ny - 1, Al, Bl, Cl, El);
        row(ny - 2, A2, B2, C2, E2);
        const double f = C2 / Bl;
        a2m = A2 - f * El;
        b2m = B2 - f * Al;
        dl = d[ROWS - 1];
        if (work) d[ROWS - 2] = d[ROWS - 2] - f * dl;
    }
    // row mm of the segment with the face rows folded in: rows 0 and n-1 are
    // identity rows, row 1 lost its A and row n-2 its C
    auto frow_of = [&](kcdouble* ytab, double yq, int mm, double& A, double& B, double& C) {
        double E;
        row_of(ytab, yq, sg * ROWS + mm, A, B, C, E);
        if (mm == 0) { A = first ? 0.0 : A; B = first ? 1.0 : B; C = first ? 0.0 : C; }
        if (mm == 1) { A = first ? 0.0 : A; B = first ? b1m : B; C = first ? c1m : C; }
        if (mm == ROWS - 2) { A = last ? a2m : A; B = last ? b2m : B; C = last ? 0.0 : C; }
        if (mm == ROWS - 1) { A = last ? 0.0 : A; B = last ? 1.0 : B; C = last ? 0.0 : C; }
    };
    auto frow = [&](int mm, double& A, double& B, double& C) { frow_of(yt, qv, mm, A, B, C); };
    bool ok = true;
    if constexpr (MINORS) {
        // C of the row before the segment (no fold reaches it: ROWS >= 8)
        double cb = 0.0;
        if (!first) {
            double A, B, E;
            row(sg * ROWS - 1, A, B, cb, E);
        }
        // the segment's transfer: (th_{b+R-1}, th_{b+R-2}) = u th_{b-1} + w th_{b-2}
        double u0 = 1.0, u1 = 0.0, w0 = 0.0, w1 = 1.0, cprev = cb;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            double A, B, C;
            frow(mm, A, B, C);
            const double P = A * cprev;
            cprev = C;
            const double nu = B * u0 - P * u1;
            const double nw = B * w0 - P * w1;
            u1 = u0; u0 = nu;
            w1 = w0; w0 = nw;
            if (mm % 8 == 7) {
                const int e = -pow2_exponent(fabs(u0) + fabs(w0));
                u0 = __builtin_ldexp(u0, e); u1 = __builtin_ldexp(u1, e);
                w0 = __builtin_ldexp(w0, e); w1 = __builtin_ldexp(w1, e);
            }
        }
        // start values of segment sg: the transfers of the segments before it
        // applied to (th_{-1}, th_{-2}) = (1, 0); the transfers sit where the
        // C inv rows go, read by every later segment before any is written
        double t1 = 1.0, t2 = 0.0;
        if (S > 1) {
            ldouble* tr = lds + 128 + l;
            if (seg < S - 1) {
                tr[(seg * 4 + 0) * 64] = u0; tr[(seg * 4 + 1) * 64] = u1;
                tr[(seg * 4 + 2) * 64] = w0; tr[(seg * 4 + 3) * 64] = w1;
            }
            __syncthreads();
            for (int qq = 0; qq < sg; ++qq) {
                const double x = tr[(qq * 4 + 0) * 64] * t1 + tr[(qq * 4 + 2) * 64] * t2;
                const double y = tr[(qq * 4 + 1) * 64] * t1 + tr[(qq * 4 + 3) * 64] * t2;
                const int e = -pow2_exponent(x);
                t1 = __builtin_ldexp(x, e);
                t2 = __builtin_ldexp(y, e);
            }
            __syncthreads();
        }
        ok = t1 > 0.0;
        if (first) ok = ok && B0 > 0.0;
        if (last) ok = ok && Bl > 0.0;
        // replay, 1 / den_k = th_{k-1} / th_k (identity rows: exactly 1), and
        // the sweep's coefficients from it at once; the rows' entries are
        // formed again (cheaper than holding them since the transfer)
        double qv2 = qv;
        kcdouble* yt2 = yt;
        asm volatile("" : "+v"(qv2), "+s"(yt2));
        cprev = cb;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            // rows in groups of 4: the scheduler would otherwise run the whole
            // minors chain ahead and hold every row's values for the divisions
            if (mm % 4 == 0) __builtin_amdgcn_sched_barrier(0);
            double A, B, C;
            frow_of(yt2, qv2, mm, A, B, C);
            const double P = A * cprev;
            cprev = C;
            const double t0 = B * t1 - P * t2;
            ok = ok && t0 > 0.0;
            const bool ident = (mm == 0 && first) || (mm == ROWS - 1 && last);
            const double inv = ident ? 1.0 : t1 * rcp_nr(t0);
            t2 = t1;
            t1 = t0;
            if (mm % 8 == 7) {
                const int e = -pow2_exponent(t1);
                t1 = __builtin_ldexp(t1, e);
                t2 = __builtin_ldexp(t2, e);
            }
            al[mm] = work ? -A * inv : 0.0;
            d[mm] = work ? d[mm] * inv : d[mm];
            // formed here, not sunk into the sweep's branches (which would keep
            // every row's A and inv live until then)
            asm volatile("" : "+v"(al[mm]), "+v"(d[mm]));
            if (seg < S) cpl[mm * 64] = C * inv;  // waves past S (batches) share segment 0's rows: no write
        }
        if (!ok && work) raise_flag(s);
    } else {
        // with inv_k = 1 / den_k the recurrences are d'_k = inv_k d_k +
        // (-A_k inv_k) d'_{k-1} and x_k = d'_k - (C_k inv_k) x_{k+1}; rows 0
        // and n-1 are identity rows (lines on a Dirichlet r face keep D)
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm) {
            double A, B, C;
            frow(mm, A, B, C);
            const double inv = iv[mm];
            if (seg < S) cpl[mm * 64] = C * inv;  // waves past S (batches) share segment 0's rows: no write
            al[mm] = work ? -A * inv : 0.0;
            d[mm] = work ? d[mm] * inv : d[mm];
        }
    }
    ldouble* xch = lds + 2 * l;
    for (int stage = 0; stage < S; ++stage) {
        if (work && seg == stage) {
            double dp = stage > 0 ? xch[0] : 0.0;
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) {
                dp = d[mm] + al[mm] * dp;
                d[mm] = dp;
            }
            xch[0] = dp;
        }
        if (S > 1) __syncthreads();
    }
    for (int stage = S - 1; stage >= 0; --stage) {
        if (work && seg == stage) {
            double x = stage < S - 1 ? xch[1] : 0.0;
#pragma unroll
            for (int mm = ROWS - 1; mm >= 0; --mm) {
                x = d[mm] - cpl[mm * 64] * x;
                d[mm] = x;
            }
            xch[1] = x;
            if (first) d[0] = (d0 - C0 * d[1] - E0 * d[2]) / B0;
            if (last) d[ROWS - 1] = (dl - El * d[ROWS - 3] - Al * d[ROWS - 2]) / Bl;
        }
        if (S > 1) __syncthreads();
    }
    if (active) {
        if constexpr (MODE == 1) {
            // first sequence of the Craig-Sneyd family: D3 stays in D, U unchanged
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) D[off + (size_t)mm * sy] = d[mm];
        } else if constexpr (MODE == 3) {
            // an intermediate Huang subiteration: X_{m+1} = X_m + E3, U unchanged
            gdouble* X = gp(s.D3);
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) X[off + (size_t)mm * sy] = X[off + (size_t)mm * sy] + d[mm];
        } else {
            double u[ROWS];
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) u[mm] = U[off + (size_t)mm * sy];
            if constexpr (MODE == 2) {
                // Hundsdorfer-Verwer: the correction is relative to U + D3
                gcdouble* D3 = gp(s.D3);
#pragma unroll
                for (int mm = 0; mm < ROWS; ++mm) u[mm] += D3[off + (size_t)mm * sy];
            }
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) U[off + (size_t)mm * sy] = u[mm] + d[mm];
        }
    }
}


// Dirichlet increments g(t_{n+1}) - g(t_n) of every step (the Douglas D0 on
// Dirichlet nodes): r_min face by k, r_max face by k, y_max face by i; zero
// where the face is not Dirichlet.  Once per solve; thread = (step, entry).
__global__ __launch_bounds__(kBlock) void k_gd(const SolveDesc* __restrict__ descs)
{
    const SolveDesc& s = descs[blockIdx.y];
    const int nr = s.nr, ny = s.ny;
    const int W = 2 * ny + nr;
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)W * s.n_steps) return;
    const int n = (int)(idx / W);
    const int e = (int)(idx - (int64_t)n * W);
    gcdouble* rt = gp(s.rt);
    gcdouble* yt = gp(s.yt);
    gcdouble* stn = gp(s.st) + (size_t)kStepStride * n;
    bool dir;
    double r, y;
    if (e < 2 * ny) {
        const bool hi = e >= ny;
        dir = hi ? s.r_hi_dir : s.r_lo_dir;
        r = rt[RT_R * nr + (hi ? nr - 1 : 0)];
        y = yt[YT_Y * ny + (hi ? e - ny : e)];
    } else {
        dir = s.y_hi_dir;
        r = rt[RT_R * nr + (e - 2 * ny)];
        y = yt[YT_Y * ny + ny - 1];
    }
    const double inc = dir ? dirichlet_value(s, stn + kStepStride, r, y) - dirichlet_value(s, stn, r, y) : 0.0;
    gp(const_cast<double*>(s.gd))[idx] = inc;
}

// Price and its r and v derivatives at (r0, v0) on the y_min plane: 4 x 4
// Lagrange interpolation in mesh coordinates (section 6), differentiated for
// the Greeks rho = dC/dr and vega = dC/dv the paper plots.
__global__ void k_readout(const SolveDesc* __restrict__ descs, const Readout* __restrict__ rq, int n,
                          double* __restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const Readout R = rq[t];
    const SolveDesc& s = descs[R.solve];
    gcdouble* U = gp(s.U);
    double acc = 0.0, acc_r = 0.0, acc_v = 0.0;
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a) {
            const double u = U[(size_t)(R.j0 + b) * s.nr + (R.i0 + a)];
            acc += R.wv[b] * R.wr[a] * u;
            acc_r += R.wv[b] * R.dwr[a] * u;
            acc_v += R.dwv[b] * R.wr[a] * u;
        }
    out[3 * t] = acc;
    out[3 * t + 1] = acc_r;
    out[3 * t + 2] = acc_v;
}

__global__ __launch_bounds__(kBlock) void k_health(const SolveDesc* __restrict__ descs)
{
    const SolveDesc& s = descs[blockIdx.y];
    const int64_t npts = (int64_t)s.nr * s.nv * s.ny;
    gcdouble* U = gp(s.U);
    bool bad = false;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < npts; p += (int64_t)gridDim.x * kBlock)
        bad = bad || !isfinite(U[p]);
    if (bad) raise_flag(s);
}

template <class K>
hipError_t allow_lds(K kernel)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <int ROWS>
hipError_t allow_yc()
{
    hipError_t e;
    if ((e = allow_lds(k_yc<ROWS, 0, false>)) || (e = allow_lds(k_yc<ROWS, 1, false>)) ||
        (e = allow_lds(k_yc<ROWS, 2, false>)) || (e = allow_lds(k_yc<ROWS, 3, false>)))
        return e;
    if ((e = allow_lds(k_yc<ROWS, 0, true>)) || (e = allow_lds(k_yc<ROWS, 1, true>)) ||
        (e = allow_lds(k_yc<ROWS, 2, true>)) || (e = allow_lds(k_yc<ROWS, 3, true>)) ||
        (e = allow_lds(k_yc<ROWS, 0, true, true>)))
        return e;
    return hipSuccess;
}

}  // namespace

// Timing events for the next sweep launch of this thread (profiling): the
// dispatch itself records them, so they bracket exactly the kernel.
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

void set_launch_events(hipEvent_t start, hipEvent_t stop)
{
    g_ev_start = start;
    g_ev_stop = stop;
}

#define HJM_LAUNCH(K, GRID, BLOCK, LDS, ST, ...)                                                     \
    do {                                                                                             \
        if (g_ev_start) {                                                                            \
            hipExtLaunchKernelGGL(K, GRID, BLOCK, LDS, ST, g_ev_start, g_ev_stop, 0, __VA_ARGS__);   \
            g_ev_start = g_ev_stop = nullptr;                                                        \
        } else {                                                                                     \
            hipLaunchKernelGGL(K, GRID, BLOCK, LDS, ST, __VA_ARGS__);                                \
        }                                                                                            \
    } while (0)

hipError_t init_kernel_attributes()
{
    static hipError_t status = [] {
        hipError_t e;
        if ((e = allow_lds(k_xr<8>)) || (e = allow_lds(k_xr<16>)) || (e = allow_lds(k_xr<32>)) ||
            (e = allow_lds(k_v<8>)) || (e = allow_lds(k_v<16>)) || (e = allow_lds(k_v<32>)) ||
            (e = allow_lds(k_yu<8>)) || (e = allow_lds(k_yu<16>)) || (e = allow_lds(k_yu<32>)) ||
            (e = allow_lds(k_rs<6>)) || (e = allow_lds(k_rs<8>)) || (e = allow_lds(k_rs<12>)) ||
            (e = allow_lds(k_rs<16>)) || (e = allow_lds(k_exr<8, false>)) || (e = allow_lds(k_exr<12, false>)) ||
            (e = allow_lds(k_exr<16, false>)) || (e = allow_lds(k_exr<8, false, true>)) ||
            (e = allow_lds(k_exr<12, false, true>)) || (e = allow_lds(k_exr<16, false, true>)) ||
            (e = allow_lds(k_exr<8, false, true, true>)) || (e = allow_lds(k_exr<12, false, true, true>)) ||
            (e = allow_lds(k_exr<16, false, true, true>)) ||
            (e = allow_lds(k_exr<8, true>)) ||
            (e = allow_lds(k_exr<12, true>)) || (e = allow_lds(k_exr<16, true>)) || (e = allow_lds(k_vs<8>)) || (e = allow_lds(k_vs<16>)) ||
            (e = allow_lds(k_vs<32>)) || (e = allow_yc<8>()) || (e = allow_yc<16>()) || (e = allow_yc<32>()))
            return e;
        return hipSuccess;
    }();
    return status;
}

hipError_t launch_terminal(const SolveDesc* d_desc, int n_solves, int64_t max_points, hipStream_t st)
{
    int64_t blocks = (max_points + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_terminal, dim3((unsigned)blocks, (unsigned)n_solves), dim3(kBlock), 0, st, d_desc);
    return hipGetLastError();
}

hipError_t launch_health(const SolveDesc* d_desc, int n_solves, int64_t max_points, hipStream_t st)
{
    int64_t blocks = (max_points + kBlock - 1) / kBlock;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_health, dim3((unsigned)blocks, (unsigned)n_solves), dim3(kBlock), 0, st, d_desc);
    return hipGetLastError();
}

hipError_t launch_readout(const SolveDesc* d_desc, const Readout* rq, int n, double* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_readout, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, d_desc, rq, n, out);
    return hipGetLastError();
}

#define HJM_DISPATCH_ROWS(rows, CALL) \
    switch (rows) {                   \
    case 8: { constexpr int R = 8; CALL; } break;   \
    case 16: { constexpr int R = 16; CALL; } break; \
    case 32: { constexpr int R = 32; CALL; } break; \
    default: return hipErrorInvalidValue;           \
    }

hipError_t launch_xr(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int step, size_t lds,
                     hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    HJM_DISPATCH_ROWS(rows, HJM_LAUNCH(k_xr<R>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step))
    return hipGetLastError();
}

hipError_t launch_v(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, size_t lds, hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    HJM_DISPATCH_ROWS(rows, HJM_LAUNCH(k_v<R>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks))
    return hipGetLastError();
}

hipError_t launch_exp(int J, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int step, hipStream_t st,
                      bool stage2)
{
    if (n_tasks <= 0) return hipSuccess;
    if (stage2) {
        switch (J) {
        case 4: HJM_LAUNCH((k_exp<4, true>), dim3(n_tasks), dim3(kBlock), 0, st, d_desc, tasks, step); break;
        case 8: HJM_LAUNCH((k_exp<8, true>), dim3(n_tasks), dim3(kBlock), 0, st, d_desc, tasks, step); break;
        case 16: HJM_LAUNCH((k_exp<16, true>), dim3(n_tasks), dim3(kBlock), 0, st, d_desc, tasks, step); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (J) {
    case 4: HJM_LAUNCH((k_exp<4, false>), dim3(n_tasks), dim3(kBlock), 0, st, d_desc, tasks, step); break;
    case 8: HJM_LAUNCH((k_exp<8, false>), dim3(n_tasks), dim3(kBlock), 0, st, d_desc, tasks, step); break;
    case 16: HJM_LAUNCH((k_exp<16, false>), dim3(n_tasks), dim3(kBlock), 0, st, d_desc, tasks, step); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool rs_rows_supported(int rows) { return rows == 6 || rows == 8 || rows == 12 || rows == 16; }

hipError_t launch_rs(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int step, int nr_max,
                     hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    // row table (kRF * ROWS + 1 per segment, at most nr_max / ROWS + 1
    // segments) and 8 doubles per thread for the reduced systems
    const size_t lds = ((size_t)kRF * nr_max + (size_t)(nr_max / rows + 1) * (kRF + 1)) * 8 + (size_t)kBlock * 8 * 8 +
                       (size_t)kFace * 8;
    switch (rows) {
    case 6: HJM_LAUNCH(k_rs<6>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
    case 8: HJM_LAUNCH(k_rs<8>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
    case 12: HJM_LAUNCH(k_rs<12>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
    case 16: HJM_LAUNCH(k_rs<16>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

void exr_lds(int nr, int rows, size_t* bytes, int* tab)
{
    const int S = nr / rows;
    const int P = exr_planes(nr, rows);
    const int lanes = P * kExrJ * S;
    const int passes = (lanes + kBlock - 1) / kBlock;
    // whole passes: the last pass's scratch stays inside; at least the
    // window variant's explicit window (J + 2 rows of nr per plane, two
    // guard doubles each side), which the tile overwrites after it
    const int tile = std::max(passes * kBlock * (rows + 1), P * (kExrJ + 2) * nr + 4);
    *tab = tile;
    // the row table, the window variant's v-table cache (kVT x kExrJ), the
    // face rows' table entries and the window variant's c of each plane
    *bytes = ((size_t)tile + (size_t)S * (kRF * rows + 1) + (size_t)kVT * kExrJ + (size_t)kFace + kExrMaxP) * 8;
}

hipError_t launch_exr(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int step, size_t lds,
                      hipStream_t st, bool stage2, bool window, bool fold)
{
    if (n_tasks <= 0) return hipSuccess;
    if (fold && (!window || stage2)) return hipErrorInvalidValue;
    if (fold) {
        switch (rows) {
        case 8: HJM_LAUNCH((k_exr<8, false, true, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        case 12: HJM_LAUNCH((k_exr<12, false, true, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        case 16: HJM_LAUNCH((k_exr<16, false, true, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (window && !stage2) {
        switch (rows) {
        case 8: HJM_LAUNCH((k_exr<8, false, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        case 12: HJM_LAUNCH((k_exr<12, false, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        case 16: HJM_LAUNCH((k_exr<16, false, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (stage2) {
        switch (rows) {
        case 8: HJM_LAUNCH((k_exr<8, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        case 12: HJM_LAUNCH((k_exr<12, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        case 16: HJM_LAUNCH((k_exr<16, true>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (rows) {
    case 8: HJM_LAUNCH((k_exr<8, false>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
    case 12: HJM_LAUNCH((k_exr<12, false>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
    case 16: HJM_LAUNCH((k_exr<16, false>), dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool vs_rows_supported(int rows) { return rows == 8 || rows == 16 || rows == 32; }
bool yc_rows_supported(int rows) { return rows == 8 || rows == 16 || rows == 32; }

hipError_t launch_vs(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int S_max, hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    if (S_max < 1 || S_max > 4) return hipErrorInvalidValue;
    const size_t lds = (size_t)2 * 4 * 64 * 8;
    HJM_DISPATCH_ROWS(rows, HJM_LAUNCH(k_vs<R>, dim3(n_tasks), dim3(64 * S_max), lds, st, d_desc, tasks))
    return hipGetLastError();
}

hipError_t launch_vfix(const SolveDesc* d_desc, const int2* tasks, int n_tasks, int segs, hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    switch (segs) {
#define HJM_VFIX(SV) case SV: HJM_LAUNCH(k_vfix<SV>, dim3(n_tasks), dim3(kBlock), 0, st, d_desc, tasks); break;
    HJM_VFIX(2) HJM_VFIX(3) HJM_VFIX(4) HJM_VFIX(5) HJM_VFIX(6) HJM_VFIX(7) HJM_VFIX(8) HJM_VFIX(9)
    HJM_VFIX(10) HJM_VFIX(11) HJM_VFIX(12) HJM_VFIX(13) HJM_VFIX(14) HJM_VFIX(15) HJM_VFIX(16)
#undef HJM_VFIX
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gd(const SolveDesc* d_desc, int n_solves, int64_t max_entries, hipStream_t st)
{
    const int64_t blocks = (max_entries + kBlock - 1) / kBlock;
    if (blocks < 1 || n_solves < 1) return hipSuccess;
    hipLaunchKernelGGL(k_gd, dim3((unsigned)blocks, (unsigned)n_solves), dim3(kBlock), 0, st, d_desc);
    return hipGetLastError();
}

hipError_t launch_ypiv(const SolveDesc* d_desc, int n_solves, int64_t max_lines, hipStream_t st)
{
    const int64_t blocks = (max_lines + kBlock - 1) / kBlock;
    if (blocks < 1 || n_solves < 1) return hipSuccess;
    hipLaunchKernelGGL(k_ypiv, dim3((unsigned)blocks, (unsigned)n_solves), dim3(kBlock), 0, st, d_desc);
    return hipGetLastError();
}

hipError_t launch_yc(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int S_max, hipStream_t st,
                     int mode, bool minors, bool fold)
{
    if (n_tasks <= 0) return hipSuccess;
    if (S_max < 1 || S_max > yc_max_segments(rows)) return hipErrorInvalidValue;
    // the exchange slots (2 per lane) and C inv of every row of the lines
    const size_t lds = (size_t)(2 + (size_t)S_max * rows) * 64 * 8;
    if (fold) {
        // the folded v sweep: Douglas (mode 0) on pivots formed in the kernel
        if (mode != 0 || !minors) return hipErrorInvalidValue;
        HJM_DISPATCH_ROWS(rows, HJM_LAUNCH((k_yc<R, 0, true, true>), dim3(n_tasks), dim3(64 * S_max), lds, st, d_desc, tasks))
        return hipGetLastError();
    }
    switch (mode) {
#define HJM_YC(M)                                                                                                       \
    if (minors) HJM_DISPATCH_ROWS(rows, HJM_LAUNCH((k_yc<R, M, true>), dim3(n_tasks), dim3(64 * S_max), lds, st, d_desc, tasks)) \
    else HJM_DISPATCH_ROWS(rows, HJM_LAUNCH((k_yc<R, M, false>), dim3(n_tasks), dim3(64 * S_max), lds, st, d_desc, tasks))
    case 0: HJM_YC(0) break;
    case 1: HJM_YC(1) break;
    case 2: HJM_YC(2) break;
    case 3: HJM_YC(3) break;
#undef HJM_YC
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_yu(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, size_t lds, hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    HJM_DISPATCH_ROWS(rows, HJM_LAUNCH(k_yu<R>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks))
    return hipGetLastError();
}

}  // namespace hjm
