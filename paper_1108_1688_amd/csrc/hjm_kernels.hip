// HIP kernels (gfx950) of the Douglas-ADI step for the single-factor HJM model
// with stochastic volatility.  FP64 throughout; no MFMA (nothing here is a
// dense contraction).
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
// Line solves.  Each tridiagonal line of n rows is split into S segments of
// at most ROWS rows held in the registers of S threads, and solved by the
// Thomas algorithm in row order with the segments chained through LDS.
// Outflow faces (section 7.3) add one entry beyond the tridiagonal band in
// rows 0 and n-1; those unknowns are eliminated from rows 1 and n-2 first and
// recovered last.  No pivoting: diagonals are >= 1 and the pivots are checked
// (> 0) into the health flag.
//
// Work is described by (solve, tile) tasks so that one launch can cover many
// independent solves of different shapes (batched mode); a null task list
// means one solve whose tile index is the workgroup index.

#include "hjm_internal.h"

namespace hjm {
namespace {

__device__ __forceinline__ double dirichlet_value(const SolveDesc& s, const double* stn, double r, double y)
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

__device__ __forceinline__ void raise_flag(const SolveDesc& s)
{
    // plain vector store of a constant; concurrent writers store the same value
    *reinterpret_cast<volatile int32_t*>(s.flag) = 1;
}

// ---------------------------------------------------------------------------
// Implicit row functors: coefficients (A, B, C) of row m of (I - theta dt A_d)
// and E, the entry beyond the band (column 2 in row 0, column n-3 in row n-1).
// ---------------------------------------------------------------------------
struct RowR {
    const double* r;
    const double* ra;
    const double* rb1;
    const double* rb2;
    double v, drift0, kappa, tdt, ih2, i2h;
    int nr;
    int lo_dir, hi_dir;
    __device__ __forceinline__ void operator()(int i, double& A, double& B, double& C, double& E) const
    {
        E = 0.0;
        if ((i == 0 && lo_dir) || (i == nr - 1 && hi_dir)) { A = 0.0; B = 1.0; C = 0.0; return; }
        const double ri = r[i];
        const double mu = (drift0 - kappa * ri) * rb1[i];  // drift of r over J_r
        if (i == 0) {
            A = 0.0;
            B = 1.0 - tdt * (-3.0 * mu * i2h - ri);
            C = -tdt * (4.0 * mu * i2h);
            E = -tdt * (-mu * i2h);
        } else if (i == nr - 1) {
            A = -tdt * (-4.0 * mu * i2h);
            B = 1.0 - tdt * (3.0 * mu * i2h - ri);
            C = 0.0;
            E = -tdt * (mu * i2h);
        } else {
            const double a = ra[i] * v;
            const double b = mu - v * rb2[i];
            A = -tdt * (a * ih2 - b * i2h);
            B = 1.0 - tdt * (-2.0 * a * ih2 - ri);
            C = -tdt * (a * ih2 + b * i2h);
        }
    }
};

struct RowV {
    const double* va;
    const double* vb;
    const double* vm;
    double tdt, ih2, i2h;
    int nv;
    __device__ __forceinline__ void operator()(int j, double& A, double& B, double& C, double& E) const
    {
        E = 0.0;
        if (j == 0) {
            const double m = vm[0];
            A = 0.0;
            B = 1.0 - tdt * (-3.0 * m * i2h);
            C = -tdt * (4.0 * m * i2h);
            E = -tdt * (-m * i2h);
        } else if (j == nv - 1) {
            const double m = vm[j];
            A = -tdt * (-4.0 * m * i2h);
            B = 1.0 - tdt * (3.0 * m * i2h);
            C = 0.0;
            E = -tdt * (m * i2h);
        } else {
            const double a = va[j], b = vb[j];
            A = -tdt * (a * ih2 - b * i2h);
            B = 1.0 - tdt * (-2.0 * a * ih2);
            C = -tdt * (a * ih2 + b * i2h);
        }
    }
};

struct RowY {
    const double* yi;
    const double* y2k;
    double qv, tdt, i2h;
    int ny;
    int hi_dir;
    __device__ __forceinline__ void operator()(int k, double& A, double& B, double& C, double& E) const
    {
        E = 0.0;
        if (k == ny - 1 && hi_dir) { A = 0.0; B = 1.0; C = 0.0; return; }
        const double b = (qv - y2k[k]) * yi[k];  // drift of y over J_y
        if (k == 0) {
            A = 0.0;
            B = 1.0 - tdt * (-3.0 * b * i2h);
            C = -tdt * (4.0 * b * i2h);
            E = -tdt * (-b * i2h);
        } else if (k == ny - 1) {
            A = -tdt * (-4.0 * b * i2h);
            B = 1.0 - tdt * (3.0 * b * i2h);
            C = 0.0;
            E = -tdt * (b * i2h);
        } else {
            A = -tdt * (-b * i2h);
            B = 1.0;
            C = -tdt * (b * i2h);
        }
    }
};

// ---------------------------------------------------------------------------
// Chained line solver: the rows of one line are split into S segments of at
// most ROWS consecutive rows, each held in the registers of one thread.  The
// elimination itself is the plain Thomas algorithm in row order: segment s
// runs its forward sweep once segment s-1 has handed over (c', d') of its last
// row, and its back substitution once segment s+1 has handed back x of its
// first row (hand-over through LDS, one workgroup barrier per stage).  Splitting
// only distributes storage and memory traffic; the arithmetic is that of one
// sequential Thomas solve, which stays accurate for the advection-dominated
// lines of this problem (a spike / partition reduction does not).
// ---------------------------------------------------------------------------
template <int ROWS>
struct Seg {
    double d[ROWS];   // right-hand side -> d' -> solution
    double cp[ROWS];  // modified super-diagonal c'
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
}

// Every thread of the workgroup calls this (barriers inside when S > 1).
// `work` marks threads holding a segment of a line that needs solving; xch is
// the line's two-double hand-over slot in LDS.
template <int ROWS, class RowFn>
__device__ __forceinline__ void line_solve(Seg<ROWS>& g, const RowFn& row, bool work, double* xch,
                                           const SolveDesc& s)
{
    const bool first = g.seg == 0;
    const bool last = g.seg == g.S - 1;
    double b1m = 0.0, c1m = 0.0, a2m = 0.0, b2m = 0.0;
    bool ok = true;
    g.lo = 0;
    g.hi = g.len - 1;
    if (work && first) {
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
    if (work && last) {
        // eliminate x_{n-1} (row n-1: e x_{n-3} + a x_{n-2} + b x_{n-1}) from row n-2
        double A, B, C, E;
        row(g.n - 1, A, B, C, E);
        g.al = A; g.bl = B; g.el = E;
        double dl = 0.0;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm == g.len - 1) dl = g.d[mm];
        g.dl = dl;
        double A2, B2, C2, E2;
        row(g.n - 2, A2, B2, C2, E2);
        const double f = C2 / B;
        a2m = A2 - f * E;
        b2m = B2 - f * A;
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm == g.len - 2) g.d[mm] = g.d[mm] - f * dl;
        g.hi = g.len - 2;
        ok = ok && (B > 0.0);
    }
    // forward sweep, segment after segment
    for (int stage = 0; stage < g.S; ++stage) {
        if (work && g.seg == stage) {
            double cprev = 0.0, dprev = 0.0;
            if (stage > 0) { cprev = xch[0]; dprev = xch[1]; }
#pragma unroll
            for (int mm = 0; mm < ROWS; ++mm) {
                if (mm >= g.lo && mm <= g.hi) {
                    double A, B, C, E;
                    if (first && mm == 1) { A = 0.0; B = b1m; C = c1m; }
                    else if (last && mm == g.len - 2) { A = a2m; B = b2m; C = 0.0; }
                    else row(g.p + mm, A, B, C, E);
                    const double den = B - A * cprev;
                    ok = ok && (den > 0.0);
                    cprev = C / den;
                    dprev = (g.d[mm] - A * dprev) / den;
                    g.cp[mm] = cprev;
                    g.d[mm] = dprev;
                }
            }
            xch[0] = cprev;
            xch[1] = dprev;
        }
        if (g.S > 1) __syncthreads();
    }
    // back substitution, segment after segment
    for (int stage = g.S - 1; stage >= 0; --stage) {
        if (work && g.seg == stage) {
            double x = (stage < g.S - 1) ? xch[0] : 0.0;
#pragma unroll
            for (int mm = ROWS - 1; mm >= 0; --mm) {
                if (mm >= g.lo && mm <= g.hi) {
                    x = g.d[mm] - g.cp[mm] * x;
                    g.d[mm] = x;
                }
            }
            xch[0] = x;
            if (first) g.d[0] = (g.d0 - g.c0 * g.d[1] - g.e0 * g.d[2]) / g.b0;
            if (last) {
                double x3 = 0.0, x2 = 0.0;
#pragma unroll
                for (int mm = 0; mm < ROWS; ++mm) {
                    if (mm == g.len - 3) x3 = g.d[mm];
                    if (mm == g.len - 2) x2 = g.d[mm];
                }
                const double xl = (g.dl - g.el * x3 - g.al * x2) / g.bl;
#pragma unroll
                for (int mm = 0; mm < ROWS; ++mm)
                    if (mm == g.len - 1) g.d[mm] = xl;
            }
        }
        if (g.S > 1) __syncthreads();
    }
    if (work && !ok) raise_flag(s);
}

// ---------------------------------------------------------------------------
// Explicit Douglas predictor at one node.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double explicit_point(const SolveDesc& s, int i, int j, int k, size_t q, double phi,
                                                 const double* stn, const double* stn1)
{
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const double* rt = s.rt;
    const double* vt = s.vt;
    const double* yt = s.yt;
    const double ri = rt[RT_R * nr + i];
    const double yk = yt[YT_Y * ny + k];
    if ((i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir) || (k == ny - 1 && s.y_hi_dir))
        return dirichlet_value(s, stn1, ri, yk) - dirichlet_value(s, stn, ri, yk);
    const double* U = s.U;
    const size_t sv = (size_t)nr;
    const size_t sy = (size_t)nr * (size_t)nv;
    const double u = U[q];
    const double vj = vt[VT_V * nv + j];
    // A1: r direction with the reaction term
    const double mu = (phi + yk - s.kappa * ri) * rt[RT_B1 * nr + i];
    double a1;
    if (i == 0) {
        a1 = mu * s.i2hr * (-3.0 * u + 4.0 * U[q + 1] - U[q + 2]) - ri * u;
    } else if (i == nr - 1) {
        a1 = mu * s.i2hr * (3.0 * u - 4.0 * U[q - 1] + U[q - 2]) - ri * u;
    } else {
        const double um = U[q - 1], up = U[q + 1];
        const double a = rt[RT_A * nr + i] * vj;
        const double b = mu - vj * rt[RT_B2 * nr + i];
        a1 = a * s.ih2r * (up - 2.0 * u + um) + b * s.i2hr * (up - um) - ri * u;
    }
    // A2: v direction
    double a2;
    if (j == 0) {
        a2 = vt[VT_M * nv] * s.i2hv * (-3.0 * u + 4.0 * U[q + sv] - U[q + 2 * sv]);
    } else if (j == nv - 1) {
        a2 = vt[VT_M * nv + j] * s.i2hv * (3.0 * u - 4.0 * U[q - sv] + U[q - 2 * sv]);
    } else {
        const double um = U[q - sv], up = U[q + sv];
        a2 = vt[VT_A * nv + j] * s.ih2v * (up - 2.0 * u + um) + vt[VT_B * nv + j] * s.i2hv * (up - um);
    }
    // A3: y direction (advection only)
    const double qy = rt[RT_Y * nr + i] * vj;
    const double by = (qy - yt[YT_K * ny + k]) * yt[YT_I * ny + k];
    double a3;
    if (k == 0) {
        a3 = by * s.i2hy * (-3.0 * u + 4.0 * U[q + sy] - U[q + 2 * sy]);
    } else if (k == ny - 1) {
        a3 = by * s.i2hy * (3.0 * u - 4.0 * U[q - sy] + U[q - 2 * sy]);
    } else {
        a3 = by * s.i2hy * (U[q + sy] - U[q - sy]);
    }
    // A0: mixed r-v derivative, interior of the (r, v) faces only
    double a0 = 0.0;
    if (i > 0 && i < nr - 1 && j > 0 && j < nv - 1) {
        const double arv = rt[RT_X * nr + i] * vt[VT_X * nv + j];
        a0 = arv * s.i4hrhv * ((U[q + 1 + sv] - U[q + 1 - sv]) - (U[q - 1 + sv] - U[q - 1 - sv]));
    }
    return s.dt * (((a1 + a2) + a3) + a0);
}

__device__ __forceinline__ int pow2_ceil(int n)
{
    int t = 1;
    while (t < n) t <<= 1;
    return t;
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_terminal(const SolveDesc* __restrict__ descs)
{
    const SolveDesc& s = descs[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) *reinterpret_cast<volatile int32_t*>(s.flag) = 0;
    const int nr = s.nr, nv = s.nv;
    const int64_t npts = (int64_t)nr * nv * s.ny;
    const double* r = s.rt + RT_R * nr;
    const double* y = s.yt + YT_Y * s.ny;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < npts; p += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(p % nr);
        const int k = (int)(p / ((int64_t)nr * nv));
        s.U[p] = dirichlet_value(s, s.st, r[i], y[k]);
    }
}

template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_xr(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks,
                                               int step)
{
    extern __shared__ double lds[];
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    if (step >= s.n_steps) return;  // whole workgroup: uniform
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int L = s.r_L, S = s.r_S, pitch = s.r_pitch;
    const int q0 = tk.y * L;
    const int nl = min(L, nv * ny - q0);
    double* tile = lds;
    double* red = lds + (size_t)L * pitch;
    const double* stn = s.st + kStepStride * step;
    const double* stn1 = stn + kStepStride;
    const double phi = stn[ST_PHI];

    // Phase A: explicit predictor of the tile's lines into LDS (coalesced along r)
    const int tpl = min(kBlock, pow2_ceil(nr));
    const int lpp = kBlock / tpl;
    for (int l = threadIdx.x / tpl; l < nl; l += lpp) {
        const int q = q0 + l;
        const int k = q / nv;
        const int j = q - k * nv;
        const size_t base = (size_t)q * nr;
        for (int i = threadIdx.x % tpl; i < nr; i += tpl)
            tile[l * pitch + i] = explicit_point(s, i, j, k, base + i, phi, stn, stn1);
    }
    __syncthreads();

    // Phase B: segmented solve of each r line in registers
    const int l = threadIdx.x % L;
    const int seg = threadIdx.x / L;
    const int q = q0 + l;
    const bool active = seg < S && l < nl;
    const int k = q / nv;
    const int j = q - k * nv;
    const bool line_dir = (k == ny - 1) && s.y_hi_dir;
    const bool work = active && !line_dir;
    Seg<ROWS> g;
    seg_init(g, nr, S, seg < S ? seg : 0);
    if (work) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) g.d[mm] = tile[l * pitch + g.p + mm];
    }
    RowR row;
    row.r = s.rt + RT_R * nr;
    row.ra = s.rt + RT_A * nr;
    row.rb1 = s.rt + RT_B1 * nr;
    row.rb2 = s.rt + RT_B2 * nr;
    row.v = active ? s.vt[VT_V * nv + j] : 0.0;
    row.drift0 = phi + (active ? s.yt[YT_Y * ny + k] : 0.0);
    row.kappa = s.kappa;
    row.tdt = s.tdt;
    row.ih2 = s.ih2r;
    row.i2h = s.i2hr;
    row.nr = nr;
    row.lo_dir = s.r_lo_dir;
    row.hi_dir = s.r_hi_dir;
    line_solve(g, row, work, red + 2 * l, s);
    if (work) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) tile[l * pitch + g.p + mm] = g.d[mm];
    }
    __syncthreads();

    // Phase C: D1 back to global memory (the tile's lines are contiguous)
    double* D = s.D + (size_t)q0 * nr;
    for (int ll = threadIdx.x / tpl; ll < nl; ll += lpp)
        for (int i = threadIdx.x % tpl; i < nr; i += tpl) D[(size_t)ll * nr + i] = tile[ll * pitch + i];
}

template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_v(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks)
{
    extern __shared__ double lds[];
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int L = s.v_L, S = s.v_S;
    const int l = threadIdx.x % L;
    const int seg = threadIdx.x / L;
    const int q = tk.y * L + l;  // line (i, k), q = k*nr + i
    const bool active = seg < S && q < nr * ny;
    const int k = q / nr;
    const int i = q - k * nr;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir) || (k == ny - 1 && s.y_hi_dir);
    const bool work = active && !line_dir;  // identity lines keep D
    Seg<ROWS> g;
    seg_init(g, nv, S, seg < S ? seg : 0);
    double* base = s.D + (size_t)k * nv * nr + i + (size_t)g.p * nr;
    if (work) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) g.d[mm] = base[(size_t)mm * nr];
    }
    RowV row;
    row.va = s.vt + VT_A * nv;
    row.vb = s.vt + VT_B * nv;
    row.vm = s.vt + VT_M * nv;
    row.tdt = s.tdt;
    row.ih2 = s.ih2v;
    row.i2h = s.i2hv;
    row.nv = nv;
    line_solve(g, row, work, lds + 2 * l, s);
    if (work) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) base[(size_t)mm * nr] = g.d[mm];
    }
}

template <int ROWS>
__global__ __launch_bounds__(kBlock) void k_yu(const SolveDesc* __restrict__ descs, const int2* __restrict__ tasks)
{
    extern __shared__ double lds[];
    const int2 tk = tasks ? tasks[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const SolveDesc& s = descs[tk.x];
    const int nr = s.nr, nv = s.nv, ny = s.ny;
    const int L = s.y_L, S = s.y_S;
    const int l = threadIdx.x % L;
    const int seg = threadIdx.x / L;
    const int q = tk.y * L + l;  // line (i, j), q = j*nr + i
    const bool active = seg < S && q < nr * nv;
    const int j = q / nr;
    const int i = q - j * nr;
    const bool line_dir = (i == 0 && s.r_lo_dir) || (i == nr - 1 && s.r_hi_dir);
    Seg<ROWS> g;
    seg_init(g, ny, S, seg < S ? seg : 0);
    const size_t sy = (size_t)nr * nv;
    const size_t off = (size_t)q + (size_t)g.p * sy;
    if (active) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) g.d[mm] = s.D[off + (size_t)mm * sy];
    }
    RowY row;
    row.yi = s.yt + YT_I * ny;
    row.y2k = s.yt + YT_K * ny;
    row.qv = active ? s.rt[RT_Y * nr + i] * s.vt[VT_V * nv + j] : 0.0;
    row.tdt = s.tdt;
    row.i2h = s.i2hy;
    row.ny = ny;
    row.hi_dir = s.y_hi_dir;
    line_solve(g, row, active && !line_dir, lds + 2 * l, s);
    if (active) {
#pragma unroll
        for (int mm = 0; mm < ROWS; ++mm)
            if (mm < g.len) s.U[off + (size_t)mm * sy] += g.d[mm];
    }
}

__global__ void k_readout(const SolveDesc* __restrict__ descs, const Readout* __restrict__ rq, int n,
                          double* __restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const Readout R = rq[t];
    const SolveDesc& s = descs[R.solve];
    double acc = 0.0;
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a)
            acc += R.wv[b] * R.wr[a] * s.U[(size_t)(R.j0 + b) * s.nr + (R.i0 + a)];
    out[t] = acc;
}

__global__ __launch_bounds__(kBlock) void k_health(const SolveDesc* __restrict__ descs)
{
    const SolveDesc& s = descs[blockIdx.y];
    const int64_t npts = (int64_t)s.nr * s.nv * s.ny;
    bool bad = false;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < npts; p += (int64_t)gridDim.x * kBlock)
        bad = bad || !isfinite(s.U[p]);
    if (bad) raise_flag(s);
}

template <class K>
hipError_t allow_lds(K kernel)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace

hipError_t init_kernel_attributes()
{
    static hipError_t status = [] {
        hipError_t e;
        if ((e = allow_lds(k_xr<8>)) || (e = allow_lds(k_xr<16>)) || (e = allow_lds(k_xr<32>)) ||
            (e = allow_lds(k_v<8>)) || (e = allow_lds(k_v<16>)) || (e = allow_lds(k_v<32>)) ||
            (e = allow_lds(k_yu<8>)) || (e = allow_lds(k_yu<16>)) || (e = allow_lds(k_yu<32>)))
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
    HJM_DISPATCH_ROWS(rows, {
        hipLaunchKernelGGL(k_xr<R>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks, step);
    })
    return hipGetLastError();
}

hipError_t launch_v(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, size_t lds, hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    HJM_DISPATCH_ROWS(rows, {
        hipLaunchKernelGGL(k_v<R>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks);
    })
    return hipGetLastError();
}

hipError_t launch_yu(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, size_t lds, hipStream_t st)
{
    if (n_tasks <= 0) return hipSuccess;
    HJM_DISPATCH_ROWS(rows, {
        hipLaunchKernelGGL(k_yu<R>, dim3(n_tasks), dim3(kBlock), lds, st, d_desc, tasks);
    })
    return hipGetLastError();
}

}  // namespace hjm
