// Host layer of libhjm: argument validation, mesh and coefficient tables,
// line-solve tiling, workspace layout and the C ABI of include/hjm.h.
#include "hjm.h"
#include "hjm_internal.h"
#include "hjm_mlp.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

using namespace hjm;

namespace {

thread_local std::string g_last_error;
int g_rows[3] = {16, 16, 16};  // rows per thread of the r, v, y line solves

hjm_status fail(hjm_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

hjm_status hip_fail(hipError_t e, const char* where)
{
    return fail(HJM_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

constexpr int kMaxNodes = 2048;  // per axis (S <= 256 segments of >= 8 rows)
constexpr double kTheta = 0.5;   // Crank-Nicolson weight

bool finite(double x) { return std::isfinite(x); }

// ---------------------------------------------------------------------------
// Curve and bond factors (sections 2 and 3.1).
// ---------------------------------------------------------------------------
// The initial curve: parametric (section 2), or discrete zero-coupon prices
// smoothed by the natural cubic spline S of -ln P(0,t) (section 6.1), held
// per interval as S = k0 + k1 u + k2 u^2 + k3 u^3, u = t - t_i; past the last
// knot S is continued linearly (constant forward, S'' = 0 as the natural end
// condition has it there).
struct Curve {
    double a = 0.0, b = 0.0, c = 0.0;
    std::vector<double> kt, k0, k1, k2, k3;
    bool spline() const { return !kt.empty(); }
    // interval of t (the last one covers t beyond the last knot: extrapolated)
    int seg(double t) const
    {
        const int n = (int)kt.size();
        const int i = (int)(std::upper_bound(kt.begin(), kt.end(), t) - kt.begin()) - 1;
        return std::min(std::max(i, 0), n - 2);
    }
    double f(double t) const
    {
        if (!spline()) return c == 0.0 ? a : a + b * (1.0 - std::exp(-c * t));
        if (t >= kt.back()) return end_slope();
        const int i = seg(t);
        const double u = t - kt[i];
        return k1[i] + u * (2.0 * k2[i] + u * 3.0 * k3[i]);
    }
    double ft(double t) const
    {
        if (!spline()) return c == 0.0 ? 0.0 : b * c * std::exp(-c * t);
        if (t >= kt.back()) return 0.0;
        const int i = seg(t);
        return 2.0 * k2[i] + 6.0 * k3[i] * (t - kt[i]);
    }
    double integral(double t) const
    {
        if (!spline()) return c == 0.0 ? a * t : a * t + b * (t - (1.0 - std::exp(-c * t)) / c);
        const int n = (int)kt.size();
        if (t >= kt.back()) {
            const double h = kt[n - 1] - kt[n - 2];
            const double end = k0[n - 2] + h * (k1[n - 2] + h * (k2[n - 2] + h * k3[n - 2]));
            return end + end_slope() * (t - kt.back());
        }
        const int i = seg(t);
        const double u = t - kt[i];
        return k0[i] + u * (k1[i] + u * (k2[i] + u * k3[i]));
    }
    double P(double t) const { return std::exp(-integral(t)); }
    double end_slope() const
    {
        const int n = (int)kt.size();
        const double h = kt[n - 1] - kt[n - 2];
        return k1[n - 2] + h * (2.0 * k2[n - 2] + h * 3.0 * k3[n - 2]);
    }
};

// Natural cubic spline through (t_i, -ln P_i): the second derivatives M_i at
// the knots solve h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1} =
// 6 (d_i - d_{i-1}), d_i = (S_{i+1} - S_i) / h_i, with M_0 = M_{n-1} = 0
// (diagonally dominant: elimination without pivoting).
Curve make_curve(const hjm_model& m)
{
    Curve cv;
    cv.a = m.f_level; cv.b = m.f_slope; cv.c = m.f_decay;
    const int n = m.curve_n;
    if (n < 2) return cv;
    std::vector<double> S(n), h(n - 1), d(n - 1), M(n, 0.0);
    for (int i = 0; i < n; ++i) S[i] = -std::log(m.curve_p[i]);
    for (int i = 0; i + 1 < n; ++i) {
        h[i] = m.curve_t[i + 1] - m.curve_t[i];
        d[i] = (S[i + 1] - S[i]) / h[i];
    }
    if (n > 2) {
        const int k = n - 2;  // unknowns M_1 .. M_{n-2}
        std::vector<double> cp(k), rp(k);
        for (int r = 0; r < k; ++r) {
            const int i = r + 1;
            const double lo = r > 0 ? h[i - 1] : 0.0, di = 2.0 * (h[i - 1] + h[i]), up = h[i];
            const double rhs = 6.0 * (d[i] - d[i - 1]);
            const double den = di - (r > 0 ? lo * cp[r - 1] : 0.0);
            cp[r] = up / den;
            rp[r] = (rhs - (r > 0 ? lo * rp[r - 1] : 0.0)) / den;
        }
        for (int r = k - 1; r >= 0; --r) M[r + 1] = rp[r] - (r + 1 < k ? cp[r] * M[r + 2] : 0.0);
    }
    cv.kt.assign(m.curve_t, m.curve_t + n);
    cv.k0.resize(n - 1); cv.k1.resize(n - 1); cv.k2.resize(n - 1); cv.k3.resize(n - 1);
    for (int i = 0; i + 1 < n; ++i) {
        cv.k0[i] = S[i];
        cv.k1[i] = d[i] - h[i] * (2.0 * M[i] + M[i + 1]) / 6.0;
        cv.k2[i] = 0.5 * M[i];
        cv.k3[i] = (M[i + 1] - M[i]) / (6.0 * h[i]);
    }
    return cv;
}

double Gfun(double kappa, double s) { return kappa == 0.0 ? s : -std::expm1(-kappa * s) / kappa; }

// ---------------------------------------------------------------------------
// Mesh (eq. (metrica)).
// ---------------------------------------------------------------------------
struct Mesh {
    std::vector<double> z, J, J2;
};

Mesh make_mesh(const hjm_axis& a)
{
    Mesh m;
    const int n = a.n;
    m.z.resize(n);
    m.J.resize(n);
    m.J2.resize(n);
    const double c1 = std::asinh((a.z_min - a.center) / a.alpha);
    const double c2 = std::asinh((a.z_max - a.center) / a.alpha);
    const double dc = c2 - c1;
    for (int q = 0; q < n; ++q) {
        const double x = (double)q / (double)(n - 1);
        const double s = c2 * x + c1 * (1.0 - x);
        m.z[q] = a.center + a.alpha * std::sinh(s);
        m.J[q] = a.alpha * std::cosh(s) * dc;
        m.J2[q] = a.alpha * std::sinh(s) * dc * dc;
    }
    m.z[0] = a.z_min;
    m.z[n - 1] = a.z_max;
    return m;
}

// the mesh map at any x (also beyond [0, 1])
double mesh_z(const hjm_axis& a, double x)
{
    const double c1 = std::asinh((a.z_min - a.center) / a.alpha);
    const double c2 = std::asinh((a.z_max - a.center) / a.alpha);
    return a.center + a.alpha * std::sinh(c2 * x + c1 * (1.0 - x));
}

double mesh_x(const hjm_axis& a, double z)
{
    const double c1 = std::asinh((a.z_min - a.center) / a.alpha);
    const double c2 = std::asinh((a.z_max - a.center) / a.alpha);
    return (std::asinh((z - a.center) / a.alpha) - c1) / (c2 - c1);
}

double rpow(double r, double g) { return g == 0.0 ? 1.0 : std::pow(r, g); }

// ---------------------------------------------------------------------------
// Validation.
// ---------------------------------------------------------------------------
hjm_status validate_axes(const hjm_axis ax[3])
{
    static const char* names[3] = {"r", "v", "y"};
    for (int a = 0; a < 3; ++a) {
        const hjm_axis& x = ax[a];
        if (x.n < 5 || x.n > kMaxNodes) return fail(HJM_EINVAL, "axis %s: n=%d outside [5, %d]", names[a], x.n, kMaxNodes);
        if (!(finite(x.z_min) && finite(x.z_max) && finite(x.center) && finite(x.alpha)))
            return fail(HJM_EINVAL, "axis %s: non-finite geometry", names[a]);
        if (!(x.alpha > 0.0)) return fail(HJM_EINVAL, "axis %s: alpha must be > 0", names[a]);
        if (!(x.z_min < x.z_max)) return fail(HJM_EINVAL, "axis %s: z_min must be < z_max", names[a]);
        for (int f : {x.lo_face, x.hi_face})
            if (f != HJM_FACE_OUTFLOW && f != HJM_FACE_DIRICHLET)
                return fail(HJM_EINVAL, "axis %s: unknown face type %d", names[a], f);
    }
    if (ax[1].lo_face != HJM_FACE_OUTFLOW || ax[1].hi_face != HJM_FACE_OUTFLOW)
        return fail(HJM_EINVAL, "the v faces must be OUTFLOW");
    if (ax[2].lo_face != HJM_FACE_OUTFLOW) return fail(HJM_EINVAL, "the y_min face must be OUTFLOW");
    if (ax[1].z_min < 0.0) return fail(HJM_EINVAL, "v_min must be >= 0");
    if (ax[2].z_min < 0.0) return fail(HJM_EINVAL, "y_min must be >= 0");
    const double pts = (double)ax[0].n * ax[1].n * ax[2].n;
    if (pts > 2147483647.0) return fail(HJM_EINVAL, "grid too large");
    return HJM_OK;
}

hjm_status validate_problem(const hjm_axis ax[3], const hjm_model* m, const hjm_payoff* p, int32_t n_steps)
{
    if (!ax || !m || !p) return fail(HJM_EINVAL, "null argument");
    hjm_status st = validate_axes(ax);
    if (st) return st;
    const double vals[] = {m->kappa, m->theta_v, m->lambda, m->gamma, m->epsilon, m->rho,
                           m->f_level, m->f_slope, m->f_decay, p->expiry, p->pay, p->strike};
    for (double v : vals)
        if (!finite(v)) return fail(HJM_EINVAL, "non-finite model or payoff parameter");
    if (m->kappa < 0.0) return fail(HJM_EINVAL, "kappa must be >= 0");
    if (m->theta_v < 0.0) return fail(HJM_EINVAL, "theta_v must be >= 0");
    if (m->lambda < 0.0) return fail(HJM_EINVAL, "lambda must be >= 0");
    if (m->epsilon < 0.0) return fail(HJM_EINVAL, "epsilon must be >= 0");
    if (std::fabs(m->rho) > 1.0) return fail(HJM_EINVAL, "|rho| must be <= 1");
    if (m->gamma < 0.0 || m->gamma > 1.0) return fail(HJM_EINVAL, "gamma must be in [0, 1]");
    if (m->gamma > 0.0 && ax[0].z_min < 0.0) return fail(HJM_EINVAL, "gamma > 0 needs r_min >= 0");
    if (m->f_decay < 0.0) return fail(HJM_EINVAL, "f_decay must be >= 0");
    if (m->curve_n != 0) {
        const int n = m->curve_n;
        if (n < 2 || n > HJM_MAX_CURVE_KNOTS)
            return fail(HJM_EINVAL, "curve_n must be 0 or in [2, %d] (got %d)", HJM_MAX_CURVE_KNOTS, n);
        if (!m->curve_t || !m->curve_p) return fail(HJM_EINVAL, "null discrete curve");
        if (m->curve_t[0] != 0.0 || m->curve_p[0] != 1.0)
            return fail(HJM_EINVAL, "a discrete curve starts at t = 0 with P = 1");
        for (int i = 0; i < n; ++i) {
            if (!finite(m->curve_t[i]) || !finite(m->curve_p[i]) || !(m->curve_p[i] > 0.0))
                return fail(HJM_EINVAL, "discrete curve knot %d is not finite or its price is not > 0", i);
            if (i > 0 && !(m->curve_t[i] > m->curve_t[i - 1]))
                return fail(HJM_EINVAL, "discrete curve maturities must increase (knot %d)", i);
        }
    }
    if (p->kind < HJM_BOND || p->kind > HJM_FORWARD) return fail(HJM_EINVAL, "unknown payoff kind %d", p->kind);
    if (p->soften < 0 || p->soften > 2) return fail(HJM_EINVAL, "soften must be 0, 1 or 2 (got %d)", p->soften);
    if (!(p->expiry > 0.0)) return fail(HJM_EINVAL, "expiry must be > 0");
    if (p->kind != HJM_BOND) {
        if (!(p->pay > p->expiry)) return fail(HJM_EINVAL, "payment date must be after expiry");
        if (!(p->strike > 0.0)) return fail(HJM_EINVAL, "strike must be > 0");
    }
    if (n_steps <= 0) return fail(HJM_EINVAL, "n_steps must be > 0");
    // Outflow faces: the drift must point out of the domain in backward time.
    const Curve cv = make_curve(*m);
    const double T = p->expiry, dt = T / n_steps;
    const double r0 = ax[0].z_min, r1 = ax[0].z_max;
    const double v0 = ax[1].z_min, v1 = ax[1].z_max;
    const double y0 = ax[2].z_min, y1 = ax[2].z_max;
    for (int n = 0; n < n_steps; ++n) {
        const double t = T - (n + 0.5) * dt;
        const double phi = cv.ft(t) + m->kappa * cv.f(t);
        if (ax[0].lo_face == HJM_FACE_OUTFLOW && phi - m->kappa * r0 + y0 < 0.0)
            return fail(HJM_EINVAL, "r_min outflow face has inflowing drift at t=%g (f_t + kappa f < kappa r_min - y_min)", t);
        if (ax[0].hi_face == HJM_FACE_OUTFLOW && phi - m->kappa * r1 + y1 > 0.0)
            return fail(HJM_EINVAL, "r_max outflow face has inflowing drift at t=%g", t);
    }
    if (m->theta_v * (1.0 - v0) < 0.0) return fail(HJM_EINVAL, "v_min outflow face needs v_min <= 1");
    if (m->theta_v * (1.0 - v1) > 0.0) return fail(HJM_EINVAL, "v_max outflow face needs v_max >= 1");
    const double l2 = m->lambda * m->lambda;
    if (l2 * rpow(r0, 2.0 * m->gamma) * v0 - 2.0 * m->kappa * y0 < 0.0)
        return fail(HJM_EINVAL, "y_min outflow face has inflowing drift");
    if (ax[2].hi_face == HJM_FACE_OUTFLOW) {
        const double rmax = std::max(std::fabs(r0), std::fabs(r1));
        if (l2 * rpow(rmax, 2.0 * m->gamma) * v1 - 2.0 * m->kappa * y1 > 0.0)
            return fail(HJM_EINVAL, "y_max outflow face has inflowing drift");
    }
    return HJM_OK;
}

// ---------------------------------------------------------------------------
// Line-solve tiling.
// ---------------------------------------------------------------------------
struct Plan {
    int rows[3];  // preferred rows per thread of the r, v, y line solves
    bool r_spike;
    int r_mode;  // R_SPIKE / R_CHAIN (k_xr), R_SPLIT (k_exp + k_rs) or R_FUSED (k_exr)
    int r_S, r_L, r_pitch, v_S, v_L, y_S, y_L;
    int r_tiles, v_tiles, y_tiles;
    size_t r_lds, v_lds, y_lds;
    int rs_rows, rs_S, rs_log2S, rs_L, rs_tiles;
    int exp_J, exp_cb, exp_tiles;
    int exr_P, exr_tiles, exr_tab;      // fused explicit + r solve
    bool exr_win;                       // its explicit phase from an LDS window
    size_t exr_lds;
    int vs_rows, vs_S, vs_tiles;        // segmented v solve (0: chained k_v)
    int yc_rows, yc_S, yc_L, yc_tiles;  // y solve on reciprocal pivots (0: k_yu)
    bool y_minors;                      // those pivots formed in k_yc each step (else stored by k_ypiv)
    bool v_fold;                        // the v sweep folded into k_exr / k_vfix / k_yc (vs_rows = kExrJ)
};

// Segmented v solve: nv = S * ROWS with S <= 4 waves; preferred rows first.
// The host also requires the segment products to stay <= 1 in magnitude
// (decided in build_tables, where the factors are known).
int vs_rows_for(int nv, int preferred)
{
    const int cands[4] = {preferred, 32, 16, 8};
    for (int r : cands)
        if (vs_rows_supported(r) && nv % r == 0 && nv / r >= 1 && nv / r <= 4) return r;
    return 0;
}

// y solve on stored pivots: ny = S * ROWS with S <= 128 / ROWS waves per workgroup.
int yc_rows_for(int ny, int preferred)
{
    const int cands[4] = {preferred, 16, 32, 8};
    for (int r : cands)
        if (yc_rows_supported(r) && ny % r == 0 && ny / r <= yc_max_segments(r)) return r;
    return 0;
}

// Overrides of the preferred rows by line shape: (axis, nodes per line,
// lines; 0 lines: any count): the autotuner's per-shape choices.
std::map<std::tuple<int, int, int64_t>, int> g_axis_rows;

// The preferred rows of a solve on an nr x nv x ny grid: the override for
// its exact line shape, else for its line length, else the global setting.
void plan_rows(int nr, int nv, int ny, int rows[3])
{
    const int n[3] = {nr, nv, ny};
    const int64_t lines[3] = {(int64_t)nv * ny, (int64_t)nr * ny, (int64_t)nr * nv};
    for (int a = 0; a < 3; ++a) {
        rows[a] = g_rows[a];
        auto it = g_axis_rows.find(std::make_tuple(a, n[a], lines[a]));
        if (it == g_axis_rows.end()) it = g_axis_rows.find(std::make_tuple(a, n[a], (int64_t)0));
        if (it != g_axis_rows.end()) rows[a] = it->second;
    }
}

int g_exp_J = 8;      // v nodes per k_exp thread (4, 8 or 16)
bool g_fuse_r = true;  // fuse the explicit predictor with the spike r solve where k_exr applies
bool g_exr_window = true;  // the fused kernel's explicit phase reads its neighbours from an LDS window
bool g_y_minors = true;    // k_yc forms the y pivots from the minors recurrence (no stored pivot array)
bool g_v_fold = true;      // Douglas solves fold the v sweep into the other kernels where they can
constexpr int kMaxBatchLanes = 8;
int g_batch_lanes = 3;  // streams a batch spreads its solves over
bool g_batch_share = true;  // solves of one operator share tables and y pivots

// k_rs needs nr = S * ROWS with S a power of two <= 64 lanes; the preferred
// rows per lane come first.
int split_rows(int nr, int preferred)
{
    const int cands[5] = {preferred, 8, 16, 12, 6};
    for (int r : cands) {
        if (!rs_rows_supported(r) || nr % r) continue;
        const int S = nr / r;
        if (S >= 1 && S <= 64 && (S & (S - 1)) == 0) return r;
    }
    return 0;
}

constexpr size_t kTileLdsBudget = 96 * 1024;
constexpr int kLCDoubles = 16;  // per-line constants of the explicit phase

// r_spike: the r sweep uses the spike solve (reduced-system scratch per line).
Plan make_plan(int nr, int nv, int ny, const int rows[3], bool r_spike = true)
{
    Plan p;
    std::memcpy(p.rows, rows, sizeof p.rows);
    p.r_spike = r_spike;
    p.r_S = (nr + rows[0] - 1) / rows[0];
    p.r_pitch = (nr + 4) | 1;  // two zero pads per side, odd: conflict-free strided LDS access
    int L = kBlock / p.r_S;
    const size_t per_line = (size_t)p.r_pitch * 8 + (size_t)kLCDoubles * 8 +
                            (r_spike ? (size_t)p.r_S * kRed * 8 : 16);
    const size_t fixed = (size_t)4 * p.r_pitch * 8 + (size_t)6 * nr * 8;  // halo lines + r solve table
    L = std::max(1, std::min<int>(L, (int)((kTileLdsBudget - std::min(fixed, kTileLdsBudget / 2)) / per_line)));
    // the explicit phase gives each thread at most rows[0] + 1 lines of its column
    int tpl = 1;
    while (tpl < nr) tpl <<= 1;
    tpl = std::min(tpl, kBlock);
    const int lpp = kBlock / tpl;
    const int col_reps = (nr + tpl - 1) / tpl;  // columns per thread (nr > kBlock)
    // (ceil(L / lpp) lines x col_reps columns <= rows[0] + 1 points; the tile
    // with its 4 halo lines <= rows[0] + 8 points)
    L = std::max(1, std::min(L, lpp * std::max(1, (rows[0] + 1) / col_reps)));
    while (L > 1 && ((L + 4 + lpp - 1) / lpp) * col_reps > rows[0] + 8) --L;
    p.r_L = L;
    p.r_tiles = (nv * ny + L - 1) / L;
    p.r_lds = fixed + per_line * L;
    p.v_S = (nv + rows[1] - 1) / rows[1];
    p.v_L = kBlock / p.v_S;
    p.v_tiles = (nr * ny + p.v_L - 1) / p.v_L;
    p.v_lds = 2 * (size_t)p.v_L * 8;
    p.y_S = (ny + rows[2] - 1) / rows[2];
    p.y_L = kBlock / p.y_S;
    p.y_tiles = (nr * nv + p.y_L - 1) / p.y_L;
    p.y_lds = 2 * (size_t)p.y_L * 8;
    p.r_mode = r_spike ? R_SPIKE : R_CHAIN;
    p.rs_rows = r_spike ? split_rows(nr, rows[0]) : 0;
    p.rs_S = p.rs_log2S = p.rs_L = p.rs_tiles = 0;
    p.exp_J = g_exp_J;
    p.exp_cb = (nr * ny + kExpCols - 1) / kExpCols;
    p.exp_tiles = p.exp_cb * ((nv + p.exp_J - 1) / p.exp_J);
    p.vs_rows = vs_rows_for(nv, rows[1]);
    p.vs_S = p.vs_rows ? nv / p.vs_rows : 0;
    p.vs_tiles = p.vs_rows ? (nr * ny + 63) / 64 : 0;
    p.yc_rows = yc_rows_for(ny, rows[2]);
    p.yc_S = p.yc_rows ? ny / p.yc_rows : 0;
    p.yc_L = p.yc_rows ? 64 : 0;
    p.yc_tiles = p.yc_rows ? (nr * nv + p.yc_L - 1) / p.yc_L : 0;
    p.y_minors = p.yc_rows && g_y_minors;
    p.v_fold = false;
    if (p.rs_rows) {
        p.r_mode = R_SPLIT;
        p.rs_S = nr / p.rs_rows;
        while ((1 << p.rs_log2S) < p.rs_S) ++p.rs_log2S;
        p.rs_L = 4 * (64 / p.rs_S);
        p.rs_tiles = (nv * ny + p.rs_L - 1) / p.rs_L;
    }
    p.exr_P = p.exr_tiles = p.exr_tab = 0;
    p.exr_lds = 0;
    // the window variant addresses the grid as one buffer of < 4 GiB
    p.exr_win = g_exr_window && (uint64_t)nr * nv * ny * 8 < (1ull << 32);
    if (p.rs_rows >= 8 && nr <= kExrMaxNr && kBlock / nr <= kExrMaxP) {
        p.exr_P = exr_planes(nr, p.rs_rows);
        p.exr_tiles = ((ny + p.exr_P - 1) / p.exr_P) * ((nv + kExrJ - 1) / kExrJ);
        exr_lds(nr, p.rs_rows, &p.exr_lds, &p.exr_tab);
        if (g_fuse_r) p.r_mode = R_FUSED;
    }
    return p;
}

// The spike solve stays within a few ulps of the sequential elimination as
// long as no row's off-diagonal entries dwarf its diagonal: with
// rho = (|A| + |C|) / B <= kSpikeRho its error measured against an extended-
// precision Thomas solve stays below 1e-15 relative (diagonally dominant rows,
// rho <= 1, and advection-dominated rows, where A C < 0 keeps every pivot
// >= B, alike); rows with rho ~ 1e4, as in the far field of the y lines, lose
// digits.  The entries of an interior r row are affine in v and in
// c = f_t + kappa f + y, so rho is quasi-convex in (v, c) and its maximum
// over all lines and steps sits at a corner of their ranges.
constexpr double kSpikeRho = 16.0;

bool r_spike_ok(const hjm_axis ax[3], const hjm_model& m, const hjm_payoff& p, int n_steps, double theta = kTheta)
{
    const Curve cv = make_curve(m);
    const double T = p.expiry, dt = T / n_steps, tdt = theta * dt;
    double phi_lo = 1e300, phi_hi = -1e300;
    for (int n = 0; n < n_steps; ++n) {
        const double t = T - (n + 0.5) * dt;
        const double phi = cv.ft(t) + m.kappa * cv.f(t);
        phi_lo = std::min(phi_lo, phi);
        phi_hi = std::max(phi_hi, phi);
    }
    const double c_lo = phi_lo + ax[2].z_min, c_hi = phi_hi + ax[2].z_max;
    const Mesh mr = make_mesh(ax[0]);
    const int nr = ax[0].n;
    const double hr1 = nr - 1.0, ih2 = hr1 * hr1, i2h = 0.5 * hr1;
    double worst = 0.0;
    for (int i = 1; i < nr - 1; ++i) {
        const double r = mr.z[i], J = mr.J[i], J2 = mr.J2[i];
        const double rg = rpow(r, m.gamma);
        const double zr = 0.5 * m.lambda * m.lambda * rg * rg;
        const double ra = zr / (J * J), rb2 = zr * J2 / (J * J * J);
        const double alo = ra * ih2 + rb2 * i2h, adi = -2.0 * ra * ih2, aup = ra * ih2 - rb2 * i2h;
        for (double c : {c_lo, c_hi})
            for (double v : {ax[1].z_min, ax[1].z_max}) {
                const double e = (c - m.kappa * r) / J * i2h;
                const double A = -tdt * (alo * v - e), B = 1.0 - tdt * (adi * v - r), C = -tdt * (aup * v + e);
                if (!(B > 0.0)) return false;
                worst = std::max(worst, (std::fabs(A) + std::fabs(C)) / B);
            }
    }
    return worst <= kSpikeRho;
}

// Upper bound of the tiles of any plan (used to size task lists).
Plan plan_bound(int nr, int nv, int ny)
{
    static const int options[3] = {8, 16, 32};
    Plan b{};
    {
        // the most k_exp tiles: the smallest v chunk
        const int save = g_exp_J;
        g_exp_J = 4;
        const int rows[3] = {8, 8, 8};
        b.exp_tiles = make_plan(nr, nv, ny, rows, true).exp_tiles;
        g_exp_J = save;
    }
    for (int o : {8, 16, 12, 6})
        for (bool sp : {true, false}) {
            const int rows[3] = {o, 8, 8};
            Plan p = make_plan(nr, nv, ny, rows, sp);
            b.rs_tiles = std::max(b.rs_tiles, p.rs_tiles);
            b.exr_tiles = std::max(b.exr_tiles, p.exr_tiles);
        }
    for (int o : options)
        for (bool sp : {true, false}) {
            const int rows[3] = {o, o, o};
            Plan p = make_plan(nr, nv, ny, rows, sp);
            b.r_tiles = std::max(b.r_tiles, p.r_tiles);
            b.v_tiles = std::max(b.v_tiles, p.v_tiles);
            b.y_tiles = std::max(b.y_tiles, p.y_tiles);
            b.rs_tiles = std::max(b.rs_tiles, p.rs_tiles);
            b.exp_tiles = std::max(b.exp_tiles, p.exp_tiles);
            b.exr_tiles = std::max(b.exr_tiles, p.exr_tiles);
            b.vs_tiles = std::max(b.vs_tiles, p.vs_tiles);
            b.yc_tiles = std::max(b.yc_tiles, p.yc_tiles);
        }
    return b;
}

// ---------------------------------------------------------------------------
// Workspace layout: a bump allocator over the caller's buffer.
// ---------------------------------------------------------------------------
struct Layout {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    }
};

size_t table_doubles(const hjm_axis ax[3], int n_steps)
{
    return (size_t)kRT * ax[0].n + (size_t)kVT * ax[1].n + (size_t)kYT * ax[2].n + (size_t)kVF * ax[1].n + kVS +
           (size_t)kStepStride * (n_steps + 1) + (size_t)kRF * ax[0].n +
           (size_t)(2 * ax[2].n + ax[0].n) * n_steps + (size_t)kVG * ax[1].n;
}

struct SolveOffsets {
    size_t U, D, YI, E, tables;
};

// corr: the Craig-Sneyd family's correction array E after the pivots
SolveOffsets layout_solve(Layout& L, const hjm_axis ax[3], int n_steps, bool corr = false)
{
    const size_t pts = (size_t)ax[0].n * ax[1].n * ax[2].n;
    SolveOffsets o;
    o.U = L.take(pts * 8);
    o.D = L.take(pts * 8);
    o.YI = L.take(pts * 8);
    o.E = corr ? L.take(pts * 8) : 0;
    o.tables = L.take(table_doubles(ax, n_steps) * 8);
    return o;
}

// Fill the host tables of one solve: axis coefficient rows, step table.
void build_tables(const hjm_axis ax[3], const hjm_model& m, const hjm_payoff& p, int n_steps, Plan& plan,
                  std::vector<double>& out, double theta = kTheta)
{
    const int nr = ax[0].n, nv = ax[1].n, ny = ax[2].n;
    out.assign(table_doubles(ax, n_steps), 0.0);
    double* rt = out.data();
    double* vt = rt + (size_t)kRT * nr;
    double* yt = vt + (size_t)kVT * nv;
    double* vf = yt + (size_t)kYT * ny;
    double* st = vf + (size_t)kVF * nv + kVS;
    double* rf = st + (size_t)kStepStride * (n_steps + 1);
    double* gd = rf + (size_t)kRF * nr;
    double* vg = gd + (size_t)(2 * ny + nr) * n_steps;
    const Mesh mr = make_mesh(ax[0]), mv = make_mesh(ax[1]), my = make_mesh(ax[2]);
    const double lam = m.lambda, eps = m.epsilon;
    const double dt = p.expiry / n_steps, tdt = theta * dt;
    const double hr1 = nr - 1.0, hv1 = nv - 1.0, hy1 = ny - 1.0;
    const double ih2r = hr1 * hr1, i2hr = 0.5 * hr1, ih2v = hv1 * hv1, i2hv = 0.5 * hv1, i2hy = 0.5 * hy1;
    const double i4hrhv = 0.25 * hr1 * hv1;
    const bool r_lo_dir = ax[0].lo_face == HJM_FACE_DIRICHLET, r_hi_dir = ax[0].hi_face == HJM_FACE_DIRICHLET;
    const bool y_hi_dir = ax[2].hi_face == HJM_FACE_DIRICHLET;
    for (int i = 0; i < nr; ++i) {
        const double r = mr.z[i], J = mr.J[i], J2 = mr.J2[i];
        const double rg = rpow(r, m.gamma);
        const double zr = 0.5 * lam * lam * rg * rg;  // zeta_rr / v
        const double ra = zr / (J * J), rb1 = 1.0 / J, rb2 = zr * J2 / (J * J * J);
        const bool lo = i == 0, hi = i == nr - 1;
        const bool dir = (lo && r_lo_dir) || (hi && r_hi_dir);
        double mlo = -1.0, mdi = 0.0, mup = 1.0, mex = 0.0;
        double alo = ra * ih2r + rb2 * i2hr, adi = -2.0 * ra * ih2r, aup = ra * ih2r - rb2 * i2hr;
        if (lo) { mlo = 0.0; mdi = -3.0; mup = 4.0; mex = -1.0; alo = adi = aup = 0.0; }
        if (hi) { mlo = -4.0; mdi = 3.0; mup = 0.0; mex = 1.0; alo = adi = aup = 0.0; }
        if (dir) { mlo = mdi = mup = mex = 0.0; alo = adi = aup = 0.0; }
        rt[RT_R * nr + i] = r;
        rt[RT_P * nr + i] = rb1 * i2hr;
        rt[RT_Q * nr + i] = -m.kappa * r * rb1 * i2hr;
        rt[RT_MLO * nr + i] = mlo;
        rt[RT_MDI * nr + i] = mdi;
        rt[RT_MUP * nr + i] = mup;
        rt[RT_MEX * nr + i] = mex;
        rt[RT_ALO * nr + i] = alo;
        rt[RT_ADI * nr + i] = adi;
        rt[RT_AUP * nr + i] = aup;
        rt[RT_RR * nr + i] = dir ? 0.0 : r;
        rt[RT_X * nr + i] = (lo || hi) ? 0.0 : lam * rg / J;
        rt[RT_Y * nr + i] = lam * lam * rg * rg;
        rt[RT_ELO * nr + i] = mesh_z(ax[0], (i - 0.5) / hr1);
        rt[RT_EHI * nr + i] = mesh_z(ax[0], (i + 0.5) / hr1);
        // the same interior row with theta dt folded in (split path)
        rf[RF_P * nr + i] = tdt * rt[RT_P * nr + i];
        rf[RF_Q * nr + i] = tdt * rt[RT_Q * nr + i];
        rf[RF_ALO * nr + i] = -tdt * alo;
        rf[RF_ADI * nr + i] = -tdt * adi;
        rf[RF_AUP * nr + i] = -tdt * aup;
        rf[RF_B * nr + i] = 1.0 + tdt * rt[RT_RR * nr + i];
    }
    std::vector<double> va(nv), vb(nv), vm(nv);  // v operator pieces, also used by the factorisation
    for (int j = 0; j < nv; ++j) {
        const double v = mv.z[j], J = mv.J[j], J2 = mv.J2[j];
        const double zv = 0.5 * eps * eps * v;
        const double mu = m.theta_v * (1.0 - v);
        va[j] = zv / (J * J);
        vb[j] = mu / J - zv * J2 / (J * J * J);
        vm[j] = mu / J;
        double o[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (j == 0) {
            o[2] = -3.0 * vm[j] * i2hv; o[3] = 4.0 * vm[j] * i2hv; o[4] = -vm[j] * i2hv;
        } else if (j == nv - 1) {
            o[0] = vm[j] * i2hv; o[1] = -4.0 * vm[j] * i2hv; o[2] = 3.0 * vm[j] * i2hv;
        } else {
            o[1] = va[j] * ih2v - vb[j] * i2hv; o[2] = -2.0 * va[j] * ih2v; o[3] = va[j] * ih2v + vb[j] * i2hv;
        }
        vt[VT_V * nv + j] = v;
        for (int w = 0; w < 5; ++w) vt[(VT_O0 + w) * nv + j] = o[w];
        vt[VT_X * nv + j] = (j == 0 || j == nv - 1) ? 0.0 : m.rho * eps * v / J * i4hrhv;
    }
    for (int k = 0; k < ny; ++k) {
        const double y = my.z[k], yi = 1.0 / my.J[k];
        const bool lo = k == 0, hi = k == ny - 1;
        const bool dir = hi && y_hi_dir;
        double w[5] = {0.0, -i2hy, 0.0, i2hy, 0.0};
        double ma = 1.0, mb = 0.0, mc = -1.0, me = 0.0;
        if (lo) { w[1] = 0.0; w[2] = -3.0 * i2hy; w[3] = 4.0 * i2hy; w[4] = -i2hy; ma = 0.0; mb = 3.0; mc = -4.0; me = 1.0; }
        if (hi) { w[0] = i2hy; w[1] = -4.0 * i2hy; w[2] = 3.0 * i2hy; w[3] = 0.0; ma = 4.0; mb = -3.0; mc = 0.0; me = -1.0; }
        if (dir) { for (double& x : w) x = 0.0; ma = mb = mc = me = 0.0; }
        yt[YT_Y * ny + k] = y;
        yt[YT_ELO * ny + k] = mesh_z(ax[2], (k - 0.5) / hy1);
        yt[YT_EHI * ny + k] = mesh_z(ax[2], (k + 0.5) / hy1);
        yt[YT_I * ny + k] = yi;
        yt[YT_K * ny + k] = 2.0 * m.kappa * y * yi;
        for (int q = 0; q < 5; ++q) yt[(YT_W0 + q) * ny + k] = w[q];
        yt[YT_T1 * ny + k] = tdt * i2hy * yi;
        yt[YT_T2 * ny + k] = -tdt * i2hy * 2.0 * m.kappa * y * yi;
        yt[YT_MA * ny + k] = ma;
        yt[YT_MB * ny + k] = mb;
        yt[YT_MC * ny + k] = mc;
        yt[YT_ME * ny + k] = me;
    }
    // LU factors of the v-line matrix (I - theta dt A2): rows depend on j
    // alone, so one elimination serves every line and every step.  Same
    // order of operations as the per-line solve: x0 eliminated from row 1,
    // x_{n-1} from row n-2, then forward elimination over rows 1..n-2.
    {
        std::vector<double> A(nv), B(nv), C(nv);
        double E0 = 0.0, El = 0.0;
        for (int j = 0; j < nv; ++j) {
            const double a = va[j], b = vb[j], mf = vm[j];
            const double ih2 = ih2v, i2h = i2hv;
            if (j == 0) {
                A[j] = 0.0; B[j] = 1.0 - tdt * (-3.0 * mf * i2h); C[j] = -tdt * (4.0 * mf * i2h);
                E0 = -tdt * (-mf * i2h);
            } else if (j == nv - 1) {
                A[j] = -tdt * (-4.0 * mf * i2h); B[j] = 1.0 - tdt * (3.0 * mf * i2h); C[j] = 0.0;
                El = -tdt * (mf * i2h);
            } else {
                A[j] = -tdt * (a * ih2 - b * i2h);
                B[j] = 1.0 - tdt * (-2.0 * a * ih2);
                C[j] = -tdt * (a * ih2 + b * i2h);
            }
        }
        double* fs = vf + (size_t)kVF * nv;
        fs[VS_B0] = B[0]; fs[VS_C0] = C[0]; fs[VS_E0] = E0;
        const double f1 = A[1] / B[0];
        fs[VS_F1] = f1;
        fs[VS_AL] = A[nv - 1]; fs[VS_BL] = B[nv - 1]; fs[VS_EL] = El;
        const double f2 = C[nv - 2] / B[nv - 1];
        fs[VS_F2] = f2;
        std::vector<double> Am(A), Bm(B), Cm(C);
        Bm[1] = B[1] - f1 * C[0];
        Cm[1] = C[1] - f1 * E0;
        Am[1] = 0.0;
        Am[nv - 2] = A[nv - 2] - f2 * El;
        Bm[nv - 2] = B[nv - 2] - f2 * A[nv - 1];
        Cm[nv - 2] = 0.0;
        double cprev = 0.0;
        for (int j = 0; j < nv; ++j) {
            vf[VF_A * nv + j] = 0.0; vf[VF_INV * nv + j] = 0.0; vf[VF_C * nv + j] = 0.0;
        }
        for (int j = 1; j <= nv - 2; ++j) {
            const double den = Bm[j] - Am[j] * cprev;
            cprev = Cm[j] / den;
            vf[VF_A * nv + j] = Am[j];
            vf[VF_INV * nv + j] = 1.0 / den;
            vf[VF_C * nv + j] = cprev;
        }
        // segmented form: rows 0 and n-1 pass through (recovered from their
        // own rows); per segment the products G (forward) and H (backward)
        for (int j = 0; j < nv; ++j) {
            const bool mid = j >= 1 && j <= nv - 2;
            vg[VG_INV * nv + j] = mid ? vf[VF_INV * nv + j] : 1.0;
            vg[VG_AL * nv + j] = mid ? -vf[VF_A * nv + j] * vf[VF_INV * nv + j] : 0.0;
            vg[VG_CP * nv + j] = mid ? vf[VF_C * nv + j] : 0.0;
        }
        // per segment of R rows: the products G and H and, for the folded
        // sweep, K (the backward sweep of G); the largest magnitude
        auto segment_products = [&](int R) {
            double worst = 0.0;
            for (int s0 = 0; R > 0 && s0 < nv; s0 += R) {
                double g = 1.0, h = 1.0, kb = 0.0;
                for (int j = s0; j < s0 + R; ++j) {
                    g *= vg[VG_AL * nv + j];
                    vg[VG_G * nv + j] = g;
                    worst = std::max(worst, std::fabs(g));
                }
                for (int j = s0 + R - 1; j >= s0; --j) {
                    h *= -vg[VG_CP * nv + j];
                    vg[VG_H * nv + j] = h;
                    kb = vg[VG_G * nv + j] - vg[VG_CP * nv + j] * kb;
                    vg[VG_K * nv + j] = kb;
                    worst = std::max(worst, std::max(std::fabs(h), std::fabs(kb)));
                }
            }
            return worst;
        };
        // the segment corrections add G d'_in and H x_in (K d'_in folded):
        // keep them from amplifying (they are products of |AL|, |CP| < 1 on
        // dominant rows); a folded sweep that fails falls back to k_vs's
        // segments, and those to the chained sweep
        double worst = segment_products(plan.vs_rows);
        if (plan.v_fold && !(worst <= 1.0)) {
            plan.v_fold = false;
            plan.vs_rows = vs_rows_for(nv, plan.rows[1]);
            plan.vs_S = plan.vs_rows ? nv / plan.vs_rows : 0;
            plan.vs_tiles = plan.vs_rows ? (nr * ny + 63) / 64 : 0;
            worst = segment_products(plan.vs_rows);
        }
        if (plan.vs_rows > 0 && !(worst <= 1.0)) {
            plan.vs_rows = plan.vs_S = plan.vs_tiles = 0;
        }
    }
    const Curve cv = make_curve(m);
    const double T = p.expiry, TM = p.kind == HJM_BOND ? p.expiry : p.pay;
    const double PT = cv.P(T), PM = cv.P(TM);
    for (int n = 0; n <= n_steps; ++n) {
        double* e = st + (size_t)kStepStride * n;
        const double t = T - n * dt;
        const double th = T - (n + 0.5) * dt;
        e[ST_PHI] = n < n_steps ? cv.ft(th) + m.kappa * cv.f(th) : 0.0;
        const double Pt = cv.P(t), ft = cv.f(t);
        const double GT = Gfun(m.kappa, T - t), GM = Gfun(m.kappa, TM - t);
        e[ST_AT] = PT / Pt * std::exp(GT * ft);
        e[ST_GT] = GT;
        e[ST_HT] = 0.5 * GT * GT;
        e[ST_AM] = PM / Pt * std::exp(GM * ft);
        e[ST_GM] = GM;
        e[ST_HM] = 0.5 * GM * GM;
    }
    // the Dirichlet increments (gd) are computed on the device (k_gd)
}

void fill_desc(SolveDesc& d, const hjm_axis ax[3], const hjm_model& m, const hjm_payoff& p, int n_steps,
               const Plan& pl, char* base, const SolveOffsets& o, int32_t* flag, double theta = kTheta)
{
    std::memset(&d, 0, sizeof d);
    d.nr = ax[0].n; d.nv = ax[1].n; d.ny = ax[2].n;
    d.n_steps = n_steps;
    d.r_lo_dir = ax[0].lo_face == HJM_FACE_DIRICHLET;
    d.r_hi_dir = ax[0].hi_face == HJM_FACE_DIRICHLET;
    d.y_hi_dir = ax[2].hi_face == HJM_FACE_DIRICHLET;
    d.kind = p.kind;
    d.soften = p.soften;
    d.r_S = pl.r_S; d.r_L = pl.r_L; d.v_S = pl.v_S; d.v_L = pl.v_L;
    d.y_S = pl.y_S; d.y_L = pl.y_L;
    d.r_tiles = pl.r_tiles; d.v_tiles = pl.v_tiles; d.y_tiles = pl.y_tiles;
    d.r_pitch = pl.r_pitch;
    d.dt = p.expiry / n_steps;
    d.tdt = theta * d.dt;
    d.kappa = m.kappa;
    d.accrual = 1.0 + (p.pay - p.expiry) * p.strike;
    const double hr1 = ax[0].n - 1.0, hv1 = ax[1].n - 1.0, hy1 = ax[2].n - 1.0;
    d.ih2r = hr1 * hr1; d.i2hr = 0.5 * hr1;
    d.ih2v = hv1 * hv1; d.i2hv = 0.5 * hv1;
    d.i2hy = 0.5 * hy1;
    d.i4hrhv = 0.25 * hr1 * hv1;
    d.U = reinterpret_cast<double*>(base + o.U);
    d.D = reinterpret_cast<double*>(base + o.D);
    double* t = reinterpret_cast<double*>(base + o.tables);
    d.rt = t;
    d.vt = t + (size_t)kRT * ax[0].n;
    d.yt = d.vt + (size_t)kVT * ax[1].n;
    d.vf = d.yt + (size_t)kYT * ax[2].n;
    d.st = d.vf + (size_t)kVF * ax[1].n + kVS;
    d.rf = d.st + (size_t)kStepStride * (n_steps + 1);
    d.gd = d.rf + (size_t)kRF * ax[0].n;
    d.flag = flag;
    d.r_mode = pl.r_mode;
    d.exp_J = pl.exp_J; d.exp_cb = pl.exp_cb; d.exp_tiles = pl.exp_tiles;
    d.rs_S = pl.rs_S; d.rs_log2S = pl.rs_log2S; d.rs_L = pl.rs_L; d.rs_tiles = pl.rs_tiles;
    d.exr_P = pl.exr_P; d.exr_tiles = pl.exr_tiles; d.exr_tab = pl.exr_tab;
    d.vg = d.gd + (size_t)(2 * ax[2].n + ax[0].n) * n_steps;
    d.yinv = reinterpret_cast<double*>(base + o.YI);
    d.vs_S = pl.vs_S; d.vs_tiles = pl.vs_tiles;
    d.yc_S = pl.yc_S; d.yc_L = pl.yc_L; d.yc_tiles = pl.yc_tiles;
    d.ypiv_skip = pl.y_minors ? 1 : 0;  // k_yc forms its own pivots: nothing to store
}

// Upload a solve's host tables, all but the Dirichlet increments (gd), which
// k_gd computes on the device.
hipError_t upload_tables(const SolveDesc& d, const std::vector<double>& t, hipStream_t st)
{
    const size_t gd_off = (size_t)(d.gd - d.rt), vg_off = (size_t)(d.vg - d.rt);
    hipError_t e = hipMemcpyAsync(const_cast<double*>(d.rt), t.data(), gd_off * 8, hipMemcpyHostToDevice, st);
    if (!e) e = hipMemcpyAsync(const_cast<double*>(d.vg), t.data() + vg_off, (t.size() - vg_off) * 8,
                               hipMemcpyHostToDevice, st);
    return e;
}

// 4-point Lagrange stencil in mesh coordinates (window centred on the
// bracketing interval, clamped to the mesh).
// dw receives the derivatives of the weights with respect to x.
void lagrange4(double x, int n, int* start, double w[4], double dw[4])
{
    const double h = 1.0 / (double)(n - 1);
    int m = (int)std::floor(x / h);
    m = std::max(0, std::min(m, n - 2));
    int s = std::max(0, std::min(m - 1, n - 4));
    for (int a = 0; a < 4; ++a) {
        const double xa = (double)(s + a) * h;
        double num = 1.0, den = 1.0;
        for (int b = 0; b < 4; ++b) {
            if (b == a) continue;
            const double xb = (double)(s + b) * h;
            num *= (x - xb);
            den *= (xa - xb);
        }
        w[a] = num / den;
        // d/dx of prod_{b != a} (x - x_b): sum over the factor left out
        double dnum = 0.0;
        for (int c = 0; c < 4; ++c) {
            if (c == a) continue;
            double pr = 1.0;
            for (int b = 0; b < 4; ++b)
                if (b != a && b != c) pr *= (x - (double)(s + b) * h);
            dnum += pr;
        }
        dw[a] = dnum / den;
    }
    *start = s;
}

// dx/dz of the sinh mesh map x(z) = (asinh((z - K)/alpha) - c1) / (c2 - c1)
double mesh_dxdz(const hjm_axis& a, double z)
{
    const double c1 = std::asinh((a.z_min - a.center) / a.alpha);
    const double c2 = std::asinh((a.z_max - a.center) / a.alpha);
    return 1.0 / ((c2 - c1) * std::sqrt(a.alpha * a.alpha + (z - a.center) * (z - a.center)));
}

hjm_status make_readout(const hjm_axis ax[3], double r0, double v0, int solve, Readout* R)
{
    if (!(finite(r0) && finite(v0))) return fail(HJM_EINVAL, "non-finite readout point");
    if (r0 < ax[0].z_min || r0 > ax[0].z_max) return fail(HJM_EINVAL, "r0=%g outside the mesh", r0);
    if (v0 < ax[1].z_min || v0 > ax[1].z_max) return fail(HJM_EINVAL, "v0=%g outside the mesh", v0);
    std::memset(R, 0, sizeof *R);
    R->solve = solve;
    lagrange4(mesh_x(ax[0], r0), ax[0].n, &R->i0, R->wr, R->dwr);
    lagrange4(mesh_x(ax[1], v0), ax[1].n, &R->j0, R->wv, R->dwv);
    const double sr = mesh_dxdz(ax[0], r0), sv = mesh_dxdz(ax[1], v0);
    for (int a = 0; a < 4; ++a) {
        R->dwr[a] *= sr;
        R->dwv[a] *= sv;
    }
    return HJM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Single grid.
// ---------------------------------------------------------------------------
struct hjm_grid {
    hjm_axis ax[3];
    hjm_model model;
    hjm_payoff payoff;
    int n_steps = 0;
    int64_t step = 0;
    int rows[3];
    Plan plan;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    SolveDesc desc;
    SolveDesc* d_desc = nullptr;  // [desc] or, for the Craig-Sneyd family, [stage 1, stage 2]
    hjm_scheme scheme{HJM_SCHEME_DOUGLAS, 0, 0.5};
    bool corr = false;            // a correction scheme (two sweep sequences per step)
    SolveDesc desc2;              // its stage-2 descriptor
    Readout* d_rq = nullptr;
    double* d_out = nullptr;
    int32_t* d_flag = nullptr;
    std::vector<double> tables;
    Readout rq;            // host copy of the last readout request
    double out_host[3] = {0.0, 0.0, 0.0};
    int32_t flag_host = 0;
    // per-pass timing
    bool profile = false;
    std::vector<hipEvent_t> events;  // pool, 2 per bracketed launch
    std::vector<int> ev_pass;        // pass of each recorded pair
    size_t ev_used = 0;              // pairs recorded since the last read
    ~hjm_grid()
    {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }
};

namespace {

struct GridLayout {
    size_t desc, rq, out, flag, total;
    SolveOffsets s;
};

GridLayout grid_layout(const hjm_axis ax[3], int n_steps, bool corr = false)
{
    Layout L;
    GridLayout g;
    g.desc = L.take(sizeof(SolveDesc) * (corr ? 2 : 1));
    g.rq = L.take(sizeof(Readout));
    g.out = L.take(sizeof(double) * 3);
    g.flag = L.take(sizeof(int32_t));
    g.s = layout_solve(L, ax, n_steps, corr);
    g.total = L.off;
    return g;
}

hjm_status validate_scheme(const hjm_scheme* sc)
{
    if (!sc) return fail(HJM_EINVAL, "null scheme");
    if (sc->kind < HJM_SCHEME_DOUGLAS || sc->kind > HJM_SCHEME_HUANG) return fail(HJM_EINVAL, "unknown scheme %d", sc->kind);
    if (sc->kind == HJM_SCHEME_HUANG && (sc->af_iters < 1 || sc->af_iters > HJM_MAX_AF_ITERS))
        return fail(HJM_EINVAL, "af_iters must lie in [1, %d] (got %d)", HJM_MAX_AF_ITERS, sc->af_iters);
    if (!(sc->theta > 0.0 && sc->theta <= 1.0)) return fail(HJM_EINVAL, "theta must lie in (0, 1] (got %g)", sc->theta);
    return HJM_OK;
}

// Stage-2 coefficients of the corrected start (see SolveDesc): CS a0 = 1/2;
// MCS a0 = 1/2, a1 = 1/2 - theta; HV a0 = a1 = 1/2, b = -1 (relative to Y3);
// Huang a0 = a1 = theta, b = -1 (the residual of the unsplit theta step).
void scheme_stage2(SolveDesc& d2, const SolveDesc& d1, const hjm_scheme& sc, double* E)
{
    const bool huang = sc.kind == HJM_SCHEME_HUANG;
    d2 = d1;
    d2.stage = 2;
    d2.D = E;
    d2.D3 = d1.D;
    d2.sc_a0 = huang ? sc.theta : 0.5;
    d2.sc_a1 = sc.kind == HJM_SCHEME_MCS ? 0.5 - sc.theta : (sc.kind == HJM_SCHEME_HV ? 0.5 : (huang ? sc.theta : 0.0));
    d2.sc_b = sc.kind == HJM_SCHEME_HV || huang ? -1.0 : 0.0;
    d2.hv = sc.kind == HJM_SCHEME_HV || huang;
}

// The solve's kernel variants (host only); HJM_EINVAL where a correction
// scheme asks for kernels the grid's shape does not allow.
hjm_status grid_plan(const hjm_axis ax[3], const hjm_model& model, const hjm_payoff& payoff, const hjm_scheme& scheme,
                     int n_steps, Plan* out)
{
    const bool corr = scheme.kind != HJM_SCHEME_DOUGLAS;
    int rows[3];
    plan_rows(ax[0].n, ax[1].n, ax[2].n, rows);
    const Plan plan = make_plan(ax[0].n, ax[1].n, ax[2].n, rows, r_spike_ok(ax, model, payoff, n_steps, scheme.theta));
    if (corr && (!(plan.r_mode == R_FUSED || plan.r_mode == R_SPLIT) || !plan.yc_rows))
        return fail(HJM_EINVAL,
                    "the correction schemes run on the lane-split r solve and the stored-pivot y solve: nr = S*ROWS "
                    "(S a power of two, rows within the spike bound) and ny = S*ROWS are needed (plan: r method %d, "
                    "y rows %d)", plan.r_mode, plan.yc_rows);
    Plan p = plan;
    // the v sweep folded into the fused kernel (its tile's 16 v rows are one
    // segment), k_vfix and k_yc: Douglas, the window form with the scanned
    // reduced system (no reduced-system scratch in the tile), the y sweep on
    // pivots formed in the kernel (its hand-over values use the pivot array),
    // whole segments; the table gate may still turn it off
    const int nr = ax[0].n, nv = ax[1].n, ny = ax[2].n;
    if (!corr && g_v_fold && p.r_mode == R_FUSED && p.exr_win && p.rs_S <= 16 && p.yc_rows && p.y_minors &&
        nv % kExrJ == 0 && nv / kExrJ >= 2 && nv / kExrJ <= kMaxFoldSegs) {
        p.v_fold = true;
        p.vs_rows = kExrJ;
        p.vs_S = nv / kExrJ;
        p.vs_tiles = (int)(((int64_t)nr * ny + kBlock - 1) / kBlock);
    }
    *out = p;
    return HJM_OK;
}

// Fill a grid handle over device memory laid out as gl at base (U at
// d_U instead when d_U is not null), upload its tables and enqueue the
// set-up kernels (Dirichlet increments, terminal data, y pivots); waits for
// them.  The problem and scheme are validated by the caller.
hjm_status grid_init(hjm_grid* g, const hjm_axis ax[3], const hjm_model& model, const hjm_payoff& payoff,
                     const hjm_scheme& scheme, int n_steps, const Plan& plan, char* base, const GridLayout& gl,
                     hipStream_t stream, double* d_U)
{
    const bool corr = scheme.kind != HJM_SCHEME_DOUGLAS;
    std::memcpy(g->ax, ax, sizeof g->ax);
    g->model = model;
    g->model.curve_t = g->model.curve_p = nullptr;  // the knots are not kept
    g->payoff = payoff;
    g->n_steps = n_steps;
    std::memcpy(g->rows, plan.rows, sizeof g->rows);
    g->plan = plan;
    // the correction schemes keep the stored pivots: their other sweep modes
    // would run at lower occupancy with the pivots formed in the kernel
    if (corr) g->plan.y_minors = false;
    g->scheme = scheme;
    g->corr = corr;
    g->stream = stream;
    g->base = base;
    g->d_desc = reinterpret_cast<SolveDesc*>(g->base + gl.desc);
    g->d_rq = reinterpret_cast<Readout*>(g->base + gl.rq);
    g->d_out = reinterpret_cast<double*>(g->base + gl.out);
    g->d_flag = reinterpret_cast<int32_t*>(g->base + gl.flag);
    build_tables(ax, model, payoff, n_steps, g->plan, g->tables, scheme.theta);
    fill_desc(g->desc, ax, model, payoff, n_steps, g->plan, g->base, gl.s, g->d_flag, scheme.theta);
    if (d_U) g->desc.U = d_U;
    if (corr) {
        g->desc.stage = 1;
        scheme_stage2(g->desc2, g->desc, scheme, reinterpret_cast<double*>(g->base + gl.s.E));
    }
    hipError_t e;
    if ((e = init_kernel_attributes()) ||
        (e = hipMemcpyAsync(g->d_desc, &g->desc, sizeof(SolveDesc), hipMemcpyHostToDevice, g->stream)) ||
        (corr && (e = hipMemcpyAsync(g->d_desc + 1, &g->desc2, sizeof(SolveDesc), hipMemcpyHostToDevice,
                                     g->stream))) ||
        (e = upload_tables(g->desc, g->tables, g->stream)) ||
        (e = launch_gd(g->d_desc, 1, (int64_t)(2 * ax[2].n + ax[0].n) * n_steps, g->stream)) ||
        (e = launch_terminal(g->d_desc, 1, (int64_t)ax[0].n * ax[1].n * ax[2].n, g->stream)) ||
        (!g->plan.y_minors && (e = launch_ypiv(g->d_desc, 1, (int64_t)ax[0].n * ax[1].n, g->stream))) ||
        (e = hipStreamSynchronize(g->stream)))
        return hip_fail(e, "grid set-up");
    return HJM_OK;
}

// ---------------------------------------------------------------------------
// Working memory of hjm_price_static: one array per GPU, held until the
// process ends.  Host code never uses the array's name as an address (on the
// host it names a stand-in, not device memory): hipGetSymbolAddress gives
// each device's copy, once per device, and only that address is used.
// ---------------------------------------------------------------------------
__device__ __align__(256) char scratch[HJM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_at[kMaxDevices] = {};

// The calling thread's current device's copy of the array; the stream (if
// not null) must belong to that device.
hjm_status static_scratch(hipStream_t stream, char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(HJM_EDEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
    if (stream) {
        hipDevice_t sdev = 0;
        if ((e = hipStreamGetDevice(stream, &sdev))) return hip_fail(e, "hipStreamGetDevice");
        if ((int)sdev != dev)
            return fail(HJM_EINVAL, "the stream belongs to device %d, the current device is %d", (int)sdev, dev);
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)))) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || reinterpret_cast<uintptr_t>(p) % 256) return fail(HJM_EDEVICE, "static scratch at a bad address");
        g_scratch_at[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_at[dev];
    return HJM_OK;
}

// hjm_price_static's layout: a grid's (descriptor, readout, flag, D, y
// pivots, tables) without U, which is the caller's.
GridLayout static_layout(const hjm_axis ax[3], int n_steps)
{
    Layout L;
    GridLayout g;
    g.desc = L.take(sizeof(SolveDesc));
    g.rq = L.take(sizeof(Readout));
    g.out = L.take(sizeof(double) * 3);
    g.flag = L.take(sizeof(int32_t));
    const size_t pts = (size_t)ax[0].n * ax[1].n * ax[2].n;
    g.s.U = 0;  // unused: the caller's d_U
    g.s.D = L.take(pts * 8);
    g.s.YI = L.take(pts * 8);
    g.s.E = 0;
    g.s.tables = L.take(table_doubles(ax, n_steps) * 8);
    g.total = L.off;
    return g;
}

}  // namespace

int32_t hjm::report_error(int32_t code, const char* msg)
{
    g_last_error = msg;
    return code;
}

extern "C" {

const char* hjm_status_str(hjm_status s)
{
    switch (s) {
    case HJM_OK: return "HJM_OK";
    case HJM_EINVAL: return "HJM_EINVAL: invalid argument";
    case HJM_ENOMEM: return "HJM_ENOMEM: workspace too small";
    case HJM_EDEVICE: return "HJM_EDEVICE: HIP runtime error";
    case HJM_ENUMERIC: return "HJM_ENUMERIC: non-finite value or non-positive pivot";
    case HJM_ESTATE: return "HJM_ESTATE: call out of order";
    default: return "unknown hjm_status";
    }
}

const char* hjm_last_error(void) { return g_last_error.c_str(); }

hjm_status hjm_set_line_tile(int32_t r_rows, int32_t v_rows, int32_t y_rows)
{
    for (int32_t v : {r_rows, v_rows, y_rows})
        if (v != 8 && v != 16 && v != 32) return fail(HJM_EINVAL, "line tile rows must be 8, 16 or 32 (got %d)", v);
    g_rows[0] = r_rows;
    g_rows[1] = v_rows;
    g_rows[2] = y_rows;
    return HJM_OK;
}

hjm_status hjm_set_axis_tile(int32_t axis, int32_t n, int64_t lines, int32_t rows)
{
    if (axis < 0 || axis > 2) return fail(HJM_EINVAL, "axis must be 0 (r), 1 (v) or 2 (y) (got %d)", axis);
    if (n < 5 || n > kMaxNodes) return fail(HJM_EINVAL, "node count %d outside [5, %d]", n, kMaxNodes);
    if (lines < 0) return fail(HJM_EINVAL, "negative line count");
    if (rows != 0 && rows != 8 && rows != 16 && rows != 32)
        return fail(HJM_EINVAL, "line tile rows must be 0 (no override), 8, 16 or 32 (got %d)", rows);
    const auto key = std::make_tuple((int)axis, (int)n, (int64_t)lines);
    if (rows) g_axis_rows[key] = rows;
    else g_axis_rows.erase(key);
    return HJM_OK;
}

hjm_status hjm_get_axis_tile(int32_t axis, int32_t n, int64_t lines, int32_t* rows)
{
    if (!rows) return fail(HJM_EINVAL, "null argument");
    auto it = g_axis_rows.find(std::make_tuple((int)axis, (int)n, (int64_t)lines));
    *rows = it == g_axis_rows.end() ? 0 : it->second;
    return HJM_OK;
}

hjm_status hjm_clear_axis_tiles(void)
{
    g_axis_rows.clear();
    return HJM_OK;
}

hjm_status hjm_set_explicit_chunk(int32_t J)
{
    if (J != 4 && J != 8 && J != 16) return fail(HJM_EINVAL, "explicit chunk must be 4, 8 or 16 (got %d)", J);
    g_exp_J = J;
    return HJM_OK;
}

hjm_status hjm_set_r_fusion(int32_t on)
{
    g_fuse_r = on != 0;
    return HJM_OK;
}

hjm_status hjm_set_exr_window(int32_t on)
{
    g_exr_window = on != 0;
    return HJM_OK;
}

hjm_status hjm_get_exr_window(int32_t* on)
{
    if (!on) return fail(HJM_EINVAL, "null argument");
    *on = g_exr_window ? 1 : 0;
    return HJM_OK;
}

hjm_status hjm_set_v_fold(int32_t on)
{
    g_v_fold = on != 0;
    return HJM_OK;
}

hjm_status hjm_get_v_fold(int32_t* on)
{
    if (!on) return fail(HJM_EINVAL, "null argument");
    *on = g_v_fold ? 1 : 0;
    return HJM_OK;
}

hjm_status hjm_set_y_minors(int32_t on)
{
    g_y_minors = on != 0;
    return HJM_OK;
}

hjm_status hjm_get_y_minors(int32_t* on)
{
    if (!on) return fail(HJM_EINVAL, "null argument");
    *on = g_y_minors ? 1 : 0;
    return HJM_OK;
}

hjm_status hjm_set_batch_streams(int32_t n)
{
    if (n < 1 || n > kMaxBatchLanes) return fail(HJM_EINVAL, "batch streams must be 1..%d (got %d)", kMaxBatchLanes, n);
    g_batch_lanes = n;
    return HJM_OK;
}

hjm_status hjm_get_batch_streams(int32_t* n)
{
    if (!n) return fail(HJM_EINVAL, "null argument");
    *n = g_batch_lanes;
    return HJM_OK;
}

hjm_status hjm_set_batch_share(int32_t on)
{
    g_batch_share = on != 0;
    return HJM_OK;
}

hjm_status hjm_get_batch_share(int32_t* on)
{
    if (!on) return fail(HJM_EINVAL, "null argument");
    *on = g_batch_share ? 1 : 0;
    return HJM_OK;
}

hjm_status hjm_get_r_fusion(int32_t* on)
{
    if (!on) return fail(HJM_EINVAL, "null argument");
    *on = g_fuse_r ? 1 : 0;
    return HJM_OK;
}

hjm_status hjm_get_explicit_chunk(int32_t* J)
{
    if (!J) return fail(HJM_EINVAL, "null argument");
    *J = g_exp_J;
    return HJM_OK;
}

hjm_status hjm_get_line_tile(int32_t* r_rows, int32_t* v_rows, int32_t* y_rows)
{
    if (!r_rows || !v_rows || !y_rows) return fail(HJM_EINVAL, "null argument");
    *r_rows = g_rows[0];
    *v_rows = g_rows[1];
    *y_rows = g_rows[2];
    return HJM_OK;
}

hjm_status hjm_workspace_bytes(const hjm_axis ax[3], int32_t n_steps, size_t* bytes)
{
    if (!ax || !bytes) return fail(HJM_EINVAL, "null argument");
    hjm_status st = validate_axes(ax);
    if (st) return st;
    if (n_steps <= 0) return fail(HJM_EINVAL, "n_steps must be > 0");
    *bytes = grid_layout(ax, n_steps).total;
    return HJM_OK;
}

hjm_status hjm_scheme_workspace_bytes(const hjm_axis ax[3], int32_t n_steps, const hjm_scheme* scheme,
                                      size_t* bytes)
{
    if (!ax || !bytes) return fail(HJM_EINVAL, "null argument");
    hjm_status st = validate_scheme(scheme);
    if (st) return st;
    st = validate_axes(ax);
    if (st) return st;
    if (n_steps <= 0) return fail(HJM_EINVAL, "n_steps must be > 0");
    *bytes = grid_layout(ax, n_steps, scheme->kind != HJM_SCHEME_DOUGLAS).total;
    return HJM_OK;
}

hjm_status hjm_grid_create(const hjm_axis ax[3], const hjm_model* model, const hjm_payoff* payoff, int32_t n_steps,
                           void* d_workspace, size_t ws_bytes, void* hip_stream, hjm_grid** out)
{
    const hjm_scheme douglas{HJM_SCHEME_DOUGLAS, 0, 0.5};
    return hjm_grid_create_scheme(ax, model, payoff, &douglas, n_steps, d_workspace, ws_bytes, hip_stream, out);
}

hjm_status hjm_grid_create_scheme(const hjm_axis ax[3], const hjm_model* model, const hjm_payoff* payoff,
                                  const hjm_scheme* scheme, int32_t n_steps, void* d_workspace, size_t ws_bytes,
                                  void* hip_stream, hjm_grid** out)
{
    if (!out) return fail(HJM_EINVAL, "null output handle");
    *out = nullptr;
    hjm_status st = validate_problem(ax, model, payoff, n_steps);
    if (st) return st;
    st = validate_scheme(scheme);
    if (st) return st;
    Plan plan;
    st = grid_plan(ax, *model, *payoff, *scheme, n_steps, &plan);
    if (st) return st;
    const bool corr = scheme->kind != HJM_SCHEME_DOUGLAS;
    if (!d_workspace) return fail(HJM_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256) return fail(HJM_EINVAL, "workspace must be 256-byte aligned");
    const GridLayout gl = grid_layout(ax, n_steps, corr);
    if (ws_bytes < gl.total) return fail(HJM_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, gl.total);
    hjm_grid* g = new (std::nothrow) hjm_grid;
    if (!g) return fail(HJM_EINVAL, "host allocation failed");
    st = grid_init(g, ax, *model, *payoff, *scheme, n_steps, plan, reinterpret_cast<char*>(d_workspace), gl,
                   reinterpret_cast<hipStream_t>(hip_stream), nullptr);
    if (st) {
        delete g;
        return st;
    }
    *out = g;
    return HJM_OK;
}

hjm_status hjm_adi_step(hjm_grid* g, int32_t k)
{
    if (!g) return fail(HJM_EINVAL, "null grid");
    if (k < 0) return fail(HJM_EINVAL, "negative step count");
    if (g->step + k > g->n_steps)
        return fail(HJM_ESTATE, "%d more steps would pass n_steps=%d (at step %lld)", k, g->n_steps, (long long)g->step);
    const Plan& p = g->plan;
    const bool split = p.r_mode == R_SPLIT;
    for (int32_t c = 0; c < k; ++c) {
        const int n = (int)g->step;
        // one sweep sequence (Douglas), two (the Craig-Sneyd family: the
        // second on the stage-2 descriptor) or 1 + af_iters (Huang)
        const int n_seq = !g->corr ? 1 : (g->scheme.kind == HJM_SCHEME_HUANG ? 1 + g->scheme.af_iters : 2);
        for (int q = 0; q < n_seq * HJM_N_PASSES; ++q) {
            const int pass = q % HJM_N_PASSES;
            const bool st2 = q >= HJM_N_PASSES;
            const bool last_seq = q >= (n_seq - 1) * HJM_N_PASSES;
            const SolveDesc* dd = g->d_desc + (st2 ? 1 : 0);
            if (pass == 1 && !split) continue;
            hipError_t e = hipSuccess;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (g->profile) {
                if (g->events.size() < 2 * (g->ev_used + 1)) {
                    for (int q = 0; q < 2 && !e; ++q) {
                        hipEvent_t ev;
                        e = hipEventCreate(&ev);
                        if (!e) g->events.push_back(ev);
                    }
                    g->ev_pass.resize(g->events.size() / 2);
                }
                if (e) return hip_fail(e, "hjm_adi_step (profile events)");
                e0 = g->events[2 * g->ev_used];
                e1 = g->events[2 * g->ev_used + 1];
                g->ev_pass[g->ev_used] = pass;
                set_launch_events(e0, e1);
            }
            if (pass == 0 && split) e = launch_exp(p.exp_J, dd, nullptr, p.exp_tiles, n, g->stream, st2);
            else if (pass == 0 && p.r_mode == R_FUSED)
                e = launch_exr(p.rs_rows, dd, nullptr, p.exr_tiles, n, p.exr_lds, g->stream, st2, p.exr_win, p.v_fold);
            else if (pass == 0) e = launch_xr(g->rows[0], dd, nullptr, p.r_tiles, n, p.r_lds, g->stream);
            else if (pass == 1) e = launch_rs(p.rs_rows, dd, nullptr, p.rs_tiles, n, g->ax[0].n, g->stream);
            else if (pass == 2 && p.v_fold) e = launch_vfix(dd, nullptr, p.vs_tiles, p.vs_S, g->stream);
            else if (pass == 2 && p.vs_rows) e = launch_vs(p.vs_rows, dd, nullptr, p.vs_tiles, p.vs_S, g->stream);
            else if (pass == 2) e = launch_v(g->rows[1], dd, nullptr, p.v_tiles, p.v_lds, g->stream);
            else if (p.yc_rows)
                e = launch_yc(p.yc_rows, dd, nullptr, p.yc_tiles, p.yc_S, g->stream,
                              !g->corr ? 0 : (!st2 ? 1 : (!last_seq ? 3 : (g->desc2.hv ? 2 : 0))), p.y_minors,
                              p.v_fold);
            else e = launch_yu(g->rows[2], dd, nullptr, p.y_tiles, p.y_lds, g->stream);
            if (e) return hip_fail(e, "hjm_adi_step");
            if (g->profile) {
                set_launch_events(nullptr, nullptr);  // a launch with no tiles records nothing
                g->ev_used += 1;
            }
        }
        g->step += 1;
    }
    return HJM_OK;
}

hjm_status hjm_price(hjm_grid* g, double r0, double v0, double* out)
{
    if (!out) return fail(HJM_EINVAL, "null argument");
    double three[3];
    hjm_status st = hjm_price_greeks(g, r0, v0, three);
    if (st) return st;
    *out = three[0];
    return HJM_OK;
}

hjm_status hjm_price_greeks(hjm_grid* g, double r0, double v0, double out[3])
{
    if (!g || !out) return fail(HJM_EINVAL, "null argument");
    if (g->step != g->n_steps)
        return fail(HJM_ESTATE, "price needs all %d steps (taken %lld)", g->n_steps, (long long)g->step);
    hjm_status st = make_readout(g->ax, r0, v0, 0, &g->rq);
    if (st) return st;
    hipError_t e;
    if ((e = hipMemcpyAsync(g->d_rq, &g->rq, sizeof g->rq, hipMemcpyHostToDevice, g->stream)) ||
        (e = launch_health(g->d_desc, 1, (int64_t)g->ax[0].n * g->ax[1].n * g->ax[2].n, g->stream)) ||
        (e = launch_readout(g->d_desc, g->d_rq, 1, g->d_out, g->stream)) ||
        (e = hipMemcpyAsync(g->out_host, g->d_out, sizeof(double) * 3, hipMemcpyDeviceToHost, g->stream)) ||
        (e = hipMemcpyAsync(&g->flag_host, g->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream)) ||
        (e = hipStreamSynchronize(g->stream)))
        return hip_fail(e, "hjm_price");
    if (g->flag_host) return fail(HJM_ENUMERIC, "non-finite value or non-positive pivot in the solve");
    for (int q = 0; q < 3; ++q) out[q] = g->out_host[q];
    return HJM_OK;
}

hjm_status hjm_grid_solution(hjm_grid* g, double** d_U, int64_t* step)
{
    if (!g || !d_U || !step) return fail(HJM_EINVAL, "null argument");
    *d_U = g->desc.U;
    *step = g->step;
    return HJM_OK;
}

hjm_status hjm_grid_set_step(hjm_grid* g, int64_t step)
{
    if (!g) return fail(HJM_EINVAL, "null grid");
    if (step < 0 || step > g->n_steps) return fail(HJM_EINVAL, "step %lld outside [0, %d]", (long long)step, g->n_steps);
    g->step = step;
    return HJM_OK;
}

hjm_status hjm_grid_destroy(hjm_grid* g)
{
    delete g;
    return HJM_OK;
}

hjm_status hjm_grid_plan(const hjm_grid* g, int32_t plan[10])
{
    if (!g || !plan) return fail(HJM_EINVAL, "null argument");
    for (int q = 0; q < 10; ++q) plan[q] = 0;
    plan[0] = g->plan.r_mode;
    plan[1] = g->plan.rs_rows;
    plan[2] = g->rows[0];
    plan[3] = g->rows[1];
    plan[4] = g->rows[2];
    plan[5] = g->plan.vs_rows;
    plan[6] = g->plan.yc_rows;
    plan[7] = g->scheme.kind;
    plan[8] = g->plan.y_minors ? 1 : 0;
    plan[9] = g->plan.v_fold ? 1 : 0;
    return HJM_OK;
}

hjm_status hjm_grid_profile(hjm_grid* g, int32_t enable)
{
    if (!g) return fail(HJM_EINVAL, "null grid");
    g->profile = enable != 0;
    return HJM_OK;
}

hjm_status hjm_grid_profile_read(hjm_grid* g, double ms[HJM_N_PASSES], int64_t launches[HJM_N_PASSES])
{
    if (!g || !ms || !launches) return fail(HJM_EINVAL, "null argument");
    for (int q = 0; q < HJM_N_PASSES; ++q) { ms[q] = 0.0; launches[q] = 0; }
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e) return hip_fail(e, "hjm_grid_profile_read");
    for (size_t u = 0; u < g->ev_used; ++u) {
        float t = 0.0f;
        if ((e = hipEventElapsedTime(&t, g->events[2 * u], g->events[2 * u + 1])))
            return hip_fail(e, "hipEventElapsedTime");
        ms[g->ev_pass[u]] += t;
        launches[g->ev_pass[u]] += 1;
    }
    g->ev_used = 0;
    return HJM_OK;
}

hjm_status hjm_static_scratch_bytes(const hjm_axis ax[3], int32_t n_steps, size_t* bytes)
{
    if (!ax || !bytes) return fail(HJM_EINVAL, "null argument");
    hjm_status st = validate_axes(ax);
    if (st) return st;
    if (n_steps <= 0) return fail(HJM_EINVAL, "n_steps must be > 0");
    *bytes = static_layout(ax, n_steps).total;
    return HJM_OK;
}

hjm_status hjm_price_static(const hjm_axis ax[3], const hjm_model* model, const hjm_payoff* payoff, int32_t n_steps,
                            double r0, double v0, double* d_U, void* hip_stream, double out[3])
{
    if (!out || !d_U) return fail(HJM_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(d_U) % 256) return fail(HJM_EINVAL, "d_U must be 256-byte aligned");
    hjm_status st = validate_problem(ax, model, payoff, n_steps);
    if (st) return st;
    const hjm_scheme douglas{HJM_SCHEME_DOUGLAS, 0, kTheta};
    Plan plan;
    st = grid_plan(ax, *model, *payoff, douglas, n_steps, &plan);
    if (st) return st;
    Readout probe;
    st = make_readout(ax, r0, v0, 0, &probe);  // reject a bad readout point before any device work
    if (st) return st;
    const GridLayout gl = static_layout(ax, n_steps);
    if (gl.total > HJM_STATIC_SCRATCH_BYTES)
        return fail(HJM_ENOMEM, "the solve needs %zu bytes of scratch, more than the %zu of the static array",
                    gl.total, (size_t)HJM_STATIC_SCRATCH_BYTES);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    char* base = nullptr;
    st = static_scratch(stream, &base);
    if (st) return st;
    hjm_grid g;
    st = grid_init(&g, ax, *model, *payoff, douglas, n_steps, plan, base, gl, stream, d_U);
    if (st) return st;
    st = hjm_adi_step(&g, n_steps);
    if (st) return st;
    return hjm_price_greeks(&g, r0, v0, out);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched solves.
// ---------------------------------------------------------------------------
// A batch launches each kernel of a Douglas step once for all the solves
// that use it.  Launch groups: one per (kernel, rows per thread); a group
// holds the (solve, tile) tasks of its solves, ordered by step count (longest
// first) so that the solves still running at step n are a prefix.
enum { G_XR = 0, G_EXR, G_EXP, G_RS, G_V, G_VS, G_YU, G_YC, kGroupKinds };

struct LaunchGroup {
    int kind = 0, rows = 0;   // rows per thread (k_exp: v nodes per thread)
    bool flag = false;        // k_exr: explicit phase from the LDS window; k_yc: pivots formed in the kernel
    int segs = 0;             // k_vs, k_yc: segments per line (one group per count)
    int seq = 0;              // sweep sequence of the step (0; 1.. the stage-2 sequences of a correction scheme)
    int mode = 0;             // k_yc: what the sweep does with D3 (launch_yc's mode)
    bool fold = false;        // the folded v sweep (k_exr, k_vfix in place of k_vs, k_yc)
    size_t off = 0;           // first task in the batch's task array
    std::vector<int2> tasks;
    std::vector<int> cnt;     // active task prefix per step
    std::vector<int64_t> pts; // grid points of the solves active per step
    size_t lds = 0;           // dynamic LDS (k_xr, k_v, k_yu)
    int aux = 0;              // k_rs: largest nr; k_vs: most segments
    int lane = 0;             // the batch stream lane it is launched on
};

struct hjm_batch {
    int n = 0;
    std::vector<hjm_axis> ax;  // 3 per solve
    std::vector<int> n_steps;
    int rows[3];
    hipStream_t stream = nullptr;
    char* base = nullptr;
    SolveDesc* d_desc = nullptr;
    int2* d_tasks = nullptr;
    Readout* d_rq = nullptr;
    double* d_out = nullptr;
    int32_t* d_flags = nullptr;
    std::vector<SolveDesc> descs;  // n stage-1 (Douglas) descriptors, then n stage-2 ones (correction schemes)
    std::vector<hjm_scheme> schemes;
    std::vector<std::vector<double>> tables;
    std::vector<int> owner;  // the solve whose tables and y pivots each solve uses (itself, unless shared)
    int n_operators = 0;
    std::vector<LaunchGroup> groups;
    int max_steps = 0;
    int64_t max_points = 0, max_ylines = 0;
    hipGraphExec_t graph = nullptr;
    bool ran = false;
    std::vector<Readout> rq;
    std::vector<int32_t> flags_host;
    // per-kernel timing of the first profile_steps steps of eager runs
    int profile_steps = 0;
    std::vector<hipEvent_t> events;  // pool, 2 per timed launch
    std::vector<int> ev_pass;
    std::vector<int64_t> ev_pts;
    size_t ev_used = 0;
    // stream lanes: the solves are split into n_lanes groups of similar work,
    // each launched on a stream of its own, forked from and joined back to
    // `stream` with events, so that kernels of different groups overlap
    int n_lanes = 1;
    std::vector<hipStream_t> lane_st;
    std::vector<hipEvent_t> fork_ev, join_ev;
    ~hjm_batch()
    {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipEvent_t e : fork_ev) (void)hipEventDestroy(e);
        for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
        for (hipStream_t st : lane_st) (void)hipStreamDestroy(st);
    }
};

namespace {

struct BatchLayout {
    size_t desc, tasks, rq, out, flags, total;
    std::vector<SolveOffsets> s;
};

// Upper bound of the tasks of one solve over every plan it could get.
size_t task_bound(const hjm_axis* a)
{
    const Plan pb = plan_bound(a[0].n, a[1].n, a[2].n);
    // (plus the folded v sweep's k_vfix tasks, one per kBlock v lines)
    return (size_t)std::max(std::max(pb.r_tiles, pb.exp_tiles), pb.exr_tiles) + pb.rs_tiles +
           std::max(pb.v_tiles, pb.vs_tiles) + ((size_t)a[0].n * a[2].n + kBlock - 1) / kBlock +
           std::max(pb.y_tiles, pb.yc_tiles) + (size_t)pb.exp_tiles;
}

// Two solves discretise the same operator (the same coefficient tables and
// y pivots) when they differ at most in the payoff's kind, strike and
// softening: same axes, model (discrete curve values included), expiry,
// bond-factor date and steps.
bool same_operator(const hjm_axis* a, const hjm_model& m, const hjm_payoff& p, int ns, const hjm_axis* b,
                   const hjm_model& q, const hjm_payoff& r, int nt)
{
    if (ns != nt) return false;
    for (int d = 0; d < 3; ++d)
        if (a[d].n != b[d].n || a[d].lo_face != b[d].lo_face || a[d].hi_face != b[d].hi_face ||
            a[d].z_min != b[d].z_min || a[d].z_max != b[d].z_max || a[d].center != b[d].center ||
            a[d].alpha != b[d].alpha)
            return false;
    if (m.kappa != q.kappa || m.theta_v != q.theta_v || m.lambda != q.lambda || m.gamma != q.gamma ||
        m.epsilon != q.epsilon || m.rho != q.rho || m.curve_n != q.curve_n)
        return false;
    if (m.curve_n == 0 && (m.f_level != q.f_level || m.f_slope != q.f_slope || m.f_decay != q.f_decay)) return false;
    for (int i = 0; i < m.curve_n; ++i)
        if (m.curve_t[i] != q.curve_t[i] || m.curve_p[i] != q.curve_p[i]) return false;
    const double pm = p.kind == HJM_BOND ? p.expiry : p.pay, rm = r.kind == HJM_BOND ? r.expiry : r.pay;
    return p.expiry == r.expiry && pm == rm;
}

// A solve that shares another's operator reads that solve's tables and, if
// the pivots are stored (stored_pivots), its y pivots; its own grid,
// Dirichlet increments and flag stay its own.  With the pivots formed in the
// sweep the pivot array stays the solve's own: the folded v sweep keeps its
// per-solve hand-over values there.
void share_operator(SolveDesc& d, const SolveDesc& o, bool stored_pivots)
{
    d.rt = o.rt; d.vt = o.vt; d.yt = o.yt; d.vf = o.vf;
    d.st = o.st; d.rf = o.rf; d.vg = o.vg;
    if (stored_pivots) {
        d.yinv = o.yinv;
        d.ypiv_skip = 1;
    }
}

// Sweep sequences per Douglas step: 1 (Douglas), 2 (the Craig-Sneyd family),
// 1 + q (Huang's correction with q subiterations).
int sweep_sequences(const hjm_scheme& sc)
{
    return sc.kind == HJM_SCHEME_DOUGLAS ? 1 : (sc.kind == HJM_SCHEME_HUANG ? 1 + sc.af_iters : 2);
}

const hjm_scheme kDouglasHalf{HJM_SCHEME_DOUGLAS, 0, kTheta};

// schemes: n entries, or null for Douglas with theta = 1/2 throughout.
BatchLayout batch_layout(int n, const hjm_axis* ax, const int32_t* n_steps, const hjm_scheme* schemes)
{
    Layout L;
    BatchLayout b;
    size_t nt = 0;
    for (int s = 0; s < n; ++s) nt += task_bound(ax + 3 * s) * sweep_sequences(schemes ? schemes[s] : kDouglasHalf);
    b.desc = L.take(sizeof(SolveDesc) * 2 * n);
    b.tasks = L.take(sizeof(int2) * std::max<size_t>(nt, 1));
    b.rq = L.take(sizeof(Readout) * n);
    b.out = L.take(sizeof(double) * 3 * n);
    b.flags = L.take(sizeof(int32_t) * n);
    b.s.resize(n);
    for (int s = 0; s < n; ++s)
        b.s[s] = layout_solve(L, ax + 3 * s, n_steps[s], schemes && schemes[s].kind != HJM_SCHEME_DOUGLAS);
    b.total = L.off;
    return b;
}

hipError_t launch_group(const hjm_batch* b, const LaunchGroup& g, int step, hipStream_t st)
{
    const int nt = g.cnt[step];
    const int2* t = b->d_tasks + g.off;
    switch (g.kind) {
    case G_XR: return launch_xr(g.rows, b->d_desc, t, nt, step, g.lds, st);
    case G_EXR: return launch_exr(g.rows, b->d_desc, t, nt, step, g.lds, st, g.seq > 0, g.flag, g.fold);
    case G_EXP: return launch_exp(g.rows, b->d_desc, t, nt, step, st, g.seq > 0);
    case G_RS: return launch_rs(g.rows, b->d_desc, t, nt, step, g.aux, st);
    case G_V: return launch_v(g.rows, b->d_desc, t, nt, g.lds, st);
    case G_VS: return g.fold ? launch_vfix(b->d_desc, t, nt, g.segs, st) : launch_vs(g.rows, b->d_desc, t, nt, g.aux, st);
    case G_YU: return launch_yu(g.rows, b->d_desc, t, nt, g.lds, st);
    default: return launch_yc(g.rows, b->d_desc, t, nt, g.aux, st, g.mode, g.flag, g.fold);
    }
}

int group_pass(int kind)
{
    switch (kind) {
    case G_XR: case G_EXR: case G_EXP: return 0;
    case G_RS: return 1;
    case G_V: case G_VS: return 2;
    default: return 3;
    }
}

// Enqueue a whole solve of the batch.  Steps before fork_at run on the
// batch's stream one group after another (the timed steps: each launch alone
// on the GPU); from fork_at on, each lane's launches go to its own stream.
hjm_status batch_enqueue(hjm_batch* b, bool timed)
{
    hipError_t e;
    if ((e = launch_terminal(b->d_desc, b->n, b->max_points, b->stream))) return hip_fail(e, "batch terminal");
    const int fork_at = b->n_lanes < 2 ? b->max_steps : (timed ? std::min(b->profile_steps, b->max_steps) : 0);
    for (int step = 0; step < b->max_steps; ++step) {
        if (step == fork_at) {
            if ((e = hipEventRecord(b->fork_ev[0], b->stream))) return hip_fail(e, "batch fork");
            for (hipStream_t st : b->lane_st)
                if ((e = hipStreamWaitEvent(st, b->fork_ev[0], 0))) return hip_fail(e, "batch fork");
        }
        for (const LaunchGroup& g : b->groups) {  // lane by lane, each in step-pass order
            const hipStream_t st = step < fork_at ? b->stream : b->lane_st[g.lane];
            const bool time_it = timed && step < b->profile_steps && g.cnt[step] > 0;
            if (time_it) {
                if (b->events.size() < 2 * (b->ev_used + 1)) {
                    for (int q = 0; q < 2; ++q) {
                        hipEvent_t ev;
                        if ((e = hipEventCreate(&ev))) return hip_fail(e, "batch profile events");
                        b->events.push_back(ev);
                    }
                    b->ev_pass.resize(b->events.size() / 2);
                    b->ev_pts.resize(b->events.size() / 2);
                }
                b->ev_pass[b->ev_used] = group_pass(g.kind);
                b->ev_pts[b->ev_used] = g.pts[step];
                set_launch_events(b->events[2 * b->ev_used], b->events[2 * b->ev_used + 1]);
            }
            e = launch_group(b, g, step, st);
            if (time_it) {
                set_launch_events(nullptr, nullptr);
                b->ev_used += 1;
            }
            if (e) return hip_fail(e, "batch step");
        }
    }
    if (fork_at < b->max_steps)
        for (size_t l = 0; l < b->lane_st.size(); ++l)
            if ((e = hipEventRecord(b->join_ev[l], b->lane_st[l])) ||
                (e = hipStreamWaitEvent(b->stream, b->join_ev[l], 0)))
                return hip_fail(e, "batch join");
    return HJM_OK;
}

}  // namespace

extern "C" {

hjm_status hjm_batch_scheme_workspace_bytes(int32_t n, const hjm_axis* ax, const int32_t* n_steps,
                                            const hjm_scheme* schemes, size_t* bytes)
{
    if (n <= 0 || !ax || !n_steps || !bytes) return fail(HJM_EINVAL, "invalid batch arguments");
    for (int s = 0; s < n; ++s) {
        hjm_status st = validate_axes(ax + 3 * s);
        if (st) return fail(st, "solve %d: %s", s, g_last_error.c_str());
        if (n_steps[s] <= 0) return fail(HJM_EINVAL, "solve %d: n_steps must be > 0", s);
        if (schemes && (st = validate_scheme(schemes + s))) return fail(st, "solve %d: %s", s, g_last_error.c_str());
    }
    *bytes = batch_layout(n, ax, n_steps, schemes).total;
    return HJM_OK;
}

hjm_status hjm_batch_workspace_bytes(int32_t n, const hjm_axis* ax, const int32_t* n_steps, size_t* bytes)
{
    return hjm_batch_scheme_workspace_bytes(n, ax, n_steps, nullptr, bytes);
}

hjm_status hjm_batch_create(int32_t n, const hjm_axis* ax, const hjm_model* model, const hjm_payoff* payoff,
                            const int32_t* n_steps, void* d_workspace, size_t ws_bytes, void* hip_stream,
                            hjm_batch** out)
{
    return hjm_batch_create_scheme(n, ax, model, payoff, nullptr, n_steps, d_workspace, ws_bytes, hip_stream, out);
}

hjm_status hjm_batch_create_scheme(int32_t n, const hjm_axis* ax, const hjm_model* model, const hjm_payoff* payoff,
                                   const hjm_scheme* schemes, const int32_t* n_steps, void* d_workspace,
                                   size_t ws_bytes, void* hip_stream, hjm_batch** out)
{
    if (!out) return fail(HJM_EINVAL, "null output handle");
    *out = nullptr;
    if (n <= 0 || !ax || !model || !payoff || !n_steps) return fail(HJM_EINVAL, "invalid batch arguments");
    std::vector<Plan> plans(n);
    for (int s = 0; s < n; ++s) {
        hjm_status st = validate_problem(ax + 3 * s, model + s, payoff + s, n_steps[s]);
        if (!st && schemes) st = validate_scheme(schemes + s);
        // the solve's kernel variants (a correction scheme needs the lane-split
        // r solve and the y solve on reciprocal pivots)
        if (!st) st = grid_plan(ax + 3 * s, model[s], payoff[s], schemes ? schemes[s] : kDouglasHalf, n_steps[s],
                                &plans[s]);
        if (st) return fail(st, "solve %d: %s", s, g_last_error.c_str());
    }
    if (!d_workspace) return fail(HJM_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256) return fail(HJM_EINVAL, "workspace must be 256-byte aligned");
    const BatchLayout bl = batch_layout(n, ax, n_steps, schemes);
    if (ws_bytes < bl.total) return fail(HJM_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, bl.total);
    hjm_batch* b = new (std::nothrow) hjm_batch;
    if (!b) return fail(HJM_EINVAL, "host allocation failed");
    b->n = n;
    b->schemes.assign(n, kDouglasHalf);
    if (schemes) b->schemes.assign(schemes, schemes + n);
    b->ax.assign(ax, ax + 3 * n);
    b->n_steps.assign(n_steps, n_steps + n);
    std::memcpy(b->rows, g_rows, sizeof b->rows);
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->base = reinterpret_cast<char*>(d_workspace);
    b->d_desc = reinterpret_cast<SolveDesc*>(b->base + bl.desc);
    b->d_tasks = reinterpret_cast<int2*>(b->base + bl.tasks);
    b->d_rq = reinterpret_cast<Readout*>(b->base + bl.rq);
    b->d_out = reinterpret_cast<double*>(b->base + bl.out);
    b->d_flags = reinterpret_cast<int32_t*>(b->base + bl.flags);
    b->descs.resize(2 * n);
    b->tables.resize(n);
    b->owner.resize(n);
    for (int s = 0; s < n; ++s) {
        const hjm_axis* a = ax + 3 * s;
        const hjm_scheme& sc = b->schemes[s];
        const bool corr = sc.kind != HJM_SCHEME_DOUGLAS;
        // the correction schemes keep the stored y pivots (as on a grid)
        if (corr) plans[s].y_minors = false;
        int own = s;
        // one operator: the same tables (theta folded in) and the same pivot form
        for (int q = 0; g_batch_share && q < s && own == s; ++q)
            if (b->owner[q] == q && b->schemes[q].theta == sc.theta &&
                (b->schemes[q].kind != HJM_SCHEME_DOUGLAS) == corr &&
                same_operator(ax + 3 * q, model[q], payoff[q], n_steps[q], a, model[s], payoff[s], n_steps[s]))
                own = q;
        b->owner[s] = own;
        if (own == s) {
            build_tables(a, model[s], payoff[s], n_steps[s], plans[s], b->tables[s], sc.theta);
            b->n_operators += 1;
        } else {
            plans[s] = plans[own];
        }
        fill_desc(b->descs[s], a, model[s], payoff[s], n_steps[s], plans[s], b->base, bl.s[s], b->d_flags + s,
                  sc.theta);
        if (own != s) share_operator(b->descs[s], b->descs[own], !plans[s].y_minors);
        if (corr) {
            b->descs[s].stage = 1;
            scheme_stage2(b->descs[n + s], b->descs[s], sc, reinterpret_cast<double*>(b->base + bl.s[s].E));
        }
        b->max_steps = std::max(b->max_steps, n_steps[s]);
        b->max_points = std::max<int64_t>(b->max_points, (int64_t)a[0].n * a[1].n * a[2].n);
        b->max_ylines = std::max<int64_t>(b->max_ylines, (int64_t)a[0].n * a[1].n);
    }
    std::vector<int> order(n);
    for (int s = 0; s < n; ++s) order[s] = s;
    // longest first; the right-hand sides of one operator next to each other
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return n_steps[a] != n_steps[c] ? n_steps[a] > n_steps[c] : b->owner[a] < b->owner[c];
    });
    // stream lanes: solves by decreasing work (points x steps) dealt to the
    // lanes in snake order, which balances the lanes' work
    b->n_lanes = std::max(1, std::min(g_batch_lanes, n));
    std::vector<int> lane_of(n, 0);
    {
        std::vector<int> by_work(order);
        auto work = [&](int q) { return (double)ax[3 * q].n * ax[3 * q + 1].n * ax[3 * q + 2].n * n_steps[q]; };
        std::stable_sort(by_work.begin(), by_work.end(), [&](int a, int c) { return work(a) > work(c); });
        for (int r = 0; r < n; ++r) {
            const int m = r % (2 * b->n_lanes);
            lane_of[by_work[r]] = m < b->n_lanes ? m : 2 * b->n_lanes - 1 - m;
        }
    }
    // (lane, sequence, kind, variant) -> group, created lane by lane, and in
    // a lane by sweep sequence and pass, the order in which a step launches
    // them on the lane's stream
    auto group = [&](int lane, int seq, int kind, int rows, bool flag, int segs, int mode, bool fold) -> LaunchGroup& {
        for (LaunchGroup& g : b->groups)
            if (g.lane == lane && g.seq == seq && g.kind == kind && g.rows == rows && g.flag == flag &&
                g.segs == segs && g.mode == mode && g.fold == fold)
                return g;
        b->groups.emplace_back();
        LaunchGroup& g = b->groups.back();
        g.lane = lane;
        g.seq = seq;
        g.kind = kind;
        g.rows = rows;
        g.flag = flag;
        g.segs = segs;
        g.mode = mode;
        g.fold = fold;
        g.cnt.assign(b->max_steps, 0);
        g.pts.assign(b->max_steps, 0);
        return g;
    };
    for (int lane = 0; lane < b->n_lanes; ++lane) {
        std::vector<int> lane_order;
        int lane_seqs = 1;
        for (int s : order)
            if (lane_of[s] == lane) {
                lane_order.push_back(s);
                lane_seqs = std::max(lane_seqs, sweep_sequences(b->schemes[s]));
            }
        for (int seq = 0; seq < lane_seqs; ++seq) {
            // the lane's solves with this sweep sequence (a prefix of the
            // order still holds: the order is by steps within every subset)
            std::vector<int> seq_order;
            for (int s : lane_order)
                if (seq < sweep_sequences(b->schemes[s])) seq_order.push_back(s);
            for (int kind = 0; kind < kGroupKinds; ++kind)
                for (size_t oi = 0; oi < seq_order.size(); ++oi) {
                    const int s = seq_order[oi];
                    const Plan& pl = plans[s];
                    const hjm_scheme& sc = b->schemes[s];
                    const bool corr = sc.kind != HJM_SCHEME_DOUGLAS;
                    const int nseq = sweep_sequences(sc);
                    // the descriptor of this sequence: stage 1, or stage 2 (the
                    // corrected start, the sweeps of E) at n + s
                    const int di = seq == 0 ? s : n + s;
                    const int ns = n_steps[s];
                    int rows = 0, tiles = 0, segs = 0, mode = 0;
                    bool flag = false;
                    size_t lds = 0;
                    int aux = 0;
                    switch (kind) {
                    case G_XR:
                        if (pl.r_mode == R_SPIKE || pl.r_mode == R_CHAIN) { rows = pl.rows[0]; tiles = pl.r_tiles; lds = pl.r_lds; }
                        break;
                    case G_EXR:
                        // the window form for the predictor only (the corrected
                        // start keeps the per-lane loads)
                        if (pl.r_mode == R_FUSED) {
                            rows = pl.rs_rows;
                            flag = pl.exr_win && seq == 0;
                            tiles = pl.exr_tiles;
                            lds = pl.exr_lds;
                        }
                        break;
                    case G_EXP: if (pl.r_mode == R_SPLIT) { rows = pl.exp_J; tiles = pl.exp_tiles; } break;
                    case G_RS: if (pl.r_mode == R_SPLIT) { rows = pl.rs_rows; tiles = pl.rs_tiles; aux = ax[3 * s].n; } break;
                    case G_V: if (!pl.vs_rows) { rows = pl.rows[1]; tiles = pl.v_tiles; lds = pl.v_lds; } break;
                    // the segmented sweeps run one wave per segment, in workgroups
                    // sized for the group's most segments: solves with fewer
                    // segments would leave waves idle for the workgroup's whole
                    // life, so each segment count is a group of its own
                    case G_VS:
                        // (folded: k_vfix, vs_tiles tasks of kBlock v lines)
                        if (pl.vs_rows) { rows = pl.vs_rows; segs = pl.vs_S; tiles = pl.vs_tiles; aux = pl.vs_S; }
                        break;
                    case G_YU: if (!pl.yc_rows) { rows = pl.rows[2]; tiles = pl.y_tiles; lds = pl.y_lds; } break;
                    default:
                        if (pl.yc_rows) {
                            rows = pl.yc_rows;
                            flag = pl.y_minors;
                            segs = pl.yc_S;
                            tiles = pl.yc_tiles;
                            aux = pl.yc_S;
                            // as on a grid: U += D3 (Douglas, the last CS / MCS
                            // sequence), D3 stays in D (stage 1), U += D3 + E3 (HV,
                            // Huang's last), D3 += E3 (Huang's intermediate ones)
                            mode = !corr ? 0 : (seq == 0 ? 1 : (seq < nseq - 1 ? 3 : (sc.kind == HJM_SCHEME_HV ||
                                                                                      sc.kind == HJM_SCHEME_HUANG ? 2 : 0)));
                        }
                        break;
                    }
                    if (!tiles) continue;
                    LaunchGroup& g = group(lane, seq, kind, rows, flag, segs, mode, pl.v_fold && (kind == G_EXR ||
                                                                                       kind == G_VS || kind == G_YC));
                    if (kind != G_YC) {
                        for (int t = 0; t < tiles; ++t) g.tasks.push_back(make_int2(di, t));
                    } else if (oi == 0 || b->owner[seq_order[oi - 1]] != b->owner[s]) {
                        // the right-hand sides of one operator (adjacent in the
                        // order, same plan and steps) read one table (and, stored,
                        // one pivot array): their tiles go in 8 at a time, each
                        // block for every right-hand side in turn, so that tasks
                        // t, t + 8, ... (dealt to one XCD) meet in that XCD's cache
                        std::vector<int> rhs{s};
                        for (size_t oj = oi + 1; oj < seq_order.size() && b->owner[seq_order[oj]] == b->owner[s]; ++oj)
                            rhs.push_back(seq_order[oj]);
                        for (int tb = 0; tb < tiles; tb += 8)
                            for (int r : rhs)
                                for (int x = tb; x < std::min(tiles, tb + 8); ++x)
                                    g.tasks.push_back(make_int2(seq == 0 ? r : n + r, x));
                    }
                    const int64_t pts = (int64_t)ax[3 * s].n * ax[3 * s + 1].n * ax[3 * s + 2].n;
                    for (int step = 0; step < ns; ++step) {
                        g.cnt[step] += tiles;
                        g.pts[step] += pts;
                    }
                    g.lds = std::max(g.lds, lds);
                    g.aux = std::max(g.aux, aux);
                }
        }
    }
    std::vector<int2> all;
    for (LaunchGroup& g : b->groups) {
        g.off = all.size();
        all.insert(all.end(), g.tasks.begin(), g.tasks.end());
    }
    hipError_t e = init_kernel_attributes();
    if (b->n_lanes > 1) {
        // default priority streams; events without timing (fork and join only)
        for (int l = 0; l < b->n_lanes && !e; ++l) {
            hipStream_t st = nullptr;
            hipEvent_t f = nullptr, j = nullptr;
            if (!(e = hipStreamCreate(&st))) b->lane_st.push_back(st);
            if (!e && !(e = hipEventCreateWithFlags(&f, hipEventDisableTiming))) b->fork_ev.push_back(f);
            if (!e && !(e = hipEventCreateWithFlags(&j, hipEventDisableTiming))) b->join_ev.push_back(j);
        }
    }
    if (!e) e = hipMemcpyAsync(b->d_desc, b->descs.data(), sizeof(SolveDesc) * 2 * n, hipMemcpyHostToDevice, b->stream);
    if (!e && !all.empty())
        e = hipMemcpyAsync(b->d_tasks, all.data(), sizeof(int2) * all.size(), hipMemcpyHostToDevice, b->stream);
    int64_t max_gd = 0;
    for (int s = 0; s < n && !e; ++s) {
        if (b->owner[s] == s) e = upload_tables(b->descs[s], b->tables[s], b->stream);
        max_gd = std::max<int64_t>(max_gd, (int64_t)(2 * ax[3 * s + 2].n + ax[3 * s].n) * n_steps[s]);
    }
    if (!e) e = launch_gd(b->d_desc, n, max_gd, b->stream);
    bool stored_pivots = false;
    for (int s = 0; s < n; ++s) stored_pivots = stored_pivots || (plans[s].yc_rows && !plans[s].y_minors);
    if (!e && stored_pivots) e = launch_ypiv(b->d_desc, n, b->max_ylines, b->stream);
    if (!e) e = hipStreamSynchronize(b->stream);
    if (e) {
        delete b;
        return hip_fail(e, "hjm_batch_create");
    }
    *out = b;
    return HJM_OK;
}

hjm_status hjm_batch_operators(const hjm_batch* b, int32_t* n_operators)
{
    if (!b || !n_operators) return fail(HJM_EINVAL, "null argument");
    *n_operators = b->n_operators;
    return HJM_OK;
}

hjm_status hjm_batch_run(hjm_batch* b, int32_t use_graph)
{
    if (!b) return fail(HJM_EINVAL, "null batch");
    if (!use_graph) {
        hjm_status st = batch_enqueue(b, true);
        if (st) return st;
        b->ran = true;
        return HJM_OK;
    }
    if (!b->stream) return fail(HJM_EINVAL, "graph mode needs a non-null stream");
    hipError_t e;
    if (!b->graph) {
        hipGraph_t graph = nullptr;
        if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)))
            return hip_fail(e, "hipStreamBeginCapture");
        hjm_status st = batch_enqueue(b, false);
        e = hipStreamEndCapture(b->stream, &graph);
        if (st) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e) {
            b->graph = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
    }
    if ((e = hipGraphLaunch(b->graph, b->stream))) return hip_fail(e, "hipGraphLaunch");
    b->ran = true;
    return HJM_OK;
}

hjm_status hjm_batch_prices(hjm_batch* b, const double* r0, const double* v0, double* out)
{
    if (!b || !out) return fail(HJM_EINVAL, "null argument");
    std::vector<double> three(3 * (size_t)b->n);
    hjm_status st = hjm_batch_greeks(b, r0, v0, three.data());
    if (st) return st;
    for (int s = 0; s < b->n; ++s) out[s] = three[3 * (size_t)s];
    return HJM_OK;
}

hjm_status hjm_batch_greeks(hjm_batch* b, const double* r0, const double* v0, double* out)
{
    if (!b || !r0 || !v0 || !out) return fail(HJM_EINVAL, "null argument");
    if (!b->ran) return fail(HJM_ESTATE, "hjm_batch_run has not been called");
    b->rq.resize(b->n);
    b->flags_host.assign(b->n, 0);
    for (int s = 0; s < b->n; ++s) {
        hjm_status st = make_readout(&b->ax[3 * s], r0[s], v0[s], s, &b->rq[s]);
        if (st) return fail(st, "solve %d: %s", s, g_last_error.c_str());
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(b->d_rq, b->rq.data(), sizeof(Readout) * b->n, hipMemcpyHostToDevice, b->stream)) ||
        (e = launch_health(b->d_desc, b->n, b->max_points, b->stream)) ||
        (e = launch_readout(b->d_desc, b->d_rq, b->n, b->d_out, b->stream)) ||
        (e = hipMemcpyAsync(out, b->d_out, sizeof(double) * 3 * b->n, hipMemcpyDeviceToHost, b->stream)) ||
        (e = hipMemcpyAsync(b->flags_host.data(), b->d_flags, sizeof(int32_t) * b->n, hipMemcpyDeviceToHost,
                            b->stream)) ||
        (e = hipStreamSynchronize(b->stream)))
        return hip_fail(e, "hjm_batch_greeks");
    for (int s = 0; s < b->n; ++s)
        if (b->flags_host[s]) return fail(HJM_ENUMERIC, "solve %d: non-finite value or non-positive pivot", s);
    return HJM_OK;
}

hjm_status hjm_batch_profile(hjm_batch* b, int32_t steps)
{
    if (!b) return fail(HJM_EINVAL, "null batch");
    if (steps < 0) return fail(HJM_EINVAL, "negative step count");
    b->profile_steps = steps;
    return HJM_OK;
}

hjm_status hjm_batch_profile_read(hjm_batch* b, double ms[HJM_N_PASSES], int64_t launches[HJM_N_PASSES],
                                  int64_t points[HJM_N_PASSES])
{
    if (!b || !ms || !launches || !points) return fail(HJM_EINVAL, "null argument");
    for (int q = 0; q < HJM_N_PASSES; ++q) { ms[q] = 0.0; launches[q] = 0; points[q] = 0; }
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e) return hip_fail(e, "hjm_batch_profile_read");
    for (size_t u = 0; u < b->ev_used; ++u) {
        float t = 0.0f;
        if ((e = hipEventElapsedTime(&t, b->events[2 * u], b->events[2 * u + 1])))
            return hip_fail(e, "hipEventElapsedTime");
        ms[b->ev_pass[u]] += t;
        launches[b->ev_pass[u]] += 1;
        points[b->ev_pass[u]] += b->ev_pts[u];
    }
    b->ev_used = 0;
    return HJM_OK;
}

hjm_status hjm_batch_destroy(hjm_batch* b)
{
    if (b && b->graph) (void)hipGraphExecDestroy(b->graph);
    delete b;
    return HJM_OK;
}

}  // extern "C"
