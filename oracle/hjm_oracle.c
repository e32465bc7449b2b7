/*
 * CPU oracle for the single-factor HJM model with stochastic volatility
 * (Valero, Torrealba, Lacasa, Fraysse, "Fast resolution of a single factor
 * Heath-Jarrow-Morton model with stochastic volatility").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library: every formula below is
 * written out again from the paper, in plain FP64 loops, with no blocking,
 * fusion or reordering beyond what the paper's algorithm states.
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 *
 * What it computes (the canonical discrete scheme):
 *   - discount curve, forward curve and its slope (section 2; parametric curve);
 *   - the bond reconstruction formula, eq. (gs) of section 3.1;
 *   - terminal data and Dirichlet data for the bond, caplet, floorlet and the
 *     linear (forward) payoff, section 3.2;
 *   - the hyperbolic (sinh) mesh of eq. (metrica), section 4.3 / 7.1, and the
 *     metric-transformed coefficients g1..g6 (section 4.3), in physical units;
 *   - the centred stencils of eq. (esquema) and the split operators
 *     L_r, L_v, L_y, L_rv of eq. (discreta) / (adiecu), section 5;
 *   - one-sided second-order rows at outflow faces (section 7.3);
 *   - tridiagonal line solves by Gaussian elimination without pivoting
 *     (the Thomas algorithm, section 5);
 *   - the Douglas ADI step of section 5.1 with theta = 1/2, and the three
 *     correction schemes of the same family (Craig-Sneyd, which the paper
 *     tried, modified Craig-Sneyd, Hundsdorfer-Verwer) with any theta;
 *   - Huang's approximate-factorisation correction (section 5.1):
 *     subiterations of the factored operator on the residual of the unsplit
 *     theta scheme, starting from the Douglas increment;
 *   - the readout C(t=0; r0, v0, y=0) by 4-point Lagrange interpolation;
 *   - the Gaussian (gamma = 0, epsilon = 0) caplet closed form used as a pin.
 *
 * Readings of passages that are garbled or silent in the paper (each one is
 * listed with its reason in the design notes):
 *   - centred first difference over 2h and mixed difference over 4 h_x h_z
 *     (section 5, eq. (esquema) prints h and h_x h_z);
 *   - metric Jacobian alpha*cosh(.)*(c2-c1) and second derivative
 *     alpha*sinh(.)*(c2-c1)^2 (section 7.1 prints sinh for the Jacobian);
 *   - g5 divides the v drift by J_v (section 4.3 prints J_r);
 *   - the exponent of r in the coefficients of eq. (1) is gamma;
 *   - the Douglas stages carry the factor theta (section 5.1 drops it);
 *   - every operator, explicit and implicit, is evaluated at t_{n+1/2};
 *   - the reaction term -rC belongs to the r operator;
 *   - n nodes per axis include both end nodes;
 *   - faces: one-sided outflow rows where the drift points out of the domain
 *     in backward time (r = 0, v = 0, v = v_max, y = 0), Dirichlet data from
 *     the closed form at r_max and y_max;
 *   - the computation is done in physical (r, v, y, t) with the mesh, not in
 *     the rescaled variables of section 4.2 (same nodes, same discrete
 *     equations up to rounding).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Problem description (the oracle's own layout; mirrored by its ctypes      */
/* wrapper only).                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n[3];           /* nodes on the r, v, y axes, both end nodes included */
    int face[6];        /* r_lo, r_hi, v_lo, v_hi, y_lo, y_hi: 0 outflow, 1 Dirichlet */
    double geom[3][4];  /* per axis: z_min, z_max, centre K, stretch alpha */
    double kappa;       /* rate mean reversion */
    double theta_v;     /* variance mean reversion */
    double lambda;      /* volatility level */
    double gamma;       /* CEV exponent of r */
    double epsilon;     /* vol of variance */
    double rho;         /* correlation of dW and dZ */
    double f_level, f_slope, f_decay; /* f(0,t) = level + slope*(1 - exp(-decay t)) */
    int kind;           /* 0 bond, 1 caplet, 2 floorlet, 3 linear forward payoff */
    double expiry;      /* T */
    double pay;         /* T_M */
    double strike;      /* K */
    int n_steps;        /* N: dt = T / N */
    int scheme;         /* ORC_DOUGLAS (the paper's), ORC_CS, ORC_MCS, ORC_HV */
    double theta;       /* implicit weight of the line solves (the paper: 1/2) */
    int soften;         /* terminal data averaged over control elements (section 7.2):
                           0 no, 1 every non-Dirichlet node, 2 the nodes whose element the kink crosses */
    int af_iters;       /* ORC_HUANG: correction subiterations after the Douglas increment (>= 1) */
    int curve_n;        /* > 0: discrete curve of curve_n knots replaces f_level/f_slope/f_decay */
    const double* curve_t;  /* maturities, curve_t[0] = 0 */
    const double* curve_p;  /* zero-coupon prices P(0, t_i), curve_p[0] = 1 */
} orc_problem;

#define ORC_OUTFLOW 0
#define ORC_DIRICHLET 1
/* ADI schemes: the paper's Douglas scheme (section 5.1) and the three
   schemes that add a correction stage for the mixed derivative: Craig and
   Sneyd (the paper tried it, section 5.1, without giving its stages), and
   the modified Craig-Sneyd and Hundsdorfer-Verwer schemes (in 't Hout and
   Welfert, "Stability of ADI schemes applied to convection-diffusion
   equations with mixed derivative terms", Appl. Numer. Math. 57 (2007)). */
#define ORC_DOUGLAS 0
#define ORC_CS 1
#define ORC_MCS 2
#define ORC_HV 3
/* Huang's approximate-factorisation correction (section 5.1 mentions trying
   it; it removes the factorisation error of the Douglas step). */
#define ORC_HUANG 4

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Section 2: the initial curve.  f(0,t) = a + b (1 - e^{-c t}).             */
/* Section 6.1: a discrete zero-coupon curve, smoothed by a spline so that   */
/* df(0,t)/dt is continuous.  Here S is the natural cubic spline of          */
/* Y(t) = -ln P(0,t) through the knots (t_i, Y_i): a cubic on each interval, */
/* S, S', S'' continuous at the knots, S'' = 0 at both ends; then            */
/* f(0,t) = S'(t), df(0,t)/dt = S''(t), P(0,t) = exp(-S(t)).  Past the last  */
/* knot S continues as its tangent line (the forward stays at its end value).*/
/* ------------------------------------------------------------------------ */

/* S(t), S'(t), S''(t) from the moments M_i = S''(t_i).  On [t_i, t_{i+1}],
   h = t_{i+1} - t_i, a = (t_{i+1} - t) / h, b = (t - t_i) / h:
     S   = a Y_i + b Y_{i+1} + h^2 ((a^3 - a) M_i + (b^3 - b) M_{i+1}) / 6,
     S'  = (Y_{i+1} - Y_i) / h + h ((1 - 3 a^2) M_i + (3 b^2 - 1) M_{i+1}) / 6,
     S'' = a M_i + b M_{i+1};
   continuity of S' at the inner knots gives, for i = 1 .. n-2,
     h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1}
       = 6 ((Y_{i+1} - Y_i) / h_i - (Y_i - Y_{i-1}) / h_{i-1}),
   with M_0 = M_{n-1} = 0, solved here on every call (Gaussian elimination
   of the tridiagonal system, which is diagonally dominant). */
#define ORC_MAX_KNOTS 64
static void spline_eval(const orc_problem* p, double t, double* S, double* S1, double* S2)
{
    int n = p->curve_n;
    double Y[ORC_MAX_KNOTS], M[ORC_MAX_KNOTS], lo[ORC_MAX_KNOTS], di[ORC_MAX_KNOTS], up[ORC_MAX_KNOTS],
        rhs[ORC_MAX_KNOTS];
    if (n < 2 || n > ORC_MAX_KNOTS) {  /* no such curve: every value is NaN */
        *S = *S1 = *S2 = NAN;
        return;
    }
    for (int i = 0; i < n; ++i) { Y[i] = -log(p->curve_p[i]); M[i] = 0.0; }
    for (int i = 1; i + 1 < n; ++i) {
        double hl = p->curve_t[i] - p->curve_t[i - 1], hr = p->curve_t[i + 1] - p->curve_t[i];
        lo[i] = hl;
        di[i] = 2.0 * (hl + hr);
        up[i] = hr;
        rhs[i] = 6.0 * ((Y[i + 1] - Y[i]) / hr - (Y[i] - Y[i - 1]) / hl);
    }
    for (int i = 2; i + 1 < n; ++i) {      /* forward elimination */
        double w = lo[i] / di[i - 1];
        di[i] -= w * up[i - 1];
        rhs[i] -= w * rhs[i - 1];
    }
    for (int i = n - 2; i >= 1; --i)       /* back substitution, M_{n-1} = 0 */
        M[i] = (rhs[i] - up[i] * M[i + 1]) / di[i];
    double tn = p->curve_t[n - 1];
    if (t >= tn) {
        /* the end: S(t_n) = Y_n, S'(t_n) from the last interval (b = 1, a = 0) */
        double h = tn - p->curve_t[n - 2];
        double s1 = (Y[n - 1] - Y[n - 2]) / h + h * (M[n - 2] + 2.0 * M[n - 1]) / 6.0;
        *S = Y[n - 1] + s1 * (t - tn);
        *S1 = s1;
        *S2 = 0.0;
        return;
    }
    int i = 0;
    while (i + 2 < n && t >= p->curve_t[i + 1]) ++i;
    double h = p->curve_t[i + 1] - p->curve_t[i];
    double a = (p->curve_t[i + 1] - t) / h, b = (t - p->curve_t[i]) / h;
    *S = a * Y[i] + b * Y[i + 1] + h * h * ((a * a * a - a) * M[i] + (b * b * b - b) * M[i + 1]) / 6.0;
    *S1 = (Y[i + 1] - Y[i]) / h + h * ((1.0 - 3.0 * a * a) * M[i] + (3.0 * b * b - 1.0) * M[i + 1]) / 6.0;
    *S2 = a * M[i] + b * M[i + 1];
}

double orc_forward(const orc_problem* p, double t)
{
    if (p->curve_n > 0) {
        double S, S1, S2;
        spline_eval(p, t, &S, &S1, &S2);
        return S1;
    }
    if (p->f_decay == 0.0) return p->f_level;
    return p->f_level + p->f_slope * (1.0 - exp(-p->f_decay * t));
}

/* d f(0,t) / dt, needed by the drift of r (eq. (1) coefficients). */
double orc_forward_dt(const orc_problem* p, double t)
{
    if (p->curve_n > 0) {
        double S, S1, S2;
        spline_eval(p, t, &S, &S1, &S2);
        return S2;
    }
    if (p->f_decay == 0.0) return 0.0;
    return p->f_slope * p->f_decay * exp(-p->f_decay * t);
}

/* p(0,t) = exp(-int_0^t f(0,s) ds). */
double orc_discount(const orc_problem* p, double t)
{
    double integral;
    if (p->curve_n > 0) {
        double S1, S2;
        spline_eval(p, t, &integral, &S1, &S2);
    } else if (p->f_decay == 0.0) {
        integral = p->f_level * t;
    } else {
        integral = p->f_level * t
                 + p->f_slope * (t - (1.0 - exp(-p->f_decay * t)) / p->f_decay);
    }
    return exp(-integral);
}

/* G(s) = (1 - e^{-kappa s}) / kappa, eq. (gs); G(s) = s when kappa = 0. */
double orc_G(double kappa, double s)
{
    if (kappa == 0.0) return s;
    return -expm1(-kappa * s) / kappa;
}

/* Bond price p(t,T) given the state (r, y), eq. (gs) with x = r - f(0,t). */
double orc_bond(const orc_problem* p, double t, double T, double r, double y)
{
    double G = orc_G(p->kappa, T - t);
    double x = r - orc_forward(p, t);
    return orc_discount(p, T) / orc_discount(p, t) * exp(-G * x - 0.5 * G * G * y);
}

/* Delta_M = 1 + (T_M - T) K, section 3.2. */
static double accrual(const orc_problem* p)
{
    return 1.0 + (p->pay - p->expiry) * p->strike;
}

/* Terminal data at t = T, section 3.2: bond 1; caplet max(1 - Delta p(T,T_M), 0);
   floorlet max(Delta p(T,T_M) - 1, 0); linear forward 1 - Delta p(T,T_M). */
double orc_payoff(const orc_problem* p, double r, double y)
{
    double T = p->expiry;
    if (p->kind == 0) return 1.0;
    double lin = 1.0 - accrual(p) * orc_bond(p, T, p->pay, r, y);
    if (p->kind == 1) return lin > 0.0 ? lin : 0.0;
    if (p->kind == 2) return -lin > 0.0 ? -lin : 0.0;
    return lin;
}

/* Dirichlet data at time t: the value of the same contract when the payoff
   is linear in bonds (deep in or out of the money): p(t,T) for the bond,
   max(p(t,T) - Delta p(t,T_M), 0) for the caplet and its mirror for the
   floorlet, section 3.2 and section 4.1 (closed form used as boundary data). */
double orc_dirichlet(const orc_problem* p, double t, double r, double y)
{
    double pT = orc_bond(p, t, p->expiry, r, y);
    if (p->kind == 0) return pT;
    double lin = pT - accrual(p) * orc_bond(p, t, p->pay, r, y);
    if (p->kind == 1) return lin > 0.0 ? lin : 0.0;
    if (p->kind == 2) return -lin > 0.0 ? -lin : 0.0;
    return lin;
}

/* Standard normal distribution function. */
static double norm_cdf(double x)
{
    return 0.5 * erfc(-x / sqrt(2.0));
}

/* Caplet price when gamma = 0 and epsilon = 0 with v = 1: the volatility
   of r is the constant lambda (Gaussian one-factor model, mentioned among
   the Hull-White family in section 1).  The caplet is Delta_M zero-bond puts
   with strike 1/Delta_M:
     C = P(0,T) N(-h + s) - Delta P(0,T_M) N(-h),
     s^2 = lambda^2 G(T_M - T)^2 (1 - e^{-2 kappa T}) / (2 kappa),
     h = ln(Delta P(0,T_M) / P(0,T)) / s + s / 2.                           */
double orc_gaussian_caplet(const orc_problem* p)
{
    double T = p->expiry, TM = p->pay;
    double var_factor;
    if (p->kappa == 0.0) var_factor = T;
    else var_factor = -expm1(-2.0 * p->kappa * T) / (2.0 * p->kappa);
    double G = orc_G(p->kappa, TM - T);
    double s = p->lambda * G * sqrt(var_factor);
    double PT = orc_discount(p, T), PM = orc_discount(p, TM);
    double D = accrual(p);
    double h = log(D * PM / PT) / s + 0.5 * s;
    return PT * norm_cdf(-h + s) - D * PM * norm_cdf(-h);
}

/* ------------------------------------------------------------------------ */
/* Section 4.3 / 7.1: the hyperbolic mesh z = K + alpha sinh(c2 x + c1 (1-x)),*/
/* x in [0, 1] uniform.  J = dz/dx, J2 = d^2 z / dx^2.                       */
/* ------------------------------------------------------------------------ */
void orc_axis(int n, double zmin, double zmax, double K, double alpha,
              double* z, double* J, double* J2)
{
    double c1 = asinh((zmin - K) / alpha);
    double c2 = asinh((zmax - K) / alpha);
    for (int m = 0; m < n; ++m) {
        double x = (double)m / (double)(n - 1);
        double s = c2 * x + c1 * (1.0 - x);
        z[m] = K + alpha * sinh(s);
        J[m] = alpha * cosh(s) * (c2 - c1);
        J2[m] = alpha * sinh(s) * (c2 - c1) * (c2 - c1);
    }
    /* the end nodes are the domain ends exactly */
    z[0] = zmin;
    z[n - 1] = zmax;
}

/* Inverse of the mesh map: x(z). */
double orc_axis_x(double z, double zmin, double zmax, double K, double alpha)
{
    double c1 = asinh((zmin - K) / alpha);
    double c2 = asinh((zmax - K) / alpha);
    return (asinh((z - K) / alpha) - c1) / (c2 - c1);
}

/* ------------------------------------------------------------------------ */
/* Mesh tables of one problem.                                               */
/* ------------------------------------------------------------------------ */
/* r^gamma on r >= 0; r^0 = 1 for every r (Gaussian limit). */
static double rpow(double r, double g)
{
    if (g == 0.0) return 1.0;
    return pow(r, g);
}

typedef struct {
    int nr, nv, ny;
    double *rg;             /* r_i^gamma */
    double *r, *Jr, *J2r;
    double *v, *Jv, *J2v;
    double *y, *Jy, *J2y;
    double hr, hv, hy;
} mesh;

static int mesh_build(const orc_problem* p, mesh* M)
{
    M->nr = p->n[0]; M->nv = p->n[1]; M->ny = p->n[2];
    int tot = 3 * (M->nr + M->nv + M->ny) + M->nr;
    double* buf = (double*)malloc(sizeof(double) * (size_t)tot);
    if (!buf) return -2;
    M->rg = buf + 3 * (M->nr + M->nv + M->ny);
    M->r = buf;            M->Jr = M->r + M->nr;  M->J2r = M->Jr + M->nr;
    M->v = M->J2r + M->nr; M->Jv = M->v + M->nv;  M->J2v = M->Jv + M->nv;
    M->y = M->J2v + M->nv; M->Jy = M->y + M->ny;  M->J2y = M->Jy + M->ny;
    orc_axis(M->nr, p->geom[0][0], p->geom[0][1], p->geom[0][2], p->geom[0][3], M->r, M->Jr, M->J2r);
    orc_axis(M->nv, p->geom[1][0], p->geom[1][1], p->geom[1][2], p->geom[1][3], M->v, M->Jv, M->J2v);
    orc_axis(M->ny, p->geom[2][0], p->geom[2][1], p->geom[2][2], p->geom[2][3], M->y, M->Jy, M->J2y);
    for (int i = 0; i < M->nr; ++i) M->rg[i] = rpow(M->r[i], p->gamma);
    M->hr = 1.0 / (double)(M->nr - 1);
    M->hv = 1.0 / (double)(M->nv - 1);
    M->hy = 1.0 / (double)(M->ny - 1);
    return 0;
}

static void mesh_free(mesh* M) { free(M->r); }

static size_t idx3(const mesh* M, int i, int j, int k)
{
    return ((size_t)k * (size_t)M->nv + (size_t)j) * (size_t)M->nr + (size_t)i;
}

static int is_dirichlet(const orc_problem* p, const mesh* M, int i, int j, int k)
{
    if (i == 0 && p->face[0] == ORC_DIRICHLET) return 1;
    if (i == M->nr - 1 && p->face[1] == ORC_DIRICHLET) return 1;
    if (j == 0 && p->face[2] == ORC_DIRICHLET) return 1;
    if (j == M->nv - 1 && p->face[3] == ORC_DIRICHLET) return 1;
    if (k == 0 && p->face[4] == ORC_DIRICHLET) return 1;
    if (k == M->ny - 1 && p->face[5] == ORC_DIRICHLET) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Coefficients of eq. (1) at a node and physical time t, then their         */
/* metric-transformed forms (section 4.3, g1..g6, in physical units).       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double a_rr, b_r;   /* coefficient of d2/dxr2 and d/dxr */
    double a_vv, b_v;   /* coefficient of d2/dxv2 and d/dxv */
    double m_r, m_v;    /* drift part alone of b_r, b_v: mu / J */
    double b_y;         /* coefficient of d/dxy */
    double a_rv;        /* coefficient of d2/dxr dxv */
    double react;       /* r (the -rC term) */
} coeffs;

/* f and ft are f(0,t) and df(0,t)/dt at the physical time of evaluation. */
static coeffs node_coeffs(const orc_problem* p, const mesh* M, int i, int j, int k, double f, double ft)
{
    double r = M->r[i], v = M->v[j], y = M->y[k];
    double rg = M->rg[i];
    double lam = p->lambda, eps = p->epsilon, kap = p->kappa;
    /* eq. (1) coefficients */
    double zeta_rr = 0.5 * lam * lam * rg * rg * v;
    double zeta_vv = 0.5 * eps * eps * v;
    double zeta_rv = lam * rg * eps * p->rho * v;
    double mu_r = ft - kap * (r - f) + y;
    double mu_v = p->theta_v * (1.0 - v);
    double mu_y = lam * lam * rg * rg * v - 2.0 * kap * y;
    /* chain rule through the mesh map */
    double Jr = M->Jr[i], J2r = M->J2r[i];
    double Jv = M->Jv[j], J2v = M->J2v[j];
    double Jy = M->Jy[k];
    coeffs c;
    c.a_rr = zeta_rr / (Jr * Jr);
    c.b_r = mu_r / Jr - zeta_rr * J2r / (Jr * Jr * Jr);
    c.a_vv = zeta_vv / (Jv * Jv);
    c.b_v = mu_v / Jv - zeta_vv * J2v / (Jv * Jv * Jv);
    c.m_r = mu_r / Jr;
    c.m_v = mu_v / Jv;
    c.b_y = mu_y / Jy;
    c.a_rv = zeta_rv / (Jr * Jv);
    c.react = r;
    return c;
}

/* ------------------------------------------------------------------------ */
/* One row of a directional operator A_d at node (i,j,k):                   */
/*   (A_d U)_m = lo U_{m-1} + di U_m + up U_{m+1} + ex U_{m+-2}              */
/* where ex sits at m+2 on a low outflow face and at m-2 on a high one.      */
/* d = 0: r (L_r with the reaction term), 1: v (L_v), 2: y (L_y).            */
/* Interior rows: centred stencils of eq. (esquema) (first difference over   */
/* 2h).  Outflow faces: one-sided second-order first difference of section   */
/* 7.3, no second-difference term.                                           */
/* ------------------------------------------------------------------------ */
typedef struct { double lo, di, up, ex; } oprow;

static oprow op_row(const orc_problem* p, const mesh* M, int d, int i, int j, int k, double f, double ft)
{
    coeffs c = node_coeffs(p, M, i, j, k, f, ft);
    /* a, b: interior coefficients; bf: face coefficient.  On a face the whole
       second-derivative term of eq. (1) is taken as zero (it vanishes at r = 0
       and v = 0; section 3.2 assumes C_vv = 0 at the v faces), metric
       correction included, so only the drift mu/J remains. */
    double a, b, bf, h, react;
    int m, n;
    if (d == 0) { a = c.a_rr; b = c.b_r; bf = c.m_r; h = M->hr; react = c.react; m = i; n = M->nr; }
    else if (d == 1) { a = c.a_vv; b = c.b_v; bf = c.m_v; h = M->hv; react = 0.0; m = j; n = M->nv; }
    else { a = 0.0; b = c.b_y; bf = c.b_y; h = M->hy; react = 0.0; m = k; n = M->ny; }
    oprow o = {0.0, 0.0, 0.0, 0.0};
    if (m == 0) {
        /* low face: (-3 U_0 + 4 U_1 - U_2) / (2h) */
        o.di = -3.0 * bf / (2.0 * h) - react;
        o.up = 4.0 * bf / (2.0 * h);
        o.ex = -1.0 * bf / (2.0 * h);
    } else if (m == n - 1) {
        /* high face: (3 U_{n-1} - 4 U_{n-2} + U_{n-3}) / (2h) */
        o.di = 3.0 * bf / (2.0 * h) - react;
        o.lo = -4.0 * bf / (2.0 * h);
        o.ex = 1.0 * bf / (2.0 * h);
    } else {
        o.lo = a / (h * h) - b / (2.0 * h);
        o.di = -2.0 * a / (h * h) - react;
        o.up = a / (h * h) + b / (2.0 * h);
    }
    return o;
}

/* Apply A_d (d = 0,1,2) or the mixed operator A_0 (d = 3) to U at time t on
   every non-Dirichlet node; Dirichlet nodes get 0. */
int orc_apply(const orc_problem* p, int d, double t, const double* U, double* out)
{
    mesh M;
    if (mesh_build(p, &M)) return -2;
    int nr = M.nr, nv = M.nv, ny = M.ny;
    double f = orc_forward(p, t), ft = orc_forward_dt(p, t);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < ny; ++k) {
        for (int j = 0; j < nv; ++j) {
            for (int i = 0; i < nr; ++i) {
                size_t q = idx3(&M, i, j, k);
                if (is_dirichlet(p, &M, i, j, k)) { out[q] = 0.0; continue; }
                if (d == 3) {
                    if (i == 0 || i == nr - 1 || j == 0 || j == nv - 1) { out[q] = 0.0; continue; }
                    coeffs c = node_coeffs(p, &M, i, j, k, f, ft);
                    double cross = U[idx3(&M, i + 1, j + 1, k)] - U[idx3(&M, i + 1, j - 1, k)]
                                 - U[idx3(&M, i - 1, j + 1, k)] + U[idx3(&M, i - 1, j - 1, k)];
                    out[q] = c.a_rv * cross / (4.0 * M.hr * M.hv);
                    continue;
                }
                oprow o = op_row(p, &M, d, i, j, k, f, ft);
                int m = (d == 0) ? i : (d == 1) ? j : k;
                int n = (d == 0) ? nr : (d == 1) ? nv : ny;
                size_t stride = (d == 0) ? 1 : (d == 1) ? (size_t)nr : (size_t)nr * (size_t)nv;
                double s = o.di * U[q];
                if (m > 0) s += o.lo * U[q - stride];
                if (m < n - 1) s += o.up * U[q + stride];
                if (m == 0) s += o.ex * U[q + 2 * stride];
                if (m == n - 1) s += o.ex * U[q - 2 * stride];
                out[q] = s;
            }
        }
    }
    mesh_free(&M);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Tridiagonal line solve (Gaussian elimination, no pivoting; the Thomas     */
/* algorithm of section 5) for rows                                          */
/*   row 0:     b0 x0 + c0 x1 + e_lo x2                         = d0         */
/*   row m:     a_m x_{m-1} + b_m x_m + c_m x_{m+1}             = d_m        */
/*   row n-1:   e_hi x_{n-3} + a_{n-1} x_{n-2} + b_{n-1} x_{n-1} = d_{n-1}    */
/* The end unknowns are first eliminated from rows 1 and n-2, the interior   */
/* rows 1..n-2 are solved by forward elimination and back substitution, then */
/* x0 and x_{n-1} are recovered from their own rows.  n >= 4.                */
/* ------------------------------------------------------------------------ */
int orc_line_solve(int n, const double* a, const double* b, const double* c,
                   double e_lo, double e_hi, const double* d, double* x)
{
    if (n < 4) return -1;
    double* A = (double*)malloc(sizeof(double) * 5 * (size_t)n);
    if (!A) return -2;
    double* B = A + n; double* C = B + n; double* D = C + n; double* W = D + n;
    for (int m = 0; m < n; ++m) { A[m] = a[m]; B[m] = b[m]; C[m] = c[m]; D[m] = d[m]; }
    /* eliminate x0 from row 1 */
    double f = A[1] / B[0];
    B[1] = B[1] - f * C[0];
    C[1] = C[1] - f * e_lo;
    D[1] = D[1] - f * D[0];
    A[1] = 0.0;
    /* eliminate x_{n-1} from row n-2 */
    f = C[n - 2] / B[n - 1];
    A[n - 2] = A[n - 2] - f * e_hi;
    B[n - 2] = B[n - 2] - f * A[n - 1];
    D[n - 2] = D[n - 2] - f * D[n - 1];
    C[n - 2] = 0.0;
    /* Thomas on rows 1..n-2: W holds the modified super-diagonal */
    W[1] = C[1] / B[1];
    D[1] = D[1] / B[1];
    for (int m = 2; m <= n - 2; ++m) {
        double den = B[m] - A[m] * W[m - 1];
        W[m] = C[m] / den;
        D[m] = (D[m] - A[m] * D[m - 1]) / den;
    }
    x[n - 2] = D[n - 2];
    for (int m = n - 3; m >= 1; --m) x[m] = D[m] - W[m] * x[m + 1];
    x[0] = (d[0] - c[0] * x[1] - e_lo * x[2]) / b[0];
    x[n - 1] = (d[n - 1] - e_hi * x[n - 3] - a[n - 1] * x[n - 2]) / b[n - 1];
    free(A);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Implicit sweep along direction d: solve (I - theta dt A_d) X = D in place */
/* on every line; identity rows on Dirichlet nodes.                         */
/* ------------------------------------------------------------------------ */
static int sweep(const orc_problem* p, const mesh* M, int d, double t, double dt, double* Dd)
{
    int nr = M->nr, nv = M->nv, ny = M->ny;
    int n = (d == 0) ? nr : (d == 1) ? nv : ny;
    int n_lines = (d == 0) ? nv * ny : (d == 1) ? nr * ny : nr * nv;
    size_t stride = (d == 0) ? 1 : (d == 1) ? (size_t)nr : (size_t)nr * (size_t)nv;
    int err = 0;
    double f = orc_forward(p, t), ft = orc_forward_dt(p, t);
#pragma omp parallel
    {
        double* buf = (double*)malloc(sizeof(double) * 5 * (size_t)n);
        if (!buf) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (int L = 0; L < n_lines; ++L) {
            if (!buf) continue;
            double *a = buf, *b = a + n, *c = b + n, *rhs = c + n, *x = rhs + n;
            int i0, j0, k0;
            if (d == 0) { i0 = 0; j0 = L % nv; k0 = L / nv; }
            else if (d == 1) { i0 = L % nr; j0 = 0; k0 = L / nr; }
            else { i0 = L % nr; j0 = L / nr; k0 = 0; }
            size_t base = idx3(M, i0, j0, k0);
            double e_lo = 0.0, e_hi = 0.0;
            for (int m = 0; m < n; ++m) {
                int i = (d == 0) ? m : i0, j = (d == 1) ? m : j0, k = (d == 2) ? m : k0;
                rhs[m] = Dd[base + (size_t)m * stride];
                if (is_dirichlet(p, M, i, j, k)) {
                    a[m] = 0.0; b[m] = 1.0; c[m] = 0.0;
                    continue;
                }
                oprow o = op_row(p, M, d, i, j, k, f, ft);
                a[m] = -p->theta * dt * o.lo;
                b[m] = 1.0 - p->theta * dt * o.di;
                c[m] = -p->theta * dt * o.up;
                if (m == 0) e_lo = -p->theta * dt * o.ex;
                if (m == n - 1) e_hi = -p->theta * dt * o.ex;
            }
            orc_line_solve(n, a, b, c, e_lo, e_hi, rhs, x);
            for (int m = 0; m < n; ++m) Dd[base + (size_t)m * stride] = x[m];
        }
        free(buf);
    }
    return err;
}

/* ------------------------------------------------------------------------ */
/* One ADI step, backward time tau_n = n dt -> tau_{n+1}, physical time      */
/* t_n = T - n dt.  Every operator is frozen at t_{n+1/2}, so F(V) = A V is   */
/* linear within the step, with A = A0 + A1 + A2 + A3.                        */
/*                                                                           */
/* Douglas (section 5.1), in delta form D = Y - U^n:                         */
/*   D0 = dt A U^n on non-Dirichlet nodes, g(t_{n+1}) - g(t_n) on Dirichlet   */
/*   nodes; (I - theta dt A_j) D_j = D_{j-1}, j = 1, 2, 3; U^{n+1} = U^n + D3. */
/* The three correction schemes take Y3 = U^n + D3 as a predictor and sweep  */
/* once more from a corrected start:                                         */
/*   CS:  Yt0 = Y0 + 1/2 dt (A0 Y3 - A0 U^n),                                */
/*        Yt_j = Yt_{j-1} + theta dt (A_j Yt_j - A_j U^n),  U^{n+1} = Yt3;    */
/*   MCS: Yh0 = Y0 + theta dt (A0 Y3 - A0 U^n),                              */
/*        Yt0 = Yh0 + (1/2 - theta) dt (F(Y3) - F(U^n)),                     */
/*        Yt_j = Yt_{j-1} + theta dt (A_j Yt_j - A_j U^n),  U^{n+1} = Yt3;    */
/*   HV:  Yt0 = Y0 + 1/2 dt (F(Y3) - F(U^n)),                                */
/*        Yt_j = Yt_{j-1} + theta dt (A_j Yt_j - A_j Y3),   U^{n+1} = Yt3.    */
/* In delta form, E = Yt - U^n (CS, MCS) or E = Yt - Y3 (HV), the corrected   */
/* start on non-Dirichlet nodes is                                           */
/*   CS:  E0 = D0 + 1/2 dt A0 D3                                             */
/*   MCS: E0 = D0 + theta dt A0 D3 + (1/2 - theta) dt A D3                   */
/*   HV:  E0 = D0 + 1/2 dt A D3 - D3                                         */
/* and every E_j solves (I - theta dt A_j) E_j = E_{j-1}.  On Dirichlet nodes */
/* the solution takes g(t_{n+1}): E0 = g(t_{n+1}) - g(t_n) (CS, MCS) or 0     */
/* (HV, whose Y3 already holds it).  U^{n+1} = U^n + E3 (CS, MCS) or         */
/* U^n + D3 + E3 (HV).                                                       */
/*                                                                          */
/* Huang's correction iterates towards the unsplit theta scheme             */
/*   (I - theta dt A) X = D0,  U^{n+1} = U^n + X,                            */
/* whose factored approximation M = (I - theta dt A1)(I - theta dt A2)       */
/* (I - theta dt A3) the Douglas step solves instead: X_1 = M^{-1} D0 = D3,  */
/* then for m = 1 .. q                                                       */
/*   X_{m+1} = X_m + M^{-1} (D0 - (I - theta dt A) X_m)                      */
/* (the residual is 0 on Dirichlet nodes, where X_m already holds the        */
/* increment), and U^{n+1} = U^n + X_{q+1}.  As q grows X tends to the       */
/* unsplit step wherever the iteration contracts.                            */
/* ------------------------------------------------------------------------ */

/* out = dt (A0 + A1 + A2 + A3) V on non-Dirichlet nodes, 0 on Dirichlet nodes */
static int apply_all(const orc_problem* p, double t, double dt, const double* V, double* out, double* tmp,
                     size_t npts)
{
    for (size_t q = 0; q < npts; ++q) out[q] = 0.0;
    for (int d = 0; d < 4; ++d) {
        int e = orc_apply(p, d, t, V, tmp);
        if (e) return e;
        for (size_t q = 0; q < npts; ++q) out[q] += tmp[q];
    }
    for (size_t q = 0; q < npts; ++q) out[q] = dt * out[q];
    return 0;
}

/* the three line sweeps in place: (I - theta dt A_j) X_j = X_{j-1} */
static int sweeps(const orc_problem* p, const mesh* M, double t, double dt, double* X)
{
    int err = sweep(p, M, 0, t, dt, X);
    if (!err) err = sweep(p, M, 1, t, dt, X);
    if (!err) err = sweep(p, M, 2, t, dt, X);
    return err;
}

int orc_step(const orc_problem* p, int n, double* U)
{
    if (p->scheme == ORC_HUANG && p->af_iters < 1) return -1;
    mesh M;
    if (mesh_build(p, &M)) return -2;
    int nr = M.nr, nv = M.nv, ny = M.ny;
    size_t npts = (size_t)nr * nv * ny;
    double dt = p->expiry / (double)p->n_steps;
    double t_now = p->expiry - (double)n * dt;
    double t_next = p->expiry - (double)(n + 1) * dt;
    double t_half = p->expiry - ((double)n + 0.5) * dt;
    int corr = p->scheme != ORC_DOUGLAS;
    double* Dd = (double*)malloc(sizeof(double) * npts * (corr ? 5 : 2));
    if (!Dd) { mesh_free(&M); return -2; }
    double* tmp = Dd + npts;
    double* D0 = corr ? tmp + npts : NULL;   /* the explicit predictor, kept */
    double* E = corr ? D0 + npts : NULL;     /* the corrected start, swept */
    double* W = corr ? E + npts : NULL;      /* dt A0 D3 or dt A D3 */
    /* explicit predictor: sum of the four operators */
    int err = apply_all(p, t_half, 1.0, U, Dd, tmp, npts);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < ny; ++k)
        for (int j = 0; j < nv; ++j)
            for (int i = 0; i < nr; ++i) {
                size_t q = idx3(&M, i, j, k);
                if (is_dirichlet(p, &M, i, j, k))
                    Dd[q] = orc_dirichlet(p, t_next, M.r[i], M.y[k]) - orc_dirichlet(p, t_now, M.r[i], M.y[k]);
                else
                    Dd[q] = dt * Dd[q];
            }
    if (corr)
        for (size_t q = 0; q < npts; ++q) D0[q] = Dd[q];
    if (!err) err = sweeps(p, &M, t_half, dt, Dd);   /* Dd = D3 */
    if (!err && p->scheme == ORC_HUANG) {
        /* Dd holds X_1; each pass sweeps the residual of the unsplit step */
        for (int m = 0; m < p->af_iters && !err; ++m) {
            err = apply_all(p, t_half, dt, Dd, W, tmp, npts);   /* W = dt A X_m */
            for (int k = 0; k < ny && !err; ++k)
                for (int j = 0; j < nv; ++j)
                    for (int i = 0; i < nr; ++i) {
                        size_t q = idx3(&M, i, j, k);
                        E[q] = is_dirichlet(p, &M, i, j, k) ? 0.0 : D0[q] + p->theta * W[q] - Dd[q];
                    }
            if (!err) err = sweeps(p, &M, t_half, dt, E);
            for (size_t q = 0; q < npts && !err; ++q) Dd[q] = Dd[q] + E[q];
        }
        for (size_t q = 0; q < npts && !err; ++q) U[q] = U[q] + Dd[q];
    } else if (!err && corr) {
        /* corrected start E0 on non-Dirichlet nodes */
        if (p->scheme == ORC_CS) {
            err = orc_apply(p, 3, t_half, Dd, W);
            for (size_t q = 0; q < npts && !err; ++q) E[q] = D0[q] + 0.5 * dt * W[q];
        } else if (p->scheme == ORC_MCS) {
            err = orc_apply(p, 3, t_half, Dd, W);
            for (size_t q = 0; q < npts && !err; ++q) E[q] = D0[q] + p->theta * dt * W[q];
            if (!err) err = apply_all(p, t_half, dt, Dd, W, tmp, npts);
            for (size_t q = 0; q < npts && !err; ++q) E[q] = E[q] + (0.5 - p->theta) * W[q];
        } else {
            err = apply_all(p, t_half, dt, Dd, W, tmp, npts);
            for (size_t q = 0; q < npts && !err; ++q) E[q] = D0[q] + 0.5 * W[q] - Dd[q];
        }
        /* Dirichlet nodes */
        for (int k = 0; k < ny && !err; ++k)
            for (int j = 0; j < nv; ++j)
                for (int i = 0; i < nr; ++i) {
                    size_t q = idx3(&M, i, j, k);
                    if (is_dirichlet(p, &M, i, j, k)) E[q] = p->scheme == ORC_HV ? 0.0 : D0[q];
                }
        if (!err) err = sweeps(p, &M, t_half, dt, E);
        if (!err) {
            if (p->scheme == ORC_HV)
                for (size_t q = 0; q < npts; ++q) U[q] = U[q] + Dd[q] + E[q];
            else
                for (size_t q = 0; q < npts; ++q) U[q] = U[q] + E[q];
        }
    } else if (!err) {
        for (size_t q = 0; q < npts; ++q) U[q] = U[q] + Dd[q];
    }
    free(Dd);
    mesh_free(&M);
    return err;
}

/* Gauss-Legendre rule of n points on [-1, 1]: the roots of P_n, by Newton's
   method from cos(pi (q + 3/4) / (n + 1/2)), with weights
   2 / ((1 - x^2) P_n'(x)^2). */
void orc_gauss_legendre(int n, double* x, double* w)
{
    for (int q = 0; q < n; ++q) {
        double z = cos(acos(-1.0) * ((double)q + 0.75) / ((double)n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;   /* P_0, P_1; recurrence up to P_n */
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / (double)m;
                p0 = p1;
                p1 = p2;
            }
            dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[q] = z;
        w[q] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

#define ORC_SOFT_Q 16   /* Gauss-Legendre points across a control element in y */

/* Section 7.2: the terminal data averaged over the control element
   [rlo, rhi] x [ylo, yhi] of a node (it does not depend on v).  At t = T the
   contract pays 1 - Delta p(T, T_M; r, y) (caplet: its positive part,
   floorlet: the negative part's size, forward: all of it), where
   Delta p = c e^{-G r - G^2 y / 2}, c = Delta P(0,T_M) / P(0,T) e^{G f(0,T)},
   G = G(T_M - T).  For each y the
   r-integral is closed form on either side of the kink
   r* = (ln c - G^2 y / 2) / G; the y-average uses ORC_SOFT_Q Gauss-Legendre
   points.  The bond pays 1 everywhere. */
double orc_payoff_cell(const orc_problem* p, double rlo, double rhi, double ylo, double yhi)
{
    if (p->kind == 0) return 1.0;
    double T = p->expiry, TM = p->pay;
    double G = orc_G(p->kappa, TM - T);
    double c = accrual(p) * orc_discount(p, TM) / orc_discount(p, T) * exp(G * orc_forward(p, T));
    double x[ORC_SOFT_Q], w[ORC_SOFT_Q];
    orc_gauss_legendre(ORC_SOFT_Q, x, w);
    double ym = 0.5 * (ylo + yhi), hy = 0.5 * (yhi - ylo), sum = 0.0;
    for (int q = 0; q < ORC_SOFT_Q; ++q) {
        double y = ym + hy * x[q];
        double cy = c * exp(-0.5 * G * G * y);        /* Delta p = cy e^{-G r} */
        double rs = log(cy) / G;                     /* kink: 1 = cy e^{-G r*} */
        double a = rlo, b = rhi, sign = 1.0;
        if (p->kind == 1) { if (rs > a) a = rs; }            /* caplet: r > r* */
        else if (p->kind == 2) { if (rs < b) b = rs; sign = -1.0; } /* floorlet: r < r* */
        double I = 0.0;
        /* integral of sign (1 - cy e^{-G r}) over [a, b]; the exponential's
           part is e^{-G a} (1 - e^{-G (b - a)}) / G, formed with expm1 so that
           a short element loses no digits to the difference */
        if (b > a)
            I = sign * ((b - a) + cy * exp(-G * a) * expm1(-G * (b - a)) / G);
        sum += w[q] * I;
    }
    return 0.5 * sum / (rhi - rlo);
}

/* The mesh map at any x (also beyond [0, 1]): z = K + alpha sinh(c2 x + c1 (1 - x)). */
static double axis_z(double x, double zmin, double zmax, double K, double alpha)
{
    double c1 = asinh((zmin - K) / alpha), c2 = asinh((zmax - K) / alpha);
    return K + alpha * sinh(c2 * x + c1 * (1.0 - x));
}

/* Terminal data on every node (independent of v), section 3.2; softened
   (section 7.2) where p->soften asks: the control element of node (i, k) is
   centred on it in the mesh coordinates, [z(x_i - h/2), z(x_i + h/2)] in r
   and in y (reaching beyond the domain at its ends), and the node takes the
   payoff's average over it.  soften 2 averages only the elements the
   payoff's kink crosses (where the pointwise data are not smooth).
   Dirichlet nodes keep the pointwise data. */
int orc_terminal(const orc_problem* p, double* U)
{
    mesh M;
    if (mesh_build(p, &M)) return -2;
    int kinked = p->kind == 1 || p->kind == 2;
    double G = 0.0, c = 0.0;
    if (kinked) {
        G = orc_G(p->kappa, p->pay - p->expiry);
        c = accrual(p) * orc_discount(p, p->pay) / orc_discount(p, p->expiry) * exp(G * orc_forward(p, p->expiry));
    }
    for (int k = 0; k < M.ny; ++k)
        for (int i = 0; i < M.nr; ++i) {
            double u = orc_payoff(p, M.r[i], M.y[k]);
            if (p->soften && !is_dirichlet(p, &M, i, 0, k)) {
                const double* gr = p->geom[0];
                const double* gy = p->geom[2];
                double hr = 1.0 / (double)(M.nr - 1), hy = 1.0 / (double)(M.ny - 1);
                double rlo = axis_z(((double)i - 0.5) * hr, gr[0], gr[1], gr[2], gr[3]);
                double rhi = axis_z(((double)i + 0.5) * hr, gr[0], gr[1], gr[2], gr[3]);
                double ylo = axis_z(((double)k - 0.5) * hy, gy[0], gy[1], gy[2], gy[3]);
                double yhi = axis_z(((double)k + 0.5) * hy, gy[0], gy[1], gy[2], gy[3]);
                int take = p->soften == 1;
                if (p->soften == 2 && kinked) {
                    /* the kink r*(y) = (ln c - G^2 y / 2) / G falls with y */
                    double rs_top = (log(c) - 0.5 * G * G * ylo) / G, rs_bot = (log(c) - 0.5 * G * G * yhi) / G;
                    take = rs_top >= rlo && rs_bot <= rhi;
                }
                if (take) u = orc_payoff_cell(p, rlo, rhi, ylo, yhi);
            }
            for (int j = 0; j < M.nv; ++j) U[idx3(&M, i, j, k)] = u;
        }
    mesh_free(&M);
    return 0;
}

/* Terminal data, then steps [first, last) of the Douglas loop. */
int orc_run(const orc_problem* p, int first, int last, double* U)
{
    if (first == 0) {
        int e = orc_terminal(p, U);
        if (e) return e;
    }
    for (int n = first; n < last; ++n) {
        int e = orc_step(p, n, U);
        if (e) return e;
    }
    return 0;
}

/* Closed-form bond price on every node at time t (the pin of section 4.1). */
int orc_bond_grid(const orc_problem* p, double t, double* out)
{
    mesh M;
    if (mesh_build(p, &M)) return -2;
    for (int k = 0; k < M.ny; ++k)
        for (int j = 0; j < M.nv; ++j)
            for (int i = 0; i < M.nr; ++i)
                out[idx3(&M, i, j, k)] = orc_bond(p, t, p->expiry, M.r[i], M.y[k]);
    mesh_free(&M);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Readout: C(t=0) at (r0, v0) on the y = y_min plane, by tensor 4-point     */
/* Lagrange interpolation in the mesh coordinates (x_r, x_v).                */
/* ------------------------------------------------------------------------ */
static void lagrange4(double x, int n, int* start, double w[4])
{
    double h = 1.0 / (double)(n - 1);
    int m = (int)floor(x / h);
    if (m < 0) m = 0;
    if (m > n - 2) m = n - 2;
    int s = m - 1;
    if (s < 0) s = 0;
    if (s > n - 4) s = n - 4;
    for (int a = 0; a < 4; ++a) {
        double xa = (double)(s + a) * h;
        double num = 1.0, den = 1.0;
        for (int b = 0; b < 4; ++b) {
            if (b == a) continue;
            double xb = (double)(s + b) * h;
            num *= (x - xb);
            den *= (xa - xb);
        }
        w[a] = num / den;
    }
    *start = s;
}

double orc_readout(const orc_problem* p, const double* U, double r0, double v0)
{
    int nr = p->n[0], nv = p->n[1];
    double xr = orc_axis_x(r0, p->geom[0][0], p->geom[0][1], p->geom[0][2], p->geom[0][3]);
    double xv = orc_axis_x(v0, p->geom[1][0], p->geom[1][1], p->geom[1][2], p->geom[1][3]);
    int si, sj;
    double wr[4], wv[4];
    lagrange4(xr, nr, &si, wr);
    lagrange4(xv, nv, &sj, wv);
    double s = 0.0;
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a)
            s += wv[b] * wr[a] * U[(size_t)(sj + b) * (size_t)nr + (size_t)(si + a)];
    return s;
}

/* The Greeks the paper plots (section 6): rho = dC/dr and vega = dC/dv at
   (r0, v0) on the y = y_min plane, as the derivatives of the same tensor
   4-point Lagrange interpolant.  In mesh coordinates x the derivative of the
   basis function of node a is sum_{c != a} prod_{b != a, c} (x - x_b) /
   prod_{b != a} (x_a - x_b); the chain rule multiplies it by dx/dz =
   1 / ((c2 - c1) sqrt(alpha^2 + (z - K)^2)) of the sinh map.
   out = (C, dC/dr, dC/dv). */
static void lagrange4_d(double x, int n, double dw[4])
{
    double h = 1.0 / (double)(n - 1);
    int m = (int)floor(x / h);
    if (m < 0) m = 0;
    if (m > n - 2) m = n - 2;
    int s = m - 1;
    if (s < 0) s = 0;
    if (s > n - 4) s = n - 4;
    for (int a = 0; a < 4; ++a) {
        double xa = (double)(s + a) * h, den = 1.0, sum = 0.0;
        for (int b = 0; b < 4; ++b)
            if (b != a) den *= (xa - (double)(s + b) * h);
        for (int c = 0; c < 4; ++c) {
            if (c == a) continue;
            double prod = 1.0;
            for (int b = 0; b < 4; ++b)
                if (b != a && b != c) prod *= (x - (double)(s + b) * h);
            sum += prod;
        }
        dw[a] = sum / den;
    }
}

static double axis_dxdz(double z, double zmin, double zmax, double K, double alpha)
{
    double c1 = asinh((zmin - K) / alpha), c2 = asinh((zmax - K) / alpha);
    return 1.0 / ((c2 - c1) * sqrt(alpha * alpha + (z - K) * (z - K)));
}

void orc_greeks(const orc_problem* p, const double* U, double r0, double v0, double* out)
{
    int nr = p->n[0], nv = p->n[1];
    double xr = orc_axis_x(r0, p->geom[0][0], p->geom[0][1], p->geom[0][2], p->geom[0][3]);
    double xv = orc_axis_x(v0, p->geom[1][0], p->geom[1][1], p->geom[1][2], p->geom[1][3]);
    int si, sj;
    double wr[4], wv[4], dr[4], dv[4];
    lagrange4(xr, nr, &si, wr);
    lagrange4(xv, nv, &sj, wv);
    lagrange4_d(xr, nr, dr);
    lagrange4_d(xv, nv, dv);
    double gr = axis_dxdz(r0, p->geom[0][0], p->geom[0][1], p->geom[0][2], p->geom[0][3]);
    double gv = axis_dxdz(v0, p->geom[1][0], p->geom[1][1], p->geom[1][2], p->geom[1][3]);
    double c = 0.0, cr = 0.0, cv = 0.0;
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a) {
            double u = U[(size_t)(sj + b) * (size_t)nr + (size_t)(si + a)];
            c += wv[b] * wr[a] * u;
            cr += wv[b] * dr[a] * u;
            cv += dv[b] * wr[a] * u;
        }
    out[0] = c;
    out[1] = cr * gr;
    out[2] = cv * gv;
}

/* Full solve from t = T to t = 0 and readout; U (nr*nv*ny) receives the
   final grid. */
int orc_price(const orc_problem* p, double r0, double v0, double* U, double* price)
{
    int e = orc_run(p, 0, p->n_steps, U);
    if (e) return e;
    *price = orc_readout(p, U, r0, v0);
    return 0;
}
