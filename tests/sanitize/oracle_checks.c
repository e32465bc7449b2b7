/* Runs the oracle's entry points on small problems, for a build with the
   address and undefined-behaviour sanitizers: every scheme, both softening
   modes, a discrete curve, the line solve, the readout and Greeks, the
   Gauss-Legendre rule, and a discrete curve with too many knots (refused:
   NaN, no write past the spline's arrays).  Exit status 0 when every
   result is finite where it should be. */
/* the oracle itself, compiled into this program */
#include "../../oracle/hjm_oracle.c"

#include <stdio.h>

typedef orc_problem problem;

static problem base(int nr, int nv, int ny)
{
    problem p;
    memset(&p, 0, sizeof p);
    p.n[0] = nr; p.n[1] = nv; p.n[2] = ny;
    p.face[1] = 1; p.face[5] = 1;  /* Dirichlet at r_max and y_max */
    double g[3][4] = {{0.0, 2.5, 0.03, 0.005}, {0.0, 30.0, 0.5, 0.5}, {0.0, 0.025, 0.0, 5e-5}};
    memcpy(p.geom, g, sizeof g);
    p.kappa = 0.08; p.theta_v = 0.25; p.lambda = 0.15; p.gamma = 0.9; p.epsilon = 0.45; p.rho = -0.6;
    p.f_level = 0.02; p.f_slope = 0.01; p.f_decay = 0.5;
    p.kind = 1; p.expiry = 1.0; p.pay = 2.0; p.strike = 0.03; p.n_steps = 6;
    p.scheme = 0; p.theta = 0.5;
    return p;
}

static int check_price(const char* what, const problem* p)
{
    size_t pts = (size_t)p->n[0] * p->n[1] * p->n[2];
    double* U = malloc(sizeof(double) * pts);
    double price = NAN, g[3];
    int st = orc_price(p, 0.02, 1.0, U, &price);
    orc_greeks(p, U, 0.02, 1.0, g);
    free(U);
    if (st != 0 || !isfinite(price) || !isfinite(g[1]) || !isfinite(g[2])) {
        fprintf(stderr, "%s: status %d price %g\n", what, st, price);
        return 1;
    }
    return 0;
}

int main(void)
{
    int bad = 0;
    orc_set_threads(2);
    problem p = base(13, 9, 10);
    for (int sc = 0; sc <= 4; ++sc) {
        problem q = p;
        q.scheme = sc;
        q.af_iters = sc == 4 ? 2 : 0;
        bad += check_price("scheme", &q);
    }
    for (int soft = 1; soft <= 2; ++soft) {
        problem q = p;
        q.soften = soft;
        bad += check_price("soften", &q);
    }
    for (int kind = 0; kind <= 3; ++kind) {
        problem q = p;
        q.kind = kind;
        bad += check_price("kind", &q);
    }
    {
        double t[6] = {0.0, 0.5, 1.0, 2.0, 3.0, 5.0};
        double P[6];
        for (int i = 0; i < 6; ++i) P[i] = exp(-(0.02 + 0.002 * t[i]) * t[i]);
        problem q = p;
        q.curve_n = 6; q.curve_t = t; q.curve_p = P;
        bad += check_price("discrete curve", &q);
        double* G = malloc(sizeof(double) * 13 * 9 * 10);
        bad += orc_bond_grid(&q, 0.5, G) != 0;
        free(G);
    }
    {
        /* more knots than the spline holds: refused, nothing written past its arrays */
        enum { N = 80 };
        double t[N], P[N];
        for (int i = 0; i < N; ++i) { t[i] = 0.25 * i; P[i] = exp(-0.02 * t[i]); }
        problem q = p;
        q.curve_n = N; q.curve_t = t; q.curve_p = P;
        bad += !isnan(orc_forward(&q, 1.0));
    }
    {
        double a[7], b[7], c[7], d[7];
        for (int i = 0; i < 7; ++i) { a[i] = -0.3; b[i] = 2.0; c[i] = -0.4; d[i] = 1.0 + i; }
        double x[7];
        bad += orc_line_solve(7, a, b, c, 0.1, -0.2, d, x) != 0;
        for (int i = 0; i < 7; ++i) bad += !isfinite(x[i]);
    }
    {
        double x[16], w[16];
        orc_gauss_legendre(16, x, w);
        double sw = 0.0;
        for (int i = 0; i < 16; ++i) sw += w[i];
        bad += fabs(sw - 2.0) > 1e-13;
    }
    printf("oracle checks: %d failures\n", bad);
    return bad != 0;
}
