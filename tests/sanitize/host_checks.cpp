// Calls the C ABI's host-side paths that need no GPU (sizes, argument
// validation, refusals before any device work), for a build of the library
// with the address and undefined-behaviour sanitizers on its host code.
// Exit status 0 when every call returns what the ABI documents.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "hjm.h"

static int bad = 0;

static void expect(const char* what, hjm_status got, hjm_status want)
{
    if (got != want) {
        std::fprintf(stderr, "%s: got %d (%s), want %d\n", what, got, hjm_last_error(), want);
        ++bad;
    }
}

static void axes(hjm_axis ax[3], int nr, int nv, int ny)
{
    std::memset(ax, 0, sizeof(hjm_axis) * 3);
    ax[0] = {nr, HJM_FACE_OUTFLOW, HJM_FACE_DIRICHLET, 0, 0.0, 2.5, 0.03, 0.005};
    ax[1] = {nv, HJM_FACE_OUTFLOW, HJM_FACE_OUTFLOW, 0, 0.0, 30.0, 0.5, 0.5};
    ax[2] = {ny, HJM_FACE_OUTFLOW, HJM_FACE_DIRICHLET, 0, 0.0, 0.025, 0.0, 5e-5};
}

int main()
{
    hjm_axis ax[3];
    axes(ax, 33, 24, 20);
    hjm_model m;
    std::memset(&m, 0, sizeof m);
    m.kappa = 0.08; m.theta_v = 0.25; m.lambda = 0.15; m.gamma = 0.9; m.epsilon = 0.45; m.rho = -0.6;
    m.f_level = 0.02; m.f_slope = 0.01; m.f_decay = 0.5;
    hjm_payoff pay;
    std::memset(&pay, 0, sizeof pay);
    pay.kind = HJM_CAPLET; pay.expiry = 1.0; pay.pay = 2.0; pay.strike = 0.03;
    size_t nb = 0;
    expect("workspace bytes", hjm_workspace_bytes(ax, 25, &nb), HJM_OK);
    if (nb < (size_t)3 * 33 * 24 * 20 * 8) ++bad;
    expect("static scratch bytes", hjm_static_scratch_bytes(ax, 25, &nb), HJM_OK);
    hjm_scheme sc{HJM_SCHEME_HV, 0, 0.7};
    expect("scheme workspace bytes", hjm_scheme_workspace_bytes(ax, 25, &sc, &nb), HJM_OK);
    void* fake = reinterpret_cast<void*>(uintptr_t(1) << 20);  // never dereferenced: refusals come first
    hjm_grid* g = nullptr;
    // invalid problems, each refused on the host
    {
        hjm_axis b[3];
        std::memcpy(b, ax, sizeof b);
        b[0].n = 4;
        expect("n < 5", hjm_grid_create(b, &m, &pay, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
        std::memcpy(b, ax, sizeof b);
        b[1].alpha = 0.0;
        expect("alpha 0", hjm_grid_create(b, &m, &pay, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
        std::memcpy(b, ax, sizeof b);
        b[2].z_max = b[2].z_min;
        expect("empty axis", hjm_grid_create(b, &m, &pay, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
    }
    {
        hjm_model q = m;
        q.rho = 1.5;
        expect("|rho| > 1", hjm_grid_create(ax, &q, &pay, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
        q = m;
        q.gamma = 1.2;
        expect("gamma > 1", hjm_grid_create(ax, &q, &pay, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
        q = m;
        q.curve_n = HJM_MAX_CURVE_KNOTS + 1;
        std::vector<double> t(q.curve_n), p(q.curve_n);
        for (int i = 0; i < q.curve_n; ++i) { t[i] = 0.25 * i; p[i] = std::exp(-0.02 * t[i]); }
        q.curve_t = t.data();
        q.curve_p = p.data();
        expect("too many knots", hjm_grid_create(ax, &q, &pay, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
        q.curve_n = 6;
        t[2] = t[1];
        expect("knots not increasing", hjm_grid_create(ax, &q, &pay, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
    }
    {
        hjm_payoff q = pay;
        q.pay = q.expiry;
        expect("pay <= expiry", hjm_grid_create(ax, &m, &q, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
        q = pay;
        q.strike = -0.01;
        expect("K <= 0", hjm_grid_create(ax, &m, &q, 25, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
    }
    expect("n_steps 0", hjm_grid_create(ax, &m, &pay, 0, fake, 1ull << 30, nullptr, &g), HJM_EINVAL);
    expect("null workspace", hjm_grid_create(ax, &m, &pay, 25, nullptr, 1ull << 30, nullptr, &g), HJM_EINVAL);
    expect("small workspace", hjm_grid_create(ax, &m, &pay, 25, fake, 64, nullptr, &g), HJM_ENOMEM);
    expect("misaligned workspace",
           hjm_grid_create(ax, &m, &pay, 25, reinterpret_cast<void*>(uintptr_t(1) << 20 | 8), 1ull << 30, nullptr, &g),
           HJM_EINVAL);
    // the static-scratch entry point: too large a grid, a readout outside the mesh
    {
        hjm_axis b[3];
        axes(b, 256, 128, 128);
        double out[3];
        expect("static: too large", hjm_price_static(b, &m, &pay, 400, 0.02, 1.0, (double*)fake, nullptr, out),
               HJM_ENOMEM);
        expect("static: r0 outside", hjm_price_static(ax, &m, &pay, 25, 5.0, 1.0, (double*)fake, nullptr, out),
               HJM_EINVAL);
        expect("static: null grid", hjm_price_static(ax, &m, &pay, 25, 0.02, 1.0, nullptr, nullptr, out), HJM_EINVAL);
    }
    // batches: sizes and refusals
    {
        std::vector<hjm_axis> bax(9);
        for (int s = 0; s < 3; ++s) axes(&bax[3 * s], 32 + 16 * s, 24, 20);
        std::vector<int32_t> steps{10, 20, 30};
        expect("batch bytes", hjm_batch_workspace_bytes(3, bax.data(), steps.data(), &nb), HJM_OK);
        steps[1] = 0;
        expect("batch steps 0", hjm_batch_workspace_bytes(3, bax.data(), steps.data(), &nb), HJM_EINVAL);
    }
    // tuning knobs
    expect("line tile 12", hjm_set_line_tile(12, 16, 16), HJM_EINVAL);
    expect("explicit chunk 5", hjm_set_explicit_chunk(5), HJM_EINVAL);
    expect("batch streams 0", hjm_set_batch_streams(0), HJM_EINVAL);
    expect("mlp bytes", hjm_mlp_workspace_bytes(4096, &nb), HJM_OK);
    for (int s = -6; s <= 0; ++s)
        if (!hjm_status_str(s)) ++bad;
    std::printf("host checks: %d failures\n", bad);
    return bad != 0;
}
