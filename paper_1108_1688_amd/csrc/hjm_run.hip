// hjm_run: price a list of solves through the C ABI from a plain-text spec,
// without Python (for profilers and for callers that embed the library).
//
//   hjm_run SPEC [--repeat N] [--warmup W] [--steps K] [--tile R,V,Y] [--batch [--graph]]
//   hjm_run --copy MIB
//
// SPEC holds one solve per line ('#' starts a comment), 37 numbers:
//   3 axes (r, v, y), each:  n z_min z_max center alpha lo_face hi_face
//   model:                   kappa theta_v lambda gamma epsilon rho f_level f_slope f_decay
//   payoff:                  kind expiry pay strike
//   solve:                   n_steps r0 v0
// Each repeat creates every grid (workspaces are allocated once), runs every
// Douglas step and reads the price out, as one pass over the list.  With
// --steps K only the first K steps of each solve run and no price is read.
// With --batch the list is priced as one batch (hjm_batch_*: at every Douglas
// step one launch per kernel covers all solves still running); --steps does
// not apply there.  With --graph each pass runs the batch twice from a HIP
// graph (captured on the first run, replayed on the second) before reading
// the prices.
// Prints the prices of the last repeat and the throughput in grid-point
// Douglas steps per second.  Exit status 0 on success, 1 on a bad spec or
// argument, 2 on a library or HIP error.
//
// --copy MIB runs a plain device-to-device copy kernel over MIB mebibytes
// (read once, written once): the reference dispatch against which hardware
// byte counters of the solver kernels are scaled.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "hjm.h"

namespace {

struct Solve {
    hjm_axis ax[3];
    hjm_model model;
    hjm_payoff payoff;
    int32_t n_steps;
    double r0, v0;
    int64_t points() const { return int64_t(ax[0].n) * ax[1].n * ax[2].n; }
};

bool parse_line(const std::string& line, Solve* s) {
    std::istringstream in(line);
    double f[37];
    int m = 0;
    while (m < 37 && (in >> f[m])) ++m;
    std::string rest;
    if (m != 37 || (in >> rest)) return false;
    std::memset(s, 0, sizeof *s);
    for (int a = 0; a < 3; ++a) {
        const double* q = f + 7 * a;
        s->ax[a].n = int32_t(q[0]);
        s->ax[a].z_min = q[1];
        s->ax[a].z_max = q[2];
        s->ax[a].center = q[3];
        s->ax[a].alpha = q[4];
        s->ax[a].lo_face = int32_t(q[5]);
        s->ax[a].hi_face = int32_t(q[6]);
    }
    const double* q = f + 21;
    s->model = {q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], q[8]};
    s->payoff.kind = int32_t(q[9]);
    s->payoff.expiry = q[10];
    s->payoff.pay = q[11];
    s->payoff.strike = q[12];
    s->n_steps = int32_t(q[13]);
    s->r0 = q[14];
    s->v0 = q[15];
    return true;
}

int lib_fail(const char* what, hjm_status st) {
    std::fprintf(stderr, "hjm_run: %s: %s (%s)\n", what, hjm_status_str(st), hjm_last_error());
    return 2;
}

int usage() {
    std::fprintf(stderr, "usage: hjm_run SPEC [--repeat N] [--warmup W] [--steps K] [--tile R,V,Y] [--batch [--graph]]\n"
                         "       hjm_run --copy MIB\n");
    return 1;
}

__global__ void __launch_bounds__(256) k_copy(const double2* __restrict__ src, double2* __restrict__ dst, int64_t n) {
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += stride) dst[q] = src[q];
}

int run_copy(int mib) {
    if (mib < 1 || mib > 4096) return usage();
    const int64_t n = int64_t(mib) * (1 << 20) / int64_t(sizeof(double2));
    double2 *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, n * sizeof(double2)) != hipSuccess || hipMalloc(&dst, n * sizeof(double2)) != hipSuccess) {
        std::fprintf(stderr, "hjm_run: hipMalloc failed\n");
        return 2;
    }
    if (hipMemset(src, 0, n * sizeof(double2)) != hipSuccess) return 2;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 2;
    const int grid = 256 * 32;
    for (int it = 0; it < 3; ++it) {
        hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, 0, src, dst, n);
        if (hipGetLastError() != hipSuccess) return 2;
    }
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, 0, src, dst, n);
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) return 2;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    std::printf("hjm_run: copy of %d MiB (%d MiB read + %d MiB written) in %.3f us: %.1f GB/s\n", mib, mib, mib,
                1e3 * ms, 2.0 * n * sizeof(double2) / (ms * 1e-3) / 1e9);
    (void)hipFree(src);
    (void)hipFree(dst);
    return 0;
}

int run_batch(const std::vector<Solve>& solves, hipStream_t stream, int repeat, int warmup, bool graph) {
    const int32_t n = int32_t(solves.size());
    std::vector<hjm_axis> ax(3 * solves.size());
    std::vector<hjm_model> model(solves.size());
    std::vector<hjm_payoff> payoff(solves.size());
    std::vector<int32_t> steps(solves.size());
    std::vector<double> r0(solves.size()), v0(solves.size()), prices(solves.size(), 0.0);
    int64_t per_pass = 0;
    for (size_t q = 0; q < solves.size(); ++q) {
        for (int a = 0; a < 3; ++a) ax[3 * q + a] = solves[q].ax[a];
        model[q] = solves[q].model;
        payoff[q] = solves[q].payoff;
        steps[q] = solves[q].n_steps;
        r0[q] = solves[q].r0;
        v0[q] = solves[q].v0;
        per_pass += solves[q].points() * solves[q].n_steps;
    }
    size_t bytes = 0;
    hjm_status st = hjm_batch_workspace_bytes(n, ax.data(), steps.data(), &bytes);
    if (st != HJM_OK) return lib_fail("batch workspace size", st);
    void* ws = nullptr;
    if (hipMalloc(&ws, bytes) != hipSuccess) {
        std::fprintf(stderr, "hjm_run: hipMalloc of %zu bytes failed\n", bytes);
        return 2;
    }
    int64_t point_steps = 0;
    double seconds = 0.0;
    for (int it = 0; it < warmup + repeat; ++it) {
        if (hipStreamSynchronize(stream) != hipSuccess) return lib_fail("sync", HJM_EDEVICE);
        auto t0 = std::chrono::steady_clock::now();
        hjm_batch* b = nullptr;
        st = hjm_batch_create(n, ax.data(), model.data(), payoff.data(), steps.data(), ws, bytes, stream, &b);
        if (st != HJM_OK) return lib_fail("batch create", st);
        st = hjm_batch_run(b, graph ? 1 : 0);
        if (graph && st == HJM_OK) st = hjm_batch_run(b, 1);
        if (st == HJM_OK) st = hjm_batch_prices(b, r0.data(), v0.data(), prices.data());
        hjm_batch_destroy(b);
        if (st != HJM_OK) return lib_fail("batch run", st);
        double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        std::printf("hjm_run: batch pass %d of %d%s: %.3f ms\n", it + 1, warmup + repeat,
                    it < warmup ? " (warmup)" : "", 1e3 * el);
        std::fflush(stdout);
        if (it >= warmup) {
            point_steps += per_pass * (graph ? 2 : 1);
            seconds += el;
        }
    }
    for (size_t q = 0; q < solves.size(); ++q)
        std::printf("solve %zu: %dx%dx%d, %d steps, price %.17g\n", q, solves[q].ax[0].n, solves[q].ax[1].n,
                    solves[q].ax[2].n, solves[q].n_steps, prices[q]);
    std::printf("hjm_run: %lld grid-point Douglas steps in %.6f s: %.4g per second\n", (long long)point_steps,
                seconds, point_steps / seconds);
    (void)hipFree(ws);
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) return usage();
    if (!std::strcmp(argv[1], "--copy")) return argc == 3 ? run_copy(std::atoi(argv[2])) : usage();
    int repeat = 1, warmup = 0, steps_cap = 0;
    bool batch = false, graph = false;
    for (int a = 2; a < argc; ++a) {
        if (!std::strcmp(argv[a], "--batch")) {
            batch = true;
            continue;
        }
        if (!std::strcmp(argv[a], "--graph")) {
            graph = true;
            continue;
        }
        if (a + 1 >= argc) return usage();
        if (!std::strcmp(argv[a], "--repeat")) {
            repeat = std::atoi(argv[++a]);
        } else if (!std::strcmp(argv[a], "--warmup")) {
            warmup = std::atoi(argv[++a]);
        } else if (!std::strcmp(argv[a], "--steps")) {
            steps_cap = std::atoi(argv[++a]);
        } else if (!std::strcmp(argv[a], "--tile")) {
            int r, v, y;
            if (std::sscanf(argv[++a], "%d,%d,%d", &r, &v, &y) != 3) return usage();
            hjm_status st = hjm_set_line_tile(r, v, y);
            if (st != HJM_OK) return lib_fail("line tile", st);
        } else {
            return usage();
        }
    }
    if (repeat < 1 || warmup < 0 || steps_cap < 0 || (batch && steps_cap > 0) || (graph && !batch)) return usage();

    std::ifstream file(argv[1]);
    if (!file) {
        std::fprintf(stderr, "hjm_run: cannot open %s\n", argv[1]);
        return 1;
    }
    std::vector<Solve> solves;
    std::string line;
    for (int ln = 1; std::getline(file, line); ++ln) {
        size_t hash = line.find('#');
        if (hash != std::string::npos) line.resize(hash);
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        Solve s;
        if (!parse_line(line, &s)) {
            std::fprintf(stderr, "hjm_run: %s:%d: expected 37 numbers\n", argv[1], ln);
            return 1;
        }
        solves.push_back(s);
    }
    if (solves.empty()) {
        std::fprintf(stderr, "hjm_run: %s holds no solve\n", argv[1]);
        return 1;
    }

    hipStream_t stream;
    if (hipStreamCreate(&stream) != hipSuccess) {
        std::fprintf(stderr, "hjm_run: hipStreamCreate failed\n");
        return 2;
    }
    if (batch) {
        int rc = run_batch(solves, stream, repeat, warmup, graph);
        (void)hipStreamDestroy(stream);
        return rc;
    }
    std::vector<void*> ws(solves.size(), nullptr);
    std::vector<size_t> ws_bytes(solves.size(), 0);
    for (size_t q = 0; q < solves.size(); ++q) {
        hjm_status st = hjm_workspace_bytes(solves[q].ax, solves[q].n_steps, &ws_bytes[q]);
        if (st != HJM_OK) return lib_fail("workspace size", st);
        if (hipMalloc(&ws[q], ws_bytes[q]) != hipSuccess) {
            std::fprintf(stderr, "hjm_run: hipMalloc of %zu bytes failed\n", ws_bytes[q]);
            return 2;
        }
    }

    std::vector<double> prices(solves.size(), 0.0);
    int64_t point_steps = 0;
    double seconds = 0.0;
    for (int it = 0; it < warmup + repeat; ++it) {
        if (hipStreamSynchronize(stream) != hipSuccess) return lib_fail("sync", HJM_EDEVICE);
        auto t0 = std::chrono::steady_clock::now();
        int64_t done = 0;
        std::vector<hjm_grid*> grids(solves.size(), nullptr);
        for (size_t q = 0; q < solves.size(); ++q) {
            const Solve& s = solves[q];
            hjm_status st = hjm_grid_create(s.ax, &s.model, &s.payoff, s.n_steps, ws[q], ws_bytes[q], stream,
                                            &grids[q]);
            if (st != HJM_OK) return lib_fail("grid create", st);
            int32_t k = steps_cap > 0 && steps_cap < s.n_steps ? steps_cap : s.n_steps;
            st = hjm_adi_step(grids[q], k);
            if (st != HJM_OK) return lib_fail("adi step", st);
            done += s.points() * k;
        }
        for (size_t q = 0; q < solves.size(); ++q) {
            if (steps_cap == 0 || steps_cap >= solves[q].n_steps) {
                hjm_status st = hjm_price(grids[q], solves[q].r0, solves[q].v0, &prices[q]);
                if (st != HJM_OK) return lib_fail("price", st);
            }
        }
        if (hipStreamSynchronize(stream) != hipSuccess) return lib_fail("sync", HJM_EDEVICE);
        for (hjm_grid* g : grids) hjm_grid_destroy(g);
        double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        std::printf("hjm_run: pass %d of %d%s: %.3f ms\n", it + 1, warmup + repeat, it < warmup ? " (warmup)" : "",
                    1e3 * el);
        std::fflush(stdout);
        if (it >= warmup) {
            point_steps += done;
            seconds += el;
        }
    }
    for (size_t q = 0; q < solves.size(); ++q) {
        if (steps_cap == 0 || steps_cap >= solves[q].n_steps)
            std::printf("solve %zu: %dx%dx%d, %d steps, price %.17g\n", q, solves[q].ax[0].n, solves[q].ax[1].n,
                        solves[q].ax[2].n, solves[q].n_steps, prices[q]);
    }
    std::printf("hjm_run: %lld grid-point Douglas steps in %.6f s: %.4g per second\n", (long long)point_steps,
                seconds, point_steps / seconds);
    for (void* p : ws) (void)hipFree(p);
    (void)hipStreamDestroy(stream);
    return 0;
}
