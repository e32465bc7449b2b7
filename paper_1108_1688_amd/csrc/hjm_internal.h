// Internal layout shared by the HIP kernels and the host layer of libhjm.
// Not part of the C ABI (include/hjm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hjm {

constexpr int kBlock = 256;        // threads per workgroup of every sweep kernel
constexpr int kStepStride = 8;     // doubles per time level in the step table

// Per-solve descriptor, resident in device memory (read through the scalar
// cache; never written by a kernel).
struct SolveDesc {
    int32_t nr, nv, ny, n_steps;
    int32_t r_lo_dir, r_hi_dir, y_hi_dir, kind;
    // line-solve tiling: segments per line (S) and lines per workgroup (L)
    int32_t r_S, r_L, v_S, v_L;
    int32_t y_S, y_L, r_tiles, v_tiles;
    int32_t y_tiles, r_pitch, pad0, pad1;
    double dt;          // time step
    double tdt;         // theta * dt, theta = 1/2
    double kappa;
    double accrual;     // Delta = 1 + (T_M - T) K
    double ih2r, i2hr;  // 1/h_r^2, 1/(2 h_r) with h = 1/(n-1)
    double ih2v, i2hv;
    double i2hy;
    double i4hrhv;      // 1/(4 h_r h_v)
    double* U;          // grid, nr*nv*ny
    double* D;          // Douglas increment, nr*nv*ny
    const double* rt;   // r-axis tables, kRT * nr
    const double* vt;   // v-axis tables, kVT * nv
    const double* yt;   // y-axis tables, kYT * ny
    const double* st;   // step table, kStepStride * (n_steps + 1)
    int32_t* flag;      // health flag: nonzero after a bad pivot or a non-finite value
    int32_t* flag_pad;
};

// r-axis table rows (each nr long)
enum { RT_R = 0, RT_A, RT_B1, RT_B2, RT_X, RT_Y, kRT };
// v-axis table rows (each nv long)
enum { VT_V = 0, VT_A, VT_B, VT_M, VT_X, kVT };
// y-axis table rows (each ny long)
enum { YT_Y = 0, YT_I, YT_K, kYT };
// step table entries, per time level n (t_n = T - n dt)
enum { ST_PHI = 0, ST_AT, ST_GT, ST_HT, ST_AM, ST_GM, ST_HM };

enum { KIND_BOND = 0, KIND_CAPLET = 1, KIND_FLOORLET = 2, KIND_FORWARD = 3 };

// Readout request: 4x4 Lagrange stencil on the lowest y plane of one solve.
struct Readout {
    int32_t solve;
    int32_t i0, j0;
    int32_t pad;
    double wr[4];
    double wv[4];
};

// Raise the dynamic-LDS limit of every sweep kernel (once per process).
hipError_t init_kernel_attributes();

// Launch entry points (defined in hjm_kernels.hip).  `tasks` is either null
// (single solve: workgroup b handles tile b of solve 0) or a list of
// (solve, tile) pairs, one per workgroup.
hipError_t launch_terminal(const SolveDesc* d_desc, int n_solves, int64_t max_points, hipStream_t st);
hipError_t launch_xr(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int step,
                     size_t lds_bytes, hipStream_t st);
hipError_t launch_v(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks,
                    size_t lds_bytes, hipStream_t st);
hipError_t launch_yu(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks,
                     size_t lds_bytes, hipStream_t st);
hipError_t launch_readout(const SolveDesc* d_desc, const Readout* rq, int n, double* out, hipStream_t st);
hipError_t launch_health(const SolveDesc* d_desc, int n_solves, int64_t max_points, hipStream_t st);

}  // namespace hjm
