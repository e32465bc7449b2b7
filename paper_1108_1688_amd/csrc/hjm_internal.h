// Internal layout shared by the HIP kernels and the host layer of libhjm.
// Not part of the C ABI (include/hjm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hjm {

constexpr int kBlock = 256;        // threads per workgroup of every sweep kernel
constexpr int kStepStride = 8;     // doubles per time level in the step table
constexpr int kRed = 8;            // doubles per segment in the r-sweep reduced system

// How the explicit predictor and the r lines are computed.
enum { R_SPIKE = 0,   // fused k_xr; segments eliminated in parallel, reduced system per line
       R_CHAIN = 1,   // fused k_xr; Thomas in row order, segments chained through LDS
       R_SPLIT = 2,   // k_exp (explicit predictor) then k_rs (spike, one line per S lanes of a wave)
       R_FUSED = 3 }; // k_exr: explicit predictor into LDS, then the k_rs spike solve, one kernel

constexpr int kExpCols = 256;  // r-y columns per k_exp workgroup (one thread each)
constexpr int kExrJ = 16;      // v nodes per k_exr tile (computed 8 at a time)
constexpr int kExrMaxNr = kBlock;  // k_exr: one thread per r node of a plane
constexpr int kExrMaxP = kBlock / 8;  // k_exr: planes per tile (nr >= 8)

// Per-solve descriptor, resident in device memory (read-only in kernels).
struct SolveDesc {
    int32_t nr, nv, ny, n_steps;
    int32_t r_lo_dir, r_hi_dir, y_hi_dir, kind;
    // line-solve tiling: segments per line (S) and lines per workgroup (L)
    int32_t r_S, r_L, v_S, v_L;
    int32_t y_S, y_L, r_tiles, v_tiles;
    int32_t y_tiles, r_pitch, r_mode, pad0;
    // split path (R_SPLIT): k_exp tiles = exp_cb column blocks x ceil(nv / exp_J)
    // v chunks; k_rs handles rs_L lines per workgroup, rs_S = nr / ROWS lanes
    // (a power of two <= 64) per line
    int32_t exp_J, exp_cb, exp_tiles, rs_S;
    int32_t rs_log2S, rs_L, rs_tiles, exr_P;
    // fused path (R_FUSED): k_exr tiles = ceil(ny / exr_P) plane blocks x
    // ceil(nv / kExrJ) v blocks, exr_P = exr_planes(nr, rows) planes per tile; the
    // row table sits exr_tab doubles into the dynamic LDS, after the tile
    // segmented v solve (k_vs, vs_S > 0): vs_S segments of nv / vs_S rows, one
    // wave of 64 consecutive i per segment; chained y solve on stored pivots
    // (k_yc, yc_S > 0): yc_S segments of ny / yc_S rows (one wave each), 64
    // lines per workgroup (yc_L)
    int32_t vs_S, vs_tiles, yc_S, yc_L;
    int32_t yc_tiles, exr_tiles, exr_tab, pad4;
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
    const double* vf;   // factors of the v-line matrix, kVF * nv + kVS
    const double* st;   // step table, kStepStride * (n_steps + 1)
    const double* rf;   // r rows of (I - theta dt A1), theta dt folded in: kRF * nr
    const double* gd;   // Dirichlet increments g(t_{n+1}) - g(t_n): (2 ny + nr) per step
    const double* vg;   // segmented v-solve constants, kVG * nv
    double* yinv;       // y-line reciprocal pivots 1 / den_k of (I - theta dt A3), nr*nv*ny (once per solve)
    // ADI scheme stage.  0: the Douglas step.  The Craig-Sneyd family runs the
    // Douglas sweeps as stage 1 (the y sweep leaves D3 in D, U unchanged), then
    // stage 2 on a second descriptor whose D is the correction array E:
    //   E0 = dt A U + dt (sc_a0 A0 + sc_a1 (A1 + A2 + A3)) D3 + sc_b D3
    // on non-Dirichlet nodes (D3 read from the D3 pointer), the increment
    // g(t_{n+1}) - g(t_n) on Dirichlet nodes when sc_b = 0 and 0 otherwise;
    // the same sweeps; U += E3, plus D3 when hv.  Huang's correction runs the
    // stage-2 sequence af_iters times with (sc_a0, sc_a1, sc_b) = (theta,
    // theta, -1): each but the last adds E3 to D3 (D3 holds the iterate X_m)
    int32_t stage, hv;
    int32_t soften;     // terminal data averaged over control elements (section 7.2): 0, 1 all, 2 at the kink
    int32_t ypiv_skip;  // the y pivots belong to another solve of the batch (shared operator)
    double sc_a0, sc_a1, sc_b;
    double* D3;
    int32_t* flag;      // health flag: nonzero after a bad pivot or a non-finite value
    int32_t* flag_pad;
};

// r-axis table rows (each nr long).  Row i of the r operator A1 (with the
// reaction term) on a line with variance v and c = f_t + kappa f + y is
//   e      = P c + Q                          (drift of r over J_r, / 2h)
//   A1 row = (MLO e + ALO v,  MDI e + ADI v - RR,  MUP e + AUP v,  MEX e)
// on offsets (-1, 0, +1, extra), where "extra" is +2 on the r_min face and
// -2 on the r_max face.  Centred rows, one-sided outflow rows (section 7.3)
// and Dirichlet rows (all zero) differ only in these entries.
enum { RT_R = 0,   // r_i
       RT_P,       // 1 / (2 h J_r)
       RT_Q,       // -kappa r_i / (2 h J_r)
       RT_MLO, RT_MDI, RT_MUP, RT_MEX,
       RT_ALO, RT_ADI, RT_AUP,
       RT_RR,      // r_i, 0 on a Dirichlet row
       RT_X,       // lambda r^gamma / J_r, 0 on the r faces
       RT_Y,       // lambda^2 r^{2 gamma}
       RT_ELO, RT_EHI,  // the node's control element [r(x_i - h/2), r(x_i + h/2)] (softening)
       kRT };
// v-axis table rows (each nv long): the A2 row on offsets -2..+2 and the
// v factor of the mixed term.
enum { VT_V = 0,   // v_j
       VT_O0, VT_O1, VT_O2, VT_O3, VT_O4,
       VT_X,       // rho epsilon v / J_v / (4 h_r h_v), 0 on the v faces
       kVT };
// y-axis table rows (each ny long).  Explicit A3 at (i, j, k):
//   (RT_Y[i] v_j YT_I[k] - YT_K[k]) * sum_w YT_W[w] U_{k+w}, w = -2..+2.
// Implicit row of (I - theta dt A3) on line (i, j) with q = RT_Y[i] v_j:
//   a = YT_T1 q + YT_T2,  row = (YT_MA a, 1 + YT_MB a, YT_MC a, YT_ME a).
enum { YT_Y = 0,   // y_k
       YT_I,       // 1 / J_y
       YT_K,       // 2 kappa y / J_y
       YT_W0, YT_W1, YT_W2, YT_W3, YT_W4,
       YT_T1, YT_T2,
       YT_MA, YT_MB, YT_MC, YT_ME,
       YT_ELO, YT_EHI,  // the node's control element in y (softening)
       kYT };
// v-line factors: rows (each nv long) then scalars.  Forward sweep of row j:
// d'_j = (d_j - VF_A[j] d'_{j-1}) * VF_INV[j]; back: x_j = d'_j - VF_C[j] x_{j+1}.
enum { VF_A = 0, VF_INV, VF_C, kVF };
// scalars after the rows: row 0 (b, c, e), factor eliminating x0 from row 1,
// row n-1 (a, b, e), factor eliminating x_{n-1} from row n-2
enum { VS_B0 = 0, VS_C0, VS_E0, VS_F1, VS_AL, VS_BL, VS_EL, VS_F2, kVS };
// r-row table of the split path.  Interior row i of (I - theta dt A1) on a
// line with variance v and c = f_t + kappa f + y, with e = FP c + FQ:
//   (A, B, C) = (FALO v + e,  FADI v + FB,  FAUP v - e)
enum { RF_P = 0, RF_Q, RF_ALO, RF_ADI, RF_AUP, RF_B, kRF };
// Segmented v solve (the v-line matrix depends on j alone).  With the faces
// folded into rows 1 and n-2 (rows 0 and n-1 pass through as identity and are
// recovered last), the forward sweep is d'_j = INV_j d_j + AL_j d'_{j-1} and
// the backward x_j = d'_j - CP_j x_{j+1}.  Each segment runs both from zero
// and adds G_j d'_in (G_j: product of AL from the segment start to j) and
// H_j x_in (H_j: product of -CP from j to the segment end).
// K_j, for the v sweep folded into the fused kernel: the backward sweep of G
// within the segment (K_end = G_end, K_j = G_j - CP_j K_{j+1}), so that the
// final value is x0_j + K_j d'_in + H_j x_in with x0 the segment's own
// solution from zero.
enum { VG_INV = 0, VG_AL, VG_CP, VG_G, VG_H, VG_K, kVG };
// most v segments (of kExrJ rows) a folded v sweep hands over
constexpr int kMaxFoldSegs = 16;

// Dirichlet increments of step n: r_min face (ny values, by k), r_max face
// (ny), y_max face (nr, by i); zero where the face is not Dirichlet.
enum { GD_RLO = 0, GD_RHI = 1, GD_YHI = 2 };

// step table entries, per time level n (t_n = T - n dt)
enum { ST_PHI = 0, ST_AT, ST_GT, ST_HT, ST_AM, ST_GM, ST_HM };

enum { KIND_BOND = 0, KIND_CAPLET = 1, KIND_FLOORLET = 2, KIND_FORWARD = 3 };

// Readout request: 4x4 Lagrange stencil on the lowest y plane of one solve.
// The kernel writes three values per request: the price (weights wr x wv),
// d price / dr (dwr x wv) and d price / dv (wr x dwv), the derivative
// weights being those of the interpolant in mesh coordinates times dx/dz.
struct Readout {
    int32_t solve;
    int32_t i0, j0;
    int32_t pad;
    double wr[4];
    double wv[4];
    double dwr[4];
    double dwv[4];
};

// Record the next sweep launch of the calling thread between these two
// events (written by the dispatch itself; used for per-kernel timing).
void set_launch_events(hipEvent_t start, hipEvent_t stop);

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
// J: v nodes per k_exp thread (4, 8 or 16)
hipError_t launch_exp(int J, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int step, hipStream_t st,
                      bool stage2 = false);
hipError_t launch_rs(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int step, int nr_max,
                     hipStream_t st);
// k_exr dynamic LDS (bytes) and table offset (doubles) for nr = S * rows
// (rows >= 8: a pass's scratch, 8 doubles per lane, fits in its rows); the
// same for both explicit phases
void exr_lds(int nr, int rows, size_t* bytes, int* tab);
// Whole y planes per fused tile: as many as the workgroup's threads cover
// (one per r node), fewer where the r solve's lanes (kExrJ lines of S lanes
// per plane) would leave its last pass part-full, most of that pass's lanes
// idle (nr = 48: five planes need 1.25 passes, four need one; nr = 32 at 8
// rows keeps eight planes in two full passes).
inline int exr_planes(int nr, int rows)
{
    const int per_plane = kExrJ * (nr / rows);
    int p = kBlock / nr;
    while (p > 1 && p * per_plane > kBlock && (p * per_plane) % kBlock != 0) --p;
    return p > 1 ? p : 1;
}
// window: the explicit phase reads its neighbours from an LDS window of its
// tile (else each thread loads its own).  The predictor only: the corrected
// start keeps the per-lane loads.
// fold: the v sweep folded in (window form, Douglas only): D1 stays in the
// tile and the tile's v segment is solved from zero (k_vfix and k_yc finish it)
hipError_t launch_exr(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int step, size_t lds,
                      hipStream_t st, bool stage2 = false, bool window = false, bool fold = false);
// rows per thread available to k_rs
bool rs_rows_supported(int rows);
hipError_t launch_vs(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int S_max, hipStream_t st);
// the folded v sweep's segment hand-over and face rows: one thread per v line
// (i, k), tasks of kBlock lines
// segs: the v segments of every solve of the launch (2 .. kMaxFoldSegs)
hipError_t launch_vfix(const SolveDesc* d_desc, const int2* tasks, int n_tasks, int segs, hipStream_t st);
// Dirichlet increments of every step into each solve's gd table; max_entries
// = the largest (2 ny + nr) n_steps of the solves
hipError_t launch_gd(const SolveDesc* d_desc, int n_solves, int64_t max_entries, hipStream_t st);
hipError_t launch_ypiv(const SolveDesc* d_desc, int n_solves, int64_t max_lines, hipStream_t st);
// mode 0: U += D3 (Douglas; the last sequence of CS and MCS); 1: D3 stays in
// D (the first sequence of the Craig-Sneyd family); 2: U += D3 + E3 (HV's
// last); 3: D3 += E3 (an intermediate Huang subiteration).  minors: the
// reciprocal pivots are formed in the kernel from the minors recurrence, else
// read from the array k_ypiv wrote
hipError_t launch_yc(int rows, const SolveDesc* d_desc, const int2* tasks, int n_tasks, int S_max, hipStream_t st,
                     int mode = 0, bool minors = false, bool fold = false);
// k_yc holds 4 ROWS-long arrays per thread: workgroups of at most 128 / ROWS
// waves keep them in registers
constexpr int yc_max_segments(int rows) { return 128 / rows; }
// rows per thread available to k_vs and k_yc
bool vs_rows_supported(int rows);
bool yc_rows_supported(int rows);
hipError_t launch_readout(const SolveDesc* d_desc, const Readout* rq, int n, double* out, hipStream_t st);
hipError_t launch_health(const SolveDesc* d_desc, int n_solves, int64_t max_points, hipStream_t st);

}  // namespace hjm
