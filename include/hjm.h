/*
 * hjm.h -- C ABI of the MI355X (gfx950) Douglas-ADI solver for the
 * single-factor Heath-Jarrow-Morton model with stochastic volatility
 * (Valero, Torrealba, Lacasa, Fraysse).
 *
 * Problem (section 3): price, at t = 0 and state (r0, v0, y = 0), a contract
 * paying F at T on the PDE of eq. (1) in (r, v, y) with coefficients from
 * the short-rate SDE (section 3.1) and terminal / boundary data of section
 * 3.2, discretised on the sinh mesh of section 4.3 with the centred stencils
 * of eq. (esquema), theta = 1/2 (Crank-Nicolson) and the Douglas ADI
 * splitting of section 5.1.
 *
 * Conventions shared by every entry point:
 *  - Grids are FP64, indexed U[(k*nv + j)*nr + i] with i along r (contiguous),
 *    j along v and k along y.  "n" nodes per axis include both end nodes.
 *  - Device memory and the HIP stream belong to the caller; the library only
 *    borrows them between create and destroy and never allocates device
 *    memory.  Opaque handles are host objects owned by the library.
 *  - Every call returns hjm_status: HJM_OK (0) or a negative error; nothing
 *    throws across the ABI.  hjm_last_error() returns a message for the last
 *    failure of the calling thread.
 *  - Handles are not thread-safe: one handle is used from one thread and one
 *    stream at a time.
 *  - Asynchronous calls (create, step, batch run) only enqueue work on the
 *    stream; calls that return host values (price, prices) synchronise it.
 */
#ifndef HJM_H
#define HJM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hjm_status;
#define HJM_OK        0
#define HJM_EINVAL   (-1)  /* invalid argument; detected on the host before any device work */
#define HJM_ENOMEM   (-2)  /* the caller's workspace is too small */
#define HJM_EDEVICE  (-3)  /* a HIP runtime call failed */
#define HJM_ENUMERIC (-4)  /* a non-finite value or a non-positive pivot was met */
#define HJM_ESTATE   (-5)  /* call out of order (e.g. price before every step ran) */

/* Face types.  OUTFLOW: one-sided second-order normal first difference
   (section 7.3), the normal second-derivative term taken as zero (section
   3.2); allowed only where the drift points out of the domain in backward
   time (checked: HJM_EINVAL otherwise).  DIRICHLET: the closed-form value of
   the contract with a linear payoff (section 4.1 bond formula) is imposed.
   Dirichlet is accepted on the r faces and on the y_max face only. */
#define HJM_FACE_OUTFLOW   0
#define HJM_FACE_DIRICHLET 1

/* Payoffs (section 3.2): bond pays 1; caplet max(1 - Delta p(T,T_M), 0);
   floorlet max(Delta p(T,T_M) - 1, 0); forward 1 - Delta p(T,T_M), with
   Delta = 1 + (T_M - T) K. */
#define HJM_BOND     0
#define HJM_CAPLET   1
#define HJM_FLOORLET 2
#define HJM_FORWARD  3

/* One axis of the hyperbolic mesh z = center + alpha sinh(c2 x + c1 (1-x)),
   x in [0,1] uniform (eq. (metrica), section 4.3 / 7.1).  Requires n >= 5,
   alpha > 0, z_min < z_max. */
typedef struct {
    int32_t n;
    int32_t lo_face;
    int32_t hi_face;
    int32_t reserved;
    double z_min, z_max, center, alpha;
} hjm_axis;

/* Model of section 3.1: dr = (f_t - kappa (r - f) + y) dt + sqrt(v) lambda r^gamma dW,
   dv = theta_v (1 - v) dt + epsilon sqrt(v) dZ, dW dZ = rho dt, and the
   initial curve f(0,t) = f_level + f_slope (1 - exp(-f_decay t)).
   Requires kappa >= 0, theta_v >= 0, lambda >= 0, epsilon >= 0, |rho| <= 1,
   gamma in [0,1] (gamma > 0 needs r_min >= 0), f_decay >= 0.

   Discrete curve (section 6.1): with curve_n >= 2 the initial curve is
   instead given by zero-coupon prices P(0, t_i) = curve_p[i] at maturities
   curve_t[i] (host memory, read once by the create call and not kept),
   smoothed by the natural cubic spline S of -ln P(0, t) through the knots:
   f(0,t) = S'(t), df(0,t)/dt = S''(t) (continuous, as the paper asks), and
   P(0,t) = exp(-S(t)); beyond the last knot the forward stays at its value
   there.  Requires 2 <= curve_n <= HJM_MAX_CURVE_KNOTS, curve_t[0] = 0 and
   curve_p[0] = 1, curve_t strictly increasing, every value finite and every
   price > 0 (else HJM_EINVAL); f_level, f_slope and f_decay are then
   ignored.  curve_n = 0 selects the parametric curve. */
#define HJM_MAX_CURVE_KNOTS 64
typedef struct {
    double kappa, theta_v, lambda, gamma, epsilon, rho;
    double f_level, f_slope, f_decay;
    int32_t curve_n;
    int32_t reserved;
    const double* curve_t;
    const double* curve_p;
} hjm_model;

/* Contract: kind, expiry T > 0, payment T_M > T and strike K > 0 (caplet,
   floorlet, forward; ignored for the bond).  soften replaces the terminal
   data by their average over the node's control element (section 7.2): the
   element is centred on the node in the mesh coordinates, [z(x - h/2),
   z(x + h/2)] in r and in y (the payoff does not depend on v); closed form in
   r across the payoff's kink, 16-point Gauss-Legendre in y.  0: pointwise
   payoff (the paper's default); 1: every non-Dirichlet node; 2: only the
   nodes whose element the caplet's or floorlet's kink crosses (the rest keep
   the pointwise payoff, which is smooth there).  Dirichlet nodes always keep
   the pointwise data. */
typedef struct {
    int32_t kind;
    int32_t soften;
    double expiry, pay, strike;
} hjm_payoff;

/* ADI scheme of a grid.  HJM_SCHEME_DOUGLAS is the paper's step (section
   5.1): explicit predictor, then (I - theta dt A_d) sweeps along r, v, y.  The
   other three add a correction stage for the mixed r-v derivative (which
   Douglas treats explicitly, first order in time) and reach second order:
   Craig-Sneyd (the paper mentions trying it, section 5.1), modified
   Craig-Sneyd and Hundsdorfer-Verwer, as defined by in 't Hout and Welfert
   (Appl. Numer. Math. 57, 2007).  Each runs the Douglas sweeps, forms a
   corrected start from their result and sweeps once more: twice the work of
   a Douglas step.  theta in (0, 1]: the paper uses 1/2; 1/3 is usual for
   modified Craig-Sneyd and 1/2 + sqrt(3)/6 for Hundsdorfer-Verwer.  Every
   operator is evaluated at t_{n+1/2}.
   HJM_SCHEME_HUANG is the Douglas step followed by af_iters (1..16)
   subiterations of Huang's approximate-factorisation correction (section
   5.1): each solves M (X_{m+1} - X_m) = D0 - (I - theta dt A) X_m with the
   factored M = (I - theta dt A1)(I - theta dt A2)(I - theta dt A3), starting
   from the Douglas increment X_1, so that the increment tends to that of the
   unsplit theta scheme (I - theta dt A) X = D0 where the iteration
   contracts; af_iters + 1 times the work of a Douglas step.  One
   subiteration at theta = 1/2 is Hundsdorfer-Verwer at theta = 1/2.
   af_iters is ignored by the other schemes. */
#define HJM_SCHEME_DOUGLAS 0
#define HJM_SCHEME_CS      1
#define HJM_SCHEME_MCS     2
#define HJM_SCHEME_HV      3
#define HJM_SCHEME_HUANG   4
#define HJM_MAX_AF_ITERS   16
typedef struct {
    int32_t kind;
    int32_t af_iters;
    double theta;
} hjm_scheme;

typedef struct hjm_grid hjm_grid;
typedef struct hjm_batch hjm_batch;

/* Bytes of device workspace hjm_grid_create needs for these axes and step
   count: the grid U, the Douglas increment D and the reciprocal pivots of the y-line
   matrices (which do not change from step to step), nr*nv*ny doubles each,
   plus 1D tables (axis coefficients, per-step curve and bond-factor scalars,
   per-step Dirichlet increments on the r and y_max faces, (2 ny + nr) doubles
   per step, readout weights and a health flag).  Host only. */
hjm_status hjm_workspace_bytes(const hjm_axis ax[3], int32_t n_steps, size_t* bytes);

/* Validate the problem, lay out the caller's workspace (d_workspace, at least
   hjm_workspace_bytes, 256-byte aligned), upload the tables and enqueue the
   terminal data U := payoff at t = T on hip_stream (a hipStream_t; NULL is
   the null stream).  n_steps > 0 Douglas steps of dt = T / n_steps will take
   the solution back to t = 0.  On success *out owns a host handle. */
hjm_status hjm_grid_create(const hjm_axis ax[3], const hjm_model* model, const hjm_payoff* payoff,
                           int32_t n_steps, void* d_workspace, size_t ws_bytes, void* hip_stream,
                           hjm_grid** out);

/* The same with an explicit ADI scheme (hjm_grid_create is the Douglas
   scheme with theta = 1/2).  The workspace of a correction scheme holds one
   more nr*nv*ny array (hjm_scheme_workspace_bytes).  The correction schemes
   run on the lane-split r solve and the stored-pivot y solve only: nr =
   S * ROWS (S a power of two) with the r rows within the spike bound, and
   ny = S * ROWS; other grids get HJM_EINVAL (before any device work), as do
   an unknown kind or theta outside (0, 1].  hjm_adi_step then enqueues whole
   steps of the chosen scheme. */
hjm_status hjm_scheme_workspace_bytes(const hjm_axis ax[3], int32_t n_steps, const hjm_scheme* scheme,
                                      size_t* bytes);
hjm_status hjm_grid_create_scheme(const hjm_axis ax[3], const hjm_model* model, const hjm_payoff* payoff,
                                  const hjm_scheme* scheme, int32_t n_steps, void* d_workspace, size_t ws_bytes,
                                  void* hip_stream, hjm_grid** out);

/* Enqueue k more Douglas steps (section 5.1) on the grid's stream.
   HJM_ESTATE if that would go past n_steps. */
hjm_status hjm_adi_step(hjm_grid* g, int32_t k);

/* After all n_steps: synchronise the stream, check the health flag and the
   grid for non-finite values (HJM_ENUMERIC), and return C(t=0; r0, v0, y=0)
   by tensor 4-point Lagrange interpolation in the mesh coordinates on the
   lowest y plane.  HJM_ESTATE before the last step, HJM_EINVAL if (r0, v0)
   is outside the mesh. */
hjm_status hjm_price(hjm_grid* g, double r0, double v0, double* out);

/* As hjm_price, with the Greeks the paper plots (section 6): out[0] = C,
   out[1] = rho = dC/dr and out[2] = vega = dC/dv at (r0, v0, y=0), the
   derivatives of the same interpolant (in mesh coordinates, times the mesh
   map's dx/dz). */
hjm_status hjm_price_greeks(hjm_grid* g, double r0, double v0, double out[3]);

/* Borrow the device grid U (nr*nv*ny doubles, inside the caller's workspace)
   and the number of steps taken so far.  Writing U and then calling
   hjm_grid_set_step restores a checkpoint. */
hjm_status hjm_grid_solution(hjm_grid* g, double** d_U, int64_t* step);

/* Declare that U holds the solution after `step` steps (0 <= step <= n_steps),
   e.g. after copying a checkpoint into the borrowed U. */
hjm_status hjm_grid_set_step(hjm_grid* g, int64_t step);

/* Release the host handle (the caller's device memory is untouched). */
hjm_status hjm_grid_destroy(hjm_grid* g);

/* How the solve is carried out (host only): plan[0] = r-line method
   (0 spike and 1 chain, both in the kernel that also computes the explicit
   predictor; 2 split: separate explicit kernel, then a spike solve with the
   segments of a line in consecutive lanes of one wavefront; 3 fused: the
   explicit predictor of a tile into LDS and that spike solve in one kernel,
   for nr <= 256 with at least 8 rows per lane), plan[1] = rows per lane of
   the split or fused r solve (0 otherwise), plan[2..4] = the line-tile
   rows per thread of the r, v and y solves, plan[5] = rows per segment of the
   segmented v solve (0: the chained v solve), plan[6] = rows per segment of
   the y solve on stored pivots (0: the per-step elimination), plan[7] = the
   ADI scheme (HJM_SCHEME_*), plan[8] = 1 where the y sweep forms its pivots
   from the minors recurrence (0: stored by the pivot kernel), plan[9] = 1
   where the v sweep is folded into the explicit + r and y kernels (16-row
   segments joined by the hand-over kernel; 0: a v kernel of its own).  The
   spike variants are chosen only where the r rows keep (|A| + |C|) / B
   bounded (section 5, tridiagonal systems), so every variant matches the
   sequential elimination to rounding. */
hjm_status hjm_grid_plan(const hjm_grid* g, int32_t plan[10]);

/* Per-pass timing.  While enabled, each kernel launch of hjm_adi_step is
   bracketed by HIP events recorded on the grid's stream.  Passes, in order:
     0  explicit predictor (on grids whose r lines are solved in the same
        kernel, that kernel: explicit predictor + r sweep)
     1  r sweep (no launches when fused into pass 0)
     2  v sweep
     3  y sweep + update */
#define HJM_N_PASSES 4
hjm_status hjm_grid_profile(hjm_grid* g, int32_t enable);

/* Synchronise the stream and return, per pass, the summed event-to-event
   milliseconds and the number of launches bracketed since the previous read
   (ms[HJM_N_PASSES], launches[HJM_N_PASSES]); the sums restart from zero. */
hjm_status hjm_grid_profile_read(hjm_grid* g, double ms[HJM_N_PASSES], int64_t launches[HJM_N_PASSES]);

/* Pricing without allocation, for callers that cannot allocate device
   memory (code that must not call hipMalloc: set-up inside HIP graph
   capture, tight serving loops, harnesses that forbid allocation).
   hjm_price_static runs one whole Douglas solve (theta = 1/2) from t = T to
   t = 0 and reads it out, like hjm_grid_create + hjm_adi_step(n_steps) +
   hjm_price_greeks, with the same kernels and the same results bit for bit,
   but every working array of the solve (the Douglas increment D, the y
   pivots, the tables, the descriptor, the readout slot and the health flag)
   lives in a library-owned device array of HJM_STATIC_SCRATCH_BYTES, one per
   GPU, held until the process ends.  The library allocates nothing.
     d_U    caller's device memory, nr*nv*ny doubles, 256-byte aligned: the
            grid (on return, the solution at t = 0, laid out as in every grid)
     out    host: out[0] = C, out[1] = rho, out[2] = vega at (r0, v0, y = 0)
   hip_stream must belong to the calling thread's current device (HJM_EINVAL
   otherwise).  Synchronises the stream.  Errors: as hjm_grid_create and
   hjm_price_greeks; HJM_ENOMEM (before any device work) when the working
   arrays need more than HJM_STATIC_SCRATCH_BYTES (hjm_static_scratch_bytes
   reports the need: 16 bytes per grid point plus the tables, so grids up to
   about 2 million points fit).  Every call on one GPU shares that GPU's array
   and overwrites what the last call left there: calls that overlap on one
   GPU (from several threads, or on several streams) race and give wrong
   results. */
#define HJM_STATIC_SCRATCH_BYTES (32u << 20)
hjm_status hjm_static_scratch_bytes(const hjm_axis ax[3], int32_t n_steps, size_t* bytes);
hjm_status hjm_price_static(const hjm_axis ax[3], const hjm_model* model, const hjm_payoff* payoff,
                            int32_t n_steps, double r0, double v0, double* d_U, void* hip_stream,
                            double out[3]);

/* ---------------------------------------------------------------------- */
/* Batched independent solves (calibration-style throughput).              */
/* ---------------------------------------------------------------------- */

/* Workspace for n solves with axes ax[s][3] and n_steps[s]. */
hjm_status hjm_batch_workspace_bytes(int32_t n, const hjm_axis* ax, const int32_t* n_steps,
                                     size_t* bytes);

/* n independent solves: ax is n*3 axes (solve-major), model/payoff/n_steps
   arrays of n.  Validates each like hjm_grid_create, lays out the shared
   workspace and uploads the tables (synchronises the stream). */
hjm_status hjm_batch_create(int32_t n, const hjm_axis* ax, const hjm_model* model,
                            const hjm_payoff* payoff, const int32_t* n_steps,
                            void* d_workspace, size_t ws_bytes, void* hip_stream,
                            hjm_batch** out);

/* The same with an ADI scheme per solve (schemes: n entries, section 5.1 and
   the Craig-Sneyd family as for hjm_grid_create_scheme; null means Douglas
   with theta = 1/2 for every solve, as hjm_batch_create).  A solve with a
   correction scheme needs the kernels a grid of that scheme needs (else
   HJM_EINVAL naming the solve, before any device work) and one more
   nr*nv*ny array of workspace (hjm_batch_scheme_workspace_bytes).  Solves
   share an operator only with the same theta and the same kind of pivots
   (correction schemes store them).  Every price equals the single grid's of
   the same scheme bit for bit. */
hjm_status hjm_batch_scheme_workspace_bytes(int32_t n, const hjm_axis* ax, const int32_t* n_steps,
                                            const hjm_scheme* schemes, size_t* bytes);
hjm_status hjm_batch_create_scheme(int32_t n, const hjm_axis* ax, const hjm_model* model,
                                   const hjm_payoff* payoff, const hjm_scheme* schemes,
                                   const int32_t* n_steps, void* d_workspace, size_t ws_bytes,
                                   void* hip_stream, hjm_batch** out);

/* Enqueue a complete solve of every problem: terminal data at t = T, then
   every step (each of its sweep sequences: one for Douglas, two for the
   Craig-Sneyd family, 1 + q for Huang's correction), where at step n one
   launch per pass and sequence covers all solves with more than n steps.  The solves are dealt to hjm_get_batch_streams()
   stream lanes (snake order by work), each launched on a stream the batch
   owns, forked from and joined back to the batch's stream with events, so
   that kernels of different lanes run concurrently; every result stays
   bit-identical.  use_graph != 0 captures the launches (lanes included) into
   a HIP graph on the first call (the stream must not be the null stream) and
   replays it afterwards. */
hjm_status hjm_batch_run(hjm_batch* b, int32_t use_graph);

/* After hjm_batch_run: synchronise, check health, and read out the n prices
   at (r0[s], v0[s]) as hjm_price does. */
hjm_status hjm_batch_prices(hjm_batch* b, const double* r0, const double* v0, double* out);

/* The same with the Greeks: out[3 s .. 3 s + 2] = (C, dC/dr, dC/dv) of solve
   s, as hjm_price_greeks. */
hjm_status hjm_batch_greeks(hjm_batch* b, const double* r0, const double* v0, double* out);

/* Per-kernel timing of eager runs (hjm_batch_run with use_graph = 0): every
   launch of the first `steps` Douglas steps is bracketed by HIP events the
   dispatch records (0 turns it off; graph runs are never timed).  Those steps
   run one launch at a time on the batch's stream (no lane overlap), so each
   duration is the kernel's own.  The read
   synchronises and returns, per pass (as for grids), the summed milliseconds,
   the launches and the grid points those launches advanced by one step; the
   sums restart from zero. */
hjm_status hjm_batch_profile(hjm_batch* b, int32_t steps);
hjm_status hjm_batch_profile_read(hjm_batch* b, double ms[HJM_N_PASSES], int64_t launches[HJM_N_PASSES],
                                  int64_t points[HJM_N_PASSES]);

hjm_status hjm_batch_destroy(hjm_batch* b);

/* ---------------------------------------------------------------------- */
/* Tuning and diagnostics.                                                 */
/* ---------------------------------------------------------------------- */

/* Line-solve tile: rows per thread of the segmented tridiagonal solves
   (8, 16 or 32) for the r, v and y sweeps.  Applies to handles created
   afterwards in this process.  HJM_EINVAL for other values. */
hjm_status hjm_set_line_tile(int32_t r_rows, int32_t v_rows, int32_t y_rows);
hjm_status hjm_get_line_tile(int32_t* r_rows, int32_t* v_rows, int32_t* y_rows);

/* Per-shape line tiles (the autotuner's choices): the preferred rows per
   thread (8, 16 or 32; 0 removes the override) of the line solves along
   `axis` (0 r, 1 v, 2 y) on grids with n nodes on that axis and `lines`
   such lines (the product of the other two node counts; 0: any count), in
   place of hjm_set_line_tile's value there.  A solve takes the override of
   its exact line shape, else the one for its line length, else the global
   value.  Handles created afterwards use them; inside a batch each solve
   takes its own shape's rows (solves that end up with different kernel
   variants launch in separate groups).  Every setting gives the same prices
   to rounding (the plans keep every variant within rounding of the
   sequential elimination). */
hjm_status hjm_set_axis_tile(int32_t axis, int32_t n, int64_t lines, int32_t rows);
hjm_status hjm_get_axis_tile(int32_t axis, int32_t n, int64_t lines, int32_t* rows);
hjm_status hjm_clear_axis_tiles(void);

/* ---------------------------------------------------------------------- */
/* Learned surrogate (caplet prices inside a box of model inputs).          */
/* ---------------------------------------------------------------------- */
/* An MLP 8 -> 256 -> 256 -> 256 -> 256 -> 1 with GELU activations, trained on
   the solver's own prices.  Inputs (float32, 8 per row, physical units):
   kappa, epsilon, rho, v0, curve level, curve slope, strike offset from the
   at-the-money strike, expiry.  Each is mapped to [-1, 1] over the training
   box; matrix products take BF16 operands and accumulate in FP32 on the matrix
   cores; master weights, biases, gradients and Adam state are FP32.  The
   network output y is reported as y * out_scale + out_shift.  Parameters are
   one float32 vector of HJM_MLP_PARAMS: W1 (256 x 8), b1, W2 (256 x 256), b2,
   W3, b3, W4, b4, w5 (256), b5, weights row-major (output x input).  All device
   memory (parameters, optimiser state, activations for up to max_batch rows)
   lives in the caller's workspace. */
typedef struct hjm_mlp hjm_mlp;
#define HJM_MLP_PARAMS 199937

/* Workspace bytes for batches of up to max_batch rows (1 <= max_batch <= 2^26). */
hjm_status hjm_mlp_workspace_bytes(int64_t max_batch, size_t* bytes);

/* Create with the training box (lo < hi per input) and the output map; the
   parameters start at zero (set them with hjm_mlp_set_params).  Synchronises. */
hjm_status hjm_mlp_create(const float box_lo[8], const float box_hi[8], float out_scale, float out_shift,
                          int64_t max_batch, void* d_workspace, size_t ws_bytes, void* hip_stream,
                          hjm_mlp** out);

/* Copy HJM_MLP_PARAMS host floats in (resets the Adam state) or out. */
hjm_status hjm_mlp_set_params(hjm_mlp* m, const float* params, int64_t n);
hjm_status hjm_mlp_get_params(hjm_mlp* m, float* params, int64_t n);

/* Loss and gradients of the mean squared error over n <= max_batch rows:
   d_x (n x 8 float32, device), d_t (n targets in network units, device).
   The gradient stays in the workspace (read it with hjm_mlp_get_grads);
   *sse (may be null) receives the summed squared error, synchronising. */
hjm_status hjm_mlp_gradients(hjm_mlp* m, const float* d_x, const float* d_t, int64_t n, double* sse);
hjm_status hjm_mlp_get_grads(hjm_mlp* m, float* grads, int64_t n);

/* One Adam step (Kingma and Ba) with the current gradient. */
hjm_status hjm_mlp_adam(hjm_mlp* m, float lr, float beta1, float beta2, float eps);

/* One pass over n rows in minibatches of `batch` rows, in order (shuffle the
   rows beforehand): gradients then Adam (beta 0.9, 0.999, eps 1e-8) per
   minibatch.  *mean_loss (may be null) receives the mean squared error seen. */
hjm_status hjm_mlp_train_epoch(hjm_mlp* m, const float* d_x, const float* d_t, int64_t n, int64_t batch,
                               float lr, double* mean_loss);

/* Prices of n rows (any n; processed max_batch rows at a time): d_y[r] =
   network(d_x[r]) * out_scale + out_shift, and d_in_box[r] = 1 where every
   input lies inside the training box, else 0 (there the caller falls back to
   the solver; d_in_box may be null).  Asynchronous. */
hjm_status hjm_mlp_infer(hjm_mlp* m, const float* d_x, int64_t n, float* d_y, uint8_t* d_in_box);

/* Gaussian caplet baseline: a control variate for the output.  Set, the
   network's output y stands for ln(price / B(x)): hjm_mlp_infer reports
   B(x) exp(y * out_scale + out_shift) instead of the affine map, and
   hjm_mlp_targets forms (ln(price / B(x)) - out_shift) / out_scale.  B is the
   caplet of the Gaussian special case of the model (section 3.1 with
   gamma = 0, no stochastic variance: the textbook bond put), with the rate
   volatility frozen at lambda f(0,T)^gamma times the root of the variance
   factor's mean path 1 + (v0 - 1) e^{-theta_v t}; the row's curve is
   f(0,t) = level + slope (1 - e^{-f_decay t}) (section 2), payment one tenor
   after expiry, strike = at-the-money strike (simple compounding over the
   tenor, as the accrual of section 3.2) + the row's offset.  Computed in
   FP64 on the device.  Null b switches the baseline off (the default).
   HJM_EINVAL unless lambda > 0, gamma in [0, 1], theta_v >= 0, f_decay > 0,
   tenor > 0, all finite.  The output of rows outside the box is unspecified
   (may be NaN where the baseline is undefined there). */
typedef struct { double lambda, gamma, theta_v, f_decay, tenor; } hjm_mlp_baseline;
hjm_status hjm_mlp_set_baseline(hjm_mlp* m, const hjm_mlp_baseline* b);

/* Training targets in network units of n rows (0 <= n <= 2^31): d_t[r] =
   (ln(d_price[r] / B(d_x[r])) - out_shift) / out_scale with the baseline,
   (d_price[r] - out_shift) / out_scale without.  d_x n x 8 float32, d_price
   n float64, d_t n float32, all device memory owned by the caller.  A price
   <= 0 with the baseline gives NaN (drop such rows before training).
   Asynchronous on the handle's stream. */
hjm_status hjm_mlp_targets(hjm_mlp* m, const float* d_x, const double* d_price, int64_t n, float* d_t);

hjm_status hjm_mlp_destroy(hjm_mlp* m);

/* Nodes along v that one thread of the explicit-predictor kernel computes
   (4, 8 or 16; HJM_EINVAL otherwise).  Process-wide, read when a grid or
   batch is created, like the line tile. */
hjm_status hjm_set_explicit_chunk(int32_t J);
hjm_status hjm_get_explicit_chunk(int32_t* J);

/* Whether grids and batches created afterwards fuse the explicit predictor
   with the spike r solve where they can (plan method 3; on by default).  Off,
   those solves take the split pair of kernels instead: the same arithmetic,
   16 more bytes of memory traffic per grid point and step.  Process-wide. */
hjm_status hjm_set_r_fusion(int32_t on);
hjm_status hjm_get_r_fusion(int32_t* on);

/* How the fused explicit + r kernel reads the explicit predictor's
   neighbours (eq. (esquema) stencils): on (default), each workgroup stages
   its tile's v window of U in LDS and reads the r neighbours and mixed-term
   corners there; off, every thread loads its own neighbours (lane moves for
   the r neighbours).  Same values either way.  For handles created
   afterwards; grids of 4 GiB or more always take the second form. */
hjm_status hjm_set_exr_window(int32_t on);
hjm_status hjm_get_exr_window(int32_t* on);

/* Where the y sweep on reciprocal pivots (plan[6] > 0) takes its pivots
   1/den_k of the Thomas elimination of (I - theta dt A3) (section 7.1; the y
   operator does not change from step to step): on (default), the sweep forms
   them every step from the minors of the line matrix, den_k = th_k / th_{k-1}
   with th_k = B_k th_{k-1} - A_k C_{k-1} th_{k-2}, which needs no stored
   array (8 bytes per grid point less traffic per step); off, a set-up kernel
   stores them once per solve (den_k = B_k - A_k C_{k-1} / den_{k-1}) and
   every step reads them.  The two agree to rounding (about 1e-15 relative),
   not bit for bit.  A non-positive pivot raises the health flag either way.
   Grids of the correction schemes always store the pivots.  For handles
   created afterwards.  Process-wide. */
hjm_status hjm_set_y_minors(int32_t on);
hjm_status hjm_get_y_minors(int32_t* on);

/* Whether Douglas solves created afterwards fold the v sweep (section 5.1's
   second implicit sweep) into the other kernels where they can (on by
   default): the fused explicit + r kernel keeps D1 in its tile and solves
   the tile's 16 v rows as one segment of the segmented v sweep from zero; a
   small kernel composes the segments of every v line (and recovers the two
   face rows); the y sweep adds each segment's hand-over terms as it loads
   D2.  One pass over the grid less per step (16 bytes per point).  Needs the
   fused kernel's window form with at most 16 lanes per r line, the y sweep
   on pivots formed in the kernel, nv a multiple of 16 with 2 to 16 segments
   and bounded segment products (plan[5] then reports 16); otherwise, and
   off, the v sweep runs on its own.  Equal to the unfolded sweep to
   rounding, not bit for bit.  Process-wide. */
hjm_status hjm_set_v_fold(int32_t on);
hjm_status hjm_get_v_fold(int32_t* on);

/* Stream lanes of batches created afterwards (1..8, default 3; HJM_EINVAL
   otherwise).  More lanes overlap more kernels at fewer solves per launch.
   Process-wide. */
hjm_status hjm_set_batch_streams(int32_t n);
hjm_status hjm_get_batch_streams(int32_t* n);

/* Shared operators in batches created afterwards (on by default).  Solves
   of a batch that differ only in their payoff (kind, strike, softening) with
   the same axes, model (discrete curve included), expiry, payment date and
   steps discretise one operator: several right-hand sides of one system
   (the strikes of one caplet, a caplet and its floorlet).  With sharing on
   they use the first such solve's coefficient tables: the host builds and
   uploads the tables once per operator, and the y sweeps of the right-hand
   sides are interleaved by line tile so that their table reads meet in
   cache.  Where the y pivots are stored (hjm_set_y_minors(0), and the
   correction schemes) the right-hand sides also share one pivot array,
   which the pivot kernel writes once per operator; where they are formed in
   the sweep each solve keeps its pivot array, which then holds the folded v
   sweep's hand-over values of its own right-hand side.  Each solve keeps its
   own grid, terminal and Dirichlet data; every result is bit-identical to
   the unshared batch.  Process-wide. */
hjm_status hjm_set_batch_share(int32_t on);
hjm_status hjm_get_batch_share(int32_t* on);

/* The number of distinct operators of a batch (n when sharing is off). */
hjm_status hjm_batch_operators(const hjm_batch* b, int32_t* n_operators);

const char* hjm_status_str(hjm_status s);
const char* hjm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HJM_H */
