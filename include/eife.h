/*
 * eife.h -- C ABI of the MI355X (gfx950) exponential-integrator Q1 finite
 * element library.
 *
 * The library advances u_t = D Lap u + f(t, u) on a rectangle
 * prod_a [a_a, a_a + N_a h_a] (d = 1, 2, 3) with homogeneous Dirichlet data
 * (Section 1, eq. (1.1); Section 2, eq. (2.1)), discretised in space with
 * continuous multilinear (Q1) elements on the uniform tensor grid of
 * Section 2.1 (eq. (2.4)) and in time with the explicit exponential
 * Runge-Kutta schemes EIFE1 (eq. (2.13)) and EIFE2 (eq. (2.14)).  Each step
 * uses the simultaneous diagonalisation of the mass and stiffness matrices
 * by the sine transform (Section 4, eqs. (4.1)-(4.4)): type-I sine transforms
 * along every axis, a diagonal phi_k(-tau D lambda) scaling, and the
 * pointwise reaction f evaluated at the nodes.
 *
 * Conventions shared by every call
 *   - Every call returns an int status: EIFE_OK (0) or a negative code.
 *     Nothing is thrown across the ABI.  eife_last_error() returns a message
 *     for the calling thread's most recent failure.
 *   - Nodal arrays ("u") live in device memory owned by the caller: the
 *     values at the unknown nodes, n_{d-1} x ... x n_0 contiguous elements
 *     of the grid's dtype (n_a = N_a - 1 interior nodes, boundary nodes not
 *     stored; n_a = N_a for periodic grids), axis 0 (x) fastest.  The
 *     library keeps no pointer to them after a call returns.
 *   - The grid owns its device workspaces (spectral state, work array,
 *     tables), allocated by eife_create_grid and released by
 *     eife_destroy_grid.  A grid may be used from one host thread at a time,
 *     and calls on one grid that use different streams must be ordered by
 *     the caller (they share the grid's workspaces).
 *   - Work is enqueued on the HIP stream passed in (NULL = the default
 *     stream) and is asynchronous unless stated otherwise.  Argument errors
 *     are reported synchronously; a failed kernel launch returns EIFE_EHIP.
 */
#ifndef EIFE_H
#define EIFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eife_grid_s* eife_grid;

enum eife_status {
  EIFE_OK = 0,
  EIFE_EINVAL = -1,       /* bad argument */
  EIFE_ENOMEM = -2,       /* device allocation failed */
  EIFE_EUNSUPPORTED = -3, /* valid request the library does not implement */
  EIFE_ESTATE = -4,       /* call out of order (e.g. step before set_phi) */
  EIFE_EHIP = -5,         /* HIP runtime error */
  EIFE_ENONFINITE = -6    /* a reduction produced a non-finite value */
};

enum eife_bc { EIFE_BC_DIRICHLET = 0, EIFE_BC_PERIODIC = 1 };
enum eife_dtype { EIFE_F32 = 0, EIFE_F64 = 1 };

/* Reaction terms f(t, x, u). */
enum eife_fkind {
  EIFE_F_ZERO = 0,       /* f = 0 (pure diffusion) */
  EIFE_F_ALLEN_CAHN = 1, /* f = u - u^3 (with D = eps^2) */
  EIFE_F_MMS_U2 = 2,     /* f = u^2 + g, g chosen so u = e^{-t} prod_a sin(pi x_a) solves the PDE:
                            g = (d pi^2 D - 1) e^{-t} s - e^{-2t} s^2, s = prod_a sin(pi x_a) */
  EIFE_F_EX51 = 3,       /* Section 5.1, Example 5.1 (d = 2):
                            f = -(pi^2/2) u + (pi^2/2) e^{-pi^2 t} sin(pi x) sin(pi y) */
  EIFE_F_CONST = 4,      /* f = c0, independent of u, x and t (c0 from eife_set_forcing) */
  EIFE_F_AFFINE_T = 5,   /* f = c0 + c1 t, independent of u and x */
  EIFE_F_FLORY_HUGGINS = 6, /* Section 5.2, Example 5.3: f = (theta/2) ln((1 - u)/(1 + u)) + theta_c u,
                               theta = c0, theta_c = c1 from eife_set_forcing; needs |u| < 1 */
  EIFE_F_TRAVELING_WAVE = 7 /* Section 5.1, Example 5.2: f = (u - u^3) / eps^2 (eps = c0 > 0, the equation
                               has D = 1) on a Dirichlet grid whose boundary nodes carry the exact wave
                               g = (1 - tanh((x - s t) / (2 sqrt(2) eps))) / 2, s = 3 / (sqrt(2) eps),
                               x = origin_x + i h_x.  The data enter as part of f (start of Section 4):
                               the load of interior node i gains -sum_j (M_ij g_j' + D K1_ij g_j) over
                               its boundary neighbours j (Q1 mass M, stiffness K1 for D = 1).  Lumped
                               load only (EIFE_LOAD_NODAL: EIFE_EUNSUPPORTED); no periodic grids. */
};

/* How P_h f(t, u_h) is formed from the nodal values of f (the paper's load
 * tensor has entries (f(t, u_ijk), phi_i phi_j phi_k), Section 4). */
enum eife_load {
  EIFE_LOAD_LUMPED = 0, /* default: F_i = f(t, u_i) * prod_a h_a, P_h f = M^{-1} F */
  EIFE_LOAD_NODAL = 1   /* P_h f replaced by the interpolant of the nodal values f(t, u_i) */
};

/* Create a grid: d in {1,2,3}; N[a] >= 2 intervals on axis a (N[a] <= 4096;
 * any N: prime factors of the FFT length above 7 run as direct-DFT stages of
 * the generic passes, R multiply-adds per output for a factor R, so large prime
 * factors are slow); h[a] > 0 the mesh width; D > 0 the diffusion
 * coefficient (eq. (1.1)); bc is EIFE_BC_DIRICHLET (unknowns: the N[a] - 1
 * interior nodes of each axis, the sine basis of Section 4) or
 * EIFE_BC_PERIODIC (the variant at the end of Section 4: unknowns at the
 * N[a] nodes j h[a], j = 0 .. N[a] - 1, of each axis, circulant matrices
 * diagonalised by the real orthonormal Fourier basis; wave-local passes for
 * lines of 128, 256 and 512 points, generic passes otherwise; no split-BF16
 * transform, no batches, no EIFE_F_MMS_U2 / EIFE_F_EX51 /
 * EIFE_F_TRAVELING_WAVE); dtype is
 * EIFE_F32 or EIFE_F64, the precision of nodal arrays and transforms
 * (eigenvalue and phi factors are always formed in double).  The origin
 * defaults to 0, c2 to 1/2 and the load to EIFE_LOAD_LUMPED.  On success
 * *out receives the grid.  Errors: EIFE_EINVAL, EIFE_EUNSUPPORTED,
 * EIFE_ENOMEM, EIFE_EHIP. */
int eife_create_grid(int d, const int32_t* N, const double* h, double D, int bc, int dtype,
                     eife_grid* out);

/* Release the grid and its device memory.  Waits for no stream: the caller
 * must make sure no enqueued step on the grid is still running.  NULL is
 * accepted and ignored. */
int eife_destroy_grid(eife_grid g);

/* Fix the step tau > 0 and the number of exponential Runge-Kutta stages:
 * 1 = EIFE1 (eq. (2.13)), 2 = EIFE2 (eq. (2.14)) with node c2, 3 = the
 * three-stage scheme of eq. (2.2) with nodes (0, c2, c3) of eife_set_nodes3.
 * Builds the per-axis double tables of e^{-tau D lambda} and e^{-c2 tau D
 * lambda} (and, for 3 stages, of the c3-scaled and third-order terms).  The
 * first 3-stage call allocates one more state array of the grid's size
 * (kept until eife_destroy_grid).  Must precede eife_step; repeat after
 * eife_set_c2 / eife_set_nodes3 or to change tau.  Synchronous with respect
 * to the host (tables are uploaded before return).  Errors: EIFE_EINVAL,
 * EIFE_ENOMEM. */
int eife_set_phi(eife_grid g, double tau, int stages);

/* Nodes 0 < c2 < c3 <= 1 of the three-stage scheme (default 1/3, 2/3; the
 * EIFE2 node of eife_set_c2 is separate).  Its weights follow eq. (2.2): b_i
 * from the Lagrange polynomials of (0, c2, c3), a_3j from those of (0, c2)
 * (the reading that satisfies the consistency conditions, eq. (2.3)).  The
 * three-stage column passes are the generic kernels (no specialised or
 * split-BF16 variant: eife_step returns EIFE_EUNSUPPORTED with
 * EIFE_TX_GEMM_SPLITBF16); the scheme keeps a third array X = e^{c3 z} u^ +
 * tau a31 G_1 between its first and second stage.  If the grid is set to
 * 3 stages, eife_set_phi must be called again.  Errors: EIFE_EINVAL. */
int eife_set_nodes3(eife_grid g, double c2, double c3);

/* EIFE2 node c2 in (0, 1] (Section 2.2, default 1/2).  Invalidates the phi
 * tables: call eife_set_phi again before stepping. */
int eife_set_c2(eife_grid g, double c2);

/* Lower corner a[0..d-1] of the rectangle (default 0), for domains that do
 * not start at the origin (Example 5.1 of Section 5 takes x in (1/2, 5/2)).
 * Only the reaction kinds that depend on x use it: the manufactured problem
 * and Example 5.1, whose per-axis sin(pi x) factors at the interior nodes are
 * recomputed here.  Waits for all work on the device first.  Errors:
 * EIFE_EINVAL (null or non-finite origin), EIFE_EHIP. */
int eife_set_origin(eife_grid g, const double* a);

/* Load reading, EIFE_LOAD_LUMPED or EIFE_LOAD_NODAL. */
int eife_set_load(eife_grid g, int kind);

/* How the sine transforms are computed (Section 4 uses the FFT). */
enum eife_transform {
  EIFE_TX_FFT = 0,            /* default: FFT passes, the specialised kernels where N allows */
  EIFE_TX_FFT_GENERIC = 1,    /* FFT passes, always the generic mixed-radix kernels */
  EIFE_TX_GEMM_SPLITBF16 = 2  /* dense sine-matrix products on the matrix cores */
};

/* Select the transform implementation of later eife_step calls.
 * EIFE_TX_GEMM_SPLITBF16 applies the orthonormal sine matrix of Section 4
 * along each axis as a dense product on the matrix cores, with FP32 data and
 * matrix split into BF16 high and low parts (three products, FP32
 * accumulation; relative error of order 1e-5 per step instead of FP32
 * round-off).  It needs an FP32 grid with every N <= 1024, else
 * EIFE_EUNSUPPORTED; the library builds the matrices (2 * kp^2 BF16 values
 * per axis, kp = the next power of two >= max(64, N - 1)) on the first
 * selection.  Unknown kind: EIFE_EINVAL.  Batches ignore this setting. */
int eife_set_transform(eife_grid g, int kind);

/* Parameters c0, c1 of EIFE_F_CONST / EIFE_F_AFFINE_T / EIFE_F_FLORY_HUGGINS, c0 of
 * EIFE_F_TRAVELING_WAVE. */
int eife_set_forcing(eife_grid g, double c0, double c1);

/* Advance the nodal values u (device pointer, in place) by n_steps >= 0
 * uniform steps of the scheme fixed by eife_set_phi, from time t0: step n
 * evaluates f at t0 + n tau (and at t0 + (n + c2) tau for the second EIFE2
 * stage, eq. (2.10); at t0 + (n + c_i) tau for stage i of the three-stage
 * scheme).  u must hold the grid's element count in its dtype.  Enqueued on
 * `stream` (a hipStream_t, NULL = default stream); returns after
 * enqueueing.  Errors: EIFE_EINVAL (null u, negative n_steps, unknown f_kind,
 * EX51 with d != 2, EIFE_F_TRAVELING_WAVE without eps), EIFE_ESTATE (no
 * eife_set_phi since the last change of c2 or the nodes), EIFE_EUNSUPPORTED
 * (a Dirichlet-only f_kind on a periodic grid, the traveling wave with the
 * nodal load, three stages with the split-BF16 transform), EIFE_EHIP. */
int eife_step(eife_grid g, void* u, int64_t n_steps, int f_kind, double t0, void* stream);

/* eife_step out of place: the steps start from u_in and their result goes to
 * u_out (both device pointers holding the grid's element count; u_in is read
 * only by the first pass of the call, so the two may be the same or overlap,
 * and u_in is otherwise left as it was).  With n_steps = 0, u_in is copied to
 * u_out.  The recurrence and its results are those of eife_step, bit for bit.
 * Errors: those of eife_step, and EIFE_EINVAL for a null u_in or u_out. */
int eife_step_out(eife_grid g, const void* u_in, void* u_out, int64_t n_steps, int f_kind, double t0,
                  void* stream);

/* Variable step sizes (Section 2.2 lets the step vary): advance u (device,
 * in place) by n_steps steps of sizes taus[0 .. n_steps-1] (host array, each
 * > 0 and finite), t_{n+1} = t_n + tau_n from t_0 = t0 (a running sum in
 * double), every factor of eqs. (2.13)/(2.14) formed with tau_n.  Scheme
 * (stages, c2), load reading and transform as set on the grid; the step size
 * of eife_set_phi is neither used nor changed.  The factors of up to 512
 * steps (at most 16 MB) at a time are built on the host, staged in pinned
 * memory and copied on `stream` ahead of the steps that read them, in two
 * alternating buffers that the grid allocates on its first variable-step
 * call and keeps; the host waits only before it refills a buffer whose
 * previous copy has not completed (it returns after enqueueing the last
 * step).
 * All taus equal to the grid's tau give the same bits as eife_step.
 * Errors: as eife_step, plus EIFE_EINVAL for a null or non-positive taus
 * entry and EIFE_ENOMEM. */
int eife_step_variable(eife_grid g, void* u, const double* taus, int64_t n_steps, int f_kind, double t0,
                       void* stream);

/* Double-precision norms of the finite element function with nodal values
 * e = u - uref (uref may be NULL, then e = u), both device arrays in the
 * grid's layout and dtype:
 *   out[0] = sqrt(e^T M e)                  (L2 norm, M the Q1 mass matrix)
 *   out[1] = sqrt(e^T M e + e^T K_1 e)       (H1 norm, K_1 the stiffness for D = 1)
 *   out[2] = max_i |e_i|
 *   out[3] = (D/2) u^T K_1 u + prod(h) sum_i (u_i^2 - 1)^2 / 4   (Allen-Cahn energy of u)
 * Section 5 reports ||u(t_n) - u_h^n||_0 and ||.||_1; the energy is the
 * double-well analogue of the Flory-Huggins energy of Section 5.2.
 * Blocks the host until `stream` has produced the four values (host array
 * out[4]).  Returns EIFE_ENONFINITE (values still written) if any is not
 * finite. */
int eife_norms(eife_grid g, const void* u, const void* uref, double* out, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): eife_norms with its result left in
 * device memory and no allocation of any kind.  Enqueues the same reduction
 * on `stream` and writes out_dev[0..3] (a device array of 4 doubles owned by
 * the caller) with the values eife_norms returns; does not wait for the
 * device.  The block partial sums go to a fixed device array of the library
 * (8192 rows of 5 doubles = 320 KB per GPU, held until the process ends;
 * grids whose reduction would need more rows are rejected with EIFE_EINVAL,
 * none do today) which every call on that GPU shares: calls that overlap in
 * time on one GPU (other streams, other threads) race and must be ordered by
 * the caller.  The grid must live on the current device.  Non-finite values
 * are written as they are (no EIFE_ENONFINITE).
 * Errors: EIFE_EINVAL (null pointers, another current device), EIFE_EHIP. */
int eife_norms_noalloc(eife_grid g, const void* u, const void* uref, double* out_dev, void* stream);

/* Discrete energy of the nodal values u (device array in the grid's layout
 * and dtype) for the reaction f_kind, f = -F'(u):
 *   out[0] = (D/2) u^T K_1 u + prod(h) sum_i F(u_i)
 * with F(u) = (u^2 - 1)^2 / 4 for EIFE_F_ALLEN_CAHN and, for
 * EIFE_F_FLORY_HUGGINS (Example 5.3, Section 5.2),
 *   F(u) = (theta/2)((1 + u) ln(1 + u) + (1 - u) ln(1 - u)) - (theta_c/2) u^2
 * with theta = c0, theta_c = c1 of eife_set_forcing.  The gradient term uses
 * the Q1 stiffness matrix, the potential nodal quadrature.  Accumulated in
 * double; blocks the host until `stream` has produced it (host out[1]).
 * Errors: EIFE_EINVAL (null pointers, any other f_kind), EIFE_ENONFINITE
 * (value still written; e.g. some |u_i| >= 1 for Flory-Huggins). */
int eife_energy(eife_grid g, const void* u, int f_kind, double* out, void* stream);

/* Pass kinds of eife_step, for per-pass timing. */
enum eife_pass {
  EIFE_PASS_ROW_PHYS = 0,   /* inverse x-transform -> f -> forward x-transform */
  EIFE_PASS_ROW_FWD = 1,    /* prologue: forward x-transform of the caller's u */
  EIFE_PASS_ROW_INV = 2,    /* epilogue: inverse x-transform into the caller's u */
  EIFE_PASS_MID = 3,        /* y-transform of a 3D grid */
  EIFE_PASS_LAST_PLAIN = 4, /* prologue: transform along the last axis */
  EIFE_PASS_LAST_A = 5,     /* last-axis transform with the first EIFE2 stage (eq. (2.14)) */
  EIFE_PASS_LAST_B = 6,     /* last-axis transform with the EIFE2 update */
  EIFE_PASS_LAST_ETD1 = 7,  /* last-axis transform with the EIFE1 update (eq. (2.13)) */
  EIFE_PASS_COUNT = 8
};

/* Measurement aid: on != 0 makes later eife_step calls record a pair of HIP
 * events around every pass on the step's stream (accumulated per pass kind);
 * on == 0 stops recording.  Either call clears the accumulated totals. */
int eife_profile(eife_grid g, int on);

/* Wait for the recorded events and return, per pass kind, the summed GPU
 * time in milliseconds (ms[EIFE_PASS_COUNT]) and the number of launches
 * (launches[EIFE_PASS_COUNT]) since eife_profile.  Blocks the host. */
int eife_profile_read(eife_grid g, double* ms, int64_t* launches);

/* ------------------------------------------------------------------------
 * Batches: many independent 2D problems advanced together.  Instance i is a
 * grid of N[2i] x N[2i+1] intervals with mesh widths h[2i], h[2i+1] and
 * diffusion D[i] (same conventions as eife_create_grid with d = 2).  The
 * nodal arrays of all instances lie back to back, in instance order, in one
 * device buffer of the batch dtype; eife_batch_offsets gives where each
 * starts.  Instances with equal (N, h) form a size class: each pass of a
 * step is one launch per class covering all of its instances.
 * ---------------------------------------------------------------------- */
typedef struct eife_batch_s* eife_batch;

/* Create a batch of B >= 1 instances.  Errors as eife_create_grid. */
int eife_create_batch(int B, const int32_t* N, const double* h, const double* D, int dtype, eife_batch* out);

/* Release the batch (see eife_destroy_grid for the stream caveat). */
int eife_destroy_batch(eife_batch b);

/* Element offsets of the instances in the batched nodal array:
 * offsets[0..B], offsets[B] = total element count. */
int eife_batch_offsets(eife_batch b, int64_t* offsets);

/* eife_set_phi for every instance (same tau and stages for all). */
int eife_batch_set_phi(eife_batch b, double tau, int stages);

/* Advance every instance by n_steps steps (as eife_step, same f_kind and t0).
 * With a non-null stream the whole sequence of launches is captured once
 * into a HIP graph and replayed: a later call with the same u, n_steps,
 * f_kind and t0 replays the cached graph.  Asynchronous on `stream`. */
int eife_batch_step(eife_batch b, void* u, int64_t n_steps, int f_kind, double t0, void* stream);

/* Choose, per size class, the launch shapes of the passes by timing the
 * candidates on the device (eife_batch_set_phi must come first): for the
 * specialised line lengths two row tile widths and, for columns, two tile
 * widths with one tile per block plus (FP32) both widths in a persistent
 * stage pass that prefetches each next tile across instances; for the other
 * lengths the line pairs per block of both passes.  Every choice gives the
 * same results bit for bit.  Before tuning, FP32 classes of 512-interval
 * columns use the persistent stage pass, the others the widest tiles.  With a
 * non-null cache_path, choices recorded there for this device, dtype and
 * class are reused, and new ones are added to the file (JSON).  Blocks the
 * host.  The timing runs leave the batch's internal state undefined; the
 * next eife_batch_step starts from u as always. */
int eife_batch_autotune(eife_batch b, const char* cache_path, void* stream);

/* Launch shape chosen for size class k (order of first appearance):
 * out[0] = class N_x, out[1] = N_y, out[2] = instances, out[3] = row-pass
 * variant, out[4] = column-pass variant (specialised lengths: 0 / 1 tile
 * widths, 2 / 3 the persistent stage pass at those widths; other lengths:
 * line pairs per block).
 * Returns EIFE_EINVAL past the last class. */
int eife_batch_class_info(eife_batch b, int k, int32_t* out);

/* Number of unknown nodes of the grid (elements of a nodal array). */
int eife_grid_size(eife_grid g, int64_t* count);

/* Message describing the calling thread's most recent failed call. */
const char* eife_last_error(void);

/* ABI version of this library. */
int eife_version(void);

/* ------------------------------------------------------------------------
 * Learned corrector (an addition on top of the EIFE2 step of eq. (2.14); not
 * part of the paper).  One coarse step u_c = EIFE2(u_n, tau_c) is followed by
 * a convolutional network that predicts the residual towards several fine
 * steps from u_n: u_{n+1} = u_c + delta.  Per image, with the RMS coarse
 * change c = sqrt(mean((u_c - u_n)^2)) + 1e-30, the network reads the
 * channels (u_c, (u_c - u_n) / c) and delta = s_out * c * o.
 *
 * Network: six 3x3 convolutions over the interior nodes of a 2D grid (x
 * fastest), channels 2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after the
 * first five, zero padding (the homogeneous Dirichlet boundary).  Tap
 * t = 3 (dy + 1) + (dx + 1) reads the input at (y + dy, x + dx).  The four
 * 32 -> 32 layers and the output layer run on the matrix cores with BF16
 * weights and activations and FP32 accumulation; the first layer's FP32
 * inputs and weights enter the matrix cores split into BF16 high and low
 * parts (three products: about 2^-16 relative, below the BF16 rounding of
 * its stored output).
 *
 * Parameters: EIFE_CORR_PARAMS floats, in order W1 [9][2][32] (tap, input
 * channel (u_c, (u_c - u_n) / c), output), b1 [32]; four times W [9][32][32] (tap, output,
 * input), b [32]; W6 [9][32] (tap, input), b6 [1].
 *
 * Device arrays (un, uc, uf, delta, u) are FP32, [batch][ny][nx] contiguous;
 * the library keeps no pointer to them after a call.  Calls are asynchronous
 * on `stream` (NULL = default stream) unless they return host values.  A
 * corrector's calls share its workspaces: use one corrector from one host
 * thread and one stream at a time (work of two calls on different streams
 * would race on the activations and indicator buffers). */
#define EIFE_CORR_PARAMS 37889
typedef struct eife_corr_s* eife_corr;

/* Workspace for images of nx * ny nodes (ny <= 2048) and batches up to
 * max_batch (activations: 7 arrays of max_batch * nx * ny * 64 bytes).
 * Parameters start at zero.  Errors: EIFE_EINVAL, EIFE_ENOMEM, EIFE_EHIP. */
int eife_corr_create(int nx, int ny, int max_batch, eife_corr* out);
int eife_corr_destroy(eife_corr c);

/* Copy count = EIFE_CORR_PARAMS FP32 parameters from / to host memory.
 * Setting them resets the Adam moments and step count.  Blocks the host.
 * Errors: EIFE_EINVAL (count), EIFE_ENONFINITE (a parameter not finite). */
int eife_corr_set_params(eife_corr c, const float* host, int64_t count);
int eife_corr_get_params(eife_corr c, float* host, int64_t count);

/* Output scale s_out > 0 (default 1e-3). */
int eife_corr_set_scale(eife_corr c, double s_out);

/* delta = s_out * c * o(un, uc) for `batch` images (c per image, as above). */
int eife_corr_forward(eife_corr c, const float* un, const float* uc, float* delta, int batch, void* stream);

/* Inference path of eife_corr_forward, eife_corr_infer_step and eife_corr_run:
 * fused != 0 (the default) runs all six layers in one kernel over 16 x 32 node
 * tiles with the activations in on-chip memory; fused = 0 runs one kernel per
 * layer with the activations in device memory (the training path's forward).
 * Both give the same delta bit for bit.  Errors: EIFE_EINVAL (null corrector). */
int eife_corr_set_fused(eife_corr c, int fused);

/* Loss = mean over the batch's nodes of (o - (uf - uc) / (s_out c))^2 and its
 * gradient in the parameters, copied to grad_host (EIFE_CORR_PARAMS floats);
 * *loss (if loss is not NULL) receives the loss.  Blocks the host. */
int eife_corr_grad(eife_corr c, const float* un, const float* uc, const float* uf, int batch, float* grad_host,
                   double* loss, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr >= 0) on
 * the gradient of the loss above.  With loss != NULL, blocks the host and
 * stores the batch loss (before the update). */
int eife_corr_train_step(eife_corr c, const float* un, const float* uc, const float* uf, int batch, double lr,
                         double* loss, void* stream);

/* Fall back in eife_corr_infer_step whenever the RMS coarse change exceeds
 * max_change_rms > 0 (fast transients; default: no limit). */
int eife_corr_set_guard(eife_corr c, double max_change_rms);

/* One corrected step of the single image u (in place): u_c = one step of
 * `coarse` (f = Allen-Cahn, from t0), delta from the network, and u = u_c +
 * delta if r = ||delta||_2 / (||u_c - u_n||_2 + 1e-12) <= theta,
 * max|u| <= 1 + 1e-3 (the maximum bound principle) and the RMS coarse change
 * is within the guard (eife_corr_set_guard); otherwise u = fine_steps
 * steps of `fine` from the original u and *fell_back = 1.  out2 (if not
 * NULL) receives (r, max|u_c + delta|).  Both grids must be FP32 2D grids of
 * nx * ny nodes with eife_set_phi done (coarse: the coarse step; fine: the
 * fine step, fine_steps * fine tau = coarse tau).  Blocks the host once to
 * read the indicator.  Errors: EIFE_EINVAL, errors of eife_step. */
int eife_corr_infer_step(eife_corr c, eife_grid coarse, eife_grid fine, float* u, double t0, int64_t fine_steps,
                         double theta, int* fell_back, double* out2, void* stream);

/* n_steps corrected steps of u (eife_corr_infer_step at t0 + k tau_coarse,
 * k = 0 .. n_steps - 1) in one call; *fallbacks receives the number of steps
 * that fell back to the fine steps.  The result equals n_steps calls of
 * eife_corr_infer_step bit for bit.  Step k + 1 is enqueued before the host
 * reads step k's indicator (assuming acceptance) and enqueued again after a
 * fallback, so the device does not idle while the host decides; the host
 * still waits once per step.  The state moves between u and two buffers of
 * the corrector (no copy per step; one copy into u at the end when the last
 * state is elsewhere), so u holds intermediate states until the call's work
 * has run. */
int eife_corr_run(eife_corr c, eife_grid coarse, eife_grid fine, float* u, double t0, double tau_coarse,
                  int64_t n_steps, int64_t fine_steps, double theta, int64_t* fallbacks, void* stream);

/* Message of the calling thread's most recent failed eife_corr_* call. */
const char* eife_corr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EIFE_H */
