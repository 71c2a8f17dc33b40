/*
 * stp.h -- C ABI of the MI355X (gfx950) S-TPLS channel-flow time step.
 *
 * The library advances the incompressible Navier-Stokes equations for
 * pressure-driven flow in a channel (periodic in x and y, no-slip walls at
 * z = 0 and z = lz, constant mean pressure gradient dp/dx) with the method of
 * Fannon et al., arXiv 1511.07800:
 *   - MAC staggered finite volumes with centred differences (Sec. 3.1, 3.2);
 *   - optional Smagorinsky eddy viscosity with Van Driest wall damping
 *     (Sec. 2.2, definitions of nu_t, Delta and phi_w);
 *   - projection: predictor u* with third-order Adams-Bashforth for the
 *     convection and the "convective-like" viscous part and Crank-Nicolson
 *     for the "diffusive" viscous part, then the pressure Poisson equation
 *     and the correction u = u* - dt grad p (Sec. 3.1);
 *   - the Poisson equation solved by Scheduled Relaxation Jacobi: cycles of
 *     M Jacobi-SOR sweeps with scheduled weights omega_k, repeated until the
 *     residual test passes (Sec. 3.4, Jacobi-SOR equation).
 * Beside the paper's FP64 method the library offers a mixed mode (FP32
 * relaxation sweeps inside an FP64 defect correction).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: nx*ny*nz cells of size dx = lx/nx, dy = ly/ny, dz = lz/nz.  Fields
 * are flat arrays, x fastest: index(i,j,k) = i + nx*(j + ny*k).
 *   u  x-faces at (i dx, (j+1/2) dy, (k+1/2) dz), nx*ny*nz values
 *   v  y-faces at ((i+1/2) dx, j dy, (k+1/2) dz), nx*ny*nz values
 *   w  z-faces at ((i+1/2) dx, (j+1/2) dy, k dz), k = 0..nz: nx*ny*(nz+1)
 *      values; planes k = 0 and k = nz are the walls and are kept at 0
 *   p, nu_T and the Poisson right-hand side at cell centres, nx*ny*nz.
 * Units are physical: the caller gives nu and dp/dx, never a Reynolds number.
 *
 * Memory: the caller allocates ONE device workspace of stp_workspace_bytes()
 * bytes (any allocator; 256-byte alignment) and keeps it alive until
 * stp_destroy().  The library carves every field and work array out of it and
 * never allocates device memory itself; it allocates a small pinned host
 * buffer for scalar read-back.  Pointers returned by stp_fields() are borrowed
 * views into the workspace.
 *
 * Streams: all device work is enqueued on cfg->stream (a hipStream_t; NULL is
 * the null stream).  stp_step() and stp_poisson_solve() synchronise that
 * stream only at residual checks and to fill their statistics; fields are
 * valid in stream order.
 *
 * Errors: every call returns an stp_status; nothing throws, aborts or exits.
 * stp_last_error() gives a message for the last failure on a context.  A
 * device fault surfaces as STP_EDEVICE at the next synchronisation.
 *
 * Threads: a context may be used by one host thread at a time.  Contexts are
 * independent.
 */
#ifndef STP_H
#define STP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STP_ABI_VERSION 2

typedef struct stp_ctx stp_ctx; /* opaque */

typedef enum {
    STP_OK = 0,
    STP_EINVAL = -1,   /* bad argument or configuration */
    STP_ENOMEM = -2,   /* workspace too small or pinned host allocation failed */
    STP_EDEVICE = -3,  /* a HIP call failed (launch, copy or a device fault) */
    STP_ENOCONV = -4,  /* Poisson solve hit its cycle limit; p holds the last iterate */
    STP_ENAN = -5      /* non-finite residual */
} stp_status;

typedef enum {
    STP_FP64 = 0,  /* every sweep and reduction in FP64 (the paper's method) */
    STP_MIXED = 1  /* FP32 relaxation sweeps inside an FP64 defect correction; each FP32 pass
                      solves for a power-of-two multiple of the residual that lies in FP32's
                      normal range, so tiny and huge right-hand sides keep FP32 precision.
                      The Crank-Nicolson increment runs in FP32 (defect form), and with
                      stencils32 = 1 also the eddy viscosity and the explicit terms; the state
                      u, v, w, p, the Crank-Nicolson right-hand side, the residual and the
                      correction stay FP64 */
} stp_precision;

typedef enum {
    STP_WS_PREV = 0,    /* Poisson solve starts from p^n */
    STP_WS_ZERO = 1,    /* Poisson solve starts from 0 */
    STP_WS_LEARNED = 2  /* from the network's guess (stp_net_init first), or from p^n when that
                           has the smaller residual */
} stp_warm;

typedef enum {
    STP_U = 0, STP_V = 1, STP_W = 2, STP_P = 3, STP_NUT = 4, STP_RHS = 5
} stp_field;

typedef enum { STP_DTYPE_F64 = 0, STP_DTYPE_F32 = 1, STP_DTYPE_F32_RHS16 = 2 } stp_dtype;

typedef struct {
    int32_t nx, ny, nz;        /* cells; nx, ny >= 1, nz >= 2 */
    int32_t les;               /* 0: nu_T = nu (DNS); 1: Smagorinsky + Van Driest */
    double lx, ly, lz;         /* domain lengths (> 0) */
    double nu;                 /* molecular kinematic viscosity (> 0) */
    double dpdx;               /* G = dp/dx, constant; G < 0 drives flow in +x */
    double dt;                 /* time step (> 0) */
    double cs;                 /* Smagorinsky coefficient C_S (paper: 0.1) */
    double vd_a;               /* Van Driest constant A (paper: 25) */
    int32_t precision;         /* stp_precision */
    int32_t warm_start;        /* stp_warm */
    double poisson_rtol;       /* stop when ||b - L p||_2 <= rtol ||b||_2; 0: run exactly maxit cycles */
    int32_t poisson_maxit;     /* cycle limit (FP64 cycles, or defect-correction passes in mixed mode) */
    int32_t srj_m;             /* length of a caller-given cycle; 0 selects the built-in schedule */
    const double* srj_omega;   /* host array of srj_m weights in sweep order (copied at init) */
    double srj_reduction;      /* built-in schedule: bound on one cycle's error reduction (e.g. 1e-3) */
    int32_t mixed_inner;       /* mixed mode: FP32 cycles per defect-correction pass (>= 1) */
    int32_t srj_adaptive;      /* built-in schedule only: 0 repeats the srj_reduction cycle; 1 sizes each
                                  cycle from the reduction still needed (see stp_poisson_solve) */
    int32_t tblock;            /* sweeps fused per relaxation launch: 1..5 (FP64 sweeps fuse at most 4), or
                                  0: the library chooses, FP32 sweeps fusing 5 on grids with ny >= 66 (tiles
                                  of 16 wavefronts x 64 rows) and otherwise 4 when a four-sweep launch fits
                                  one round of resident workgroups, else 5; FP64 sweeps fuse 4.  Grids with
                                  nx < 64 or ny < 32 always run single sweeps.  Results are bitwise
                                  identical for every value. */
    double cn_tol;             /* Crank-Nicolson iteration error target relative to the start (e.g. 1e-13) */
    int32_t learned_correction; /* mixed mode with stp_net_init: after each defect-correction pass that has
                                   not converged, try p + s_r y(r, p) from the network (a coarse
                                   correction of the residual r) and keep it when its FP64 residual is
                                   smaller; the stop test is unchanged.  0: off.  Not used in FP64 mode. */
    int32_t extrap_order;      /* Poisson initial guess from the last solutions: 0 starts from p^n; 1 or 2
                                  from whichever has the least FP64 residual of p^n and its extrapolations
                                  in time of order 1 (2 p^n - p^{n-1}) and, for 2, order 2
                                  (3 (p^n - p^{n-1}) + p^{n-2}), as far as earlier solutions exist; the
                                  learned warm start then refines that guess.  Needs STP_WS_PREV or
                                  STP_WS_LEARNED.  The stop test is unchanged. */
    int32_t proj_depth;        /* Poisson initial guess by least squares over the last k = proj_depth
                                  solutions (0: off; 1..8): x = sum_i c_i p^{n-i}, i = 0..k-1, with the c_i
                                  minimising ||b - sum_i c_i b^{n-i}||_2 over the right-hand sides those
                                  solutions were solved for (L p^{n-i} = b^{n-i} to the solve tolerance).
                                  x is kept when its FP64 residual is below that of the other candidates
                                  (p^n, the extrapolations); the learned warm start then refines the guess.
                                  Only converged solves enter the history (a failed solve empties it).
                                  Adds 2 proj_depth arrays of nx*ny*nz doubles to the workspace.  Needs
                                  STP_WS_PREV or STP_WS_LEARNED.  The stop test is unchanged. */
    int32_t mixed_rhs16;       /* STP_MIXED only: 1 stores each FP32 pass's right-hand side (the FP64
                                  residual) as FP16 after scaling it to about unit rms by a power of
                                  two (the correction is scaled back exactly), so the sweeps read 2
                                  instead of 4 bytes of it per cell; the sweeps still compute in FP32
                                  and the FP64 residual test is unchanged, but one pass then reduces
                                  the residual by at most about 1e-3 (FP16 rounds each element to
                                  within 4.9e-4), so the per-pass floor becomes max(srj_reduction,
                                  1e-3).  Adds nx*ny*nz halves to the workspace.  0: FP32. */
    int32_t stencils32;        /* STP_MIXED only: 1 runs the eddy viscosity and the explicit momentum terms
                                  in FP32 on FP32 copies of the state made each step (u as its departure
                                  from its FP64 x-y plane means, so the copy rounds the departure only),
                                  with nu_T and the Adams-Bashforth history stored in FP32, and forms the
                                  Crank-Nicolson right-hand side as the FP64 state plus the FP32
                                  increment.  The FP32 rounding of those terms enters each step's
                                  Poisson right-hand side as noise the least-squares and learned guesses
                                  cannot predict, which bounds their residual from below (about 3e-6 of
                                  ||b|| on the 512x256x192 LES against 4e-7 with FP64 stencils) and costs
                                  more sweeps than the stencils save there.  0: FP64 stencils. */
    void* stream;              /* hipStream_t for all work */
} stp_config;

typedef struct {
    int32_t cycles;    /* SRJ cycles run (FP64 cycles, or FP32 inner cycles in mixed mode) */
    int32_t outer;     /* residual checks after the first (defect-correction passes in mixed mode) */
    int32_t sweeps;    /* relaxation sweeps run */
    int32_t status;    /* stp_status of the solve */
    double relres0;    /* ||b - L p0||_2 / ||b||_2 before the solve */
    double relres;     /* after the solve */
    double bnorm;      /* ||b||_2 */
    int32_t launches;  /* relaxation kernel launches (each runs tblock sweeps or fewer) */
    int32_t corrections; /* learned coarse corrections kept (learned_correction) */
    double ms_relax;   /* device time of the back-to-back sweep sequences (events around each), ms */
} stp_solve_stats;

typedef struct {
    stp_solve_stats poisson;
    int32_t step;      /* steps completed by this context */
    int32_t cn_sweeps; /* Crank-Nicolson iterations per component */
    double max_div;    /* max |div u^{n+1}| over all cells */
    double u_bulk;     /* mean of u over all x-faces */
    double u_max;      /* max |u| */
    double cfl;        /* max(|u| dt/dx, |v| dt/dy, |w| dt/dz) */
    double u_centre;   /* mean u on the channel centreline z = lz/2 */
    double nut_max;    /* max nu_T */
    double ms_total;   /* wall time of the step (stream-ordered events), ms */
    double ms_poisson; /* of which the Poisson solve, ms */
    double relres_prev;    /* learned warm start or extrapolation: relative residual of p^n ... */
    double relres_learned; /* ... of the network's guess (0 when not used) */
    int32_t learned_used;  /* 1 if the solve started from the network's guess */
    int32_t extrap_used;   /* extrapolation order of the guess kept (0: p^n) */
    double ms_net;         /* network inference time, ms */
    double relres_extrap;  /* ... and of the extrapolated guess kept (0 when extrap_order = 0) */
    double relres_proj;    /* ... and of the least-squares guess (0 when not formed) */
    int32_t proj_used;     /* 1 if the solve started from the least-squares guess (or its refinement) */
    int32_t proj_rank;     /* history columns the least-squares guess used (0 when not formed) */
    /* Device time of the step's phases in the order of Sec. 3.1 (stream-ordered events; with
       ms_poisson they add up to ms_total), ms.  The same phases are roctx ranges named
       "stp_step: <phase>" for rocprofv3 --marker-trace; with STP_TRACE_SYNC=1 in the
       environment at stp_init each range also waits for its phase's device work. */
    double ms_nut;         /* eddy viscosity (and the mixed mode's FP32 copies of the state) */
    double ms_momentum;    /* explicit terms, Crank-Nicolson right-hand sides and iterations */
    double ms_divergence;  /* b = div u* / dt and its mean removal */
    double ms_guess;       /* Poisson guess: extrapolation, least squares, network (ms_net) */
    double ms_projection;  /* history update, u = u* - dt grad p, diagnostics */
} stp_step_stats;

/* Bytes of device workspace the configuration needs (0 if cfg is invalid). */
size_t stp_workspace_bytes(const stp_config* cfg);

/* Validate cfg, carve the workspace, build the SRJ schedule and zero every
 * field (state at rest, p = 0, empty Adams-Bashforth history, step 0).
 * STP_EINVAL on a bad configuration, STP_ENOMEM if bytes is too small.
 * On success *out owns a context to release with stp_destroy(). */
stp_status stp_init(const stp_config* cfg, void* dev_workspace, size_t bytes, stp_ctx** out);

/* Advance nsteps time steps (Sec. 3.1): eddy viscosity (if les), explicit
 * terms, Crank-Nicolson predictor, b = div(u*)/dt minus its mean, SRJ solve
 * for p from the warm start, p minus its mean, correction, diagnostics.
 * Stops at the first step whose solve fails and returns its status
 * (STP_ENOCONV leaves the step completed with the last iterate).
 * last (nullable) receives the statistics of the last step taken. */
stp_status stp_step(stp_ctx* ctx, int32_t nsteps, stp_step_stats* last);

/* Solve L_p p = b (Sec. 3.1 Poisson equation, zero normal gradient at the
 * walls, periodic in x and y) with the context's schedule and precision.
 * With srj_adaptive = 1 each cycle is a Chebyshev/Leja cycle whose degree M
 * (rounded up to a multiple of 16) meets the bound 1/T_M <= rho on the residual
 * reduction, rho = max(rtol ||b|| / ||r||, floor), floor = 1e-10 in FP64 and
 * srj_reduction for the FP32 passes of the mixed mode; a cycle of degree M
 * multiplies every residual mode by at most 1/T_M, so one cycle usually meets
 * the test.
 * b_dev: device FP64 array of nx*ny*nz values, mean-free (borrowed, read).
 * p_dev: device FP64 array, initial guess in, solution out (mean removed).
 * rtol, maxit as in stp_config.  stats nullable.  Returns STP_OK,
 * STP_ENOCONV, STP_ENAN or an error. */
stp_status stp_poisson_solve(stp_ctx* ctx, const void* b_dev, void* p_dev, double rtol, int32_t maxit,
                             stp_solve_stats* stats);

/* Apply an explicit list of Jacobi-SOR sweeps (Sec. 3.4):
 * p <- p + (omega_s / D)(L_p p - b) for s = 0..nsweeps-1, with
 * D = 2/dx^2 + 2/dy^2 + 2/dz^2.  dtype selects FP64 or FP32 arrays for
 * b_dev and p_dev (nx*ny*nz values each, borrowed), or STP_DTYPE_F32_RHS16:
 * FP32 p with an FP16 b (widened exactly to FP32 on load).  omega is a host array.
 * Uses the context's fused-sweep setting.  Enqueues only; no sync. */
stp_status stp_relax(stp_ctx* ctx, int32_t dtype, const void* b_dev, void* p_dev, const double* omega,
                     int32_t nsweeps);

/* ||b - L_p p||_2 in FP64 for FP64 device arrays (synchronises). */
stp_status stp_residual_norm(stp_ctx* ctx, const void* b_dev, const void* p_dev, double* norm);

/* Allocation-free variant of stp_residual_norm, for callers that cannot
 * allocate device or pinned memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It needs no context (the
 * grid comes as arguments: nx, ny, nz cells, domain lx, ly, lz, with the
 * limits of stp_config), computes the same FP64 residual norm with the same
 * kernels, and writes it to the device double *norm_dev, enqueued on stream
 * (a hipStream_t; NULL is the null stream) without synchronising or reading
 * anything back.  b_dev and p_dev are FP64 device arrays of nx*ny*nz values
 * (borrowed, read).  The reduction partials live in a static scratch array
 * of the library (512 KiB per GPU, held until the process ends); it allocates
 * nothing and every partial is written before it is read.  Calls on one GPU
 * share that scratch: calls that may overlap on the same GPU (different
 * streams, or host threads) race, and the caller must order them.
 * Returns STP_EINVAL for a null pointer, an invalid grid or one that needs
 * more partials than the scratch holds (an x-y plane of more than 65536
 * column tiles of 64 x 4 cells), STP_EDEVICE if the scratch address cannot be
 * found or a launch fails; stp_last_error(NULL) then gives the reason. */
stp_status stp_residual_norm_noalloc(int32_t nx, int32_t ny, int32_t nz, double lx, double ly, double lz,
                                     const void* b_dev, const void* p_dev, void* norm_dev, void* stream);

/* The least-squares guess of proj_depth on caller-given histories (not in the
 * paper; the paper starts each solve from the previous pressure, Sec. 3.4):
 * out = sum_i c_i x_i with c minimising ||b - sum_i c_i y_i||_2, for k (1..8)
 * earlier solutions x[i] and the right-hand sides y[i] they solve (newest
 * first; the order only decides which of two dependent columns is dropped).
 * x_dev and y_dev are host arrays of k device pointers; every array holds
 * nx*ny*nz doubles and is borrowed.  Columns whose part orthogonal to the
 * newer ones is below 1e-5 of their norm are left out; *rank receives the
 * number used (0: out is not written).  STP_EINVAL for k outside 1..8 or a
 * null pointer.  Synchronises. */
stp_status stp_lsq_guess(stp_ctx* ctx, int32_t k, const void* const* x_dev, const void* const* y_dev,
                         const void* b_dev, void* out_dev, int32_t* rank);

/* Borrowed view of a field on the staggered (MAC) grid of Sec. 3.1: device
 * pointer, shape {nz or nz+1, ny, nx} (slowest first), strides in elements
 * in the same order ({nx ny, nx, 1}), dtype, and offset = the position (z, y,
 * x) of element [0][0][0] in the box [0, lz] x [0, ly] x [0, lx]; element
 * [k][j][i] lies at offset + (k dz, j dy, i dx):
 *   STP_U (x-faces)  (dz/2, dy/2, 0)
 *   STP_V (y-faces)  (dz/2, 0, dx/2)
 *   STP_W (z-faces)  (0, dy/2, dx/2), nz+1 planes, planes 0 and nz on the walls
 *   STP_P, STP_NUT, STP_RHS (cell centres)  (dz/2, dy/2, dx/2).
 * strides and offset may be NULL.  Every field is FP64, except STP_NUT with
 * stencils32, which computes and keeps nu_T in FP32 (STP_DTYPE_F32). */
stp_status stp_fields(stp_ctx* ctx, int32_t field, void** dev_ptr, int64_t shape[3], int64_t strides[3],
                      int32_t* dtype, double offset[3]);

/* Plane averages of the current state at every height, the x-y means from
 * which the paper's space-time averages, bulk velocity, centreline velocity
 * and skin friction are formed (Sec. 6).  out: host array of 8 (nz + 1)
 * doubles, out[q (nz + 1) + k]:
 *   q = 0 <u>, 1 <v>, 2 <u^2>, 3 <v^2>, 4 <nu_T> on the cell planes
 *       z = (k + 1/2) dz, k < nz (out[q (nz + 1) + nz] = 0);
 *   q = 5 <w>, 6 <w^2> on the face planes z = k dz, k = 0..nz;
 *   q = 7 <u w> on the x-z edges (i dx, k dz), k = 0..nz, with u averaged
 *       over the planes k - 1 and k (odd ghosts beyond the walls) and w over
 *       the columns i - 1 and i.
 * nu_T is the eddy viscosity of the last step (computed from its starting
 * velocity).  FP64, fixed summation order; synchronises the stream. */
stp_status stp_plane_stats(stp_ctx* ctx, double* out);

/* The relaxation cycle in use: writes min(cap, M) weights, *m = M. */
stp_status stp_schedule(const stp_ctx* ctx, double* omega, int32_t cap, int32_t* m);

/* ---- checkpoint and restart ----------------------------------------------------
 * Not in the paper (it writes periodic dumps and describes no restart).  Apart
 * from the caller-owned workspace, which holds every field and history array,
 * a context's state is the number of steps taken (it also selects the
 * Adams-Bashforth start-up and history slots, and the slots of the
 * least-squares history) and the numbers of earlier solutions held for the
 * extrapolated and the least-squares warm starts.  A checkpoint is a copy of
 * the workspace plus stp_get_state(); copying both into a context made with
 * the same configuration and calling stp_set_state() continues the run
 * bitwise.  The network's workspace (weights) is not part of it. */
typedef struct {
    int32_t step;   /* steps completed */
    int32_t nhist;  /* earlier solutions held for extrap_order (0..extrap_order) */
    int32_t nproj;  /* earlier solutions and right-hand sides held for proj_depth (0..proj_depth) */
} stp_state;

stp_status stp_get_state(const stp_ctx* ctx, stp_state* out);
/* STP_EINVAL if step < 0, nhist lies outside 0..extrap_order or nproj outside
 * 0..proj_depth. */
stp_status stp_set_state(stp_ctx* ctx, const stp_state* in);

/* ---- learned warm start ------------------------------------------------------
 * Not part of the paper: a 3-level 3-D convolutional network (16/32/64
 * channels, 3x3x3 kernels, ReLU, 2x average pooling, nearest upsampling with
 * skip concatenation; periodic in x and y, zero padding beyond the walls)
 * predicts the pressure increment of a step from (b, p^n).  BF16 weights and
 * activations, FP32 accumulation on the matrix cores.  The exact increment is
 * L^-1 r with r = b - L p^n, so the inputs are the residual (computed in
 * FP64) and p^n, each scaled by its own rms: x = (r/(D s_r), (p^n - mean)/s_p),
 * s_r = rms(r/D), s_p = rms(p^n - mean p^n) (1 where zero); the guess is
 * p^n + s_r y.  The relaxation always runs to the same residual,
 * so the network only changes the starting point.  Requires nx, ny, nz
 * divisible by 4.  Parameters: one FP32 vector, per layer W[27][cout][cin]
 * (tap = 9(dz+1) + 3(dy+1) + (dx+1)) then bias[cout], channel counts padded
 * to multiples of 16 with zero weights (layout from stp_net_layout). */

/* Bytes of device workspace the network needs for this context's grid
 * (training adds the backward buffers); 0 if the grid is not supported. */
size_t stp_net_workspace_bytes(const stp_ctx* ctx, int32_t training);

/* Carve the network out of a caller-owned device workspace (kept alive until
 * stp_destroy), initialise the weights from seed (He-uniform), zero the
 * biases.  training = 0 allows prediction only. */
stp_status stp_net_init(stp_ctx* ctx, void* dev_workspace, size_t bytes, int32_t training, uint64_t seed);

/* Borrowed device pointers to the FP32 parameter vector and its gradient
 * (gradient NULL without training) and their length. */
stp_status stp_net_params(stp_ctx* ctx, float** params, float** grads, int64_t* count);

/* Layer l (0..5): out = {weight offset, bias offset, cin, cout, logical cin, logical cout}. */
stp_status stp_net_layout(const stp_ctx* ctx, int32_t layer, int64_t out[6]);

/* After the caller wrote the parameter vector: refresh the BF16 copies and
 * restart Adam. */
stp_status stp_net_sync(stp_ctx* ctx);

/* p_guess = p_prev + s y(b, p_prev); FP64 device arrays of nx*ny*nz (borrowed). */
stp_status stp_net_predict(stp_ctx* ctx, const void* b_dev, const void* p_prev_dev, void* p_guess_dev);

/* One training step on a (b, p_prev, p_next) triple from the solver: forward,
 * loss = mean((y - (p_next - p_prev)/s_r)^2), backward into the gradient
 * vector, then Adam (beta 0.9, 0.999, eps 1e-8) with learning rate lr when
 * lr > 0 (lr = 0 leaves the weights and only computes gradients).  *loss
 * (nullable) receives the loss; synchronises when loss is not NULL. */
stp_status stp_net_train_step(stp_ctx* ctx, const void* b_dev, const void* p_prev_dev, const void* p_next_dev,
                              float lr, double* loss);

/* Release the context (not the caller's workspace). NULL is accepted. */
stp_status stp_destroy(stp_ctx* ctx);

/* Message for the last failure on ctx ("" if none); valid until the next call.
 * With ctx = NULL: the message of the last failed stp_residual_norm_noalloc
 * call on this thread, or "null context". */
const char* stp_last_error(const stp_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* STP_H */
