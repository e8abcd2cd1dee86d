/*
 * lbm.h -- C ABI of the MI355X (gfx950) free-energy lattice Boltzmann library.
 *
 * The library advances the liquid-gas free-energy lattice Boltzmann model of
 * Pooley & Furtado, "Eliminating spurious velocities in the free energy
 * lattice Boltzmann method", on periodic D2Q9 and D3Q19 lattices:
 *   - density and momentum moments                 Section "Model", Eq. (rho)
 *   - isotropic gradient / Laplacian stencils      Eqs. (xderiv), (laplace), (best),
 *                                                  3D: Eq. (laplacian3d)
 *   - van der Waals bulk pressure                  Eq. (p0)
 *   - tuned equilibrium (scheme LBM_SCHEME_EQ)     Eq. (equilibrium), Eq. (feq0),
 *                                                  2D weights: Section "Summary",
 *                                                  3D weights: Eq. (3dres)
 *   - momentum-conserving body force               Section "Using a forcing method"
 *     (scheme LBM_SCHEME_FORCE, 2-site halo)
 *   - BGK collision and streaming                  Eq. (latbolt)
 *   - the lambda (Galilean invariance) terms       Eq. (viscous), Appendix A
 * Units are lattice units: dx = dt = c = 1.
 *
 * Conventions shared by every entry point
 *   - Every pointer named dev_* is a device pointer on the current HIP device;
 *     host_* pointers are host memory.  The caller owns every buffer.  The
 *     library allocates no device memory: all device scratch lives in the
 *     caller's workspace (lbm_workspace_bytes / lbm_init).
 *   - Fields are FP64, SoA, x fastest: a scalar field is [nz][ny][nx]
 *     (nz = 1 for D2Q9), a vector field is [3][nz][ny][nx] (the z component
 *     of a D2Q9 vector field is written as zero), populations are
 *     [q][nz][ny][nx] in the paper's numbering of the velocities (D2Q9:
 *     e1,2 = (+-1,0), e3,4 = (0,+-1), e5,6 = (+-1,+-1), e7,8 = (-+1,+-1);
 *     D3Q19: faces e1..e6 then e7..e18 as printed in Section "Extension to
 *     3D").  Populations exchanged through the ABI are the paper's f_i(r,t),
 *     the values at site r after streaming.
 *   - All work is enqueued on the HIP stream given to lbm_init (NULL = the
 *     default stream).  Entry points that return host values synchronise
 *     that stream; the others only enqueue work.
 *   - Every function returns an int status: LBM_OK (0) or a negative
 *     LBM_E_* code; lbm_strerror() names it.  No C++ exception crosses the
 *     ABI.  A failed call leaves the context usable unless it returned
 *     LBM_E_DEVICE.
 *   - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19, LBM_D3Q15 = 15 /* binary stepper only */ };
enum { LBM_SCHEME_EQ = 0, LBM_SCHEME_FORCE = 1 };
/* FP64 populations, or FP32 deviations delta_i = f_i - s_i from a fixed
 * per-direction shift s_i (arithmetic in FP32, reductions in FP64). */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32_SHIFTED = 1 };
/* Shift of the FP32 storage: the rest equilibrium at rho_shift
 * (s_i = f_i^eq(rho_shift, u = 0)), or the normalised lattice weights times
 * rho_shift (2D 4/9, 1/9, 1/36; 3D 1/3, 1/18, 1/36). */
enum { LBM_SHIFT_REST_EQ = 0, LBM_SHIFT_WEIGHTS = 1 };
/* Arithmetic of the step kernels: the storage precision (FP64 storage ->
 * FP64, FP32 storage -> FP32), or FP64 arithmetic on FP32-stored deviations. */
enum { LBM_COMPUTE_NATIVE = 0, LBM_COMPUTE_F64 = 1 };

enum {
    LBM_OK = 0,
    LBM_E_INVAL = -1,     /* bad argument or unphysical parameter          */
    LBM_E_NOMEM = -2,     /* workspace smaller than lbm_workspace_bytes()  */
    LBM_E_DEVICE = -3,    /* a HIP call or kernel launch failed            */
    LBM_E_NONFINITE = -4, /* non-finite value or b*rho >= 1 in the state   */
    LBM_E_STATE = -5,     /* call not valid in the context's current state */
    LBM_E_LIMIT = -6      /* input beyond the fixed scratch of an allocation-free call */
};

typedef struct {
    double a, b, T;       /* van der Waals constants and temperature, Eq. (p0)  */
    double kappa;         /* square-gradient coefficient, Eq. (pt)              */
    double tau;           /* BGK relaxation time, Eq. (latbolt); > 1/2          */
    int lattice;          /* LBM_D2Q9 or LBM_D3Q19                              */
    int scheme;           /* LBM_SCHEME_EQ or LBM_SCHEME_FORCE                  */
    int storage;          /* LBM_STORE_F64 or LBM_STORE_F32_SHIFTED             */
    int nx, ny, nz;       /* lattice extent; nz = 1 for D2Q9                    */
    /* Stencil and weight overrides for parameter scans; NaN = the paper's
     * optimum.  B: gradient off-axis coefficient (Eq. (xderiv), 2A + 4B = 1
     * in 2D, 2A + 8B = 1 in 3D); D: Laplacian off-axis coefficient
     * (Eq. (laplace), C + 2D = 1 in 2D, C + 4D = 1 in 3D); F: force stencil
     * off-axis coefficient.  wp_diag, wt_diag, wxx_diag: the D2Q9
     * equilibrium weights w^p_5-8, w^t_5-8, w^xx_5-8 (the axis weights follow
     * from the constraints after Eq. (fi)); must be NaN for D3Q19. */
    double B, D, F;
    double wp_diag, wt_diag, wxx_diag;
    int galilean_lambda;  /* 1 = include the lambda terms (default), 0 = drop */
    int shift_mode;       /* LBM_SHIFT_REST_EQ or LBM_SHIFT_WEIGHTS            */
    double rho_shift;     /* FP32 shift density; NaN = mean of the initial rho */
    int tile;             /* launch shape id (lbm_tile_count); -1 = default     */
    int planes_per_block; /* planes marched by one workgroup; <= 0 = default    */
    int compute;          /* LBM_COMPUTE_NATIVE or LBM_COMPUTE_F64              */
} lbm_params;

/* Fill *p with the paper's drop-experiment defaults (a = 9/49, b = 2/21,
 * T = 0.56, kappa = 0.025, tau = 1, D2Q9, equilibrium scheme, FP64, 100x100,
 * every override NaN, lambda terms on, tile -1, native arithmetic). */
void lbm_params_default(lbm_params *p);

/* Bytes of device workspace lbm_init needs for these parameters (0 if the
 * parameters are invalid).  The workspace holds two population buffers, the
 * observation fields and the reduction partials. */
size_t lbm_workspace_bytes(const lbm_params *p);

/* Create a context and set the populations to the equilibrium of the
 * active scheme for density dev_rho0 [n] and velocity dev_u0 [3][n]
 * (dev_u0 may be NULL: fluid at rest).  The equilibrium includes the
 * gradient terms of Eq. (equilibrium) evaluated with the stencils.
 * dev_workspace must stay valid, and untouched by the caller, until
 * lbm_destroy.  stream is a hipStream_t (NULL = default stream).
 * Returns LBM_E_INVAL for bad parameters or an initial density that is
 * non-finite, <= 0 or >= 1/b somewhere; LBM_E_NOMEM if bytes is too small.
 * Synchronises the stream. */
int lbm_init(lbm_ctx **out, const lbm_params *p, void *dev_workspace, size_t bytes,
             void *stream, const double *dev_rho0, const double *dev_u0);

/* Advance the state by nsteps >= 0 time steps, Eq. (latbolt).  Only
 * enqueues work. */
int lbm_step(lbm_ctx *ctx, long long nsteps);

/* Density [n] and velocity [3][n] of the current state: u = j / rho for the
 * equilibrium scheme, v = u + g / (2 rho) for the forcing scheme (end of
 * Appendix A).  Either pointer may be NULL.  Only enqueues work. */
int lbm_moments(lbm_ctx *ctx, double *dev_rho, double *dev_vel);

/* Spurious velocity: the maximum velocity magnitude in the system (Section
 * "Numerical results"), |u| or |v| as in lbm_moments, reduced in FP64.
 * Returns LBM_E_NONFINITE if the state holds a non-finite value or
 * b*rho >= 1.  Synchronises. */
int lbm_max_spurious_u(lbm_ctx *ctx, double *host_out);

/* FP64 totals of the current state: mass sum_r rho and momentum
 * sum_r sum_i f_i e_i (host_mom[3]).  Synchronises. */
int lbm_invariants(lbm_ctx *ctx, double *host_mass, double *host_mom);

/* Advance nsteps >= 1 steps and report, for the last step t -> t+1, the
 * steady-state residual max_r |vel(r,t+1) - vel(r,t)| and max_r |vel(r,t+1)|
 * (FP64).  Either host pointer may be NULL.  Returns LBM_E_NONFINITE (after
 * advancing) if the new state is non-finite or has b*rho >= 1.
 * Synchronises. */
int lbm_step_observed(lbm_ctx *ctx, long long nsteps, double *host_residual,
                      double *host_max_vel);

/* Copy the state out as FP64 post-streaming populations f_i(r,t) [q][n]
 * (FP32 storage is decoded, shift added).  Only enqueues work. */
int lbm_get_state(lbm_ctx *ctx, double *dev_f);

/* Replace the state with FP64 post-streaming populations f_i(r,t) [q][n]
 * (rounded to FP32 deviations for FP32 storage).  Only enqueues work. */
int lbm_set_state(lbm_ctx *ctx, const double *dev_f);

/* Number of time steps taken since lbm_init (lbm_set_state keeps it). */
long long lbm_steps_done(const lbm_ctx *ctx);

/* The per-direction FP32 shift s_i actually in use (host_shift[q]); zeros
 * for FP64 storage. */
int lbm_shift(const lbm_ctx *ctx, double *host_shift);

/* Launch shapes: lbm_tile_count(lattice) shapes exist per lattice; shape k
 * covers tile_x x tile_y sites of a plane per workgroup (tile_y = 1 for
 * D2Q9, which marches along y; D3Q19 marches along z). */
int lbm_tile_count(int lattice);
int lbm_tile_shape(int lattice, int k, int *tile_x, int *tile_y);

/* Select the launch shape and planes per workgroup for later steps
 * (tile < 0 or planes <= 0 keep the current value).  Results do not depend
 * on the shape. */
int lbm_set_launch(lbm_ctx *ctx, int tile, int planes_per_block);
int lbm_get_launch(const lbm_ctx *ctx, int *tile, int *planes_per_block, int *workgroups);

/* Free the context (host memory only; the workspace stays the caller's). */
int lbm_destroy(lbm_ctx *ctx);

/* Coexisting gas and liquid densities of the van der Waals fluid of
 * Eq. (p0) at temperature T < T_c = 8a/(27b): equal pressure and equal
 * chemical potential mu = T ln(rho/(1-b rho)) + T/(1-b rho) - 2 a rho
 * (Maxwell construction).  Host computation.  LBM_E_INVAL if T >= T_c. */
int lbm_coexistence(double a, double b, double T, double *rho_gas, double *rho_liq);

/* ---- many independent problems in one launch per step -------------------
 *
 * A batch holds nprob independent periodic problems that share lattice,
 * scheme, storage and compute (each has its own extent, a, b, T, kappa,
 * tau, stencil overrides and shift).  Problem k's sites occupy
 * [lbm_batch_offset(k), lbm_batch_offset(k+1)) of concatenated FP64 fields:
 * a scalar field is [n_total], a vector field [3][n_total], each segment x
 * fastest as in the single-problem API.  Every step is one persistent
 * launch over a flat list of (problem, tile, plane chunk) work items; a
 * problem that has been retired (converged, diverging, non-finite, out of
 * steps) is skipped and keeps its state.  lbm_batch_run captures K steps
 * plus the convergence check in a hipGraph and replays it; it needs a
 * non-default stream (graph capture). */
typedef struct lbm_batch lbm_batch;

enum {
    LBM_BATCH_RUNNING = 0,
    LBM_BATCH_CONVERGED = 1,  /* residual <= tol                              */
    LBM_BATCH_MAXSTEPS = 2,   /* max_steps reached first                      */
    LBM_BATCH_DIVERGED = 3,   /* residual rose 10x above its minimum for `patience` checks */
    LBM_BATCH_NONFINITE = 4   /* non-finite state or b*rho >= 1              */
};

/* Workspace bytes for these problems (0 if any is invalid or they do not
 * share lattice, scheme, storage and compute). */
size_t lbm_batch_workspace_bytes(int nprob, const lbm_params *per_problem);

/* Create a batch and set every problem to the equilibrium of its initial
 * density dev_rho0 [n_total] and velocity dev_u0 [3][n_total] (may be NULL).
 * The launch shape comes from per_problem[0].tile / planes_per_block.
 * stream must be a non-default hipStream_t.  Synchronises. */
int lbm_batch_init(lbm_batch **out, int nprob, const lbm_params *per_problem,
                   void *dev_workspace, size_t bytes, void *stream,
                   const double *dev_rho0, const double *dev_u0);

/* Advance every active problem by nsteps (no checks).  Only enqueues.
 * A problem that lbm_batch_run retired is skipped and keeps its state; its
 * populations stay in the buffer the batch returns to after an even number
 * of steps, so while any problem is retired an odd nsteps is refused with
 * LBM_E_STATE (lbm_batch_reactivate lifts this). */
int lbm_batch_step(lbm_batch *bt, long long nsteps);

/* Run until no problem is active or max_steps more steps have been taken.
 * Every K = check_every (rounded up to even) steps each active problem's
 * residual max_r |vel(r,t+1) - vel(r,t)| (vel as in lbm_moments, FP64) is
 * measured; the problem is retired as LBM_BATCH_CONVERGED when it is <= tol,
 * LBM_BATCH_DIVERGED when, at `patience` consecutive checks after `grace`
 * steps, it exceeded 10 times the smallest residual seen after `grace`
 * (patience <= 0 disables this), LBM_BATCH_NONFINITE on a bad
 * state, LBM_BATCH_MAXSTEPS when its step count reaches max_steps.
 * Per-problem outputs (host, may be NULL): steps taken while active, last
 * residual, status.  Synchronises once per K steps (4 bytes read back).
 * While few problems remain active, work items march fewer planes (the
 * caller's launch is restored on return); results do not depend on it. */
int lbm_batch_run(lbm_batch *bt, double tol, int check_every, long long max_steps, int patience,
                  long long grace, long long *host_steps, double *host_residual, int *host_status);

/* Per-problem spurious velocity of the current state: host_out[k] = max |u|
 * (equilibrium scheme) or max |v| (forcing scheme, v = u + g / 2 rho) over
 * problem k's sites, the same quantity as lbm_max_spurious_u (section
 * "Numerical results": the maximum velocity magnitude in the system).
 * A problem with a non-finite velocity reports +inf, and the call then
 * returns LBM_E_NONFINITE (host_out is filled either way).  Synchronises. */
int lbm_batch_max_spurious_u(lbm_batch *bt, double *host_out);

/* Make every problem active again with a fresh status (step count,
 * residual history), keeping its populations, so that a later lbm_batch_run
 * continues all of them (e.g. to a tighter residual).  Synchronises. */
int lbm_batch_reactivate(lbm_batch *bt);

/* Density [n_total] and velocity [3][n_total] of every problem (retired ones
 * included).  Only enqueues. */
int lbm_batch_moments(lbm_batch *bt, double *dev_rho, double *dev_vel);

/* First site of problem k in the concatenated fields (k = nprob gives
 * n_total); -1 for a bad k. */
long long lbm_batch_offset(const lbm_batch *bt, int k);

/* Launch shape of the batched step (as lbm_set_launch) and the number of
 * work items it makes. */
int lbm_batch_set_launch(lbm_batch *bt, int tile, int planes_per_block);
int lbm_batch_get_launch(const lbm_batch *bt, int *tile, int *planes_per_block, int *items);

/* Free the batch (host memory and its graph; the workspace stays the
 * caller's). */
int lbm_batch_destroy(lbm_batch *bt);

/* ---- warm-start network kernels ------------------------------------------
 *
 * Building blocks of the small convolutional network that predicts a
 * near-steady (rho, u) field from the drop parameters, so a batch can start
 * close to its steady state.  3x3 convolutions wrap periodically in x and y
 * (like the lattice).  They run as implicit GEMMs on bf16 matrix cores with
 * FP32 accumulation: FP32 operands are rounded to bf16 (nearest even) as they
 * enter the MFMA.  Tensors are FP32, NHWC, 16-byte aligned, with padded
 * channel counts cin, cout in {16, 32}; nb * h * w must be a multiple of 16
 * and below 2^31.
 * Weights are [9][cout][cin] with tap 3 (dy + 1) + (dx + 1):
 *   out[p][co] = bias[co] + sum_{tap, ci} W[tap][co][ci] act(in[p + (dy, dx)][ci])
 * with act = max(., 0) when relu_in, else the identity.  Channels co >=
 * cout_real are written as zero.  All functions only enqueue on `stream`
 * except lbm_net_mse with a non-NULL host_loss, which synchronises. */
typedef struct {
    int nb, h, w;       /* images, rows, columns */
    int cin, cout;      /* padded channel counts */
    int cout_real;      /* channels actually produced */
} lbm_conv_shape;

int lbm_net_conv3x3_fwd(const lbm_conv_shape *s, const float *dev_in, int relu_in,
                        const float *dev_w, const float *dev_bias, float *dev_out, void *stream);

/* Gradient with respect to the convolution input:
 * din[q][ci] = sum_{tap, co} W[tap][co][ci] dout[q - (dy, dx)][co], multiplied
 * by (zin[q][ci] > 0) when dev_zin is not NULL (the previous layer's relu). */
int lbm_net_conv3x3_bwd_data(const lbm_conv_shape *s, const float *dev_dout, const float *dev_w,
                             const float *dev_zin, float *dev_din, void *stream);

/* Workspace bytes for lbm_net_conv3x3_bwd_weight (per-workgroup partials). */
size_t lbm_net_conv3x3_bwd_weight_workspace(const lbm_conv_shape *s);

/* Gradients with respect to the weights [9][cout][cin] and bias [cout]:
 * dW[tap][co][ci] = sum_p dout[p][co] act(in[p + (dy, dx)][ci]),
 * dbias[co] = sum_p dout[p][co]; partial sums are combined in a fixed order
 * (deterministic). */
int lbm_net_conv3x3_bwd_weight(const lbm_conv_shape *s, const float *dev_dout, const float *dev_in,
                               int relu_in, float *dev_dw, float *dev_dbias, void *dev_workspace,
                               size_t bytes, void *stream);

/* Allocation-free variant of lbm_net_conv3x3_bwd_weight, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving
 * loops, hosts that forbid hipMalloc): the same kernels, the same partial
 * sums and the same fixed summation order, so dW and dbias are bitwise those
 * of lbm_net_conv3x3_bwd_weight.  The per-workgroup partials live in a fixed
 * 16 MiB device array of the library (one per GPU, held until the process
 * ends) instead of a caller workspace; the call allocates nothing, host or
 * device.  Returns LBM_E_LIMIT, before any device work, when the partials
 * would exceed it: lbm_net_conv3x3_bwd_weight_workspace(s) > 16 MiB
 * (nb*h*w <= 463,872 pixels at cin = cout = 32).  The array is shared by
 * every call on a GPU and keeps the last call's contents (every call writes
 * all the partials it reads): calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  stream must
 * belong to the current device. */
int lbm_net_conv3x3_bwd_weight_noalloc(const lbm_conv_shape *s, const float *dev_dout,
                                       const float *dev_in, int relu_in, float *dev_dw,
                                       float *dev_dbias, void *stream);

/* Mean squared error over the first creal of c channels of npix pixels;
 * writes grad = 2 (pred - target) / (npix creal) (zero in padded channels)
 * and, if host_loss is not NULL, the loss.  dev_part holds >= 1024 doubles. */
int lbm_net_mse(long long npix, int c, int creal, const float *dev_pred, const float *dev_target,
                float *dev_grad, double *dev_part, double *host_loss, void *stream);

/* One Adam step (Kingma & Ba) on n parameters, step number t >= 1. */
int lbm_net_adam(int n, float *dev_param, const float *dev_grad, float *dev_m, float *dev_v,
                 double lr, double beta1, double beta2, double eps, long long t, void *stream);

/* ---- warm-start data preparation ----------------------------------------
 *
 * For nprob square side x side D2Q9 problems stored back to back (site
 * s = y side + x of problem k at k side^2 + s), each a drop centred on the
 * node (side/2, side/2).  Only enqueue on `stream`. */

/* Network input [nprob][side][side][16] FP32 (16-byte aligned): channels
 * 0..4 = dev_consts[k][0..4] (per-problem normalised constants: a, b, T,
 * kappa, R / side), channel 5 = (rho0 - rho_mean) / rho_scale, others 0. */
int lbm_warm_features(int nprob, int side, const double *dev_consts, const double *dev_rho0, double rho_mean,
                      double rho_scale, float *dev_x, void *stream);

/* Training target [ntot][16] FP32 (16-byte aligned) from a steady state:
 * channel 0 = (rho - rho0) / s_rho, channels 1, 2 = (u_x, u_y) / s_u with
 * dev_vel [3][ntot], others 0. */
int lbm_warm_targets(long long ntot, const double *dev_rho, const double *dev_rho0, const double *dev_vel,
                     double s_rho, double s_u, float *dev_y, void *stream);

/* Initial field from a network prediction pred [nprob][side][side][cpad]
 * (channel 0 = (rho - rho0) / s_rho, channels 1, 2 = u / s_u): decode; if
 * symmetrize, average over the eight symmetries of the square about the
 * centre (scalar rho(g p), vector M_g^T u(g p)); add the uniform density that
 * gives the cold start's mass; clamp rho to [rho_lo, rho_hi]; subtract the
 * mass-weighted mean velocity.  with_velocity = 0 starts from u = 0.  A
 * problem with a non-finite prediction gets rho0 and u = 0.  Outputs FP64:
 * dev_rho [nprob side^2], dev_u [3][nprob side^2] (z component 0). */
int lbm_warm_project(int nprob, int side, int cpad, const float *dev_pred, const double *dev_rho0, double s_rho,
                     double s_u, int with_velocity, int symmetrize, double rho_lo, double rho_hi, double *dev_rho,
                     double *dev_u, void *stream);

/* ---- binary fluid -------------------------------------------------------
 *
 * The Introduction states that the analysis carries over to other multiphase
 * systems such as binary fluids.  This stepper is that carry-over for the
 * symmetric binary fluid: a carrier density rho with ideal-gas pressure
 * rho/3 and an order parameter phi with bulk free energy
 * phi_a phi^2/2 + phi_b phi^4/4 plus kappa |grad phi|^2/2 (phi_a < 0 gives
 * two phases phi = +-sqrt(-phi_a/phi_b) with a tanh interface of width
 * sqrt(-2 kappa/phi_a)).  Two FP64 distributions advance together on a
 * D2Q9, D3Q19 or D3Q15 lattice, periodic or between two walls (wall):
 *   - f_i relaxes (time tau) to the tuned equilibrium of Eq. (equilibrium)/
 *     (feq0) with phi in the place of the differentiated density: bulk
 *     pressure rho/3 + phi_a phi^2/2 + 3 phi_b phi^4/4 on the w^p weights,
 *     -w^t_i kappa phi lap(phi) and the w^ab_i kappa d_a phi d_b phi terms,
 *     at the paper's optimum stencils and weights; no lambda term (it
 *     vanishes for c_s^2 = 1/3, Eq. (viscous));
 *   - g_i relaxes (time tau_phi) to the equilibrium with moments phi, phi u
 *     and gamma mu delta_ab + phi u_a u_b, chemical potential
 *     mu = phi_a phi + phi_b phi^3 - kappa lap(phi).
 * Gradients and Laplacians use Eqs. (xderiv), (laplace), (laplacian3d).
 * Fields and populations follow the conventions of the liquid-gas API
 * (SoA, x fastest, post-streaming populations f_i(r,t) and g_i(r,t) in the
 * paper's velocity numbering); the caller owns every buffer, and the
 * context allocates no device memory. */
typedef struct lbm_bin_ctx lbm_bin_ctx;

typedef struct {
    double phi_a, phi_b;  /* bulk free energy phi_a phi^2/2 + phi_b phi^4/4; phi_b >= 0 */
    double kappa;         /* square-gradient coefficient, >= 0                     */
    double gamma;         /* mobility coefficient of the mu term, >= 0             */
    double tau, tau_phi;  /* relaxation times of f and g, Eq. (latbolt); > 1/2     */
    /* LBM_D2Q9, LBM_D3Q19, or LBM_D3Q15 for the lattice comparison of
     * section "Extension to 3D" (which gives no D3Q15 tables): faces e1..e6,
     * then the eight corners in opposite pairs; weights with the moments of
     * Appendix A, w = faces 1/3, corners 1/24; w^p, w^t corner weights
     * wp_diag, wt_diag (faces 1/2 - 4 corner; default 1/24), w^xx corner
     * weight wxx_diag = c (faces along x 1/4 - 4c, others -1/4 - 4c;
     * default 0), w^xy = e_x e_y / 8; stencil corner coefficients B, D
     * (2A + 8B = 1, C + 4D = 1; defaults 1/24, 1/12).  Equilibrium scheme
     * only. */
    int lattice;
    int nx, ny, nz;       /* lattice extent; nz = 1 for D2Q9                       */
    /* 0: periodic.  1: walls at both ends of the marching axis (y for D2Q9,
     * z for D3Q19), halfway between planes (at -1/2 and n - 1/2): a
     * population streaming into a wall returns to its site reversed
     * (halfway bounce-back, no slip) and the stencils mirror phi about the
     * wall (zero normal derivative, a neutral wall).  The paper defines no
     * walls; the forcing section only notes they are harder with forcing.
     * In the forcing scheme the force stencil reaches one plane further:
     * beyond a wall it reads the gradient of the mirrored phi (its normal
     * component reversed). */
    int wall;
    /* LBM_SCHEME_EQ (the tuned equilibrium above) or LBM_SCHEME_FORCE: the
     * forcing scheme of section "Using a forcing method" carried over, i.e.
     * an f equilibrium without the w^ab terms and a body force
     * g = -div(kappa d phi d phi - delta kappa |d phi|^2 / 2) with the force
     * stencil (F_i as in the liquid-gas API), phi advected by and the
     * reported velocity equal to v = u + g / (2 rho); with walls or
     * periodic.  Not on LBM_D3Q15 (LBM_E_INVAL). */
    int scheme;
    /* Stencil and weight overrides as in lbm_params (NaN = the paper's
     * optimum): B, D the gradient and Laplacian off-axis coefficients;
     * wp_diag, wt_diag, wxx_diag the D2Q9 weights w^p_5-8, w^t_5-8,
     * w^xx_5-8 (NaN for D3Q19; the corner weights for D3Q15).  The
     * gamma mu term of g uses the same w^p. */
    double B, D;
    double wp_diag, wt_diag, wxx_diag;
    int tile;             /* launch shape id (lbm_bin_tile_count); -1 = default    */
    int planes_per_block; /* planes marched by one workgroup; <= 0 = default       */
} lbm_bin_params;

/* phi_a = -0.02, phi_b = 0.02, kappa = 0.04, gamma = 1, tau = tau_phi = 1,
 * D2Q9 100 x 100, periodic, equilibrium scheme, every override NaN, default
 * launch. */
void lbm_bin_params_default(lbm_bin_params *p);

/* Bytes of device workspace (four population buffers, observation fields,
 * reduction partials); 0 if the parameters are invalid. */
size_t lbm_bin_workspace_bytes(const lbm_bin_params *p);

/* Create a context with f = f^eq(rho0, rho0 u0, phi0) and g = g^eq(phi0,
 * u0), the stencils applied to dev_phi0 [n]; dev_rho0 [n] must be finite and
 * positive, dev_phi0 finite; dev_u0 [3][n] may be NULL (rest).
 * dev_workspace (256-byte aligned) must stay valid until lbm_bin_destroy.
 * LBM_E_INVAL for bad parameters or fields, LBM_E_NOMEM for a small
 * workspace.  Synchronises the stream. */
int lbm_bin_init(lbm_bin_ctx **out, const lbm_bin_params *p, void *dev_workspace, size_t bytes,
                 void *stream, const double *dev_rho0, const double *dev_phi0, const double *dev_u0);

/* Advance both distributions by nsteps >= 0 time steps (one fused launch
 * per step).  Only enqueues work. */
int lbm_bin_step(lbm_bin_ctx *ctx, long long nsteps);

/* rho [n], phi [n], the velocity [3][n] (u = j / rho; v = u + g / (2 rho)
 * for the forcing scheme) and mu [n] of the current state; any pointer may
 * be NULL.  Only enqueues work. */
int lbm_bin_moments(lbm_bin_ctx *ctx, double *dev_rho, double *dev_phi, double *dev_vel,
                    double *dev_mu);

/* Maximum velocity magnitude max_r |u| (the spurious velocity of a static
 * interface, Section "Numerical results"), FP64.  LBM_E_NONFINITE if the
 * state holds a non-finite value or rho <= 0.  Synchronises. */
int lbm_bin_max_spurious_u(lbm_bin_ctx *ctx, double *host_out);

/* FP64 totals of the post-streaming state: mass sum f, order parameter
 * sum g and momentum sum f e (host_mom[3]).  Synchronises. */
int lbm_bin_invariants(lbm_bin_ctx *ctx, double *host_mass, double *host_phi, double *host_mom);

/* Copy out / replace the state as post-streaming populations f_i(r,t),
 * g_i(r,t), FP64 [q][n] each.  Only enqueue work. */
int lbm_bin_get_state(lbm_bin_ctx *ctx, double *dev_f, double *dev_g);
int lbm_bin_set_state(lbm_bin_ctx *ctx, const double *dev_f, const double *dev_g);

/* Time steps taken since lbm_bin_init. */
long long lbm_bin_steps_done(const lbm_bin_ctx *ctx);

/* Launch shapes of the binary step (as lbm_tile_count / lbm_tile_shape /
 * lbm_set_launch / lbm_get_launch); results do not depend on the shape. */
int lbm_bin_tile_count(int lattice);
int lbm_bin_tile_shape(int lattice, int k, int *tile_x, int *tile_y);
int lbm_bin_set_launch(lbm_bin_ctx *ctx, int tile, int planes_per_block);
int lbm_bin_get_launch(const lbm_bin_ctx *ctx, int *tile, int *planes_per_block, int *workgroups);

/* Free the context (host memory only). */
int lbm_bin_destroy(lbm_bin_ctx *ctx);

/* ---- measurement --------------------------------------------------------
 *
 * Copy `bytes` (a multiple of 16, below 2^43; both pointers 16-byte aligned) from
 * dev_src to dev_dst with a streaming kernel (16-byte loads, non-temporal
 * 16-byte stores).  Not part of the method: it measures the HBM rate one
 * read plus one write of every byte can reach, the ceiling the step
 * kernels' algorithmic traffic is compared with.  Only enqueues work;
 * LBM_E_INVAL for a bad size or alignment. */
int lbm_stream_copy(const void *dev_src, void *dev_dst, size_t bytes, void *stream);

/* Human-readable name of a status code. */
const char *lbm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
