/*
 * lbm.h -- C ABI of the MI355X (gfx950) phase-field lattice Boltzmann library.
 *
 * The library advances the coupled D2Q9 lattice Boltzmann equations of
 * Zhang, Liang & Guo, "On the formulations of interfacial force in the
 * phase-field-based lattice Boltzmann method" (arXiv:2012.14729):
 *   flow populations f_i   (Sec. III, Eq. 29, equilibrium Eq. 31, forcing Eq. 35)
 *   order-parameter h_i    (Sec. III, Eq. 30, equilibrium Eq. 32, forcing Eq. 36)
 * with the chemical potential of Sec. II.A (Eq. 2), one of the eight
 * interfacial forces of Sec. II.B, the macroscopic moments of Eq. (37), the
 * isotropic difference stencils of Eqs. (41)-(42) and half-way bounce-back
 * walls (Sec. IV, Eqs. 43-44).  Lattice units: dx = dt = 1, cs^2 = 1/3.
 *
 * Conventions shared by every entry point
 *  - Return value: LBM_OK (0) on success, a negative lbm_status_code on
 *    failure; nothing throws across the ABI.  lbm_last_error() returns a
 *    thread-local message for the last failing call.
 *  - Device pointers ("d_" prefix) are HIP device addresses on the current
 *    device; host pointers ("h_" prefix or plain scalars) are ordinary memory.
 *  - Every call that takes a `stream` (a hipStream_t passed as void*, NULL
 *    for the null stream) is asynchronous on that stream unless it says it
 *    synchronises.  Arguments are validated on the host before any launch.
 *  - Fields are FP32, row-major [ny][nx] with x fastest and no padding
 *    (element (x, y) at offset y*nx + x).  Node (x, y) sits at lattice
 *    position (x, y); half-way walls lie at x = -1/2, nx - 1/2 (wall_x) or
 *    y = -1/2, ny - 1/2 (wall_y).
 *  - Ownership: the caller allocates and owns all device memory (workspace,
 *    inputs, outputs).  The library owns only the small host handles, which
 *    the matching *_destroy call frees.  No entry point allocates device
 *    memory except lbm_batch_create, which allocates nothing either: the
 *    caller passes the batch workspace.
 */
#ifndef PFLBM_LBM_H
#define PFLBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Interfacial force F_sf, in the paper's order (Sec. II.B). */
enum lbm_force_form {
  LBM_STF1 = 0, /* -div(kappa grad(phi) (x) grad(phi))                         Eq. (17) */
  LBM_STF2 = 1, /*  div(kappa (|grad phi|^2 I - grad(phi) (x) grad(phi)))      Eq. (18) */
  LBM_CPF1 = 2, /* -phi grad(mu_phi)                                           Eq. (20) */
  LBM_CPF2 = 3, /*  mu_phi grad(phi)                                           Eq. (20) */
  LBM_PF1 = 4,  /* -kappa grad(phi) lap(phi)                                   Eq. (20) */
  LBM_PF2 = 5,  /*  kappa phi grad(lap phi)                                    Eq. (20) */
  LBM_CSF1 = 6, /* -kappa |grad phi|^2 n div(n), n = grad phi/sqrt(|grad phi|^2+eps^2)  Eq. (24) */
  LBM_CSF2 = 7, /* -(sigma/2) grad(phi) div(n)                                 Eq. (25) */
  LBM_NUM_FORMS = 8
};

enum lbm_status_code {
  LBM_OK = 0,
  LBM_E_INVAL = -1,       /* bad argument; nothing was launched                        */
  LBM_E_HIP = -2,         /* a HIP runtime call failed; message in lbm_last_error()    */
  LBM_E_DIVERGED = -3,    /* a non-finite velocity or order parameter was produced    */
  LBM_E_UNSUPPORTED = -4  /* valid request the library does not implement             */
};

/* Problem statement in lattice units (Sec. II.A, Sec. III, Sec. IV).
 * Validation (LBM_E_INVAL): nx, ny >= 8; (nx rounded up to 64) * ny < 2^31
 * (a lattice needs about 168 B per node, so 288 GB of HBM hold about 1.7e9
 * nodes, 41000^2); wall_x, wall_y in {0, 1, 2}; at
 * most one walled axis may have moving walls, and free-slip walls do not
 * move; rho1, rho2 > 0; nu1, nu2 > 0 (so
 * tau_f = 1/2 + 3 nu > 1/2 everywhere); sigma >= 0; W > 0; M >= 0;
 * tau_h > 1/2; eps_n > 0; all finite except rho0, which may be NaN. */
typedef struct lbm_params {
  int32_t nx, ny;          /* nodes along x and y                                          */
  int32_t wall_x, wall_y;  /* 0: periodic axis; 1: half-way no-slip (bounce-back) walls;     */
                           /* 2: half-way free-slip walls (specular reflection, Sec. V.D's  */
                           /*    side walls): a plane of mirror symmetry; links into a      */
                           /*    corner bounce back                                          */
  double u_wall_lo;        /* tangential speed of the low wall of the walled axis (Eq. 43):  */
  double u_wall_hi;        /*   a y-wall moves along +x, an x-wall along +y                   */
  double rho1, rho2;       /* densities of fluid 1 (phi = +1) and fluid 2 (phi = -1) (Eq. 9) */
  double nu1, nu2;         /* kinematic viscosities; mu = rho nu is linear in phi (Eq. 10)   */
  double sigma, W;         /* surface tension, interface width: beta = 3 sigma/(4 W),        */
                           /*   kappa = 3 W sigma / 8 (Eq. 6)                                */
  double M, tau_h;         /* mobility and CH relaxation time: M = cs^2 eta (tau_h - 1/2)    */
  double gx, gy;           /* gravity; F_g = (rho - rho0) g (Eq. 8)                          */
  double rho0;             /* background density; NaN: mean of rho(phi0) over the domain    */
  double eps_n;            /* regulariser of the CSF interface normal (1e-6 is typical)      */
} lbm_params;

typedef struct lbm_sim lbm_sim;
typedef struct lbm_batch lbm_batch;

/* Bytes of device workspace one simulation needs (state of two population
 * sets, the order parameter in FP64, the (phi u) history and small scratch). */
int lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* Create a simulation on the caller's workspace (>= lbm_workspace_bytes,
 * 256-byte aligned) and initialise it from phi0 (and u0; d_ux0 and d_uy0 may
 * both be NULL for u0 = 0): P0 = 0, f = f^eq(P0, rho(phi0), u0),
 * h = h^eq(phi0, mu_phi(phi0), u0), (phi u)^(-1) = phi0 u0 (Eqs. 31-32).
 * If p->rho0 is NaN the call synchronises `stream` once to fix rho0.
 * The workspace must stay allocated until lbm_destroy.  The inputs may be
 * freed when the call returns (they are consumed on `stream`).
 * Tiles away from the domain edge use a faster addressing path with the
 * same arithmetic; the environment variable PFLBM_GENERAL_PATH, read here
 * and by lbm_batch_create, sends every tile through the general path (=1),
 * or turns off only the batched engine's wrapped path (=2) (diagnostics:
 * every path gives bitwise identical states).  The step
 * kernels work on 64x8-node tiles; PFLBM_TILE=1, 2 or 3 (read here) runs a
 * periodic lattice's step on 32x16, 32x8 or 64x4 tiles instead (diagnostics
 * and tuning: every shape gives bitwise identical states). */
int lbm_init(lbm_sim** sim, const lbm_params* p, void* d_ws, size_t ws_bytes,
             const float* d_phi0, const float* d_ux0, const float* d_uy0, void* stream);

/* Advance nsteps >= 0 time steps (Eqs. 29-30: collide with the given force
 * form, stream with bounce-back).  Asynchronous; no host synchronisation. */
int lbm_step(lbm_sim* sim, int32_t nsteps, int32_t force_form, void* stream);

/* Macroscopic fields of the current state (Eq. 37): phi = sum h_i, rho(phi)
 * (Eq. 9), u = [sum c_i f_i + (cs^2/2)(F_sf + F_g)] / (cs^2 rho) and
 * P_sf = sum f_i + (cs^2/2) u.grad(rho).  u depends on the force form, so it
 * is an argument.  Any output pointer may be NULL to skip that field.  Each
 * output holds nx*ny floats. */
int lbm_moments(lbm_sim* sim, int32_t force_form, float* d_phi, float* d_rho, float* d_ux, float* d_uy,
                float* d_p, void* stream);

/* Hydrodynamic pressure of the current state (Sec. II.B): p_h = P_sf - D,
 * where D holds the gradient terms the force form moves into its
 * generalised pressure P_sf (Eq. 21 for CPF-1/2 and PF-1/2, with
 * f0 = beta (1 - phi^2)^2; D = 0 for STF-2, CSF-1, CSF-2; D = -kappa |grad phi|^2
 * for STF-1, the value Eqs. 19 and 26 give).  Stencils as in the step
 * (Eqs. 41-42).  d_ph: caller-owned device buffer of nx*ny floats, row-major
 * [y][x]; must not be NULL.  Asynchronous on `stream`.  LBM_E_INVAL for a
 * NULL argument or a bad form. */
int lbm_hydro_pressure(lbm_sim* sim, int32_t force_form, float* d_ph, void* stream);

/* Host-side query: synchronises `stream`; *diverged = 1 if any step since
 * init produced a non-finite velocity or order parameter, else 0.  Returns
 * LBM_E_DIVERGED in that case (with *diverged = 1). */
int lbm_status(lbm_sim* sim, int32_t* diverged, void* stream);

/* Number of completed time steps since init (host counter). */
int lbm_get_step(const lbm_sim* sim, int64_t* step);

/* Checkpoint: the complete device state (populations, FP64 order
 * parameter, (phi u) history, divergence flag) copied to/from a caller-owned
 * device blob of lbm_state_bytes bytes; the blob's unused tail is written as
 * zeros, so equal states give equal blobs.  Restoring and stepping
 * reproduces an uninterrupted run bit for bit.  The host step counter
 * (lbm_get_step) is not part of the blob and restore leaves it unchanged. */
int lbm_state_bytes(const lbm_sim* sim, size_t* bytes);
int lbm_save(lbm_sim* sim, void* d_blob, void* stream);
int lbm_restore(lbm_sim* sim, const void* d_blob, void* stream);

/* One time step (as lbm_step, same force form rules) from the state held in
 * d_blob_in to d_blob_out, both in the lbm_save layout of this simulation;
 * the simulation's own state and step counter are not touched.  The blobs
 * must not overlap (LBM_E_INVAL).  d_blob_out's divergence flag is
 * d_blob_in's plus this step's; its padding (lanes past nx of each row's last
 * 64-node segment) is not written, so a zeroed output blob keeps equal
 * states in equal blobs.  Used to recompute the states of a checkpoint
 * segment without copies. */
int lbm_step_blobs(lbm_sim* sim, const void* d_blob_in, void* d_blob_out, int32_t force_form, void* stream);

/* Kernel timing with HIP events on the launch stream that take each timed
 * kernel's own start and stop times from its dispatch (hipExtLaunchKernel:
 * no packets between the kernels).  period: 0 = off; k >= 1 = time the two
 * launches of every k-th step counted from this call, the first step after
 * it included.  kernel: 0 = fused collide-stream kernel, 1 = order-parameter
 * kernel.  Not for steps captured into a HIP graph.  lbm_kernel_time
 * synchronises and returns the summed elapsed milliseconds and the number of
 * timed launches since the last reset; every call of lbm_set_timing drains
 * the pending events and resets the counters.  LBM_E_INVAL for period < 0. */
int lbm_set_timing(lbm_sim* sim, int32_t period);
int lbm_kernel_time(lbm_sim* sim, int32_t kernel, double* total_ms, int64_t* launches);

int lbm_destroy(lbm_sim* sim);

/* ------------------------------------------------------------------------
 * Batched: `count` independent simulations of uneven size and force form
 * advanced together by persistent kernels replayed from a captured HIP graph.
 * params[k] and forms[k] describe instance k (periodic axes only in this
 * version: wall_x = wall_y = 0, else LBM_E_UNSUPPORTED); d_phi0 is a host
 * array of `count` device pointers to each instance's nx*ny initial field.
 * ------------------------------------------------------------------------ */
int lbm_batch_workspace_bytes(const lbm_params* params, int32_t count, size_t* bytes);
/* Initialise every instance (as lbm_init, u0 = 0) and choose the launch
 * shape of the batched step by timing the candidates on this batch (one
 * fused kernel for every form or one per form; addressing paths: general
 * only, interior tiles on the interior path, or every tile on the wrapped
 * path (when every instance's state array fits in 4 GiB); persistent
 * workgroups per CU or one per tile), unless a choice for the same
 * instance sizes and forms is cached in this process or in the file named
 * by PFLBM_TUNE_CACHE; PFLBM_BATCH_TUNE=0 skips the timing and
 * PFLBM_BATCH_CFG=split,paths,blocks_per_cu forces a shape.  The
 * timing steps run before the states are (re)initialised, so the returned
 * batch starts from phi0 either way.  Synchronises `stream`. */
int lbm_batch_create(lbm_batch** batch, const lbm_params* params, const int32_t* forms, int32_t count,
                     void* d_ws, size_t ws_bytes, const float* const* d_phi0, void* stream);
/* The launch shape in use: split = 1 if the fused step runs one launch per
 * force form, fast = the addressing paths (0 general, 1 interior tiles on
 * the interior path and the others general, 2 every tile wrapped),
 * blocks_per_cu = persistent workgroups per CU (0: one per tile), and the
 * measured time per step in ms (0 when not timed).  Host-only. */
int lbm_batch_config(const lbm_batch* batch, int32_t* split, int32_t* fast, int32_t* blocks_per_cu,
                     double* ms_per_step);
/* Tile shape (tile_x x tile_y nodes) the batched step kernels use for
 * instance k: the tuner picks one shape for every instance, or per instance
 * 32x8 tiles where 64-wide ones would idle more lanes of the last tile
 * column (else 64x8), whichever steps faster; PFLBM_BATCH_SHAPE (read by
 * lbm_batch_create) forces one shape for every instance (0..3: 64x8,
 * 32x16, 32x8, 64x4) or the per-instance choice (4).
 * Host-only. */
int lbm_batch_tile_shape(const lbm_batch* batch, int32_t k, int32_t* tile_x, int32_t* tile_y);
/* Advance every instance by nsteps (asynchronous). */
int lbm_batch_step(lbm_batch* batch, int32_t nsteps, void* stream);
/* Moments of instance k, same definitions and layout as lbm_moments. */
int lbm_batch_moments(lbm_batch* batch, int32_t k, float* d_phi, float* d_rho, float* d_ux, float* d_uy,
                      float* d_p, void* stream);
/* Synchronises; h_flags[k] = 1 if instance k diverged, else 0. */
int lbm_batch_status(lbm_batch* batch, int32_t* h_flags, void* stream);
int lbm_batch_destroy(lbm_batch* batch);

/* ------------------------------------------------------------------------
 * Adjoint.  The adjoint state lambda of a step is dL/ds for the physical
 * pre-collision state s = (f_0..f_8, h_0..h_8, J_x, J_y) of every node: 20
 * FP64 planes of nx*ny values, row-major (x fastest), plane order f, h, J.
 * An lbm_adj is bound to one simulation and differentiates its current
 * state (or a saved one); it keeps accumulators of dL/dsigma and dL/dM.
 * The workspace (FP64 scratch of one adjoint step, the accumulators and the
 * buffers of lbm_adjoint_init) is caller-owned, 256-byte aligned,
 * lbm_adjoint_workspace_bytes long.
 * ------------------------------------------------------------------------ */
typedef struct lbm_adj lbm_adj;
int lbm_adjoint_workspace_bytes(const lbm_params* p, size_t* bytes);
/* Requires p->sigma > 0 (dL/dsigma is formed as dL/dF * F / sigma). Zeroes
 * the parameter-gradient accumulators (asynchronously on the null stream).
 * Free-slip walls (wall_x or wall_y = 2) return LBM_E_UNSUPPORTED. */
int lbm_adjoint_create(lbm_adj** adj, lbm_sim* sim, void* d_ws, size_t ws_bytes);
/* Zero the dL/dsigma, dL/dM accumulators. */
int lbm_adjoint_reset(lbm_adj* adj, void* stream);
/* lambda_T for L = 1/2 sum_x (phi_T - phi*)^2 at the simulation's current
 * state (reading A19): dL/dh_i = phi_T - phi*, dL/df = dL/dJ = 0.  d_target:
 * nx*ny FP32.  If h_loss is not NULL the call synchronises and stores L. */
int lbm_adjoint_seed_phi_misfit(lbm_adj* adj, const float* d_target, double* d_lambda, double* h_loss,
                                void* stream);
/* One step backwards: the simulation must hold the forward state s_t of the
 * step being differentiated (restore it first).  In: d_lambda_in =
 * lambda_{t+1}; out: d_lambda_out = lambda_t = (ds_{t+1}/ds_t)^T lambda_{t+1}
 * (Eqs. 6, 29-37, 41-43 transposed).  The two arrays must not overlap
 * (LBM_E_INVAL).  Adds this step's contributions to dL/dsigma and dL/dM. */
int lbm_adjoint_step(lbm_adj* adj, int32_t force_form, const double* d_lambda_in, double* d_lambda_out,
                     void* stream);
/* The same step linearised about the state held in d_blob (written by
 * lbm_save of this adjoint's simulation) instead of the simulation's current
 * state; the simulation is not touched. */
int lbm_adjoint_step_blob(lbm_adj* adj, const void* d_blob, int32_t force_form, const double* d_lambda_in,
                          double* d_lambda_out, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as lbm_adjoint_step_blob, with its per-step scratch (15 FP64 values
 * per node) in a 64 MiB array of the library's own, one per GPU, held until
 * the process ends, instead of the adjoint workspace.  Lattices of at most
 * 559240 nodes (nx*ny); larger ones return LBM_E_INVAL before any launch.
 * Allocates nothing.  Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (different streams or host threads) race
 * and give wrong results.  No state carries over between calls (every value
 * the step reads from the array it has written in the same call).  The
 * first call on a device looks the array's address up once. */
int lbm_adjoint_step_blob_noalloc(lbm_adj* adj, const void* d_blob, int32_t force_form, const double* d_lambda_in,
                                  double* d_lambda_out, void* stream);
/* Adjoint of lbm_init (reading A11): dL/dphi0 (nx*ny FP64) from lambda_0,
 * and the initial state's contributions to dL/dsigma and dL/dM (replacing
 * those of an earlier call).  phi0, u0 as given to lbm_init. */
int lbm_adjoint_init(lbm_adj* adj, const float* d_phi0, const float* d_ux0, const float* d_uy0,
                     const double* d_lambda0, double* d_dphi0, void* stream);
/* Synchronises; returns the accumulated dL/dsigma and dL/dM. */
int lbm_adjoint_param_grads(lbm_adj* adj, double* h_dsigma, double* h_dM, void* stream);
int lbm_adjoint_destroy(lbm_adj* adj);

const char* lbm_last_error(void);
const char* lbm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PFLBM_LBM_H */
