/*
 * cfdhip -- FP64 structured multi-block Euler hot path for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libcfdhip.so.  Every entry point takes plain pointers and sizes.
 * Pointers named dev_* are device memory on the GPU that was current when the
 * context was created; pointers named *_host are host memory.  The caller
 * owns every buffer it passes; the library never keeps a caller pointer
 * beyond the call except the bound workspace (cfd_bind_workspace).
 *
 * Method (arXiv 2012.02925, "An Improved Framework of GPU Computing for CFD
 * Applications on Structured Grids using OpenACC"):
 *   - finite-volume form of the Euler equations (Sec. 2, eq. (1)-(2));
 *   - MUSCL reconstruction of primitive variables with a limiter
 *     (Sec. 7.2, V4, eq. (flux)), Roe flux-difference splitting in each index
 *     direction (Sec. 2), flux divergence on curvilinear metrics;
 *   - wall-face flux override (Sec. 7.2, V7);
 *   - ghost cells for physical and connected boundaries, connected ghosts
 *     exchanged by device pack/unpack at every Runge-Kutta stage
 *     (Sec. 2, Sec. 4, Sec. 7.2 V1/V5);
 *   - explicit M-stage Runge-Kutta time marching (Sec. 2), global CFL step.
 *
 * Layouts used at this boundary
 *   State / residual ("packed"): FP64 structure of arrays,
 *     [var][cell], var = 0..dim+1, cells of all blocks concatenated in block
 *     order, each block in k-j-i order (i fastest), interior cells only.
 *     Conservative variables (rho, rho u, rho v[, rho w], rho E) unless an
 *     entry point says primitive (rho, u, v[, w], p).
 *   Nodes of a block: [coord][k][j][i] with (ni+1)(nj+1)(nk+1) points per
 *     coordinate (nk+1 -> 1 in 2D), i fastest; concatenated over blocks in
 *     the node-sized entry points.
 *   Faces: 0..5 = imin, imax, jmin, jmax, kmin, kmax.  A face range lo/hi is a
 *     half-open cell-index range along the face's tangential axes in
 *     increasing axis order (i before j before k); in 2D only [0] is used.
 *
 * Calls are asynchronous on the stream given to cfd_create unless stated.
 * Errors: every call returns a cfd_status; cfd_last_error() gives detail.
 * Calls in the wrong order return CFD_ERR_STATE.  One context must not be
 * used from two threads at once.
 */
#ifndef CFDHIP_H
#define CFDHIP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cfd_ctx cfd_ctx;

typedef enum {
  CFD_OK = 0,
  CFD_ERR_ARG = -1,         /* bad argument (null pointer, size, enum) */
  CFD_ERR_STATE = -2,       /* call out of order (e.g. before finalize/bind) */
  CFD_ERR_TOPOLOGY = -3,    /* connection or patch extents do not match / overlap */
  CFD_ERR_GRID = -4,        /* non-positive cell volume or degenerate face */
  CFD_ERR_HIP = -5,         /* HIP runtime error */
  CFD_ERR_NONFINITE = -6,   /* non-finite or non-physical state detected */
  CFD_ERR_UNSUPPORTED = -7  /* valid request the library does not implement */
} cfd_status;

enum { CFD_LIM_NONE = 0, CFD_LIM_VANLEER = 1, CFD_LIM_VANALBADA = 2 };
/* Face flux.  ROE: rotated Roe flux with Harten smoothing (efix).  VANLEER_FVS:
 * F = A (F+(qL) + F-(qR)) with van Leer's Mach-number polynomial split;
 * STEGER_WARMING: the same with F+- = R diag((l +- |l|)/2) R^-1 Q (closed form). */
enum { CFD_FLUX_ROE = 0, CFD_FLUX_VANLEER_FVS = 1, CFD_FLUX_STEGER_WARMING = 2 };
enum {
  CFD_BC_SLIP_WALL = 1,
  CFD_BC_SUP_INFLOW = 2,
  CFD_BC_EXTRAP_OUTFLOW = 3,
  CFD_BC_FARFIELD = 4,
  CFD_BC_SUB_INFLOW = 5,
  CFD_BC_SUB_OUTFLOW = 6,
  CFD_BC_NOSLIP_WALL = 7
};
/* CFL: one global step CFL * min(Omega/lambda) from Q^n each step.  FIXED:
 * dt_fixed.  LOCAL: every cell advances with its own CFL * Omega/lambda from
 * Q^n (steady-state acceleration; time-inaccurate by design).
 * lambda = sum_d |u . Sbar_d| + c |Sbar_d|, Sbar_d the mean of the cell's two
 * area vectors in direction d. */
enum { CFD_DT_CFL = 0, CFD_DT_FIXED = 1, CFD_DT_LOCAL = 2 };
/* execution modes for cfd_set_exec */
enum { CFD_EXEC_BATCHED = 0, CFD_EXEC_PER_BLOCK = 1, CFD_EXEC_PERSISTENT = 2 };
/* connected-boundary exchange for cfd_set_ghost_exchange */
enum { CFD_GHOSTS_DIRECT = 0, CFD_GHOSTS_PACKED = 1 };

typedef struct {
  int dim;              /* 2 or 3 */
  double gamma;         /* ratio of specific heats (1.4) */
  int limiter;          /* CFD_LIM_*; symmetric limiters only (van Leer, van Albada) or none */
  double muscl_eps;     /* MUSCL epsilon of eq. (flux); 1 = second order */
  double muscl_kappa;   /* MUSCL kappa of eq. (flux); face states do not depend on it
                           for the symmetric limiters, the value is validated only */
  double lim_eps[5];    /* van Albada regularisation per primitive variable (rho,u,v[,w],p) */
  double efix;          /* Harten smoothing half-width as a fraction of the Roe sound speed; 0 = off */
  int rk_stages;        /* M of the M-stage scheme, alpha_k = 1/(M-k+1); 1..8 (4 with CFD_RK_CLASSIC4) */
  int dt_mode;          /* CFD_DT_CFL | CFD_DT_FIXED | CFD_DT_LOCAL */
  double cfl;           /* CFL number for CFD_DT_CFL and CFD_DT_LOCAL */
  double dt_fixed;      /* time step for CFD_DT_FIXED */
  int flux;             /* CFD_FLUX_*: inviscid face flux (Sec. 2 lists Roe's flux-difference
                           splitting and van Leer's and Steger-Warming's flux-vector
                           splittings); the residual VJP needs CFD_FLUX_ROE */
  double viscosity;     /* laminar Navier-Stokes when > 0: constant viscosity in these units
                           (rho_inf = c_inf = 1), mu = M_inf / Re per unit length; 0 = Euler */
  double prandtl;       /* Prandtl number (0.72) when viscosity > 0 */
  int debug_flags;      /* CFD_CHECK_FINITE | CFD_NAN_GHOSTS (0 for production runs) */
  int rk_scheme;        /* CFD_RK_MSTAGE (Sec. 2) | CFD_RK_CLASSIC4 */
} cfd_config;

/* Runge-Kutta scheme (cfd_config.rk_scheme).  CFD_RK_MSTAGE: the M-stage
 * scheme of Sec. 2, Q^(k) = Q^(0) - dt R(Q^(k-1)) / (M-k+1).  CFD_RK_CLASSIC4
 * (not in the paper): the classical fourth-order method, stage inputs
 * Y2 = Q - dt/2 R(Q), Y3 = Q - dt/2 R(Y2), Y4 = Q - dt R(Y3) and
 * Q^(n+1) = Q - dt/6 (R(Q) + 2 R(Y2) + 2 R(Y3) + R(Y4)); needs rk_stages = 4,
 * two more state buffers in the workspace, and has no step adjoint
 * (cfd_rk_step_vjp and cfd_rk_step_record return CFD_ERR_UNSUPPORTED).  Any
 * other value is CFD_ERR_ARG at cfd_create. */
enum { CFD_RK_MSTAGE = 0, CFD_RK_CLASSIC4 = 1 };

/* Debug checks (cfd_config.debug_flags; any other bit is CFD_ERR_ARG at
 * cfd_create).  With any flag set, cfd_rk_step does not use its captured graph.
 *   CFD_CHECK_FINITE  after every Runge-Kutta stage of cfd_rk_step the new
 *                     state is checked on the device (density and pressure
 *                     positive and finite, velocity finite); cfd_rk_step then
 *                     synchronises after every step and returns
 *                     CFD_ERR_NONFINITE, naming the step, if a stage failed
 *                     (the state is left as that step produced it).
 *                     cfd_residual checks its output for non-finite entries
 *                     the same way.
 *   CFD_NAN_GHOSTS    every ghost fill first writes quiet NaN into the whole
 *                     ghost region of the state buffer (both layers, edges
 *                     and corners), so a ghost value that the connections and
 *                     patches do not provide shows up as NaN in the result. */
enum { CFD_CHECK_FINITE = 1, CFD_NAN_GHOSTS = 2 };

/* Version string of the library build. */
const char* cfd_version(void);
const char* cfd_status_string(cfd_status s);
/* Last error message of a context (never NULL; "" if none). */
const char* cfd_last_error(const cfd_ctx* ctx);

/* Create a context on the current HIP device; hip_stream is a hipStream_t
 * (NULL = the default stream) on which all later work is enqueued.
 * Errors: CFD_ERR_ARG for an invalid config (dim, gamma <= 1, stages, cfl). */
cfd_status cfd_create(const cfd_config* cfg, void* hip_stream, cfd_ctx** out);
cfd_status cfd_destroy(cfd_ctx* ctx);

/* Add a block of ni x nj (x nk) cells (nk = 1 in 2D; every extent >= 2).
 * nodes_host: node coordinates as described above, copied by the call.
 * Returns the block id (0, 1, ...) in *block_id.  Only before cfd_finalize. */
cfd_status cfd_add_block(cfd_ctx* ctx, int ni, int nj, int nk, const double* nodes_host, int* block_id);

/* Physical boundary patch on a face range of a block (Sec. 2 boundary types;
 * the paper names the types but prints no formulas; these are the readings).
 * q_i is the interior cell next to the face, n the unit outward normal.
 *   CFD_BC_SLIP_WALL       mirror ghosts, wall-face flux (0, p_w S, 0), p_w = 1.5 p0 - 0.5 p1
 *   CFD_BC_SUP_INFLOW      both ghost layers = params_host[0..dim+1] (primitive)
 *   CFD_BC_EXTRAP_OUTFLOW  both ghost layers = q_i
 *   CFD_BC_FARFIELD        params_host = free-stream primitive state (dim+2);
 *                          both ghost layers = the Riemann-invariant state
 *                          q_b(q_i, q_inf, n) and the face flux is overwritten
 *                          with the exact flux F(q_b) . S (Sec. 7.2 V7)
 *   CFD_BC_SUB_INFLOW      params_host = (p0, rho0, d_1..d_dim): stagnation
 *                          pressure and density, inflow direction (normalised
 *                          by the call); p_b = min(p_i, p0), isentropic rho_b
 *                          and speed, velocity along d
 *   CFD_BC_SUB_OUTFLOW     params_host = (p_back): q_b = (rho_i, u_i, p_back),
 *                          q_i where u_i . n >= c_i
 *   CFD_BC_NOSLIP_WALL     adiabatic no-slip wall: ghost layer g copies interior
 *                          layer g with the velocity negated; the inviscid face
 *                          flux is the wall flux of CFD_BC_SLIP_WALL
 * Parameters must be finite, densities and pressures positive
 * (CFD_ERR_NONFINITE), a direction non-zero (CFD_ERR_ARG); params_host is
 * copied and ignored by the kinds without parameters.
 * Returns a patch id in *patch_id (may be NULL).  Ranges may not overlap other
 * patches or connections (checked at finalize: CFD_ERR_TOPOLOGY).  A context
 * created with the adjoint rejects the last four kinds at finalize
 * (CFD_ERR_UNSUPPORTED). */
cfd_status cfd_set_bc(cfd_ctx* ctx, int block, int face, const int lo[2], const int hi[2],
                      int bc_type, const double* params_host, int* patch_id);

/* Connect face range A of block_a with face range B of block_b (a block may
 * connect to itself: periodic).  Both sides' two ghost layers are filled from
 * the other side's first two interior layers at every stage.  orient maps an
 * offset (r1, r2) inside range A to the offset inside range B: (s1, s2) =
 * (r2, r1) if bit 2 is set else (r1, r2); then s_m is reversed along B's m-th
 * tangential axis if bit (m-1) is set.  Extents must agree under the map. */
cfd_status cfd_connect(cfd_ctx* ctx, int block_a, int face_a, const int lo_a[2], const int hi_a[2],
                       int block_b, int face_b, const int lo_b[2], const int hi_b[2], int orient);

/* Validate the topology and plan all device tables and tiles.  Returns the
 * number of workspace bytes the context needs in *workspace_bytes.
 * Errors: CFD_ERR_STATE (no blocks), CFD_ERR_TOPOLOGY. */
cfd_status cfd_finalize(cfd_ctx* ctx, size_t* workspace_bytes);

/* Bind caller-allocated device memory (>= workspace_bytes, 256-byte aligned)
 * as the context's workspace; uploads tables and nodes and computes the
 * metrics on the device.  Synchronises the stream.
 * Errors: CFD_ERR_ARG (size/alignment), CFD_ERR_GRID (non-positive volume). */
cfd_status cfd_bind_workspace(cfd_ctx* ctx, void* dev_ptr, size_t bytes);

/* Replace the node coordinates of all blocks (device, concatenated node
 * layout) and recompute the metrics.  Synchronises; CFD_ERR_GRID on a
 * non-positive volume. */
cfd_status cfd_set_nodes(cfd_ctx* ctx, const double* dev_nodes);
/* Update the parameters of a patch that has them (supersonic inflow, farfield,
 * subsonic inflow or outflow; the layout and checks of cfd_set_bc).
 * CFD_ERR_ARG for a patch kind without parameters.  Synchronises. */
cfd_status cfd_set_bc_params(cfd_ctx* ctx, int patch_id, const double* params_host);

/* Set the solution from packed conservative (cfd_set_state) or primitive
 * (cfd_set_state_primitive) variables; the CFL step of the new state is
 * recomputed.  Synchronises; CFD_ERR_NONFINITE if any density or pressure is
 * not positive and finite. */
cfd_status cfd_set_state(cfd_ctx* ctx, const double* dev_Q);
cfd_status cfd_set_state_primitive(cfd_ctx* ctx, const double* dev_q);
/* Packed conservative copy of the current solution. */
cfd_status cfd_get_state(cfd_ctx* ctx, double* dev_Q);

/* Residual R(Q) of the current state, packed conservative layout, with
 * dQ/dt = -R: ghost fill (connections, then physical patches), MUSCL face
 * states, the configured face flux on every face, wall-flux override, flux
 * divergence / volume.  With viscosity > 0 (laminar Navier-Stokes, Sec. 2,
 * eq. (governing)) R also subtracts the viscous part Rv = (1/Omega) sum
 * F_v . S_out: Stokes stresses tau = mu (grad u + grad u^T - 2/3 div u I),
 * Theta = u . tau + k grad T with T = gamma p / rho and k = mu / ((gamma-1) Pr);
 * face gradients by Green's theorem over each face's dual volume (the two cell
 * centres and the face's pseudo-nodes, which average the interior and
 * face-ghost cells around a grid node); the CFL steps then add
 * 4 max(4/3, gamma/Pr) (mu/rho) sum_d |Sbar_d|^2 / Omega to lambda. */
cfd_status cfd_residual(cfd_ctx* ctx, double* dev_R);

/* cfd_residual into dev_R, plus dev_norms[v] = sqrt(sum over all cells of
 * R_v^2 / ncells) for each conservative variable v (nvar doubles, device
 * memory): the convergence monitor of steady runs (divide by the first
 * iteration's norms for the relative history).  Deterministic: fixed
 * partition of the cells and fixed reduction order. */
cfd_status cfd_residual_norms(cfd_ctx* ctx, double* dev_R, double* dev_norms);

/* cfd_residual_norms for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * allocation): same arguments and results, but the per-part partial sums
 * live in a library-owned static device array (40 KiB per GPU, held until the
 * process ends) instead of the context workspace, and the call allocates
 * nothing.  Every call on one GPU shares that array: calls that overlap in
 * time on one GPU (different streams or threads) race and must be
 * serialised by the caller.  CFD_ERR_UNSUPPORTED if the partial sums would
 * exceed the array (1024 parts x 5 variables; not reachable with the fixed
 * partition), CFD_ERR_HIP if the array has no address on the context's
 * device. */
cfd_status cfd_residual_norms_noalloc(cfd_ctx* ctx, double* dev_R, double* dev_norms);

/* Limiter freezing for steady runs (Sec. 8.2, the laminar NACA 0012 case: the limiter is frozen late in a
 * steady run so the residual keeps falling; no formula is printed).  Reading:
 * per cell, direction and primitive variable the factor
 *   phi = S(a, b) / ((a + b)/2)   (0 where a + b = 0),
 * S the limiter's slope form and a, b the cell's forward and backward
 * differences, is taken from the current state; while frozen every limited
 * slope is phi (a + b)/2 with the current differences.  The residual is
 * unchanged at the freeze state.
 * cfd_enable_limiter_freezing reserves dim * (dim+2) padded arrays per block
 * in the workspace; call it before cfd_finalize (CFD_ERR_STATE after;
 * CFD_ERR_ARG without a limiter; an adjoint context rejects it at finalize
 * with CFD_ERR_UNSUPPORTED).  cfd_freeze_limiter(ctx, 1) computes the factors
 * from the current state (asynchronous on the stream) and switches every
 * later residual and step to them; cfd_freeze_limiter(ctx, 0) returns to the
 * live limiter.  CFD_ERR_STATE if freezing was not enabled or no state is
 * set. */
cfd_status cfd_enable_limiter_freezing(cfd_ctx* ctx, int enable);
cfd_status cfd_freeze_limiter(cfd_ctx* ctx, int freeze);

/* Global CFL time step CFL * min(Omega / lambda) of the current state, or the
 * fixed step, written to dev_dt[0]; with CFD_DT_LOCAL the smallest cell step. */
cfd_status cfd_time_step(cfd_ctx* ctx, double* dev_dt);

/* Advance nsteps M-stage Runge-Kutta steps in place.  The time step of each
 * step is computed on the device from the state at the start of the step
 * (CFD_DT_CFL) or fixed.  If dev_dt_last is not NULL the step used last is
 * written there. */
cfd_status cfd_rk_step(cfd_ctx* ctx, int nsteps, double* dev_dt_last);

/* Padded primitive arrays of all blocks after a ghost fill of the current
 * state (connections, then physical patches): block after block, each
 * [var][k+2][j+2][i+2] with extents (nk+4) (1 in 2D), (nj+4), (ni+4).
 * Corner ghost cells are undefined.  For inspection and tests. */
cfd_status cfd_padded_primitives(cfd_ctx* ctx, double* dev_out);
/* Element count of the cfd_padded_primitives output. */
cfd_status cfd_padded_size(cfd_ctx* ctx, size_t* count);

/* Execution mode of rk_step/residual: CFD_EXEC_BATCHED launches every phase
 * once for all blocks (tile list over every block, one workgroup per tile);
 * CFD_EXEC_PERSISTENT launches the stage kernel once for all blocks with as
 * many workgroups as the device holds at once, each walking the tile list
 * (grid-stride loop); CFD_EXEC_PER_BLOCK launches each phase once per block.
 * use_graph != 0 captures one Runge-Kutta step in a hipGraph (batched and
 * persistent modes).  All modes give bit-identical results. */
cfd_status cfd_set_exec(cfd_ctx* ctx, int mode, int use_graph);

/* Connected-boundary exchange (Sec. 4: ghosts of connected boundaries are
 * exchanged at every Runge-Kutta stage).  CFD_GHOSTS_DIRECT (default): every
 * receiver ghost is copied straight from the donor's interior in the same
 * launch as the physical patches (all blocks are on this GPU; Sec. 5 fills
 * self-connected ghosts by copying); along an axis that a block connects to
 * itself end to end without reorientation the stage kernel and the viscous
 * pass read the periodic neighbours through the wrap, so between the stages
 * of a step those connections are not filled at all (unless the limiter is
 * frozen; every other reader of the ghosts fills them in full).  CFD_GHOSTS_PACKED: the donor strips are
 * packed into per-connection segments of the exchange buffer, then unpacked
 * into the receivers (Sec. 7.2 V1/V5), the form a transfer between GPUs would
 * take.  Bit-identical results.  CFD_ERR_ARG for another mode. */
cfd_status cfd_set_ghost_exchange(cfd_ctx* ctx, int mode);

/* Time every compiled tile shape of the stage kernel on the bound problem
 * (reps launches each) and keep the fastest.  *chosen (may be NULL) receives
 * the index of the chosen variant.  Synchronises. */
cfd_status cfd_autotune(cfd_ctx* ctx, int reps, int* chosen);
/* Select a tile-shape variant by index (0 .. cfd_query(CFD_Q_NVARIANTS)-1). */
cfd_status cfd_set_variant(cfd_ctx* ctx, int variant);

/* Kernel timing: while enabled, rk_step records HIP events around every
 * stage-kernel launch on the context stream (graph capture is bypassed).
 * cfd_kernel_time returns the summed stage-kernel time in ms and the launch
 * count since the last enable; it synchronises. */
cfd_status cfd_profile(cfd_ctx* ctx, int enable);
cfd_status cfd_kernel_time(cfd_ctx* ctx, double* total_ms, long long* launches);

/* ---- adjoint (residual vector-Jacobian products) --------------------------
 * Not in the paper: a hand-written reverse-mode derivative of the residual
 * above (ghost fill, MUSCL with the symmetric limiters or none, Roe flux with
 * Harten smoothing, wall override, divergence), so gradients of functionals of
 * the solution with respect to the state, the node coordinates and the inflow
 * states can be formed.  The context must be created with cfd_enable_adjoint
 * before cfd_finalize (it reserves the extra workspace).  Cotangents use the
 * same layouts as their primal values (packed conservative state, node
 * layout, dim+2 values per inflow patch in patch-id order of the inflow
 * patches).  Node gradients cover 2D and 3D grids (2D: the face vectors and
 * diagonal-product areas; 3D: the half cross products of face diagonals and
 * the mean-node face sums of the cell volumes, transposed per node). */

/* Reserve adjoint workspace (call before cfd_finalize). */
cfd_status cfd_enable_adjoint(cfd_ctx* ctx, int enable);
/* dev_Qbar = (dR/dQ)^T dev_Rbar at the current state; if not NULL,
 * dev_Xbar = (dR/dX)^T dev_Rbar (nodes) and dev_BCbar = (dR/dtheta)^T dev_Rbar
 * (inflow states).  Clears the metric/inflow accumulators first.  dev_Rbar
 * and dev_Qbar must not overlap (cells are finalized while neighbouring
 * tiles still read the residual cotangent). */
cfd_status cfd_residual_vjp(cfd_ctx* ctx, const double* dev_Rbar, double* dev_Qbar, double* dev_Xbar,
                            double* dev_BCbar);
/* Zero the accumulated node-metric and inflow cotangents. */
cfd_status cfd_adjoint_reset(cfd_ctx* ctx);
/* Reverse one Runge-Kutta step taken from the current state (the state at
 * the start of that step, e.g. restored with cfd_load_state): on entry
 * dev_Qbar holds dJ/dQ^{n+1}, on return dJ/dQ^n; the metric and inflow
 * cotangents of the step accumulate.  Needs CFD_DT_FIXED and at most 4 stages. */
cfd_status cfd_rk_step_vjp(cfd_ctx* ctx, double* dev_Qbar);
/* One Runge-Kutta step like cfd_rk_step(ctx, 1, NULL) that also leaves the
 * ghost-filled inputs Q^(0..M-1) of its M stages in dev_stages: M consecutive
 * slots of cfd_state_size bytes each (device memory owned by the caller, same
 * internal layout as cfd_save_state).  Stages 1..M-1 write straight into the
 * slots; slot 0 is one copy of the step-start state. */
cfd_status cfd_rk_step_record(cfd_ctx* ctx, void* dev_stages);
/* cfd_rk_step_vjp for a step recorded by cfd_rk_step_record: the stage states
 * come from dev_stages instead of being recomputed, and the current state is
 * neither read nor changed.  Same cotangent conventions and requirements. */
cfd_status cfd_rk_step_vjp_recorded(cfd_ctx* ctx, const void* dev_stages, double* dev_Qbar);
/* J = sum over slip-wall faces of p_w |S| (integrated wall pressure) into
 * dev_J[0]; dev_Qbar (nullable) = dJ/dQ; dJ/dS accumulates. */
cfd_status cfd_objective_wall_pressure(cfd_ctx* ctx, double* dev_J, double* dev_Qbar);
/* Node gradient and inflow-state gradient of everything accumulated since
 * the last reset (both nullable). */
cfd_status cfd_adjoint_result(cfd_ctx* ctx, double* dev_Xbar, double* dev_BCbar);
/* dev_thetabar[dim+2] = (dQ/dtheta)^T sum over cells of dev_Qbar, for a
 * uniform state Q = Q(theta) with primitive theta_host[dim+2]. */
cfd_status cfd_uniform_state_vjp(cfd_ctx* ctx, const double* theta_host, const double* dev_Qbar,
                                 double* dev_thetabar);
/* Bit-exact copy of the internal solution (checkpoints): cfd_state_size
 * bytes, device memory. */
cfd_status cfd_state_size(cfd_ctx* ctx, size_t* bytes);
cfd_status cfd_save_state(cfd_ctx* ctx, void* dev_dst);
cfd_status cfd_load_state(cfd_ctx* ctx, const void* dev_src);

enum {
  CFD_Q_NBLOCKS = 0, CFD_Q_NCELLS = 1, CFD_Q_NVAR = 2, CFD_Q_NVARIANTS = 3, CFD_Q_VARIANT = 4,
  CFD_Q_NTILES = 5, CFD_Q_NTRANSFERS = 6, CFD_Q_NPATCHES = 7, CFD_Q_NNODES = 8,
  CFD_Q_EXCHANGE_DOUBLES = 9, CFD_Q_WORKSPACE_BYTES = 10, CFD_Q_TILE_X = 11, CFD_Q_TILE_Y = 12
};
/* Integer facts about a finalized context. */
cfd_status cfd_query(cfd_ctx* ctx, int what, long long* value);

/* ---- measurement ------------------------------------------------------
 * Streaming-bandwidth probe (no method arithmetic; a ceiling for the stage
 * kernel's HBM rate): a kernel that reads element e of `reads` arrays and
 * writes element e of `writes` arrays for e < n, each array n doubles
 * (dev_src holds reads * n doubles, dev_dst writes * n, caller-owned device
 * memory on the stream's device), with one double per lane per array
 * (vec = 1, the stage kernel's 8-byte coalesced accesses) or two (vec = 2,
 * 16-byte accesses; n even).  Supported (reads, writes): (1, 1), (3, 1),
 * (4, 1), (15, 5), (20, 5) -- 20 reads and 5 writes per element is the
 * stage kernel's per-cell traffic in 3D after the first stage.  One warm-up
 * launch, then reps timed launches on hip_stream (hipStream_t, NULL = default);
 * *ms_out = mean milliseconds per launch.  Synchronises.  Errors: CFD_ERR_ARG
 * (null pointer, n <= 0, reps <= 0, vec, unsupported pair), CFD_ERR_HIP. */
cfd_status cfd_stream_probe(int reads, int writes, int vec, const double* dev_src, double* dev_dst, long long n,
                            int reps, void* hip_stream, double* ms_out);

#ifdef __cplusplus
}
#endif
#endif /* CFDHIP_H */
