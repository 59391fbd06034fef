/*
 * lbm3d.h -- C ABI of the MI355X (gfx950) coupled D3Q19 / D3Q7 thermal
 * pseudopotential lattice Boltzmann step.
 *
 * Method: J. Huang, L. Wang, K. He, C. Huang, "An efficient thermal lattice
 * Boltzmann method for simulating three-dimensional liquid-vapor phase
 * change" (arXiv 2206.00946).  One call of lbm_step advances the state by the
 * paper's time step: D3Q19 non-orthogonal MRT collision in moment space with
 * exact-difference forcing (Sec. 2.1, eqs. (1)-(11), Appendix A.1), the
 * Peng-Robinson pseudopotential and its interaction force (eqs. (6), (7),
 * (54), (55)), the D3Q7 MRT temperature update with the rho*c_v blend and the
 * phase-change source (Sec. 2.2, eqs. (13)-(15), (27)-(29), Appendix A.2),
 * streaming (eq. (9)), and the boundary treatments of Sec. 3 (bounce-back
 * eq. (34), thermal non-equilibrium extrapolation eqs. (35)-(36), the wetting
 * ghost layer eq. (37), the D3Q19 constant-pressure outlet eqs. (38)-(53)).
 *
 * Conventions shared by every entry point
 *  - Grid: nx*ny*nz cells, dx = dt = 1; flat index x + nx*(y + ny*z).
 *  - Host arrays are caller-owned and only read/written during the call.
 *  - Device arrays (dst_on_device = 1, or the optional device_buffer of
 *    lbm_create) are caller-owned device pointers on the current HIP device.
 *  - Every function validates its arguments and returns an lbm_status; no
 *    exception crosses the ABI.  On LBM_EHIP the HIP error string is kept in
 *    lbm_last_error().  A ctx is used by one host thread at a time; all GPU
 *    work is enqueued on the ctx stream.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;   /* opaque, library-owned */

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = 1,        /* bad argument or inconsistent parameters            */
  LBM_ENOMEM = 2,        /* allocation failed or device_buffer too small       */
  LBM_EHIP = 3,          /* a HIP call failed (see lbm_last_error)             */
  LBM_ENONPHYS = 4,      /* rho <= 0, rho*b >= 1, T <= 0, psi^2 < 0 or NaN met */
  LBM_ESTATE = 5,        /* call out of order (e.g. lbm_step before lbm_init)  */
  LBM_EUNSUPPORTED = 6   /* valid request that this library does not implement */
} lbm_status;

/* Storage precision of the populations.  FP64 computes in double.  The other
 * three store f_i - w_i*rho_ref and g_i - w_i*T_ref (deviations from the rest
 * equilibrium) and compute in float. */
typedef enum {
  LBM_FP64 = 0,
  LBM_FP32_DEV = 1,
  LBM_FP16_DEV = 2,
  LBM_BF16_DEV = 3
} lbm_precision;

/* Face kinds, faces ordered (-x, +x, -y, +y, -z, +z).  Periodic faces come in
 * pairs.  WALL (no-slip, bounce-back eq. (34), wetting ghost layer eq. (37))
 * is accepted on the z faces only, with x and y periodic.  PRESSURE is the
 * constant-density outlet of Sec. 3.3 on any face.  Every non-periodic face is
 * a Dirichlet temperature face (eqs. (35)-(36)). */
typedef enum {
  LBM_FACE_PERIODIC = 0,
  LBM_FACE_WALL = 1,
  LBM_FACE_PRESSURE = 2
} lbm_face_kind;

typedef struct {
  int32_t nx, ny, nz;            /* cells; a bounded axis needs >= 3 cells      */
  int32_t precision;             /* lbm_precision                               */
  double a, b, R, omega;         /* Peng-Robinson, eqs. (54)-(55); paper: 3/49, 2/21, 1, 0.344 */
  double G;                      /* interaction strength, eq. (6); paper: -1    */
  double s_e, s_nu, s_q, s_pi;   /* D3Q19 relaxation rates, eq. (11)            */
  double wbar;                   /* D3Q7 rest weight parameter, 0 < wbar < 1    */
  double lambda;                 /* thermal conductivity (sets varsigma_1..3)   */
  double cv;                     /* specific heat at constant volume            */
  double s_T_other;              /* varsigma_0 and varsigma_4..6                */
  int32_t theta_corr;            /* vartheta of eq. (13): 0, or 1 for the correction S_i of
                                  * eq. (16) with d2T/dt2 = T(t) - 2T(t-1) + T(t-2) (applied
                                  * from the third step after lbm_init; unfused kernels) */
  int32_t face[6];               /* lbm_face_kind per face                      */
  double face_T[6];              /* Dirichlet temperature of each bounded face  */
  double face_rho[6];            /* outlet density of each PRESSURE face        */
  double kappa_w;                /* tan(pi/2 - theta) of eq. (37) on wall faces */
  double rho_ref, T_ref;         /* deviation-storage references               */
  double diag_rho_v, diag_rho_l; /* densities used by the liquid-volume diagnostics */
  /* Density-dependent conductivity (the liquid and vapour values of the
   * Sec. 4.1 benchmark): with lambda_vapour > 0 and lambda_liquid > 0,
   * lambda(rho) is linear in rho between (lambda_rho_v, lambda_vapour) and
   * (lambda_rho_l, lambda_liquid) and constant beyond, and varsigma_1..3 are
   * set per node from it; with both 0, lambda is uniform. */
  double lambda_vapour, lambda_liquid;
  double lambda_rho_v, lambda_rho_l;
} lbm_params;

typedef struct {
  double mass;        /* sum of rho over all cells (FP64 reduction)            */
  double energy;      /* sum of rho*c_v*T                                      */
  double vol_hard;    /* number of cells with rho > (diag_rho_v+diag_rho_l)/2  */
  double vol_smooth;  /* sum of clip((rho-rho_v)/(rho_l-rho_v), 0, 1)          */
  double evap_mass;   /* mass at lbm_init minus mass now                       */
  int64_t step;       /* time steps taken since lbm_init                       */
} lbm_diag;

/* Fill *p with the paper's parameters (Sec. 4: a = 3/49, b = 2/21, R = 1,
 * omega = 0.344, G = -1, relaxation times 1.25 (shear) and 0.8 (bulk) read
 * as rates s_nu = 0.8 and s_e = 1.25, s_q = s_pi = 1; lambda = 1/3, cv = 5
 * (Sec. 4.2); wbar = 0.75), an all-periodic nx*ny*nz box, FP32 deviation
 * storage with rho_ref = 0.3796789993997207 (vapour at 0.86 Tc) and
 * T_ref = 0.86 Tc.  Returns LBM_EINVAL if p is NULL. */
lbm_status lbm_default_params(lbm_params* p, int32_t nx, int32_t ny, int32_t nz);

/* Bytes of device memory a context needs for the state of the method: the
 * D3Q19 populations f_i and D3Q7 populations g_i of eqs. (1) and (13) at one
 * time level plus the next (streaming of eq. (9) writes a second copy).
 * state_bytes covers the two copies of
 * the populations (2 * 26 * nz * (nx*ny + 64) * element size: each direction
 * plane is padded by 64 elements), scratch_bytes for fields, wall
 * temperature planes and reduction partials.  Validates *p. */
lbm_status lbm_required_bytes(const lbm_params* p, size_t* state_bytes, size_t* scratch_bytes);

/* Create a context for the problem the paper states in Sec. 2-4: the grid
 * (dx = dt = 1), the Peng-Robinson parameters of eqs. (54)-(55), G of eq.
 * (6), the relaxation rates of eq. (11) and of the D3Q7 matrix (conductivity
 * after eq. (33)), c_v and wbar of eqs. (13)-(14), vartheta of eq. (13), and
 * the face conditions of Sec. 3.
 * Create it on the current HIP device.  device_buffer: NULL lets the
 * library allocate (and later free) its memory; otherwise a caller-owned
 * device allocation of at least state_bytes + scratch_bytes that must outlive
 * the context.  hip_stream: a hipStream_t, or NULL for the default stream.
 * Parameters are validated (LBM_EINVAL) and unsupported combinations
 * (walls on x/y faces) give LBM_EUNSUPPORTED.
 * A step runs as one single-pass kernel launch when x and y are periodic, z
 * is periodic or has a wall or pressure outlet on each of its two faces,
 * nx >= 8, ny % 8 == 0, nz >= 4 and theta_corr = 0; otherwise as four
 * launches of the general kernels (same results to rounding).  Environment
 * overrides read when the context is created, for tests and measurements:
 * LBM_FUSED=0 forces the general kernels, LBM_FUSED_CHUNK=n cuts the z march
 * of the single-pass kernel into n-plane chunks, LBM_FUSED_TY=16 selects
 * 16-row tiles (FP32/FP16/BF16, nx % 64 == 0, ny % 16 == 0), LBM_FUSED_MAP=1
 * gives each XCD a 2 x 4 block of tiles, LBM_FUSED_XDEFER=0 keeps the
 * ordinary state between the FP64 steps of one lbm_step call. */
lbm_status lbm_create(const lbm_params* p, void* device_buffer, size_t buffer_bytes,
                      void* hip_stream, lbm_ctx** out);

/* Set the state from host FP64 fields (nx*ny*nz each): f = f^eq(rho, u)
 * (eq. (2)), g = w_i T (eq. (14)).  u is 3*cells (x, then y, then z
 * components) or NULL for rest.  Resets the step counter and records the
 * initial mass for evap_mass.  Synchronous. */
lbm_status lbm_init(lbm_ctx* ctx, const double* rho, const double* u, const double* T);

/* T_b of the thermal Dirichlet condition of Sec. 3.1, eqs. (35)-(36),
 * g_i(x_b) = w_i T_b + g_i(x_f) - w_i T(x_f), as a field over a wall face:
 * replace the Dirichlet temperature of a wall face (4 = -z, 5 = +z) by a
 * host FP64 field of nx*ny values (index x + nx*y).  NULL restores the
 * uniform face_T.  Synchronous. */
lbm_status lbm_set_wall_T(lbm_ctx* ctx, int32_t face, const double* Tw);

/* Set kappa_w = tan(pi/2 - theta) of eq. (37). */
lbm_status lbm_set_kappa(lbm_ctx* ctx, double kappa_w);

/* Advance nsteps >= 0 time steps of the method: per step the boundary
 * completion of Sec. 3 (eqs. (34)-(53)), rho and T (eqs. (3), (25)), psi
 * (eqs. (7), (54)), the force (eq. (6)), the velocities (eqs. (4)-(5)), the
 * source (eqs. (15), (27)-(29)), both collisions (eqs. (8), (10), (11) and
 * (13)-(14)) and streaming with the rho c_v blend (eqs. (9), (13)).  The
 * work is enqueued on the ctx stream;
 * the call synchronises once at the end to read the non-physical-state flag
 * and returns LBM_ENONPHYS if any step met rho <= 0, rho*b >= 1, T <= 0,
 * a negative psi radicand or a NaN (the state stays readable).  If a HIP
 * call fails part-way (LBM_EHIP) the state is unspecified: between the steps
 * of one call the library may keep the populations in an internal layout. */
lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* rho, real velocity u (eq. (5); 3*cells, component-major) and T of the
 * current state with boundary nodes completed (Dirichlet temperature and
 * outlet populations filled).  Any output pointer may be NULL.  With
 * dst_on_device = 1 the pointers are device pointers.  Synchronous. */
lbm_status lbm_fields(lbm_ctx* ctx, double* rho, double* u, double* T, int32_t dst_on_device);

/* Raw populations of the current state in FP64 (f: 19*cells, g: 7*cells,
 * direction-major; deviation storage is converted back to full values).
 * Slots not yet filled by the outlet condition hold unspecified values.
 * Host pointers; either may be NULL.  Synchronous. */
lbm_status lbm_populations(lbm_ctx* ctx, double* f, double* g);

/* Checkpoint and resume (infrastructure around the method; the paper
 * defines no such operation).  lbm_save writes the whole state of the context
 * into host memory: the current populations in their device layout and
 * storage format, the step counter, the initial mass (for evap_mass), the
 * wall temperature planes set by lbm_set_wall_T, kappa_w and, with
 * theta_corr = 1, the two stored temperatures of eq. (16).  lbm_load puts
 * such an image into a context created with the same grid, precision and
 * theta_corr (the context's other parameters apply from then on), after
 * which lbm_step continues exactly as the saving context would have.
 * lbm_save_bytes gives the image size.  Errors: LBM_EINVAL for a NULL
 * pointer, a buffer smaller than the image, an image not written by
 * lbm_save or one from a different grid, precision or theta_corr;
 * LBM_ESTATE for lbm_save before lbm_init.  The caller owns the host
 * buffer.  Synchronous. */
lbm_status lbm_save_bytes(const lbm_ctx* ctx, size_t* bytes);
lbm_status lbm_save(lbm_ctx* ctx, void* host_dst, size_t bytes);
lbm_status lbm_load(lbm_ctx* ctx, const void* host_src, size_t bytes);

/* FP64 diagnostics of the current state, reduced on the GPU in a fixed
 * order: mass sum(rho), energy sum(rho c_v T), liquid volume (the droplet
 * volume behind the diameter D of the d^2 law, Sec. 4.2, eq. (56)) and the
 * evaporated mass M(init) - M(now).  Fields with the boundary nodes
 * completed (rho_out on outlet nodes).  Errors: LBM_EINVAL for NULL
 * arguments, LBM_ESTATE before lbm_init, LBM_EHIP.  Synchronous. */
lbm_status lbm_reduce(lbm_ctx* ctx, lbm_diag* out);

/* Discrete adjoint of nsteps time steps from the current state t0.
 * Objective (objective = 0): the evaporated mass J = M(t0) - M(t0 + N),
 * M = sum over all cells of rho (rho_out on outlet nodes), the quantity
 * behind the d^2 law (Sec. 4.2, eq. (56)).  The adjoint reverses every stage
 * of the step (Sec. 2, 3.1, 3.3: collisions, streaming, blend, source,
 * force and divergence stencils, wetting ghost layer eq. (37), outlet fill,
 * Dirichlet extrapolation eqs. (35)-(36)) and returns
 *   dJ_dTw[x + nx*y]: derivative with respect to the Dirichlet temperature
 *                     of node (x, y) of face spec->wall_face (the T_w field
 *                     when one is set, else the uniform face_T), nx*ny values;
 *   *dJ_dkappa:       derivative with respect to kappa_w (eq. (37)); the
 *                     derivative of |grad_t psi| at 0 is taken as 0.
 * The forward trajectory is recomputed from ceil(N / L) stored states, L =
 * ceil(N / K), K = n_checkpoints (0: ceil(sqrt(N))); the workspace (see
 * lbm_adjoint_bytes) is allocated for the call and released before it
 * returns (LBM_ENOMEM if it does not fit).  Requires periodic x and y faces
 * (LBM_EUNSUPPORTED otherwise) and a non-periodic wall_face (LBM_EINVAL).
 * On return the context holds the state at t0 + N, as after lbm_step(N).
 * J, dJ_dTw and dJ_dkappa may be NULL; dJ_dTw is a device pointer when
 * dst_on_device = 1.  Synchronous. */
typedef struct {
  int32_t nsteps;         /* N >= 1 */
  int32_t n_checkpoints;  /* K >= 0 */
  int32_t objective;      /* 0: evaporated mass */
  int32_t wall_face;      /* 4 (-z) or 5 (+z) */
} lbm_adjoint_spec;

/* Device bytes lbm_adjoint allocates for spec on this context: K + L
 * stored states, two adjoint states and a few fields; when the step runs on
 * the unfused kernels also the per-cell fields (rho, T, psi, three
 * velocities of three components) of the L states of a segment, kept from
 * its recomputation so that the reverse step does not derive them again. */
lbm_status lbm_adjoint_bytes(const lbm_ctx* ctx, const lbm_adjoint_spec* spec, size_t* bytes);

lbm_status lbm_adjoint(lbm_ctx* ctx, const lbm_adjoint_spec* spec, double* J, double* dJ_dTw, double* dJ_dkappa,
                       int32_t dst_on_device);

/* lbm_adjoint for callers that cannot allocate device memory (code under HIP
 * graph capture of the surrounding work, tight serving or optimisation loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * lbm_adjoint, computed by the same kernels, but the workspace (the
 * lbm_adjoint_bytes of the request) lives in a fixed 64 MiB device array that
 * the library holds on every GPU it runs on until the process ends; the call
 * itself allocates and frees nothing.  Requests needing more than 64 MiB
 * return LBM_ENOMEM before any work (the state stays at t0).  The context's
 * device must be the current device (LBM_EINVAL otherwise).  Every call on
 * one GPU shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (two host threads, or contexts on different streams
 * whose calls interleave) race and must be serialised by the caller.
 * Synchronous. */
lbm_status lbm_adjoint_noalloc(lbm_ctx* ctx, const lbm_adjoint_spec* spec, double* J, double* dJ_dTw,
                               double* dJ_dkappa, int32_t dst_on_device);

/* Message of the last failing call on ctx (or of the last failing
 * lbm_create when ctx is NULL).  Valid until the next call on ctx. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Release the context and, if the library allocated it, its memory. */
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */
