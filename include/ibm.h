/*
 * ibm.h -- C-ABI of the MI355X (gfx950) implementation of the per-time-step
 * hot path of the sharp-interface immersed boundary fractional-step scheme of
 * Vagnoli, Scarpolini, Verzicco and Viola ("A fast and consistent
 * sharp-interface immersed boundary method for moving bodies of arbitrary
 * thickness").
 *
 * Problem statement followed by the calls (paper Sec. 2): a box periodic and
 * uniform in x and z, stretched in y between two no-slip walls; a staggered
 * grid with the pressure at cell centres and each velocity component on the
 * faces normal to it; moving surfaces made of triangles with a prescribed wall
 * velocity; Reynolds number Re, time step dt and a fractional-step scheme
 * (RK2+CN or AB+CN).
 *
 * Conventions shared by every call
 *   - Arrays are row-major [y][z][x] (x fastest).  u, w and p hold
 *     ny*nz*nx values; v holds (ny+1)*nz*nx values including the two wall
 *     planes j = 0 and j = ny, which the library keeps at 0.
 *     u(i,j,k) sits at (i dx, yc[j], (k+1/2) dz), v(i,j,k) at
 *     ((i+1/2) dx, yf[j], (k+1/2) dz), w(i,j,k) at ((i+1/2) dx, yc[j], k dz),
 *     p(i,j,k) at ((i+1/2) dx, yc[j], (k+1/2) dz).
 *   - Precision (ibm_opts.precision).  IBM_FP64: every array is FP64.
 *     IBM_MIXED: u, v, w, phi and every right-hand side passed in stay FP64;
 *     p and the H arrays are FP32 ("f32/f64" below: FP32 in the mixed form,
 *     FP64 otherwise).  The mixed form runs the predictor (right-hand side
 *     storage and line solves) in FP32; its Poisson solve is FP64, or FP32
 *     transforms refined with FP64 residuals (ibm_opts.mixed_poisson).
 *   - "dev" pointers are device memory on the context's device; "host"
 *     pointers are host memory.  The caller owns every array it passes; the
 *     library owns its workspace and the tag buffers.
 *   - Every call is enqueued on the context's HIP stream and returns without
 *     synchronising, except ibm_check and the *_host calls.  A context is
 *     bound to one stream and one device and is not thread-safe.
 *   - Return value: IBM_OK (0) or a negative IBM_E* code.  Conditions found
 *     on the device (capacity overflow, non-finite values, geometry limits)
 *     are recorded in a sticky device word that ibm_check returns.  No call
 *     aborts or throws across the ABI.
 */
#ifndef IBM_H
#define IBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define IBM_OK 0
#define IBM_EINVAL (-1)    /* bad size, layout, pointer or grid */
#define IBM_ENOMEM (-2)    /* device allocation failed at create */
#define IBM_EHIP (-3)      /* HIP runtime error; text in ibm_strerror */
#define IBM_ECAPACITY (-4) /* forcing list or C_B list overflowed */
#define IBM_ENONFINITE (-5)
#define IBM_ECFL (-6)      /* a body vertex moves more than half the local
                              spacing in one step (device flag
                              IBM_FLAG_CFL) */
#define IBM_EGEOM (-7)     /* body too large for the periodic box, probe
                              leaving the channel, or a probe stencil that
                              contains its own forcing node */
#define IBM_ECOMPAT (-8)   /* a Poisson right-hand side that fails the
                              compatibility condition (device flag
                              IBM_FLAG_COMPAT) */

/* sticky device flags returned by ibm_check */
#define IBM_FLAG_CAPACITY 1u
#define IBM_FLAG_NONFINITE 2u
#define IBM_FLAG_GEOM 4u
#define IBM_FLAG_REFINE 8u /* mixed form: a Poisson solve ended above the
                              refinement tolerance after refine_max steps */
#define IBM_FLAG_CFL 16u   /* ibm_step: over dt a body vertex moves more
                              than half the local spacing along an axis
                              (|U_x| dt > dx/2, |U_z| dt > dz/2 or |U_y| dt >
                              dy/2 of the cell the vertex lies in): the
                              one-layer fresh-cell treatment of Sec. 3.1
                              needs less */
#define IBM_FLAG_COMPAT 32u /* poisson_solve: |sum rhs dV| > 1e-12 sum |rhs|
                               dV, so Eq. elliptic_mod has no solution (the
                               solve still returns the gauged field) */

#define IBM_FP64 0
#define IBM_MIXED 1

/* Poisson solve of the mixed form (ibm_opts.mixed_poisson) */
#define IBM_POISSON_FP64 0    /* FP64 transforms and solves (default) */
#define IBM_POISSON_REFINED 1 /* FP32 transforms, FP64 wall-normal solves,
                                 FP64-residual refinement */
#define IBM_RK2CN 0
#define IBM_AB2CN 1

/* shape of the sinks/sources q on the fluid cells (ibm_opts.use_q) */
#define IBM_Q_NONE 0    /* standard projection, D u = 0 everywhere */
#define IBM_Q_UNIFORM 1 /* uniform q_F (Sec. 3.2, Eq. q_F): mass */
#define IBM_Q_ENERGY 2  /* q_F = c0 + c1 (p - e) (App. B, Eq. unif_shape):
                           mass and kinetic energy in the inviscid limit */

typedef struct ibm_ctx ibm_ctx;

/* Grid (paper Sec. 2, Fig. 1).  y_faces: host array of ny+1 strictly
 * increasing face heights; the walls are y_faces[0] and y_faces[ny].
 * Periodic spacings are lx/nx and lz/nz. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t reserved;
  double lx, lz;
  const double* y_faces; /* host, ny+1 */
} ibm_grid;

/* Options.  dpdx is the mean pressure gradient dP/dx; the driving volume
 * force is -dpdx along x.  force_cap bounds each forcing list and the C_B
 * list (0 = automatic: max(65536, cells/16)).  use_q: IBM_Q_UNIFORM applies
 * the consistent mass correction of Sec. 3.2, IBM_Q_ENERGY its mass- and
 * energy-conserving shape of App. B (p = the sub-stage's pressure, e = the
 * cell-centred kinetic energy of u_hat, each component's square averaged
 * over the two faces; a constant p - e on C_F falls back to the uniform
 * shape), IBM_Q_NONE the standard projection.
 * Mixed form only: mixed_poisson selects the Poisson solve, FP64
 * (IBM_POISSON_FP64, the default: on stretched grids the FP32 solve's
 * rounding, amplified by the largest wall-normal eigenvalue, needs two
 * refinements to reach the divergence bound, which costs more than an FP64
 * solve) or FP32 transforms refined with FP64 residuals
 * (IBM_POISSON_REFINED); refine_max (0..16, 0 = 3) bounds the refinements of
 * one solve, which stop once max|rhs - L_c phi| * alpha_dt <= refine_tol
 * (0 = 1e-11; alpha_dt = 1 for poisson_solve); after the projection that
 * product is max|D u - q| (paper Eq. mod_div). */
typedef struct {
  int32_t precision; /* IBM_FP64 or IBM_MIXED */
  int32_t scheme;    /* IBM_RK2CN or IBM_AB2CN */
  double re;
  double dpdx;
  int64_t force_cap;
  int32_t use_q;
  int32_t refine_max;
  double refine_tol;
  int32_t mixed_poisson;
  int32_t reserved;
} ibm_opts;

/* One triangulated surface at time t^n (paper Sec. 2: the wall position
 * X(t) and velocity U(X(t))).  xyz, vel: dev f64[nv*3]; tri: dev i32[nt*3]
 * vertex indices.  Several bodies are numbered globally: the triangle id of
 * triangle t of body b is (sum of nt of bodies before b) + t. */
typedef struct {
  int32_t nv, nt;
  const double* xyz;
  const double* vel;
  const int32_t* tri;
} ibm_body;

/* Views of the context-owned tag buffers, filled by ibm_tag and valid until
 * the next ibm_tag.  idx[c]: dev i64, ascending linear node indices of the
 * forcing nodes of component c (v indices count the wall plane j = 0);
 * tri[c]: dev i32 forcing triangle of each; cb: dev i64 ascending linear
 * indices of the boundary cells C_B; count: dev i64[4] = forcing counts of
 * u, v, w and |C_B|; mask[c], cb_mask: dev bitmaps, bit n of word n/32. */
typedef struct {
  int64_t* idx[3];
  int32_t* tri[3];
  int64_t* cb;
  int64_t* count;
  uint32_t* mask[3];
  uint32_t* cb_mask;
  int64_t capacity;
} ibm_tags;

/* Flow state owned by the caller.  u, v, w: dev f64; p: dev f32/f64.
 * h[3] (AB+CN only): dev f32/f64 H^{n-1} read and H^n written; may be NULL
 * for RK2+CN. */
typedef struct {
  double *u, *v, *w;
  void* p;
  void* h[3];
} ibm_state;

/* Create a context on the current HIP device for one grid; all workspace is
 * allocated here and nothing later.  stream: hipStream_t (NULL = default). */
int ibm_create(const ibm_grid* g, const ibm_opts* o, void* stream, ibm_ctx** out);
void ibm_destroy(ibm_ctx* ctx);
int ibm_set_stream(ibm_ctx* ctx, void* stream);

/* Body transforms (the wall position and velocity at t^n from host-evaluated
 * coefficients; only +, - and * on the device, in a fixed order, so the
 * vertices are bit-identical to any implementation of the same order).
 * rigid:  X = c + R X0, U = cdot + omega x (X - c);
 *         coef (host) = [c(3), R(9 row-major), cdot(3), omega(3)];
 *         x0: dev f64[nv*3] reference positions.
 * deform: X = c + (r0 + f s) d, U = cdot + (f sdot) d (a shape carried by
 *         a centre moving at cdot); coef (host) = [c(3), r0, s, sdot,
 *         cdot(3)]; data: dev f64[nv*4] = [d(3), f].
 * Output xyz, vel: dev f64[nv*3]. */
int ibm_body_rigid(ibm_ctx* ctx, const double* x0, int32_t nv, const double* coef,
                   double* xyz, double* vel);
int ibm_body_deform(ibm_ctx* ctx, const double* data, int32_t nv, const double* coef,
                    double* xyz, double* vel);
/* ibm_body_rigid with its 18 coefficients in device memory (coef: dev
 * f64[18], e.g. written by ibm_rigid_advance), so that a free body's motion
 * never visits the host. */
int ibm_body_rigid_dev(ibm_ctx* ctx, const double* x0, int32_t nv, const double* coef,
                       double* xyz, double* vel);

/* Rigid-body dynamics of the loosely coupled FSI (paper Sec. 4.5, driven by
 * the loads of Sec. 3.3): one AB2 step (explicit Euler on a body's first)
 * of Newton's equations (fluid force plus an external force such as
 * gravity with buoyancy, inertial frame), Euler's equations (principal
 * frame; the torque is taken about the body's centre, as ibm_loads gives it
 * with pole = c) and the unit orientation quaternion, renormalised.
 * state: dev f64[nb * IBM_RIGID_STATE], per body c(3), q(4) = (w, x, y, z),
 *   V(3), Omega(3) in the body frame, then the last derivatives (13) and a
 *   started flag (0 before the first step), updated in place;
 * props: dev f64[nb * IBM_RIGID_PROPS]: mass, principal moments (3),
 *   external force (3), unused;
 * loads: dev f64[6 nb], (F, M about c) per body as ibm_loads writes them;
 * coef: dev f64[18 nb], out: the rigid-motion coefficients at the new time
 *   (c, R row-major body -> world, cdot, omega world) for ibm_body_rigid_dev.
 * The paper advances the fluid in a frame translating with the body; here
 * the body moves through the fixed grid.  IBM_EINVAL for a bad argument. */
#define IBM_RIGID_STATE 28
#define IBM_RIGID_PROPS 8
int ibm_rigid_advance(ibm_ctx* ctx, int32_t nb, double* state, const double* props,
                      const double* loads, double dt, double* coef);

/* Tagging (paper Alg. 1, Sec. 3.1) of the three staggered lattices and the
 * boundary cells C_B (Sec. 3.2: cells all of whose faces carry forcing
 * nodes).  A node x is a forcing node if for some triangle T, with X the
 * closest point of T to x and N = x - X, either |N| = 0 or N.(x_n - X) < 0
 * for one of its six same-lattice neighbours x_n; its forcing triangle is
 * the classifying triangle of least |N|^2, ties to the lowest id.  The
 * decision uses IEEE binary64 +,-,*,/ in a fixed order (no FMA), so results
 * are exact integers independent of scheduling.  Also stores the bodies for
 * the following ibm_force / ibm_step calls.  out may be NULL.  (ibm_tag has
 * no time step, so the displacement check of IBM_FLAG_CFL runs only inside
 * ibm_step.) */
int ibm_tag(ibm_ctx* ctx, const ibm_body* bodies, int32_t nbody, ibm_tags* out);
/* Synchronises and copies the four counts (u, v, w, C_B) to the host. */
int ibm_tags_count_host(ibm_ctx* ctx, int64_t* counts);
/* Stream-ordered device-to-device copy of the first n entries of a list of
 * the last ibm_tag: list 0, 1, 2 = forcing nodes of u, v, w (idx_dst: dev
 * i64[n]; tri_dst: dev i32[n] or NULL), list 3 = C_B (idx_dst only).
 * n must not exceed the list's count (IBM_EINVAL if it exceeds the
 * capacity). */
int ibm_tags_copy(ibm_ctx* ctx, int32_t list, int64_t* idx_dst, int32_t* tri_dst, int64_t n);

/* Two-sided IB forcing (paper Eqs. IB_step, probe and new_IB): every forcing
 * node of the last ibm_tag receives u^f = (1 - a) U + a u^e, a = |N|/h,
 * x^e = X + h N/|N|, h = 2 x (local cell diagonal), u^e the trilinear
 * interpolation of its component at x^e, U the barycentric wall velocity;
 * all values are computed from the input fields before any is written.
 * u, v, w: dev, updated in place. */
int ibm_force(ibm_ctx* ctx, double* u, double* v, double* w);

/* Predictor on the fluid nodes (paper Eq. NS_prov): explicit right-hand side
 * R = dt [gamma H(u) + rho H_prev - alpha (G p + dpdx e_x) + (alpha/Re) L u]
 * and the approximate factorisation (I - bL_x)(I - bL_z)(I - bL_y) du = R,
 * b = alpha dt/(2 Re), with identity rows on the forcing nodes; then
 * u <- u + du.  gamma, rho: the sub-stage coefficients; h_prev (read when
 * rho != 0) and h_out (written when not NULL): dev f32/f64 arrays of H per
 * component, all three given (IBM_EINVAL if h_out names only some).  p: dev
 * f32/f64.  u, v, w: dev f64, in
 * place (the mixed form computes R and H in FP64 arithmetic, stores them in
 * FP32, solves the three factors in FP32 and adds du to the FP64 u). */
/* Volume force on component comp (0 = u, 1 = v, 2 = w) of the predictor,
 * F = f0 + kappa u_comp (the forces that paper Sec. 4.2 and 4.3 add to
 * Eq. NS_prov; a constant driving gradient is ibm_opts.dpdx), evaluated from
 * u^s and weighted by alpha like the driving gradient, on every unknown node
 * of the component that is not a forcing node.  f0, kappa: dev f64 arrays on
 * the component's lattice (v: nx*(ny+1)*nz values, walls included and
 * ignored), owned by the caller and read by every later ibm_viscous and
 * ibm_step until replaced; NULL = 0 (both NULL clears the force).
 * IBM_EINVAL for a bad component. */
int ibm_set_volume_force(ibm_ctx* ctx, int32_t comp, const double* f0, const double* kappa);

int ibm_viscous(ibm_ctx* ctx, const void* p, const void* const* h_prev,
                void* const* h_out, double gamma, double rho, double dt,
                double* u, double* v, double* w);

/* Consistent mass correction (paper Eqs. mod_div, q_boundary, q_F,
 * elliptic_mod): q_F = -(sum_{C_B} D u dV)/|C_F| from the last ibm_tag, and
 * rhs = (D u - q_F)/alpha_dt on C_F, 0 on C_B (IBM_Q_NONE: rhs =
 * D u/alpha_dt).  IBM_Q_ENERGY: q_F = c0 + c1 (p - e) (App. B), p required
 * (dev f32/f64), the two coefficients from five fixed-order sums over all
 * cells.  rhs: dev f64 ny*nz*nx; qf: dev f64[1] (q_F) or f64[2] (c0, c1)
 * (may be NULL); p: NULL unless IBM_Q_ENERGY. */
int ibm_mass_rhs(ibm_ctx* ctx, const double* u, const double* v, const double* w,
                 const void* p, double alpha_dt, double* rhs, double* qf);

/* Direct solve of L_c phi = rhs (paper Eq. elliptic / elliptic_mod; L_c = D G
 * with homogeneous Neumann walls): real FFT in x, complex FFT in z,
 * tridiagonal solve in y per Fourier mode.  The singular (0,0) mode is fixed
 * by phi_0 = 0 and the result is shifted to zero volume-weighted mean.
 * rhs, phi: dev f64 ny*nz*nx (may alias).  The compatibility condition of
 * the Neumann problem (App. A: sum rhs dV = 0) is checked first with two
 * fixed-order device sums; |sum rhs dV| > 1e-12 sum |rhs| dV raises
 * IBM_FLAG_COMPAT (read by ibm_check; no synchronisation here).  Mixed form:
 * the transforms run
 * in FP32 and the result is refined, phi += S(rhs - L_c phi) with the
 * residual in FP64, until max|rhs - L_c phi| <= refine_tol or refine_max
 * refinements; the stopping test runs on the device (no synchronisation),
 * IBM_FLAG_REFINE is raised if the tolerance was not reached. */
int poisson_solve(ibm_ctx* ctx, const double* rhs, double* phi);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * poisson_solve for an FP64 context, with no context.  Every table and the
 * spectrum live in one static device array of IBM_STATIC_SCRATCH_BYTES per
 * device (held until the process ends); the call allocates nothing and only
 * enqueues kernels on `stream` (hipStream_t, NULL = default).  g: the grid as
 * for ibm_create (host y_faces, copied into kernel arguments); rhs, phi: dev
 * f64 ny*nz*nx (may alias).  IBM_EINVAL if the grid needs more than the
 * static array (spectrum ny*nz*(nx/2+1 rounded up to 8)*16 bytes plus small
 * tables: e.g. up to 128x96x128 fits) or is not a valid grid.  Calls that
 * overlap on one device share the array and race.  The compatibility check
 * of poisson_solve is not made (there is no context to report its flag). */
#define IBM_STATIC_SCRATCH_BYTES (64ll * 1024 * 1024)
int poisson_solve_static(const ibm_grid* g, const double* rhs, double* phi, void* stream);

/* No-slip (transpiration) error (paper Sec. 4.4): at every forcing node of
 * the last ibm_tag (or ibm_step) on this context, the flow velocity
 * extrapolated to the wall with the forcing interpolator of Eq. new_IB,
 * (u(x^f) - a u(x^e)) / (1 - a) with the node's wall point, probe x^e and
 * a = |N|/h as in the forcing (u(x^f) itself when |N| = 0), minus the wall
 * velocity U(X^f).  eps: host double[4]: the mean of the three components'
 * values, then for u, v, w the mean of |error| over that component's
 * forcing nodes (0 without any).  u, v, w: dev f64.  Uses the forcing
 * buffer of the context (not concurrent with a step on it).  Synchronises. */
int ibm_noslip_error(ibm_ctx* ctx, const double* u, const double* v, const double* w,
                     double* eps);

/* Post-projection divergence (paper Eq. mod_div, D u = q on the fluid
 * cells): out (host double[2]) = max over C_F of |D u - q_F| with the C_F of
 * the last ibm_tag (or ibm_step) and the uniform q_F of the last mass
 * correction on this context (every cell and q = 0 with IBM_Q_NONE), and
 * that q_F.  Not meaningful after the energy-conserving shape (q varies on
 * C_F).  u, v, w: dev f64.  Synchronises. */
int ibm_divergence(ibm_ctx* ctx, const double* u, const double* v, const double* w,
                   double* out);

/* Pressure on the boundary cells (paper Sec. 2, after Eq. q_F: the solve does
 * not define p on C_B; it is rebuilt from the surrounding field with the
 * strategy of the forcing, as post-processing that never enters the step).
 * Reading: for each cell of the C_B list of the last ibm_tag (or ibm_step),
 * the wall point X is the closest point of the cell centre on the forcing
 * triangles of its six faces (least |N|^2, ties to the lowest triangle id),
 * the probe x^e = X + h N/|N| with h twice the cell diagonal, and the cell
 * takes p(x^e) (zero normal gradient at the wall), trilinear on the
 * cell-centre lattice, constant beyond the first and last centres; a centre
 * on the surface takes the mean of the probes on both sides.  p: dev f32
 * (mixed form) or f64, ny*nz*nx.  out: dev f64[out_cap]; out[f] for the
 * f-th boundary cell in ascending order (ibm_tags_count_host gives the
 * count); a count above out_cap fills out_cap values and raises
 * IBM_FLAG_CAPACITY.  Enqueued on the context's stream. */
int ibm_pressure_cb(ibm_ctx* ctx, const void* p, double* out, int64_t out_cap);

/* Hydrodynamic loads (paper Sec. 3.3) on the bodies of the last ibm_tag
 * (the same triangulation; the vertices as they were then).  Markers are the
 * triangle centroids X (normal n from the triangle's winding, area A); for
 * each, a probe point X + s h n (h twice the diagonal of the grid cell that
 * holds X; side s = +1, and also -1 where sides[b] == 2: zero-thickness
 * bodies) carries second-order moving-least-squares fits of p, u, v, w (the
 * 4x4x4 nodes of each lattice around it that lie in front of the marker's
 * tangent plane, fluid cells only for p, Gaussian weights), Taylor-expanded
 * back to X; the traction t = -p n_s + (G + G^T) n_s / Re is summed over the
 * sides.  u, v, w: dev f64 state arrays; p: dev, f64 (IBM_FP64) or f32
 * (IBM_MIXED); sides: dev i32[nb] (2: two-sided, else one side); pole: dev
 * f64[3 nb], the torque pole of each body; traction: dev f64[3 ntri] (per
 * marker, bodies in tagging order); loads: dev f64[6 nb], (F, M) per body,
 * F = sum t A, M = sum (X - pole) x t A, summed in a fixed order.  All
 * buffers are the caller's.  IBM_EINVAL for a null argument or no tagged
 * body.  Enqueued on the context's stream, no synchronisation. */
int ibm_loads(ibm_ctx* ctx, const double* u, const double* v, const double* w, const void* p,
              const int32_t* sides, const double* pole, double* traction, double* loads);

/* Projection and pressure update (paper Eqs. projection, update_pressure):
 * u <- u - alpha_dt G phi on every interior velocity node;
 * p <- p + phi - alpha_dt/(2 Re) L_c phi.  phi, u, v, w: dev f64; p: dev
 * f32/f64; in place. */
int ibm_project(ibm_ctx* ctx, const double* phi, double alpha_dt, double* u,
                double* v, double* w, void* p);

/* One whole time step of the scheme (paper Sec. 2 and Sec. 3): tags the
 * bodies at t^n once, then for every sub-stage: IB forcing, predictor,
 * consistent mass correction, Poisson solve, projection and pressure update.
 * The bodies stay at t^n for all sub-stages.  The tagging also raises
 * IBM_FLAG_CFL when a vertex velocity carries the vertex more than half the
 * local spacing in dt.  A dt not seen before has its line-solve tables
 * computed on the host and copied in stream order from pinned staging (no
 * synchronisation; the host waits only if the stream is four such changes
 * behind). */
int ibm_step(ibm_ctx* ctx, ibm_state* s, const ibm_body* bodies, int32_t nbody,
             double dt);

/* ------------------------------------------------------------------ batch
 * Many independent simulations, each with its own grid, options, state and
 * one body, advanced together (the paper's method applied per simulation;
 * the batching is an execution arrangement for grids too small to fill the
 * GPU one at a time).  Each simulation runs on a context of its own with its
 * own stream, forked from and joined back into the batch's stream. */
typedef struct ibm_batch ibm_batch;

#define IBM_MOTION_RIGID 0  /* X = c + R X0, U = cdot + omega x (X - c) */
#define IBM_MOTION_DEFORM 1 /* X = c + (r0 + f s) d, U = (f sdot) d      */
#define IBM_COEF_STRIDE 18  /* doubles per simulation in the coefficient array */

#define IBM_BATCH_SERIAL 0  /* one simulation after the other */
#define IBM_BATCH_STREAMS 1 /* concurrent streams, launched every step */
#define IBM_BATCH_GRAPH 2   /* one captured HIP graph replayed every step */
#define IBM_BATCH_PLAN 3    /* the mode of the batch's current plan */
#define IBM_BATCH_GROUPED 4 /* each kernel of the step launched once for all
                               simulations, captured into one graph */

/* One simulation of a batch.  state: dev arrays as for ibm_step (the
 * batch keeps the pointers); ref: dev f64[nv*3] reference vertices (rigid)
 * or f64[nv*4] [direction, amplitude] (deform), as for ibm_body_rigid /
 * ibm_body_deform; xyz, vel: dev f64[nv*3] written by every step; tri: dev
 * i32[nt*3]. */
typedef struct {
  ibm_state state;
  int32_t motion;
  int32_t nv, nt;
  const double* ref;
  double* xyz;
  double* vel;
  const int32_t* tri;
} ibm_sim;

/* grids, opts, sims: host arrays of nsim entries (copied).  stream: the
 * batch's hipStream_t (NULL = default).  Creates nsim contexts; all device
 * workspace is allocated here, including the launch tables of the grouped
 * form (sized by recording every simulation's step once; synchronises). */
int ibm_batch_create(const ibm_grid* grids, const ibm_opts* opts, const ibm_sim* sims,
                     int32_t nsim, void* stream, ibm_batch** out);
void ibm_batch_destroy(ibm_batch* b);
/* The context of simulation `sim` (owned by the batch), or NULL. */
ibm_ctx* ibm_batch_context(ibm_batch* b, int32_t sim);
/* One time step of every simulation: body transform at t^n from
 * coef (host f64[nsim*IBM_COEF_STRIDE]; simulation s at s*IBM_COEF_STRIDE,
 * rigid: the 18 values of ibm_body_rigid, deform: the first 9 values of
 * ibm_body_deform), then ibm_step.  mode: IBM_BATCH_SERIAL, _STREAMS,
 * _GRAPH, _GROUPED or _PLAN (the current plan's mode; streams and graph
 * modes use the plan's stream groups and tile choice); the first graph call
 * for a dt captures the graph (a change of dt or of plan drops it).
 * _GROUPED: every simulation's step is recorded (no launch) and the k-th
 * launch of all simulations becomes one launch per kernel variant and block
 * size, whose blocks each run as one simulation's block with that
 * simulation's argument record; the sequence is captured into one graph (a
 * few hundred launches per batched step instead of a few dozen per
 * simulation).  IBM_EINVAL if a simulation's step uses a kernel without a
 * grouped form (the energy-conserving q_F, the refined Poisson solve, volume
 * forces).  Results are identical in every mode and to ibm_step run on
 * each simulation alone.  The first call for a dt synchronises once (line
 * tables, waiting for any earlier step before a captured graph is dropped);
 * later calls only enqueue, except that the host waits when the coefficient
 * staging ring (4 slots) is full. */
int ibm_batch_step(ibm_batch* b, const double* coef, double dt, int32_t mode);
/* Synchronise and return (and clear) the OR of every simulation's flags. */
int ibm_batch_check(ibm_batch* b, uint32_t* flags);

/* Execution plan of a batch (an arrangement of the same arithmetic: every
 * plan gives results identical to IBM_BATCH_SERIAL).
 *   mode:       IBM_BATCH_STREAMS, _GRAPH or _GROUPED, used by IBM_BATCH_PLAN
 *   streams:    stream groups, 1..nsim: the simulations, largest first, are
 *               dealt round-robin to the groups; a group runs its
 *               simulations one after the other, groups run concurrently
 *   rhs_planes: wall-normal planes per block of the predictor right-hand
 *               side, 1..64 (fewer planes, more blocks on small grids)
 *   ms_per_step: filled by ibm_batch_tune (the measured time), else ignored
 * A new batch starts with {IBM_BATCH_GRAPH, nsim, 16}. */
typedef struct {
  int32_t mode;
  int32_t streams;
  int32_t rhs_planes;
  int32_t reserved;
  double ms_per_step;
} ibm_batch_plan;
/* Apply a plan (drops a captured graph).  IBM_EINVAL for values out of
 * range. */
int ibm_batch_set_plan(ibm_batch* b, const ibm_batch_plan* plan);
int ibm_batch_get_plan(ibm_batch* b, ibm_batch_plan* plan);
/* Autotuner: SWITCHED OFF, returns IBM_EINVAL (three runs of it ended in a
 * GPU fault or an abort whose cause is not found; set plans with
 * ibm_batch_set_plan).  When enabled it times candidate plans on this
 * batch's own simulations (a
 * coordinate search over streams in {1, 2, 4, ..., nsim}, then rhs_planes in
 * {16, 48, 8, 4}, then graph vs eager streams; the grouped form is not among
 * its candidates), `steps` timed steps each after
 * one untimed step, all with the body coefficients `coef` and step dt.  The
 * simulations' states (u, v, w, p and, for AB2, h) are saved first into
 * `scratch` (dev, 256-byte aligned, at least ibm_batch_tune_scratch_bytes
 * bytes, owned by the caller; IBM_EINVAL otherwise) and restored after every
 * trial, so tuning leaves them as they were; the library allocates nothing.
 * Every stream of the batch is idle whenever a plan is applied.  Applies the
 * fastest plan and returns it in *best; if table is not NULL, up to
 * max_entries tried plans (with their times) are written there and *n_tried
 * gets their count.  Synchronises. */
int64_t ibm_batch_tune_scratch_bytes(ibm_batch* b);
int ibm_batch_tune(ibm_batch* b, const double* coef, double dt, int32_t steps, void* scratch,
                   int64_t scratch_bytes, ibm_batch_plan* best, ibm_batch_plan* table,
                   int32_t max_entries, int32_t* n_tried);

/* Mixed form: synchronise and copy the refinement statistics since the
 * last reset to stats (host double[IBM_REFINE_STATS]): Poisson solves,
 * FP64-residual corrections applied, the largest final
 * max|rhs - L_c phi| * alpha_dt, the largest such residual left by the first
 * correction, the largest such residual of the initial (uncorrected) solve,
 * and the sum over solves of that initial residual.  reset = 1 clears them. */
#define IBM_REFINE_STATS 6
int ibm_refine_stats(ibm_ctx* ctx, double* stats, int32_t reset);

/* Synchronise the stream and return (and clear) the sticky device flags. */
int ibm_check(ibm_ctx* ctx, uint32_t* flags);
const char* ibm_strerror(int code);

/* Per-kernel timing with HIP events on the context's stream.  enable = 1
 * records an event pair around every launch of a kernel whose name contains
 * `filter` (NULL or "" = all kernels); ibm_profile_read synchronises and
 * writes up to `cap` (name, launches, total ms) records, returns the number
 * written, and resets the accumulators. */
int ibm_profile(ibm_ctx* ctx, int32_t enable, const char* filter);
int ibm_profile_read(ibm_ctx* ctx, char* names, int32_t name_len, int64_t* launches,
                     double* total_ms, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* IBM_H */
