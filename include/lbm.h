/*
 * lbm.h -- C ABI of the MI355X lattice Boltzmann library (liblbm.so).
 *
 * The library advances a periodic lattice Boltzmann fluid on one gfx950 GPU
 * with no-slip solids treated either by interpolated bounce-back (IBB) on
 * fluid-solid links with momentum-exchange force and torque, or by the
 * direct-forcing immersed boundary method (IBM).  The method is the one
 * compared in Peng, Ayala & Wang, arXiv 1906.05445:
 *   - evolution: lattice BGK (Eq. 1, viscosity Eq. 2) or MRT (Eq. 3) with a
 *     second-order mesoscopic body-force term (Sec. 2.1);
 *   - IBB: halfway bounce-back (Eq. 10), quadratic Bouzidi (Eq. 11), linear
 *     Bouzidi (named in Sec. 3.3), with the link fraction q of Sec. 2.2;
 *     force and torque by the Galilean-invariant momentum exchange (Eq. 17);
 *   - IBM: Uhlmann's direct forcing (Eq. 5-9) with Peskin's 4-point delta
 *     (Eq. 6), iterated n_iter times (Sec. 3.1), force and torque from the
 *     Lagrangian forces (Sec. 3.1, App. B).
 *
 * Conventions (lattice units: dx = dt = 1, reference density rho0 = 1):
 *   - cell index n = x + nx*(y + ny*z); D2Q9 lattices have nz == 1;
 *   - velocity sets: rest first, then +/- pairs, axis pairs before diagonal
 *     pairs; D2Q9: (1,0) (-1,0) (0,1) (0,-1) (1,1) (-1,-1) (1,-1) (-1,1);
 *     D3Q19: the 6 axis directions (+x -x +y -y +z -z) then (1,1,0)
 *     (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
 *     (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1);
 *   - population arrays crossing the ABI are [Q][N] (direction-major);
 *     velocity arrays are [3][N];
 *   - MRT moment order (the rows of M): D2Q9: 1, |e|^2, |e|^4, ex,
 *     ex|e|^2, ey, ey|e|^2, ex^2-ey^2, ex ey; D3Q19: 1, |e|^2, |e|^4, ex,
 *     ex|e|^2, ey, ey|e|^2, ez, ez|e|^2, 3ex^2-|e|^2, (3ex^2-|e|^2)|e|^2,
 *     ey^2-ez^2, (ey^2-ez^2)|e|^2, ex ey, ey ez, ex ez, (ey^2-ez^2)ex,
 *     (ez^2-ex^2)ey, (ex^2-ey^2)ez (orthogonalised in that order);
 *   - forces are the hydrodynamic force ON the solid; torques are about the
 *     solid centre.
 *
 * Ownership: every pointer argument is borrowed for the duration of the call.
 * Device memory is caller-owned: the context lives inside a device workspace
 * the caller allocates (size from lbm_workspace_bytes); the library never
 * allocates device memory.  All GPU work is ordered on the caller's HIP
 * stream; the readout calls (lbm_force_torque, lbm_force_history,
 * lbm_macros, lbm_get_f, lbm_get_state, lbm_link_list) synchronise that
 * stream.  One context must not be used by two host threads at once.
 *
 * Errors: no exception crosses the ABI.  Every call returns lbm_status;
 * lbm_status_string names it and lbm_last_error(ctx) gives detail.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_EINVAL (-1)       /* invalid argument (tau <= 1/2, bad sizes, overlapping solids, ...) */
#define LBM_ENOMEM (-2)       /* workspace too small, or a link / point capacity exceeded */
#define LBM_EDEVICE (-3)      /* HIP runtime error; text in lbm_last_error */
#define LBM_EDIVERGED (-4)    /* non-finite value found by the watchdog */
#define LBM_EUNSUPPORTED (-5) /* combination not implemented */
#define LBM_ESTATE (-6)       /* call out of order */
#define LBM_EAGAIN (-7)       /* batch admission deferred: not enough free pool memory */

typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 } lbm_lattice;
typedef enum { LBM_BGK = 0, LBM_MRT = 1 } lbm_collision;
/* Storage of the populations.  All formats hold the deviation f_i - w_i from
 * the rest state; F64 computes in FP64, F32_DEV and the FP16 formats decode
 * to FP32 and compute in FP32 (force and torque are always accumulated in
 * FP64).  F16_DEV rounds to nearest on store; F16_SR (IEEE half too) rounds
 * stochastically: up with the probability of the fraction dropped, so that
 * changes smaller than half a unit in the last place survive on average (a
 * slowly developing flow stored to nearest lags behind); the dither is a
 * hash of slot and time step, so runs repeat bit for bit. */
typedef enum { LBM_F64 = 0, LBM_F32_DEV = 1, LBM_F16_DEV = 2, LBM_F16_SR = 3 } lbm_storage;
/* No-slip treatment (Sec. 2.1, 2.2): halfway bounce-back (Eq. 10), linear
 * Bouzidi (two-point form of Eq. 11), quadratic Bouzidi (Eq. 11), direct-
 * forcing IBM (Eq. 5-9), Yu's unified scheme (Eq. 12-14; the merged Eq. 15
 * with its x_ff weight read as 2(1-q)/(2+q), as Eq. 12-14 give), Zhao &
 * Yong's single-node scheme (Eq. 16).  Quadratic and Yu fall back to linear
 * where x_ff or x_fff is not fluid, linear (q < 1/2) to Eq. 10 where x_ff is
 * not; Zhao-Yong reads x_f only. */
typedef enum {
  LBM_BB = 0,
  LBM_IBB_LINEAR = 1,
  LBM_IBB_QUADRATIC = 2,
  LBM_IBM = 3,
  LBM_IBB_YU = 4,
  LBM_IBB_ZHAO_YONG = 5
} lbm_boundary;
typedef enum { LBM_SPHERE = 0, LBM_CYLINDER = 1, LBM_PLANE = 2 } lbm_solid_kind;
/* Domain boundary of one axis (Sec. 3.4: the sphere in an open domain has a
 * uniform inflow, stress-free sides and a convective outflow).
 *   PERIODIC : the default.
 *   SLIP     : stress-free planes halfway outside the first and last node
 *              layers: a population that would cross one has its normal
 *              component reversed and stays in its layer (zero normal
 *              velocity, zero normal derivative of the tangential ones).
 *   OPEN     : x only.  Velocity inlet halfway before x = 0: a population
 *              that would leave there returns reversed with the wall term of
 *              Eq. 10 for u_w = (inflow, 0, 0) and rho0 = 1.  Convective
 *              outflow at the last layer x = nx - 1: a population entering it
 *              from outside is f_i(t+1) = [f_i(t) + U_o f_i(nx-2, t+1)] /
 *              (1 + U_o), U_o = max(u_x of that node's last collision, 0)
 *              (the condition d f/dt + U_o d f/dx = 0, implicit in time,
 *              upwind in x). */
typedef enum { LBM_PERIODIC = 0, LBM_SLIP = 1, LBM_OPEN = 2 } lbm_domain;

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

/* Lattice, grid and relaxation (Eq. 1-3).
 *   tau   : BGK relaxation time, nu = (tau - 1/2)/3 (Eq. 2); must be > 1/2.
 *   rates : MRT only; NULL selects the default diagonal S: every even
 *           non-conserved moment relaxes with 1/tau, the odd non-conserved
 *           moments with s_odd from (tau - 1/2)(1/s_odd - 1/2) = 3/16; or Q
 *           caller rates in the moment order above (rates of the conserved
 *           moments have no effect).
 *   body_force        : force density g added on the fluid region.
 *   body_force_fluid_only : 1 = g acts only on nodes outside every solid's
 *           volume (the setting Sec. 3.3 finds more accurate for IBM);
 *           0 = everywhere (IBB solid nodes never carry fluid).
 *   boundary : lbm_domain per axis (zero: periodic).  OPEN is allowed on x
 *           only and needs nx >= 8; D2Q9 keeps z periodic.  A lattice with a
 *           bounded axis takes fixed solids only, each at least 4 nodes clear
 *           of every bounded face (lbm_set_solids), and is not admitted to a
 *           batch.
 *   inflow : inflow velocity U_in of an OPEN x axis (|U_in| < 0.3).
 *   cover_momentum : 1 = moving bounce-back solids exchange momentum with
 *           the nodes they cover and uncover (Sec. 3.2 needs the refill but
 *           gives no such term; this reading is an option): a node covered
 *           in a step gives the solid its momentum sum_i f_i e_i, a node
 *           uncovered (refilled with f_eq(rho_bar, u_w)) takes rho_bar u_w
 *           from it, with the torques about the solid's centre; the sums
 *           (fixed point, order-free) join the force and torque of the next
 *           step, which free solids move with.  0 = off (default). */
typedef struct {
  int32_t lattice;    /* lbm_lattice */
  int32_t collision;  /* lbm_collision */
  int32_t storage;    /* lbm_storage */
  int32_t nx, ny, nz; /* nz == 1 for D2Q9; fewer than 2^31 cells */
  double tau;
  const double *rates;
  double body_force[3];
  int32_t body_force_fluid_only;
  int32_t boundary[3]; /* lbm_domain per axis */
  double inflow;
  int32_t cover_momentum;
} lbm_params;

/* A rigid solid.  Sphere: centre, radius (in 2D a circle).  Cylinder: axis
 * along a coordinate direction (unit vector), infinite and periodic along
 * it.  Plane (a half-space, for tests): `axis` is the unit normal pointing
 * into the fluid, `centre` a point of the plane.  inverted = 1 makes the
 * solid the OUTSIDE of the sphere/cylinder (an outer Couette wall, a pipe).
 * Wall velocity u_w(x) = velocity + omega x (x - centre).  A solid with
 * nonzero velocity translates (centre(t) = centre + t*velocity).
 * density > 0 makes the solid move freely (Sec. 3.2, fluid density rho0 = 1,
 * no interaction force): density is rho_p / rho_f, gravity the external
 * acceleration; velocity and omega are the initial values (and those of the
 * step before the first).  After every step t, with the force F and torque T
 * of that step on the solid:
 *   IBB (Eq. 20, F and T by Eq. 17): rho_p V_p (v' - v) = F + (rho_p - 1)
 *   V_p gravity, I_p (w' - w) = T;
 *   IBM (Eq. 23, Feng & Michaelides, F = -sum F_l dV_l, T = -sum (X_l - Y)
 *   x F_l dV_l): rho_p V_p (v' - v) = V_p (v - v_prev) + F + (rho_p - 1) V_p
 *   gravity, I_p (w' - w) = (I_p / rho_p) (w - w_prev) + T;
 * centre' = centre + (v + v')/2 (dt = 1); sphere V_p = 4 pi R^3/3,
 * I_p = 2 rho_p V_p R^2/5; cylinder (D2Q9 only, per unit depth) V_p = pi R^2,
 * I_p = rho_p V_p R^2/2, rotation about z.  The Eq. 23 update is explicit:
 * at small radii and density ratios near one it can oscillate with growing
 * amplitude (a sphere of radius 4 at rho_p = 1.5 does; radius 7, or rho_p = 3,
 * does not).  Free solids need a sphere or (2D) cylinder that is not inverted
 * and a context outside any batch (else LBM_EUNSUPPORTED); a step that would
 * carry one faster than half a cell per step ends with LBM_EDIVERGED.  A
 * moving (translating or free) IBM solid must moreover be the only solid,
 * with no fluid-only body force (body_force zero or body_force_fluid_only 0)
 * and at least one forcing iteration (else LBM_EINVAL);
 * its Lagrangian points move rigidly with it (their orientation is kept),
 * and it uses twice the point capacity of a fixed one (at most
 * max_lagrangian / 2 points). */
typedef struct {
  int32_t kind;       /* lbm_solid_kind */
  int32_t inverted;
  double centre[3];   /* 0 <= centre < box size (per non-axial axis) */
  double radius;
  double axis[3];
  double velocity[3];
  double omega[3];
  double density;     /* rho_p / rho_f of a free solid; 0 = motion prescribed */
  double gravity[3];  /* acceleration on a free solid */
} lbm_solid;

/* IBM options: n_iter direct-forcing iterations per step (Sec. 3.1 uses 5),
 * delta the regularized delta function of Eq. 5 and Eq. 8 by its width in
 * lattice nodes: 4 = Peskin's four-point function (Eq. 6; also 0, the
 * default), 3 = the three-point function of Roma et al., 2 = the two-point
 * linear one (the three compared in Sec. 3.1), retraction R_d of the
 * Lagrangian points towards the solid (Breugem, Sec. 3.1; 0 = Uhlmann).
 * Other delta values give LBM_EINVAL. */
typedef struct {
  int32_t n_iter;
  int32_t delta;
  double retraction;
} lbm_ibm_opts;

/* Bytes of device workspace for one context.  max_links bounds the number of
 * IBB boundary links (Sec. 2.2: one per fluid node and direction whose
 * neighbour across the wall is a solid node), max_lagrangian the number of
 * IBM points (Sec. 2.1, Eq. 5-9); 0 selects a bound computed from the
 * lattice size (N / 2 links, max(1024, N / 64) points).  The IBM shell
 * (the cells within the points' delta supports) may hold min(N, 16 x the
 * point capacity) cells: a mesh of about one point per unit area needs 4 to
 * 8 per point, and a sparser one may give LBM_ENOMEM from lbm_set_solids.
 * A negative
 * max_lagrangian reserves no IBM space at all (no points, shell or spread
 * force field: 3 N force values fewer), for contexts that never take IBM
 * solids; lbm_set_solids with LBM_IBM and lbm_set_lagrangian then give
 * LBM_ENOMEM.  Returns 0 for invalid parameters. */
size_t lbm_workspace_bytes(const lbm_params *p, int32_t max_solids, int64_t max_links,
                           int64_t max_lagrangian);

/* Create a context for the lattice Boltzmann equation of Sec. 2 (BGK, Eq. 1
 * with the viscosity of Eq. 2, or MRT, Eq. 3, with the forcing of Sec. 2.1)
 * inside dev_workspace (device memory, >= ws_bytes, caller owned, 256-byte
 * aligned, kept until lbm_destroy) for work on hip_stream (a hipStream_t,
 * caller owned; NULL for the default stream).  The populations start at
 * rest (f = w).  Errors: LBM_EINVAL (tau <= 1/2, dimensions, rates),
 * LBM_ENOMEM (ws_bytes too small), LBM_EDEVICE. */
lbm_status lbm_create(const lbm_params *p, int32_t max_solids, int64_t max_links, int64_t max_lagrangian,
                      void *dev_workspace, size_t ws_bytes, void *hip_stream, lbm_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid it): lbm_create without a
 * workspace argument.  The workspace is a file-scope device array of
 * lbm_noalloc_capacity() bytes (64 MiB) that the library holds on every
 * device it runs on until the process ends; the call allocates nothing,
 * device or host.  Everything else is lbm_create's: the same parameters, the
 * same layout (lbm_workspace_bytes must not exceed the capacity: about
 * 240 bytes per cell with the default capacities, e.g. 64^3 in FP32), the
 * same calls on the context afterwards, lbm_destroy to release it.  One such
 * context at a time per device: the array keeps the last context's contents
 * and is cleared by the next lbm_create_noalloc; a second one while the
 * first lives gives LBM_ESTATE, and two host threads using the array of one
 * device at once would race.  Errors: LBM_EINVAL as lbm_create, LBM_ENOMEM
 * (the lattice does not fit the array), LBM_ESTATE, LBM_EDEVICE. */
lbm_status lbm_create_noalloc(const lbm_params *p, int32_t max_solids, int64_t max_links, int64_t max_lagrangian,
                              void *hip_stream, lbm_ctx **out);
size_t lbm_noalloc_capacity(void);

/* Set the solids and the no-slip method (replaces any previous set).
 * IBB (Sec. 2.2, Fig. 1): classifies nodes (inside iff squared distance
 * <= R^2, shortest periodic image), builds the boundary links and the wall
 * fraction q = |x_f - x_w| / |x_f - x_b| of each.  IBM (Sec. 2.1): generates
 * the Lagrangian mesh of each solid (geodesic sphere of about one point per
 * unit area; circles / rings of spacing about 1; Sec. 3.1 places the points
 * R_d inside the surface), unless points are given afterwards with
 * lbm_set_lagrangian.  opts may be NULL (5 iterations, no retraction).
 * On a lattice with a bounded axis (lbm_params.boundary) the solids are
 * fixed (velocity and rotation zero, no free motion: else LBM_EUNSUPPORTED)
 * and each keeps 4 nodes between its surface and every bounded face:
 * centre +- (radius + 4) within [0, n - 1] on that axis (else LBM_EINVAL).
 * Errors: LBM_EINVAL and LBM_EUNSUPPORTED leave the context as it was;
 * after LBM_ENOMEM (too many links or points) the context has no solids. */
lbm_status lbm_set_solids(lbm_ctx *c, const lbm_solid *s, int32_t n, int32_t method, const lbm_ibm_opts *opts);

/* IBM only: replace the Lagrangian points X_l of one solid (Eq. 5, 8) with
 * X [n][3] (FP64, lattice units), each with control volume dV (Delta V_l of
 * Eq. 8).  The points of a moving solid are given where the solid was placed
 * by lbm_set_solids, before any step (else LBM_EINVAL). */
lbm_status lbm_set_lagrangian(lbm_ctx *c, int32_t solid, const double *X, int64_t n, double dV);

/* Advance nsteps time steps t -> t+1 (no host synchronisation inside): IBM
 * forcing (Eq. 5-9, n_iter times, Sec. 3.1), then streaming and collision
 * (Eq. 1 or Eq. 3 with the body force of Sec. 2.1), then for IBB the unknown
 * populations of every boundary link (Eq. 10, 11, 12-14 or 16) and the
 * force and torque of Eq. 17.  Moving IBB solids are reclassified, their
 * uncovered nodes refilled and their links rebuilt (Sec. 3.2).  Errors:
 * LBM_ENOMEM (a moving solid outgrew a capacity), LBM_EDIVERGED (a free
 * solid reached half a cell per step), LBM_EDEVICE. */
lbm_status lbm_step(lbm_ctx *c, int64_t nsteps);

/* Centre, velocity and angular velocity of every solid now, state [n][9]
 * (a free solid's from its integration; others' from their prescribed
 * motion).  Synchronizes the stream. */
lbm_status lbm_solid_state(lbm_ctx *c, double *state);

/* Force and torque on every solid in the most recent step, [n][3] each:
 * IBB by the Galilean-invariant momentum exchange of Eq. 17 (lever arm from
 * the solid centre to the wall point x_w = x_f - q e_i of each link); IBM
 * -sum F_l dV_l and -sum (X_l - Y) x F_l dV_l (Sec. 3.1, App. B).  FP64.
 * Synchronizes the stream. */
lbm_status lbm_force_torque(lbm_ctx *c, double *force, double *torque);

/* Per-step force and torque (as lbm_force_torque: Eq. 17, or the IBM sums of
 * Sec. 3.1), ft [count][nsolid][6] = (Fx Fy Fz Tx Ty Tz), for steps first ..
 * first+count-1 (step k is the update k -> k+1).  The library keeps the last
 * lbm_history_capacity() steps; older ones give LBM_EINVAL.  Synchronizes
 * the stream. */
lbm_status lbm_force_history(lbm_ctx *c, int64_t first, int64_t count, double *ft);
int64_t lbm_history_capacity(void);

/* Macroscopic fields of the most recent collision: rho [N] = sum_i f_i and
 * u [3][N] = (j + F/2)/rho with j = sum_i f_i e_i and F the total force
 * density of that collision (the second-order forcing of Sec. 2.1 uses this
 * velocity); IBB solid nodes report rho = 0 and the wall velocity of Eq. 10.
 * node_type [N] (may be NULL), in the geometry of that collision: 0 fluid,
 * 1 IBB solid node, 2 fluid inside an IBM solid.  Before the first step (or
 * after lbm_set_f / lbm_set_state): the fields of the current populations,
 * u = j/rho. */
lbm_status lbm_macros(lbm_ctx *c, double *rho, double *u, uint8_t *node_type);

/* Strain rate and dissipation of the most recent collision (Sec. 3.1,
 * Eq. 19), from the non-equilibrium moments of the populations it relaxed:
 * S [6][N] = s_xx, s_yy, s_zz, s_xy, s_yz, s_xz with s_ab = (d_a u_b +
 * d_b u_a)/2, eps [N] = 2 nu s_ab s_ab (nu of Eq. 2); either may be NULL,
 * not both.  Each second-order moment row k of M (lbm_params) is taken with
 * its own rate s_k: row k of s = -(3/2) s_k (m_k - m_k^eq) - (3/4) s_k
 * (row k of u F + F u), rho0 = 1 (for D2Q9 this is Eq. 19).  IBB solid nodes
 * give 0.  FP64 whatever the storage.  LBM_ESTATE before the first step
 * after lbm_create / lbm_set_f / lbm_set_state.  Synchronizes the stream. */
lbm_status lbm_strain(lbm_ctx *c, double *S, double *eps);

/* Populations f_i(x, t) of Eq. 1 / Eq. 3 before the next collision, [Q][N]
 * FP64 (solid nodes give 0); lbm_set_f replaces them (time and history are
 * kept).  Both synchronize the stream. */
lbm_status lbm_get_f(lbm_ctx *c, double *f);
lbm_status lbm_set_f(lbm_ctx *c, const double *f);

/* Set every population to the equilibrium f_eq(rho, u) of a uniform flow
 * (the second-order polynomial equilibrium of Eq. 1 and Eq. 3, c_s^2 = 1/3),
 * u [3] (u[2] ignored for D2Q9); the same start as from rest, with a mean
 * flow.  Time and history are kept.  Errors: LBM_EINVAL (rho <= 0,
 * non-finite values).  Synchronizes the stream. */
lbm_status lbm_set_equilibrium(lbm_ctx *c, double rho, const double *u);

/* Raw deviations f_i - w_i before the next collision, [Q][N] in the storage
 * format (double, float or IEEE half), bit for bit.  With an OPEN x axis the
 * populations entering at the inlet are given without the inlet term of
 * Eq. 10 (6 w_i e_ix U_in), which the next collision adds: the raw state is
 * what is stored, so that a restore is exact. */
lbm_status lbm_get_state(lbm_ctx *c, void *host);
lbm_status lbm_set_state(lbm_ctx *c, const void *host);

/* Boundary links of Sec. 2.2 in canonical order (by fluid cell x_f, then
 * direction i, the population f_i(x_f) that bounce-back supplies): cell,
 * dir, solid, q = |x_f - x_w| / |x_f - x_b| in (0, 1] (FP64, Fig. 1).  Pass
 * NULL arrays to get the count only; otherwise *count holds the capacity of
 * the arrays on entry (LBM_EINVAL if smaller than the link count) and the
 * count on return.  Synchronizes the stream. */
lbm_status lbm_link_list(lbm_ctx *c, int64_t *count, uint32_t *cell, uint8_t *dir, int32_t *solid, double *q);

/* Node classification [N]: 0 fluid, 1 IBB solid node, 2 inside an IBM solid. */
lbm_status lbm_node_types(lbm_ctx *c, uint8_t *node_type);

/* Completed time steps. */
int64_t lbm_time(const lbm_ctx *c);

/* Scan the current populations for NaN/Inf: LBM_OK or LBM_EDIVERGED. */
lbm_status lbm_check(lbm_ctx *c);

/* Release the host side of a context (not a step of the method); the
 * workspace stays the caller's.  Members of a batch are released with
 * lbm_batch_release instead (LBM_ESTATE here). */
lbm_status lbm_destroy(lbm_ctx *c);
/* Name of a status code, and the detail text of a context's last error. */
const char *lbm_status_string(lbm_status st);
const char *lbm_last_error(const lbm_ctx *c);

/* Profiling: with every = k >= 1, lbm_step records HIP events on the
 * context's stream around its stream-collide launches: when only fixed IBB
 * solids are present, the launches of steps 2 .. n of a call run back to back
 * and one pair of events spans all of them; otherwise a pair surrounds every
 * k-th launch (k = 1: all of them; a larger k keeps the event overhead out of
 * a timed run).  every = 0 stops recording (every < 0: LBM_EINVAL).
 * lbm_profile_read synchronises the stream, returns the summed duration (ms)
 * and the number of launches timed since the last read, and clears them. */
lbm_status lbm_profile(lbm_ctx *c, int32_t every);
lbm_status lbm_profile_read(lbm_ctx *c, double *sweep_ms, int64_t *launches);

/* Result of the sweep autotuner, which runs on the first lbm_step of a
 * context (or reuses a choice made for an identical lattice in this process):
 * nontemporal = 1 if the sweep writes with non-temporal stores (-1 before
 * tuning), and the measured sweep times of both store kinds (us). */
lbm_status lbm_autotune_info(lbm_ctx *c, int32_t *nontemporal, double *us_plain, double *us_nontemporal);

/* Sweep policy, kept per lattice signature: bit 0 of *policy = non-temporal
 * stores (always set: the tuner does not change the store kind), bit 1 =
 * workgroups take tiles in an order that gives each of the 8 XCDs (which
 * receive workgroups in turn) one contiguous range, so neighbouring tiles
 * share an L2; the tuner picks the tile order.  *policy = -1 before tuning;
 * us[4] (may be NULL) receives, per policy, the time per step measured over
 * back-to-back tuning steps in microseconds (the sweeps and any other kernels
 * of those steps; 0 for the policies not tried).  lbm_autotune_info above
 * reports the store half for the chosen tile order. */
lbm_status lbm_autotune_policy(lbm_ctx *c, int32_t *policy, double *us);

/* Copy `bytes` from src to dst (device pointers) with the library's
 * streaming copy kernel, the bandwidth yardstick for the sweep. */
lbm_status lbm_copy_probe(const void *src, void *dst, size_t bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batches: many independent lattices (uneven sizes, own solids, own
 * relaxation rates and body force) advanced together.  Not in the paper,
 * which treats one lattice at a time; every member follows exactly the
 * single-context definition of a step above, so a member's results are bit
 * for bit those of the same context stepped alone.
 *
 * A batch owns a device pool (caller-owned memory, 256-byte aligned, kept
 * until lbm_batch_destroy).  The first lbm_batch_table_bytes(max_slots)
 * bytes hold the batch's tables; members are contexts whose workspaces are
 * carved from the rest.  All members share one lattice and one storage
 * format, and all batch work runs on one stream (lbm_batch_stream): the
 * caller's, or one the batch creates when the caller passes none.  Each step is one launch per stage over the units of
 * all members, replayed from a captured HIP graph; the first steps of a new
 * total size tune the sweep's launch shape and store policy.
 * A batch and its members must not be used by two host threads at once.
 * ------------------------------------------------------------------------ */

/* Bytes at the head of the pool taken by the tables of max_slots members. */
size_t lbm_batch_table_bytes(int32_t max_slots);

/* Create a batch of up to max_slots members in dev_pool.  lattice is an
 * lbm_lattice and storage an lbm_storage shared by every member (each member
 * a lattice of Sec. 2 with its own solids, stepped as lbm_step defines).
 * hip_stream (a hipStream_t, caller owned, kept until lbm_batch_destroy) is
 * the stream of every batch and member call; it must not be the legacy null
 * stream, because the batched steps are captured as HIP graphs on it.  NULL:
 * the batch creates a non-blocking stream of its own (default priority) and
 * destroys it with the batch.  Errors: LBM_EINVAL, LBM_ENOMEM (pool smaller
 * than the tables), LBM_EDEVICE. */
lbm_status lbm_batch_create(int32_t lattice, int32_t storage, int32_t max_slots, void *dev_pool, size_t pool_bytes,
                            void *hip_stream, lbm_batch **out);

/* Admit a member (a lattice of Sec. 2, as lbm_create defines it): a context
 * with the same parameters as lbm_create whose
 * workspace of lbm_workspace_bytes(p, ...) bytes is taken from the pool.
 * It is configured and read with the ordinary context calls (lbm_set_solids,
 * lbm_force_torque, lbm_macros, ...) and may even be stepped alone with
 * lbm_step; lbm_destroy refuses it.  LBM_EAGAIN: no free slot, or no
 * contiguous free range of that size (retry after a release). */
lbm_status lbm_batch_admit(lbm_batch *b, const lbm_params *p, int32_t max_solids, int64_t max_links,
                           int64_t max_lagrangian, lbm_ctx **out);

/* Release a member: its context is destroyed and its pool range returned
 * (its results, the Eq. 17 or Sec. 3.1 force history and the fields, are
 * read before, with the context calls). */
lbm_status lbm_batch_release(lbm_batch *b, lbm_ctx *c);

/* Advance every member by nsteps steps, each step exactly the one lbm_step
 * takes (Sec. 2: forcing, Eq. 5-9; stream and collide, Eq. 1 / Eq. 3;
 * bounce-back, Eq. 10-16, and Eq. 17; Sec. 3.2 rebuild of moving solids),
 * one launch per stage over all members.  Returns after enqueueing, except
 * when a member has translating solids: then the stream is synchronised and
 * the members' link capacities are checked (LBM_ENOMEM when exceeded, with
 * the member's lbm_last_error naming the capacity). */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Wait for the batch's stream. */
lbm_status lbm_batch_sync(lbm_batch *b);

/* Members, free pool bytes, largest contiguous free range, total cells. */
lbm_status lbm_batch_info(lbm_batch *b, int32_t *members, size_t *bytes_free, size_t *largest_free,
                          int64_t *total_cells);

/* Sweep launch shape chosen by the tuner: non-temporal stores (0/1), unit
 * order (0 contiguous share per block, 1 round-robin), persistent blocks, or
 * 0 with tiles_per_block tiles per block (0 for persistent grids), and its
 * measured time per step (us, all members).  LBM_ESTATE before the tuner has
 * finished. */
lbm_status lbm_batch_tune_info(lbm_batch *b, int32_t *nontemporal, int32_t *order, int32_t *blocks,
                               int32_t *tiles_per_block, double *sweep_us);

/* The tuner's candidates: fills up to cap entries (fields as in
 * lbm_batch_tune_info, mean measured sweep time per step in us or -1 before
 * tuning) and returns the number of candidates. */
int32_t lbm_batch_tune_table(lbm_batch *b, int32_t cap, int32_t *nontemporal, int32_t *order, int32_t *blocks,
                             int32_t *tiles_per_block, double *sweep_us);

/* Advance nsteps steps launched one by one (not from the graph) with events
 * on the sweep dispatches; returns the mean sweep time per step (us).  For
 * measurement; needs a tuned batch whose members have not changed since its
 * last lbm_batch_step (LBM_ESTATE otherwise). */
lbm_status lbm_batch_time_sweep(lbm_batch *b, int64_t nsteps, double *sweep_us);

/* Convergence check of every member (serving): for slot k, members[k] is
 * the member context (NULL for a free slot) and change[k] the largest
 * relative change of a solid's force over the last `lag` steps,
 * |F(t-1) - F(t-1-lag)| / |F(t-1)| (Euclidean norms, F the force of step
 * t-1), NaN when one of those forces is not finite (the member diverged:
 * its populations went non-finite; the other members are not affected), or
 * -1 when the member has no solid or fewer than lag + 1 steps.
 * Both arrays hold max_slots entries.  One launch and one small read-back;
 * synchronises the batch's stream. */
lbm_status lbm_batch_force_change(lbm_batch *b, int64_t lag, lbm_ctx **members, double *change);

/* Members whose drag has converged (serving): after lbm_batch_force_change
 * with the same lag, the members whose change is >= 0 and < tol, in slot
 * order; up to cap of them go to converged, *n gets how many there are.
 * The change is the relative change of the Eq. 17 (IBB) or Sec. 3.1 (IBM)
 * force over lag steps.  Synchronises the batch's stream.  Errors:
 * LBM_EINVAL (tol <= 0, lag <= 0 or beyond the history). */
lbm_status lbm_batch_poll(lbm_batch *b, int64_t lag, double tol, lbm_ctx **converged, int32_t cap, int32_t *n);

/* The batch's HIP stream (a hipStream_t). */
void *lbm_batch_stream(lbm_batch *b);

const char *lbm_batch_last_error(const lbm_batch *b);

/* Destroy the batch and every member left in it (the pool is not freed). */
lbm_status lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
