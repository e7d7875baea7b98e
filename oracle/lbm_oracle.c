/*
 * lbm_oracle.c -- plain, slow, FP64 CPU oracle for the lattice Boltzmann hot
 * path compared in Peng, Ayala & Wang, "A comparative study of immersed
 * boundary method and interpolated bounce-back scheme for no-slip boundary
 * treatment in the lattice Boltzmann method: Part I, laminar flows"
 * (arXiv 1906.05445).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against an
 * independent, obviously-correct implementation.  It shares no code, table or
 * header with the HIP library.
 *
 * What it computes, in the order of one time step t -> t+1 (push scheme):
 *   1. density and momentum of the current (post-streaming) populations;
 *   2. body force density g on the fluid region (Sec. 3.3 discussion of where
 *      the driving force is applied);
 *   3. IBM only: direct-forcing boundary force by Uhlmann's steps, Eq. 5-9,
 *      with Peskin's 4-point delta, Eq. 6 (or the 3-point delta of Roma et
 *      al. or the 2-point linear one, compared in Sec. 3.1), repeated n_iter
 *      times (Sec. 3.1);
 *   4. collision: lattice BGK, Eq. 1 + Eq. 2, or MRT, Eq. 3, with the
 *      second-order (Guo) mesoscopic forcing named in Sec. 2.1;
 *   5. streaming to the neighbour along e_i (periodic box);
 *   6. IBB only: the unknown populations of every boundary link by halfway
 *      bounce-back (Eq. 10), linear Bouzidi, quadratic Bouzidi (Eq. 11), Yu's
 *      unified scheme (Eq. 12-14) or Zhao & Yong's single-node scheme
 *      (Eq. 16), then the force and torque on each solid by the
 *      Galilean-invariant momentum exchange method, Eq. 17;
 *   7. moving IBB solids only: advance the solid (prescribed translation, or
 *      free motion by Eq. 20 under the force and torque of step 6), reclassify,
 *      refill the newly uncovered nodes and rebuild the boundary links
 *      (Sec. 3.2).  Moving IBM solids: advance the solid (prescribed
 *      translation, or free motion by Feng & Michaelides's discretisation,
 *      Eq. 23, under the force and torque of step 3) and carry its Lagrangian
 *      points with it.
 *
 * Two representations of the same step (orc_set_form):
 *   - literal (the default): the populations f_i themselves, the equilibrium
 *     f_eq(rho, u), rho = sum f_i, and the momentum exchange of Eq. 17 summed
 *     term by term with plain additions, as the equations are written;
 *   - deviation: h_i = f_i - w_i from the rest state (rho = 1, u = 0).  Every
 *     relation used is linear in f apart from f_eq, and all bounce-back
 *     weights sum to one, so the step is the same computation written for h
 *     (f - f_eq = h - h_eq, and the rest-state part of each Eq. 17 term,
 *     w_i (e_ibar - e_i), is added in closed form); Eq. 17 is summed with
 *     compensated additions.  This keeps the stored numbers small, which
 *     lowers the rounding by about three decades.
 * tests/test_oracle_forms.py pins the two against each other within the
 * literal form's measured rounding, for every boundary scheme and the IBM.
 *
 * Threads (orc_set_threads, default 1) split only the per-cell loops
 * (moments, collision, streaming, classification), whose results do not
 * depend on the split; every sum across cells keeps its serial order.
 *
 * The paper does not print the velocity sets, the equilibrium, the MRT
 * matrix, the relaxation rates, the forcing term, the linear Bouzidi formula
 * or the refill rule (Sec. 2 defers them to textbooks).  The readings used are the
 * standard ones and are listed where they are used.
 *
 * Pins (see tests/test_oracle_*.py): velocity-set moments, equilibrium and
 * forcing moments, MRT orthogonality and MRT(S = I/tau) == BGK, exact
 * streaming permutation, mass/momentum balance (with the momentum exchange
 * force), Taylor-Green decay, exact plane Poiseuille for the default MRT rates
 * with halfway bounce-back, second-order IBB convergence, steady Couette
 * (App. A, Eq. 31) and its torque, pipe flow (Eq. 28), delta-function moment
 * identities (App. B), interpolation/spreading invariants, link
 * classification and q by exact arithmetic on tiny grids; free IBM solids by
 * the closed-form solution of the Eq. 23 recurrence without fluid force and
 * by the exact balance of fluid plus solid momentum (tests/test_oracle_free_ibm.py).
 *
 * PARITY UNPINNED (no closed form or independent reference exists): the
 * default MRT rates beyond what exact Poiseuille pins, and of the refill rule
 * for newly uncovered nodes of a moving IBB solid the choice of the density
 * (the mean over the neighbours that stay fluid; the co-moving uniform flow
 * fixes it only where the density is uniform).  These are checked only
 * against the GPU library (same reading on both sides) and by convergence
 * order.  (The IBM coupling reading -- which velocity is interpolated, force
 * factor 1, Sec. 2.1 -- is pinned by the one-point closed form of
 * tests/test_oracle_comoving.py.)
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 *        -o liblbm_oracle.so lbm_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 19

/* ------------------------------------------------------------------------ */
/* Velocity sets.  Not printed in the paper (Sec. 2 refers to textbooks).    */
/* Standard D2Q9 and D3Q19 with c_s^2 = 1/3.  Order: rest, then +/- pairs,   */
/* axis pairs before diagonal pairs, so the opposite of i is i+1 (odd i) or  */
/* i-1 (even i > 0).                                                         */
/* ------------------------------------------------------------------------ */
static const int E2[9][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                             {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const int E3[19][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* Weights from the isotropy conditions: sum w = 1, sum w e_a e_b = delta_ab/3,
 * fourth moment isotropic.  Rest 4/9 (D2Q9) or 1/3 (D3Q19); speed-1 links
 * 1/9 or 1/18; speed-sqrt2 links 1/36 in both. */
static double weight_of(int D, const int e[3]) {
  int s = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
  if (D == 2) return s == 0 ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
  return s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* ------------------------------------------------------------------------ */
/* Solids                                                                    */
/* ------------------------------------------------------------------------ */
enum { K_SPHERE = 0, K_CYLINDER = 1, K_PLANE = 2 };
enum { M_BB = 0, M_LINEAR = 1, M_QUADRATIC = 2, M_IBM = 3, M_YU = 4, M_ZHAO_YONG = 5 };

typedef struct {
  int kind, inverted;
  double c0[3];  /* centre (sphere, cylinder) or a point on the plane, at t = 0 */
  double c[3];   /* current centre */
  double R;
  int ax;        /* cylinder axis / plane normal axis (0, 1, 2) */
  int sgn;       /* plane normal sign (+1 / -1): the fluid side is sgn*(x-p) > 0 */
  double U[3], W[3];
  int moving;
  /* free motion (Eq. 20): density ratio rho_p / rho_f, external acceleration
   * (gravity), volume and moment of inertia of the solid */
  int free;
  double rho_p, grav[3], Vp, Ip;
  /* IBM: displacement of the solid since its Lagrangian points were placed
   * (unwrapped; the points move rigidly with it), and the velocities of the
   * step before (Eq. 23 reads v^{n-1}, w^{n-1}) */
  double disp[3], Up[3], Wp[3];
  /* Kempe's inner-fluid integrals (Eq. 24-26) of the last step and of the
   * step before: sum alpha u and sum alpha r x u; kfirst: no step yet */
  double Ik[6], Ikp[6];
  int kfirst;
} solid_t;

typedef struct {
  long cell;
  int dir, sid;
  double q;
  int ff_ok, fff_ok;
} link_t;

typedef struct orc {
  int D, Q, nx, ny, nz;
  long N;
  int collision;
  double tau, S[QMAX];
  int e[QMAX][3], opp[QMAX];
  double w[QMAX];
  double M[QMAX][QMAX], Minv[QMAX][QMAX];
  double g[3];
  int g_fluid_only;
  double *f, *fpost, *fnew;
  unsigned char *excl;    /* node removed from the fluid (IBB solid node) */
  unsigned char *inside;  /* node inside the physical volume of some solid */
  int *owner;             /* solid index of an inside node, -1 otherwise */
  double *rho_out, *u_out; /* macros of the most recent collision */
  double *strain_out;      /* [6][N] strain rate of the most recent collision (Eq. 19) */
  unsigned char *type_out;
  int nsolid, method;
  solid_t *sol;
  long nlink;
  link_t *links;
  /* IBM */
  int n_iter;
  int inner;      /* free IBM solids: 0 Feng & Michaelides (Eq. 23), 1 Kempe (Eq. 24-26) */
  int delta;      /* points of the delta function: 4 (Eq. 6), 3 or 2 */
  long nlag;
  double *X;      /* [nlag][3] */
  double *dV;     /* [nlag] */
  int *lag_sid;   /* [nlag] */
  double *Flag;   /* [nlag][3] total boundary force of the last step */
  double *fibm;   /* [3][N] Eulerian boundary force of the last step */
  /* force/torque */
  double *FT;     /* [nsolid][6] of the last step */
  double *hist;
  long hist_len, hist_cap;
  long t;
  int stepped;
  int literal;   /* 1: f stores f_i; 0: f stores h_i = f_i - w_i */
  int nthreads;  /* threads of the per-cell loops */
  /* domain boundaries per axis (Sec. 3.4): BC_PERIODIC, BC_SLIP (stress-free
   * planes halfway outside the first and last node layers) or, on x only,
   * BC_OPEN (velocity inlet halfway before x = 0, convective outflow at the
   * last layer); Uin the inflow velocity; mir[a][i] the direction i with its
   * axis-a component reversed */
  int bc[3];
  double Uin;
  int mir[3][QMAX];
  /* covering / uncovering momentum of moving IBB solids (R38): on or off, and
   * per solid the force and torque [6] of the last move, added to the force
   * of the next step */
  int cover;
  double *cu;
} orc;

enum { BC_PERIODIC = 0, BC_SLIP = 1, BC_OPEN = 2 };

static void solid_node_output(struct orc *o);

/* Compensated (Neumaier) summation: the momentum-exchange sum adds O(0.1)
 * rest-state terms that cancel to a small force, so a plain running sum
 * would carry an error of ~1e-12; this keeps it at the last bit. */
typedef struct {
  double s, c;
} acc_t;
static void acc_add(acc_t *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static double acc_get(const acc_t *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */
static int wrap(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}
static long cell_of(const orc *o, int x, int y, int z) {
  return (long)wrap(x, o->nx) + (long)o->nx * ((long)wrap(y, o->ny) + (long)o->ny * (long)wrap(z, o->nz));
}
static void coords_of(const orc *o, long n, int *x, int *y, int *z) {
  *x = (int)(n % o->nx);
  *y = (int)((n / o->nx) % o->ny);
  *z = (int)(n / ((long)o->nx * o->ny));
}
/* Shortest periodic image of a separation d along an axis of length L. */
static double min_image(double d, int L) {
  if (d > 0.5 * (double)L) d -= (double)L;
  else if (d < -0.5 * (double)L) d += (double)L;
  return d;
}
static int dims_of(const orc *o, int a) { return a == 0 ? o->nx : (a == 1 ? o->ny : o->nz); }

/* ------------------------------------------------------------------------ */
/* Equilibrium and forcing.                                                  */
/* f_eq: the compressible second-order polynomial (not printed in Sec. 2).  */
/* Forcing: Guo's second-order scheme, the one Sec. 2.1 names for BGK; its  */
/* MRT form is (I - S/2) M F_hat, the inverse-design construction.          */
/* ------------------------------------------------------------------------ */
static void feq_all(const orc *o, double rho, const double u[3], double *feq) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < o->Q; i++) {
    double eu = o->e[i][0] * u[0] + o->e[i][1] * u[1] + o->e[i][2] * u[2];
    feq[i] = o->w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}
/* The same equilibrium written as a deviation from the rest state:
 * f_eq_i - w_i = w_i [ (rho - 1) + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u) ]. */
static void heq_all(const orc *o, double drho, const double u[3], double *heq) {
  double rho = 1.0 + drho;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < o->Q; i++) {
    double eu = o->e[i][0] * u[0] + o->e[i][1] * u[1] + o->e[i][2] * u[2];
    heq[i] = o->w[i] * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
  }
}
static void guo_all(const orc *o, const double u[3], const double F[3], double *Fi) {
  for (int i = 0; i < o->Q; i++) {
    double eu = o->e[i][0] * u[0] + o->e[i][1] * u[1] + o->e[i][2] * u[2];
    double eF = o->e[i][0] * F[0] + o->e[i][1] * F[1] + o->e[i][2] * F[2];
    double emuF = (o->e[i][0] - u[0]) * F[0] + (o->e[i][1] - u[1]) * F[1] + (o->e[i][2] - u[2]) * F[2];
    /* w_i [ (e_i - u)/c_s^2 + (e_i.u) e_i / c_s^4 ] . F */
    Fi[i] = o->w[i] * (3.0 * emuF + 9.0 * eu * eF);
  }
}

/* ------------------------------------------------------------------------ */
/* MRT transform: rows of the unweighted Gram-Schmidt orthogonalisation of   */
/* monomials of e_i (the matrix M of Eq. 3 is not printed).  Row order:      */
/*  D2Q9 : 1, |e|^2, |e|^4, ex, ex|e|^2, ey, ey|e|^2, ex^2-ey^2, ex ey       */
/*  D3Q19: 1, |e|^2, |e|^4, ex, ex|e|^2, ey, ey|e|^2, ez, ez|e|^2,           */
/*         3ex^2-|e|^2, (3ex^2-|e|^2)|e|^2, ey^2-ez^2, (ey^2-ez^2)|e|^2,     */
/*         ex ey, ey ez, ex ez, (ey^2-ez^2)ex, (ez^2-ex^2)ey, (ex^2-ey^2)ez  */
/* The inverse is computed by Gauss-Jordan elimination with partial pivots.  */
/* ------------------------------------------------------------------------ */
static double monomial(int D, int k, const int e[3]) {
  double x = e[0], y = e[1], z = e[2];
  double s = x * x + y * y + z * z;
  if (D == 2) {
    switch (k) {
      case 0: return 1.0;
      case 1: return s;
      case 2: return s * s;
      case 3: return x;
      case 4: return x * s;
      case 5: return y;
      case 6: return y * s;
      case 7: return x * x - y * y;
      default: return x * y;
    }
  }
  switch (k) {
    case 0: return 1.0;
    case 1: return s;
    case 2: return s * s;
    case 3: return x;
    case 4: return x * s;
    case 5: return y;
    case 6: return y * s;
    case 7: return z;
    case 8: return z * s;
    case 9: return 3.0 * x * x - s;
    case 10: return (3.0 * x * x - s) * s;
    case 11: return y * y - z * z;
    case 12: return (y * y - z * z) * s;
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}

static void build_mrt(orc *o) {
  int Q = o->Q;
  for (int k = 0; k < Q; k++) {
    double v[QMAX];
    for (int i = 0; i < Q; i++) v[i] = monomial(o->D, k, o->e[i]);
    for (int p = 0; p < k; p++) {
      double num = 0.0, den = 0.0;
      for (int i = 0; i < Q; i++) {
        num += v[i] * o->M[p][i];
        den += o->M[p][i] * o->M[p][i];
      }
      for (int i = 0; i < Q; i++) v[i] -= (num / den) * o->M[p][i];
    }
    for (int i = 0; i < Q; i++) o->M[k][i] = v[i];
  }
  /* Gauss-Jordan inverse */
  double a[QMAX][2 * QMAX];
  for (int r = 0; r < Q; r++)
    for (int c = 0; c < 2 * Q; c++) a[r][c] = c < Q ? o->M[r][c] : (c - Q == r ? 1.0 : 0.0);
  for (int col = 0; col < Q; col++) {
    int piv = col;
    for (int r = col + 1; r < Q; r++)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * Q; c++) {
        double tmp = a[col][c];
        a[col][c] = a[piv][c];
        a[piv][c] = tmp;
      }
    double d = a[col][col];
    for (int c = 0; c < 2 * Q; c++) a[col][c] /= d;
    for (int r = 0; r < Q; r++) {
      if (r == col) continue;
      double m = a[r][col];
      if (m == 0.0) continue;
      for (int c = 0; c < 2 * Q; c++) a[r][c] -= m * a[col][c];
    }
  }
  for (int r = 0; r < Q; r++)
    for (int c = 0; c < Q; c++) o->Minv[r][c] = a[r][Q + c];
}

/* Default relaxation rates (the paper does not print S).  Conserved moments
 * (density, momentum) 1.0 -- their rate has no effect; every even
 * non-conserved moment relaxes with s_nu = 1/tau (so Eq. 2 holds for the
 * shear viscosity); the odd non-conserved moments (energy flux q and the
 * third-order m group) take s_odd from (1/s_nu - 1/2)(1/s_odd - 1/2) = 3/16. */
static void default_rates(orc *o) {
  double snu = 1.0 / o->tau;
  double sodd = 1.0 / (0.5 + (3.0 / 16.0) / (1.0 / snu - 0.5));
  for (int k = 0; k < o->Q; k++) o->S[k] = snu;
  if (o->D == 2) {
    o->S[0] = o->S[3] = o->S[5] = 1.0;
    o->S[4] = o->S[6] = sodd;
  } else {
    o->S[0] = o->S[3] = o->S[5] = o->S[7] = 1.0;
    o->S[4] = o->S[6] = o->S[8] = sodd;
    o->S[16] = o->S[17] = o->S[18] = sodd;
  }
}

/* ------------------------------------------------------------------------ */
/* Classification of nodes against solids (the fluid/solid split of Fig. 1) */
/* A node is inside an ordinary sphere/cylinder when its squared distance   */
/* (shortest periodic image, summed x then y then z) is <= R^2; inverted     */
/* solids (solid outside the surface) flip the test; a plane's solid side is */
/* sgn*(x - p) <= 0.                                                         */
/* ------------------------------------------------------------------------ */
static void sep(const orc *o, const solid_t *s, double px, double py, double pz, double d[3]) {
  /* shortest periodic image along periodic axes; the plain difference along bounded ones */
  d[0] = o->bc[0] == BC_PERIODIC ? min_image(px - s->c[0], o->nx) : px - s->c[0];
  d[1] = o->bc[1] == BC_PERIODIC ? min_image(py - s->c[1], o->ny) : py - s->c[1];
  d[2] = o->D == 2 ? 0.0 : (o->bc[2] == BC_PERIODIC ? min_image(pz - s->c[2], o->nz) : pz - s->c[2]);
  if (s->kind == K_CYLINDER) d[s->ax] = 0.0;
}
static int in_solid(const orc *o, const solid_t *s, int x, int y, int z) {
  int in;
  if (s->kind == K_PLANE) {
    double p = s->ax == 0 ? (double)x : (s->ax == 1 ? (double)y : (double)z);
    in = (double)s->sgn * (p - s->c[s->ax]) <= 0.0;
  } else {
    double d[3];
    sep(o, s, (double)x, (double)y, (double)z, d);
    double r2 = d[0] * d[0];
    r2 = r2 + d[1] * d[1];
    r2 = r2 + d[2] * d[2];
    in = r2 <= s->R * s->R;
  }
  return s->inverted ? !in : in;
}

static void classify(orc *o) {
#pragma omp parallel for num_threads(o->nthreads) schedule(static)
  for (long n = 0; n < o->N; n++) {
    int x, y, z;
    coords_of(o, n, &x, &y, &z);
    o->inside[n] = 0;
    o->owner[n] = -1;
    for (int k = 0; k < o->nsolid; k++)
      if (in_solid(o, &o->sol[k], x, y, z)) {
        o->inside[n] = 1;
        o->owner[n] = k;
        break;
      }
    o->excl[n] = (o->method != M_IBM) && o->inside[n];
  }
}

/* q = |x_f - x_w| / |x_f - x_b| (Sec. 2.2), from the intersection of the
 * segment x_f + t e_ibar, t in (0, 1], with the surface of solid s. */
static double link_q(const orc *o, const solid_t *s, int x, int y, int z, int i) {
  double e[3] = {(double)-o->e[i][0], (double)-o->e[i][1], (double)-o->e[i][2]};
  double t;
  if (s->kind == K_PLANE) {
    double p = s->ax == 0 ? (double)x : (s->ax == 1 ? (double)y : (double)z);
    double dist = (double)s->sgn * (p - s->c[s->ax]);
    t = dist / (-(double)s->sgn * e[s->ax]);
  } else {
    double d[3];
    sep(o, s, (double)x, (double)y, (double)z, d);
    if (s->kind == K_CYLINDER) e[s->ax] = 0.0;
    if (o->D == 2) e[2] = 0.0;
    double a = e[0] * e[0];
    a = a + e[1] * e[1];
    a = a + e[2] * e[2];
    double b = d[0] * e[0];
    b = b + d[1] * e[1];
    b = b + d[2] * e[2];
    double dd = d[0] * d[0];
    dd = dd + d[1] * d[1];
    dd = dd + d[2] * d[2];
    double cc = dd - s->R * s->R;
    double disc = b * b - a * cc;
    if (disc < 0.0) disc = 0.0;
    /* Root of a t^2 + 2 b t + cc = 0 in (0, 1], each case written without
     * cancellation: entering an ordinary solid from outside (cc > 0, b < 0)
     * takes the smaller root; leaving the inside of an inverted solid
     * (cc <= 0) takes the larger one. */
    if (!s->inverted)
      t = cc / (-b + sqrt(disc));
    else if (b > 0.0)
      t = -cc / (b + sqrt(disc));
    else
      t = (-b + sqrt(disc)) / a;
  }
  if (!(t >= 0x1p-52)) t = 0x1p-52;
  if (t > 1.0) t = 1.0;
  return t;
}

static void build_links(orc *o) {
  o->nlink = 0;
  if (o->method == M_IBM) return;
  long cap = 1024, cnt = 0;
  link_t *L = (link_t *)malloc(sizeof(link_t) * cap);
  for (long n = 0; n < o->N; n++) {
    if (o->excl[n]) continue;
    int x, y, z;
    coords_of(o, n, &x, &y, &z);
    for (int i = 1; i < o->Q; i++) {
      long nb = cell_of(o, x - o->e[i][0], y - o->e[i][1], z - o->e[i][2]);
      if (!o->excl[nb]) continue;
      if (cnt == cap) {
        cap *= 2;
        L = (link_t *)realloc(L, sizeof(link_t) * cap);
      }
      link_t *l = &L[cnt++];
      l->cell = n;
      l->dir = i;
      l->sid = o->owner[nb];
      l->q = link_q(o, &o->sol[l->sid], x, y, z, i);
      long ff = cell_of(o, x + o->e[i][0], y + o->e[i][1], z + o->e[i][2]);
      long fff = cell_of(o, x + 2 * o->e[i][0], y + 2 * o->e[i][1], z + 2 * o->e[i][2]);
      l->ff_ok = !o->excl[ff];
      l->fff_ok = !o->excl[fff];
    }
  }
  free(o->links);
  o->links = L;
  o->nlink = cnt;
}

/* Wall velocity of rigid-body motion at a point with lever r from the centre */
static void wall_velocity(const solid_t *s, const double r[3], double uw[3]) {
  uw[0] = s->U[0] + (s->W[1] * r[2] - s->W[2] * r[1]);
  uw[1] = s->U[1] + (s->W[2] * r[0] - s->W[0] * r[2]);
  uw[2] = s->U[2] + (s->W[0] * r[1] - s->W[1] * r[0]);
}
static void lever(const orc *o, const solid_t *s, double px, double py, double pz, double r[3]) {
  if (s->kind == K_PLANE) {
    r[0] = px - s->c[0];
    r[1] = py - s->c[1];
    r[2] = o->D == 2 ? 0.0 : pz - s->c[2];
    return;
  }
  r[0] = min_image(px - s->c[0], o->nx);
  r[1] = min_image(py - s->c[1], o->ny);
  r[2] = o->D == 2 ? 0.0 : min_image(pz - s->c[2], o->nz);
}

/* ------------------------------------------------------------------------ */
/* Interpolated bounce-back value of the unknown f_i(x_f, t+1).              */
/*   fb_f, fb_ff, fb_fff : f*_ibar at x_f, x_ff, x_fff (post-collision, t)   */
/*   fi_ff, fi_fff       : f_i at x_ff, x_fff at t+1, i.e. by streaming      */
/*                         f*_i(x_f, t) and f*_i(x_ff, t)                    */
/*   B                   : wall term 2 rho0 w_i e_i.u_w / c_s^2 of Eq. 10    */
/* Halfway bounce-back, Eq. 10.  Quadratic Bouzidi, Eq. 11a (q < 1/2) and    */
/* Eq. 11b (q >= 1/2).  Yu's unified scheme, Eq. 12-14 (any q).              */
/* Linear Bouzidi (named in Sec. 3.3, not printed):                         */
/* the same construction with two-point Lagrange interpolation,             */
/*   q < 1/2 : 2q f*_ibar(x_f) + (1-2q) f*_ibar(x_ff) + B                    */
/*   q >= 1/2: [f*_ibar(x_f) + B]/(2q) + (2q-1)/(2q) f*_i(x_f)               */
/* Where the extra nodes are not fluid (narrow gaps) the scheme degrades:    */
/* quadratic or Yu -> linear -> halfway bounce-back (Sec. 2.2: Eq. 10 takes  */
/* over where the interpolation nodes are missing).                          */
/* ------------------------------------------------------------------------ */
double orc_ibb_value(int method, double q, int ff_ok, int fff_ok, double fb_f, double fb_ff,
                     double fb_fff, double fi_f, double fi_ff, double fi_fff, double B) {
  if (method == M_QUADRATIC && ff_ok && fff_ok) {
    if (q < 0.5)
      return q * (2.0 * q + 1.0) * fb_f + (1.0 + 2.0 * q) * (1.0 - 2.0 * q) * fb_ff -
             q * (1.0 - 2.0 * q) * fb_fff + B;
    return (fb_f + B) / (q * (2.0 * q + 1.0)) + ((2.0 * q - 1.0) / q) * fi_ff -
           ((2.0 * q - 1.0) / (1.0 + 2.0 * q)) * fi_fff;
  }
  if (method == M_YU && ff_ok && fff_ok) {
    /* Yu's three steps, Eq. 12-14, taken in turn:
     * (12) the population that reaches the wall point after one step starts
     *      1 - q from x_f towards x_ff; quadratic interpolation there from
     *      f*_ibar at x_f, x_ff, x_fff;
     * (13) it bounces back at the wall with the wall term B;
     * (14) f_i(x_f, t+1) by quadratic interpolation at x_f from the wall
     *      value (at -q along e_i) and f_i(x_ff), f_i(x_fff) at t+1.
     * (Eq. 15 merges the three steps; as printed its x_ff coefficient,
     * 2(1-q)/(1+q), does not follow from Eq. 12-14, which give 2(1-q)/(2+q).) */
    double fw_in = 0.5 * q * (q + 1.0) * fb_f + (1.0 + q) * (1.0 - q) * fb_ff -
                   0.5 * q * (1.0 - q) * fb_fff;
    double fw_out = fw_in + B;
    return 2.0 / ((1.0 + q) * (2.0 + q)) * fw_out + (2.0 * q / (1.0 + q)) * fi_ff -
           (q / (2.0 + q)) * fi_fff;
  }
  if (method == M_QUADRATIC || method == M_YU || method == M_LINEAR) {
    if (q < 0.5) {
      if (ff_ok) return 2.0 * q * fb_f + (1.0 - 2.0 * q) * fb_ff + B;
      return fb_f + B;
    }
    return (fb_f + B) / (2.0 * q) + ((2.0 * q - 1.0) / (2.0 * q)) * fi_f;
  }
  return fb_f + B;
}

/* Zhao & Yong's single-node scheme, Eq. 16: the unknown f_i(x_f, t+1) from
 * the post-collision f*_i(x_f, t) leaving the wall, the pre-collision
 * f_ibar(x_f, t) heading to it, and the wall term B scaled by 1/(1 + 2q).
 * Only x_f is read, so there is no fallback for narrow gaps. */
double orc_zhao_yong_value(double q, double fi_post, double fb_pre, double B) {
  return (2.0 * q / (1.0 + 2.0 * q)) * fi_post + (1.0 / (1.0 + 2.0 * q)) * fb_pre + B / (1.0 + 2.0 * q);
}

/* ------------------------------------------------------------------------ */
/* Peskin's 4-point regularized delta, Eq. 6 (one factor).                   */
/* ------------------------------------------------------------------------ */
double orc_phi(double r) {
  r = fabs(r);
  if (r >= 2.0) return 0.0;
  if (r >= 1.0) return 0.125 * (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r));
  return 0.125 * (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r));
}

/* The other two delta functions of the comparison in Sec. 3.1, which the
 * paper names but does not print; written from their published definitions.
 * Three-point (Roma, Peskin & Berger 1999): support |r| < 3/2, the unique
 * piecewise form with sum_j phi(r - j) = 1, sum_j (r - j) phi(r - j) = 0 and
 * sum_j phi(r - j)^2 = 1/2 for every r:
 *   |r| <= 1/2      : (1 + sqrt(1 - 3 r^2)) / 3
 *   1/2 <= |r| < 3/2: (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6
 * Two-point: the linear hat 1 - |r| on |r| < 1 (bilinear / trilinear
 * interpolation). */
double orc_phi3(double r) {
  r = fabs(r);
  if (r >= 1.5) return 0.0;
  if (r >= 0.5) return (5.0 - 3.0 * r - sqrt(1.0 - 3.0 * (1.0 - r) * (1.0 - r))) / 6.0;
  return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
}
double orc_phi2(double r) {
  r = fabs(r);
  return r >= 1.0 ? 0.0 : 1.0 - r;
}
double orc_phi_n(int points, double r) {
  return points == 3 ? orc_phi3(r) : (points == 2 ? orc_phi2(r) : orc_phi(r));
}

/* Stencil of a Lagrangian point: the w nodes per axis whose distance to X is
 * below w/2 (the support of the w-point delta; w = 4: floor(X)-1 ..
 * floor(X)+2), with the weight phi(x - X) per axis. */
typedef struct {
  long cell[64];
  double wgt[64];
  int n;
} stencil_t;

static void stencil_of(const orc *o, const double X[3], stencil_t *st) {
  int b[3];
  const int w = o->delta;
  double wx[4], wy[4], wz[4];
  for (int a = 0; a < 3; a++) b[a] = (int)floor(X[a] - 0.5 * w) + 1;
  for (int k = 0; k < w; k++) {
    wx[k] = orc_phi_n(w, (double)(b[0] + k) - X[0]);
    wy[k] = orc_phi_n(w, (double)(b[1] + k) - X[1]);
    wz[k] = orc_phi_n(w, (double)(b[2] + k) - X[2]);
  }
  st->n = 0;
  int kzn = o->D == 2 ? 1 : w;
  for (int kz = 0; kz < kzn; kz++)
    for (int ky = 0; ky < w; ky++)
      for (int kx = 0; kx < w; kx++) {
        double wgt = wx[kx] * wy[ky];
        int z = 0;
        if (o->D == 3) {
          wgt *= wz[kz];
          z = b[2] + kz;
        }
        st->cell[st->n] = cell_of(o, b[0] + kx, b[1] + ky, z);
        st->wgt[st->n] = wgt;
        st->n++;
      }
}

/* Position of Lagrangian point l now: where it was placed, moved with its
 * solid (rigid translation; the points of a sphere or cylinder keep their
 * orientation, which the shape does not see). */
static void lag_pos(const orc *o, long l, double X[3]) {
  const solid_t *s = &o->sol[o->lag_sid[l]];
  for (int a = 0; a < 3; a++) X[a] = o->X[3 * l + a] + s->disp[a];
  if (o->D == 2) X[2] = 0.0;
}

/* Eq. 5: U(X_l) = sum_x u(x) delta_h(x - X_l) h^3, with h = 1. */
static void interpolate(const orc *o, const double *u, double *Ut) {
  for (long l = 0; l < o->nlag; l++) {
    stencil_t st;
    double X[3];
    lag_pos(o, l, X);
    stencil_of(o, X, &st);
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < st.n; k++)
      for (int a = 0; a < 3; a++) s[a] += u[a * o->N + st.cell[k]] * st.wgt[k];
    for (int a = 0; a < 3; a++) Ut[3 * l + a] = s[a];
  }
}

/* Eq. 8: f(x) = sum_X F(X) delta_h(x - X) dV  (accumulated into f). */
static void spread(const orc *o, const double *F, double *f) {
  for (long l = 0; l < o->nlag; l++) {
    stencil_t st;
    double X[3];
    lag_pos(o, l, X);
    stencil_of(o, X, &st);
    for (int k = 0; k < st.n; k++)
      for (int a = 0; a < 3; a++) f[a * o->N + st.cell[k]] += F[3 * l + a] * st.wgt[k] * o->dV[l];
  }
}

/* Direct forcing, Sec. 2.1, repeated n_iter times ("iterated for 5 times",
 * Sec. 3.1).  u0 is the velocity of the current populations with half of the
 * body force and none of the boundary force; then for each iteration:
 *   U~_l = interpolation of u (Eq. 5)
 *   F_l  = rho0 (U^d_l - U~_l) / dt (Eq. 7, rho0 = 1, dt = 1)
 *   f    = spreading of F (Eq. 8)
 *   u   += f dt / rho0 (Eq. 9)
 * The boundary force used in the collision is the sum over iterations; the
 * force on solid s is -sum_l F_l dV_l and the torque -sum_l (X_l - Y) x F_l
 * dV_l (Sec. 3.1 and App. B, Eq. 45, with the fluid inside the solid taken
 * to move rigidly, Sec. 3.2, so its inertia term vanishes for a fixed
 * solid). */
static void ibm_force(orc *o, const double *rho, const double *j, const double *Fb) {
  long N = o->N;
  double *u = (double *)malloc(sizeof(double) * 3 * N);
  double *fk = (double *)malloc(sizeof(double) * 3 * N);
  double *Ut = (double *)malloc(sizeof(double) * 3 * (o->nlag + 1));
  double *Fk = (double *)malloc(sizeof(double) * 3 * (o->nlag + 1));
  for (long n = 0; n < N; n++)
    for (int a = 0; a < 3; a++) u[a * N + n] = (j[a * N + n] + 0.5 * Fb[a * N + n]) / rho[n];
  memset(o->fibm, 0, sizeof(double) * 3 * N);
  memset(o->Flag, 0, sizeof(double) * 3 * (o->nlag + 1));
  for (int it = 0; it < o->n_iter; it++) {
    interpolate(o, u, Ut);
    for (long l = 0; l < o->nlag; l++) {
      const solid_t *s = &o->sol[o->lag_sid[l]];
      double r[3], Ud[3], X[3];
      lag_pos(o, l, X);
      lever(o, s, X[0], X[1], X[2], r);
      wall_velocity(s, r, Ud);
      for (int a = 0; a < 3; a++) Fk[3 * l + a] = Ud[a] - Ut[3 * l + a];
      if (o->D == 2) Fk[3 * l + 2] = 0.0;
    }
    memset(fk, 0, sizeof(double) * 3 * N);
    spread(o, Fk, fk);
    for (long n = 0; n < 3 * N; n++) {
      u[n] += fk[n];
      o->fibm[n] += fk[n];
    }
    for (long l = 0; l < 3 * o->nlag; l++) o->Flag[l] += Fk[l];
  }
  acc_t *acc = (acc_t *)calloc(6 * (o->nsolid > 0 ? o->nsolid : 1), sizeof(acc_t));
  for (long l = 0; l < o->nlag; l++) {
    int k = o->lag_sid[l];
    const solid_t *s = &o->sol[k];
    double r[3], F[3], X[3];
    lag_pos(o, l, X);
    lever(o, s, X[0], X[1], X[2], r);
    for (int a = 0; a < 3; a++) F[a] = -o->Flag[3 * l + a] * o->dV[l];
    acc_add(&acc[6 * k + 0], F[0]);
    acc_add(&acc[6 * k + 1], F[1]);
    acc_add(&acc[6 * k + 2], F[2]);
    acc_add(&acc[6 * k + 3], r[1] * F[2] - r[2] * F[1]);
    acc_add(&acc[6 * k + 4], r[2] * F[0] - r[0] * F[2]);
    acc_add(&acc[6 * k + 5], r[0] * F[1] - r[1] * F[0]);
  }
  for (int k = 0; k < 6 * o->nsolid; k++) o->FT[k] = acc_get(&acc[k]);
  free(acc);
  free(u);
  free(fk);
  free(Ut);
  free(Fk);
}

/* ------------------------------------------------------------------------ */
/* construction                                                              */
/* ------------------------------------------------------------------------ */
orc *orc_create(int lattice, int collision, int nx, int ny, int nz, double tau, const double *rates,
                const double *g, int g_fluid_only) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || !(tau > 0.5)) return NULL;
  if (lattice == 0 && nz != 1) return NULL;
  orc *o = (orc *)calloc(1, sizeof(orc));
  o->D = lattice == 0 ? 2 : 3;
  o->Q = lattice == 0 ? 9 : 19;
  o->nx = nx;
  o->ny = ny;
  o->nz = nz;
  o->N = (long)nx * ny * nz;
  o->collision = collision;
  o->tau = tau;
  for (int i = 0; i < o->Q; i++) {
    for (int a = 0; a < 3; a++) o->e[i][a] = o->D == 2 ? E2[i][a] : E3[i][a];
    o->w[i] = weight_of(o->D, o->e[i]);
  }
  for (int i = 0; i < o->Q; i++)
    for (int k = 0; k < o->Q; k++)
      if (o->e[k][0] == -o->e[i][0] && o->e[k][1] == -o->e[i][1] && o->e[k][2] == -o->e[i][2]) o->opp[i] = k;
  build_mrt(o);
  default_rates(o);
  if (rates)
    for (int k = 0; k < o->Q; k++) o->S[k] = rates[k];
  for (int a = 0; a < 3; a++) o->g[a] = g ? g[a] : 0.0;
  if (o->D == 2) o->g[2] = 0.0;
  o->g_fluid_only = g_fluid_only;
  long QN = (long)o->Q * o->N;
  o->f = (double *)malloc(sizeof(double) * QN);
  o->fpost = (double *)malloc(sizeof(double) * QN);
  o->fnew = (double *)malloc(sizeof(double) * QN);
  o->excl = (unsigned char *)calloc(o->N, 1);
  o->inside = (unsigned char *)calloc(o->N, 1);
  o->owner = (int *)malloc(sizeof(int) * o->N);
  o->rho_out = (double *)malloc(sizeof(double) * o->N);
  o->u_out = (double *)calloc(3 * o->N, sizeof(double));
  o->strain_out = (double *)calloc(6 * o->N, sizeof(double));
  o->type_out = (unsigned char *)calloc(o->N, 1);
  o->fibm = (double *)calloc(3 * o->N, sizeof(double));
  o->literal = 1;
  o->nthreads = 1;
  for (int a = 0; a < 3; a++) {
    o->bc[a] = BC_PERIODIC;
    for (int i = 0; i < o->Q; i++)
      for (int k = 0; k < o->Q; k++) {
        int same = 1;
        for (int b = 0; b < 3; b++) same &= o->e[k][b] == (b == a ? -o->e[i][b] : o->e[i][b]);
        if (same) o->mir[a][i] = k;
      }
  }
  o->Uin = 0.0;
  for (long n = 0; n < o->N; n++) {
    o->owner[n] = -1;
    o->rho_out[n] = 1.0;
    for (int i = 0; i < o->Q; i++) o->f[(long)i * o->N + n] = o->w[i]; /* rest: f = w, rho = 1 */
  }
  o->n_iter = 5;
  o->delta = 4;
  o->method = M_BB;
  return o;
}

void orc_destroy(orc *o) {
  if (!o) return;
  free(o->f);
  free(o->fpost);
  free(o->fnew);
  free(o->excl);
  free(o->inside);
  free(o->owner);
  free(o->rho_out);
  free(o->u_out);
  free(o->strain_out);
  free(o->type_out);
  free(o->fibm);
  free(o->sol);
  free(o->links);
  free(o->X);
  free(o->dV);
  free(o->lag_sid);
  free(o->Flag);
  free(o->FT);
  free(o->cu);
  free(o->hist);
  free(o);
}

/* kind/inverted/axis arrays per solid; centre, U, W as [n][3]. For planes
 * `axis` is the normal axis and `sign` its orientation (fluid on the side
 * sign*(x - p) > 0); for cylinders the axis (0, 1, 2). */
int orc_set_solids(orc *o, int n, const int *kind, const int *inverted, const double *centre,
                   const double *radius, const int *axis, const int *sign, const double *U,
                   const double *W, int method) {
  free(o->sol);
  o->sol = (solid_t *)calloc(n > 0 ? n : 1, sizeof(solid_t));
  o->nsolid = n;
  o->method = method;
  for (int k = 0; k < n; k++) {
    solid_t *s = &o->sol[k];
    s->kind = kind[k];
    s->inverted = inverted[k];
    s->R = radius[k];
    s->ax = axis ? axis[k] : 2;
    s->sgn = sign ? sign[k] : 1;
    for (int a = 0; a < 3; a++) {
      s->c0[a] = centre[3 * k + a];
      s->c[a] = s->c0[a];
      s->U[a] = U ? U[3 * k + a] : 0.0;
      s->W[a] = W ? W[3 * k + a] : 0.0;
    }
    if (o->D == 2) s->U[2] = 0.0;
    if (s->kind != K_PLANE)
      for (int a = 0; a < o->D; a++)
        if (!(s->c0[a] >= 0.0 && s->c0[a] < (double)dims_of(o, a)) && !(s->kind == K_CYLINDER && a == s->ax))
          return -1;
    for (int a = 0; a < 3; a++) {
      s->disp[a] = 0.0;
      s->Up[a] = s->U[a];
      s->Wp[a] = s->W[a];
    }
    for (int a = 0; a < 6; a++) s->Ik[a] = s->Ikp[a] = 0.0;
    s->kfirst = 1;
    s->moving = (s->U[0] != 0.0 || s->U[1] != 0.0 || s->U[2] != 0.0);
    if (s->moving && (s->kind == K_PLANE || (method == M_IBM && s->inverted))) return -5;
  }
  free(o->FT);
  o->FT = (double *)calloc(6 * (n > 0 ? n : 1), sizeof(double));
  free(o->cu);
  o->cu = (double *)calloc(6 * (n > 0 ? n : 1), sizeof(double));
  o->hist_len = 0;
  classify(o);
  build_links(o);
  solid_node_output(o);
  return 0;
}

int orc_set_lagrangian(orc *o, int sid, const double *X, long n, double dV) {
  long old = o->nlag;
  o->nlag += n;
  o->X = (double *)realloc(o->X, sizeof(double) * 3 * (o->nlag + 1));
  o->dV = (double *)realloc(o->dV, sizeof(double) * (o->nlag + 1));
  o->lag_sid = (int *)realloc(o->lag_sid, sizeof(int) * (o->nlag + 1));
  o->Flag = (double *)realloc(o->Flag, sizeof(double) * 3 * (o->nlag + 1));
  for (long l = 0; l < n; l++) {
    for (int a = 0; a < 3; a++) o->X[3 * (old + l) + a] = X[3 * l + a];
    if (o->D == 2) o->X[3 * (old + l) + 2] = 0.0;
    o->dV[old + l] = dV;
    o->lag_sid[old + l] = sid;
  }
  return 0;
}

void orc_clear_lagrangian(orc *o) { o->nlag = 0; }
void orc_set_ibm_iters(orc *o, int n_iter) { o->n_iter = n_iter; }

/* Make solid k free (Eq. 20 with bounce-back, Eq. 23 with the IBM) with
 * density ratio rho_p / rho_f and external acceleration g; its velocity and
 * angular velocity start at the values given to orc_set_solids, and so do
 * those of the step before.  Spheres, and cylinders in D2Q9; not inverted.
 * -1 invalid, -5 unsupported. */
int orc_set_free(orc *o, int k, double rho_p, const double *g) {
  if (k < 0 || k >= o->nsolid || !(rho_p > 0.0)) return -1;
  solid_t *s = &o->sol[k];
  if (s->inverted || s->kind == K_PLANE || (s->kind == K_CYLINDER && o->D != 2)) return -5;
  s->free = 1;
  s->moving = 1;
  s->rho_p = rho_p;
  for (int a = 0; a < 3; a++) s->grav[a] = g ? g[a] : 0.0;
  if (o->D == 2) s->grav[2] = 0.0;
  const double pi = 3.14159265358979323846;
  if (s->kind == K_SPHERE) {
    s->Vp = 4.0 / 3.0 * pi * s->R * s->R * s->R;
    s->Ip = 0.4 * rho_p * s->Vp * s->R * s->R;
  } else {
    s->Vp = pi * s->R * s->R;
    s->Ip = 0.5 * rho_p * s->Vp * s->R * s->R;
  }
  return 0;
}

/* Centre, velocity and angular velocity of every solid now: [n][9]. */
void orc_solid_state(const orc *o, double *st) {
  for (int k = 0; k < o->nsolid; k++)
    for (int a = 0; a < 3; a++) {
      st[9 * k + a] = o->sol[k].c[a];
      st[9 * k + 3 + a] = o->sol[k].U[a];
      st[9 * k + 6 + a] = o->sol[k].W[a];
    }
}
int orc_set_ibm_inner(orc *o, int mode) {
  if (mode != 0 && mode != 1) return -1;
  o->inner = mode;
  return 0;
}
/* Eq. 25 with the signed distance of Eq. 26 (a = b = c = R): the solid
 * fraction of the grid cell centred on node (x, y, z), from phi at its 8
 * corners x +- 1/2 (4 in 2D); phi < 0 inside. */
static double kempe_alpha(const orc *o, const solid_t *s, int x, int y, int z) {
  double num = 0.0, den = 0.0;
  const int nz = o->D == 2 ? 1 : 2;
  for (int kz = 0; kz < nz; kz++)
    for (int ky = 0; ky < 2; ky++)
      for (int kx = 0; kx < 2; kx++) {
        double r[3];
        lever(o, s, (double)x + kx - 0.5, (double)y + ky - 0.5, o->D == 2 ? 0.0 : (double)z + kz - 0.5, r);
        const double phi = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) / s->R - 1.0;
        if (phi < 0.0) num += -phi;
        den += fabs(phi);
      }
  return den > 0.0 ? num / den : 0.0;
}
/* Kempe's integrals over solid k of the velocity u of the collision just
 * taken (Eq. 24, h = 1): I = sum alpha u, L = sum alpha (x - Y) x u. */
static void kempe_integrals(const orc *o, const solid_t *s, double out[6]) {
  for (int a = 0; a < 6; a++) out[a] = 0.0;
  for (long n = 0; n < o->N; n++) {
    int x, y, z;
    coords_of(o, n, &x, &y, &z);
    const double al = kempe_alpha(o, s, x, y, z);
    if (al == 0.0) continue;
    double r[3], u[3];
    lever(o, s, (double)x, (double)y, (double)z, r);
    for (int a = 0; a < 3; a++) u[a] = o->u_out[a * o->N + n];
    out[0] += al * u[0];
    out[1] += al * u[1];
    out[2] += al * u[2];
    out[3] += al * (r[1] * u[2] - r[2] * u[1]);
    out[4] += al * (r[2] * u[0] - r[0] * u[2]);
    out[5] += al * (r[0] * u[1] - r[1] * u[0]);
  }
}
/* Sum of alpha over the box (the level-set volume of solid k) and the last
 * step's Kempe integrals of solid k. */
double orc_kempe_volume(const orc *o, int k) {
  double v = 0.0;
  for (long n = 0; n < o->N; n++) {
    int x, y, z;
    coords_of(o, n, &x, &y, &z);
    v += kempe_alpha(o, &o->sol[k], x, y, z);
  }
  return v;
}
void orc_kempe_inner(const orc *o, int k, double out[6]) {
  for (int a = 0; a < 6; a++) out[a] = o->sol[k].Ik[a];
}
int orc_set_ibm_delta(orc *o, int points) {
  if (points != 2 && points != 3 && points != 4) return -1;
  o->delta = points;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* one time step                                                             */
/* ------------------------------------------------------------------------ */
/* Collision of every fluid node.  h holds f - w; with rho = 1 + drho and
 * f - f_eq = h - h_eq the formulas below are Eq. 1 and Eq. 3 as written. */
/* Strain rate s_ab = (d_a u_b + d_b u_a)/2 from the non-equilibrium moments
 * of the populations a collision relaxes (Sec. 3.1, Eq. 19).  hi, heq, Fi:
 * the deviations, their equilibrium part and Guo's forcing term F_hat of one
 * node; S: xx, yy, zz, xy, yz, xz.  rho0 = 1, dt = 1.
 *
 * D2Q9 is Eq. 19 as printed, in the moment basis its text names (energy
 * e = 3|e|^2 - 4, normal stress n = e_x^2 - e_y^2, shear c = e_x e_y); psi
 * is the moment of the forcing term of Eq. 3, (1 - s/2) M F_hat.  For D3Q19
 * the same first-order Chapman-Enskog balance of every second-order moment
 * row k (with rate s_k), -(s_k/dt) m_k^(1) + psi_k = (D_0 of the equilibrium
 * moment)_k = 2 rho0 c_s^2 (row k of s) + (row k of uF + Fu), is solved for
 * s over the rows |e|^2, 3e_x^2 - |e|^2, e_y^2 - e_z^2, e_x e_y, e_y e_z,
 * e_x e_z (c_s^2 = 1/3); for D2Q9 it reduces to Eq. 19.  The rates are
 * those of the same rows of M (R4 order); BGK: all 1/tau. */
static double rate_of_row(const orc *o, int k) { return o->collision == 0 ? 1.0 / o->tau : o->S[k]; }

static void strain_node(const orc *o, const double *hi, const double *heq, const double *Fi, double S[6]) {
  for (int a = 0; a < 6; a++) S[a] = 0.0;
  if (o->D == 2) {
    const double se = rate_of_row(o, 1), sn = rate_of_row(o, 7), sc = rate_of_row(o, 8);
    double me = 0.0, mn = 0.0, mc = 0.0, pe = 0.0, pn = 0.0, pc = 0.0;
    for (int i = 0; i < o->Q; i++) {
      const double ex = o->e[i][0], ey = o->e[i][1];
      const double re = 3.0 * (ex * ex + ey * ey) - 4.0, rn = ex * ex - ey * ey, rc = ex * ey;
      me += re * (hi[i] - heq[i]);
      mn += rn * (hi[i] - heq[i]);
      mc += rc * (hi[i] - heq[i]);
      pe += re * Fi[i];
      pn += rn * Fi[i];
      pc += rc * Fi[i];
    }
    pe *= 1.0 - 0.5 * se;
    pn *= 1.0 - 0.5 * sn;
    pc *= 1.0 - 0.5 * sc;
    const double fe = (se / (2.0 - se)) * pe, fn = (3.0 * sn / (2.0 - sn)) * pn;
    S[0] = -se / 4.0 * me - 3.0 * sn / 4.0 * mn - 0.25 * (fe + fn);  /* Eq. 19a */
    S[1] = -se / 4.0 * me + 3.0 * sn / 4.0 * mn - 0.25 * (fe - fn);  /* Eq. 19b */
    S[3] = -3.0 * sc / 2.0 * mc - 0.5 * (3.0 * sc / (2.0 - sc)) * pc; /* Eq. 19c */
    return;
  }
  /* D3Q19: rows T, P, W, xy, yz, xz and their rates (R4 row indices 1, 9, 11, 13, 14, 15) */
  static const int rows[6] = {1, 9, 11, 13, 14, 15};
  double X[6];
  for (int k = 0; k < 6; k++) {
    double m1 = 0.0, psi = 0.0;
    for (int i = 0; i < o->Q; i++) {
      const double ex = o->e[i][0], ey = o->e[i][1], ez = o->e[i][2];
      double r;
      switch (k) {
        case 0: r = ex * ex + ey * ey + ez * ez; break;
        case 1: r = 3.0 * ex * ex - (ex * ex + ey * ey + ez * ez); break;
        case 2: r = ey * ey - ez * ez; break;
        case 3: r = ex * ey; break;
        case 4: r = ey * ez; break;
        default: r = ex * ez; break;
      }
      m1 += r * (hi[i] - heq[i]);
      psi += r * Fi[i];
    }
    const double s = rate_of_row(o, rows[k]);
    psi *= 1.0 - 0.5 * s;
    /* 2 c_s^2 = 2/3: row k of s = -(3 s / 2) m1 - (3 / 2) (s / (2 - s)) psi */
    X[k] = -1.5 * s * m1 - 1.5 * (s / (2.0 - s)) * psi;
  }
  /* T = sxx + syy + szz, P = 2 sxx - syy - szz, W = syy - szz */
  const double sxx = (X[0] + X[1]) / 3.0, rest = (2.0 * X[0] - X[1]) / 3.0;
  S[0] = sxx;
  S[1] = 0.5 * (rest + X[2]);
  S[2] = 0.5 * (rest - X[2]);
  S[3] = X[3];
  S[4] = X[4];
  S[5] = X[5];
}

/* Collision of every fluid node (Eq. 1 or Eq. 3 with the forcing of Sec.
 * 2.1), from the moments rho (and drho = rho - 1) and j of the stored
 * populations; hi and heq below are f and f_eq in the literal form, h and
 * h_eq = f_eq - w in the deviation form. */
static void collide(orc *o, const double *rhoa, const double *drho, const double *j, const double *Ftot) {
  int Q = o->Q;
  long N = o->N;
#pragma omp parallel for num_threads(o->nthreads) schedule(static)
  for (long n = 0; n < N; n++) {
    if (o->excl[n]) continue;
    double hi[QMAX], heq[QMAX], Fi[QMAX], u[3], F[3];
    double rho = rhoa[n];
    for (int i = 0; i < Q; i++) hi[i] = o->f[(long)i * N + n];
    for (int a = 0; a < 3; a++) F[a] = Ftot[a * N + n];
    for (int a = 0; a < 3; a++) u[a] = (j[a * N + n] + 0.5 * F[a]) / rho;
    if (o->literal) feq_all(o, rho, u, heq);
    else heq_all(o, drho[n], u, heq);
    guo_all(o, u, F, Fi);
    if (o->collision == 0) {
      /* Eq. 1 with F_i = (1 - 1/(2 tau)) F_hat_i */
      for (int i = 0; i < Q; i++)
        o->fpost[(long)i * N + n] = hi[i] - (hi[i] - heq[i]) / o->tau + (1.0 - 0.5 / o->tau) * Fi[i];
    } else {
      /* Eq. 3: f + [-M^-1 S (m - m_eq) + M^-1 Psi], Psi = (I - S/2) M F_hat */
      double m[QMAX], meq[QMAX], mF[QMAX], dm[QMAX];
      for (int k = 0; k < Q; k++) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int i = 0; i < Q; i++) {
          a += o->M[k][i] * hi[i];
          b += o->M[k][i] * heq[i];
          c += o->M[k][i] * Fi[i];
        }
        m[k] = a;
        meq[k] = b;
        mF[k] = c;
      }
      for (int k = 0; k < Q; k++) dm[k] = -o->S[k] * (m[k] - meq[k]) + (1.0 - 0.5 * o->S[k]) * mF[k];
      for (int i = 0; i < Q; i++) {
        double s = 0.0;
        for (int k = 0; k < Q; k++) s += o->Minv[i][k] * dm[k];
        o->fpost[(long)i * N + n] = hi[i] + s;
      }
    }
    o->rho_out[n] = rho;
    for (int a = 0; a < 3; a++) o->u_out[a * N + n] = u[a];
    double S[6];
    strain_node(o, hi, heq, Fi, S);
    for (int a = 0; a < 6; a++) o->strain_out[a * N + n] = S[a];
  }
}

static void solid_node_output(orc *o) {
  for (long n = 0; n < o->N; n++) {
    o->type_out[n] = o->excl[n] ? 1 : (o->inside[n] ? 2 : 0);
    if (!o->excl[n]) continue;
    int x, y, z;
    coords_of(o, n, &x, &y, &z);
    const solid_t *s = &o->sol[o->owner[n]];
    double r[3], uw[3];
    lever(o, s, (double)x, (double)y, (double)z, r);
    wall_velocity(s, r, uw);
    o->rho_out[n] = 0.0;
    for (int a = 0; a < 3; a++) o->u_out[a * o->N + n] = uw[a];
    for (int a = 0; a < 6; a++) o->strain_out[a * o->N + n] = 0.0;
  }
}

static void push_history(orc *o) {
  long need = (o->hist_len + 1) * 6 * (o->nsolid > 0 ? o->nsolid : 1);
  if (need > o->hist_cap) {
    o->hist_cap = need * 2 + 64;
    o->hist = (double *)realloc(o->hist, sizeof(double) * o->hist_cap);
  }
  for (int k = 0; k < 6 * o->nsolid; k++) o->hist[o->hist_len * 6 * o->nsolid + k] = o->FT[k];
  o->hist_len++;
}

/* Advance moving IBB solids to t+1, reclassify, refill the nodes uncovered
 * this step and rebuild the links (Sec. 3.2 needs a refill; its scheme is not
 * given there).  Refill: f = f_eq(rho_bar, u_w(x)) where rho_bar is the mean
 * density, at t+1, of the neighbours x + e_i that are fluid both before and
 * after the move (1 if there is none).  Covered nodes are dropped.  The
 * position is recomputed as Y0 + t U (never accumulated) and wrapped to the
 * box. */
/* Free solid, Eq. 20 with the fluid density rho_f = rho0 = 1 and no
 * interaction force: explicit in the force and torque F, T of the step just
 * taken (Eq. 17, on the solid),
 *   rho_p V_p (v^{n+1} - v^n) = F + (rho_p - 1) V_p g,
 *   I_p (w^{n+1} - w^n) = T,
 *   Y^{n+1} = Y^n + (v^n + v^{n+1}) / 2     (dt = 1),
 * the position wrapped into the box.  With interpolated bounce-back there is
 * no fluid inside the solid, so none of the inner-fluid terms of Eq. 21-24
 * enter.  Sphere: V_p = 4 pi R^3 / 3, I_p = 2 rho_p V_p R^2 / 5; cylinder
 * (D2Q9, per unit depth): V_p = pi R^2, I_p = rho_p V_p R^2 / 2, rotation
 * about z only. */
static double wrap_pos(double y, int L) {
  if (y >= 0.0 && y < (double)L) return y;
  y = fmod(y, (double)L);
  if (y < 0.0) y += (double)L;
  return y;
}

/* With the IBM the fluid fills the solid, and the update is Feng &
 * Michaelides's discretisation, Eq. 23, with rho_f = 1 and dt = 1:
 *   rho_p V_p (v^{n+1} - v^n) = V_p (v^n - v^{n-1}) + F + (rho_p - 1) V_p g,
 *   I_p (w^{n+1} - w^n) = (I_p / rho_p) (w^n - w^{n-1}) + T,
 * F, T being the IBM force and torque of the step (-sum F_l dV_l and
 * -sum (X_l - Y) x F_l dV_l); the position as above.  At the first step
 * v^{n-1} = v^n (the solid moved steadily before).  With Kempe's treatment
 * (Eq. 24-26, orc_set_ibm_inner(o, 1)) the inner-fluid terms are the change
 * over the step of I = sum alpha u and L = sum alpha r x u (u of the
 * collision, h = 1):
 *   rho_p V_p (v^{n+1} - v^n) = (I^n - I^{n-1}) + F + (rho_p - 1) V_p g,
 *   I_p (w^{n+1} - w^n) = (L^n - L^{n-1}) + T,
 * with I^{-1} = I^0 at the first step. */
static void advance_free(orc *o, int k) {
  solid_t *s = &o->sol[k];
  const double *F = &o->FT[6 * k], *T = &o->FT[6 * k + 3];
  const double m = s->rho_p * s->Vp;
  double vn[3], wn[3];
  for (int a = 0; a < 3; a++) {
    if (o->method == M_IBM && o->inner == 1) {
      vn[a] = s->U[a] + ((s->Ik[a] - s->Ikp[a]) + F[a] + (s->rho_p - 1.0) * s->Vp * s->grav[a]) / m;
      wn[a] = s->W[a] + ((s->Ik[3 + a] - s->Ikp[3 + a]) + T[a]) / s->Ip;
    } else if (o->method == M_IBM) {
      vn[a] = s->U[a] + (s->Vp * (s->U[a] - s->Up[a]) + F[a] + (s->rho_p - 1.0) * s->Vp * s->grav[a]) / m;
      wn[a] = s->W[a] + (s->Ip / s->rho_p * (s->W[a] - s->Wp[a]) + T[a]) / s->Ip;
    } else {
      vn[a] = s->U[a] + (F[a] + (s->rho_p - 1.0) * s->Vp * s->grav[a]) / m;
      wn[a] = s->W[a] + T[a] / s->Ip;
    }
  }
  if (o->D == 2) {
    vn[2] = 0.0;
    wn[0] = 0.0;
    wn[1] = 0.0;
  }
  for (int a = 0; a < (o->D == 2 ? 2 : 3); a++) {
    s->c[a] = wrap_pos(s->c[a] + 0.5 * (s->U[a] + vn[a]), dims_of(o, a));
    s->disp[a] = s->disp[a] + 0.5 * (s->U[a] + vn[a]);
  }
  for (int a = 0; a < 3; a++) {
    s->Up[a] = s->U[a];
    s->Wp[a] = s->W[a];
    s->U[a] = vn[a];
    s->W[a] = wn[a];
  }
  for (int a = 0; a < 6; a++) s->Ikp[a] = s->Ik[a];
}

static void move_solids(orc *o) {
  int any = 0;
  for (int k = 0; k < o->nsolid; k++) any |= o->sol[k].moving;
  if (!any) return;
  long N = o->N;
  unsigned char *old = (unsigned char *)malloc(N);
  int *old_owner = (int *)malloc(sizeof(int) * N);
  memcpy(old, o->excl, N);
  memcpy(old_owner, o->owner, sizeof(int) * N);
  for (int k = 0; k < o->nsolid; k++) {
    solid_t *s = &o->sol[k];
    if (!s->moving) continue;
    if (s->free) {
      advance_free(o, k);
      continue;
    }
    for (int a = 0; a < 3; a++) {
      int L = dims_of(o, a);
      double y = s->c0[a] + (double)(o->t + 1) * s->U[a];
      y = fmod(y, (double)L);
      if (y < 0.0) y += (double)L;
      s->c[a] = y;
      s->disp[a] = (double)(o->t + 1) * s->U[a];
    }
  }
  classify(o);
  /* covering (R38): a node fluid at t and solid at t+1 takes its momentum,
   * sum_i f_i e_i of the populations that streamed into it, into the solid
   * that now holds it (torque about that solid's centre at t+1) */
  if (o->cover)
    for (long n = 0; n < N; n++) {
      if (old[n] || !o->excl[n] || o->owner[n] < 0) continue;
      int x, y, z;
      coords_of(o, n, &x, &y, &z);
      double m[3] = {0.0, 0.0, 0.0}, r[3];
      for (int i = 0; i < o->Q; i++)
        for (int a = 0; a < 3; a++) m[a] += o->f[(long)i * N + n] * o->e[i][a];
      const int sid = o->owner[n];
      lever(o, &o->sol[sid], (double)x, (double)y, (double)z, r);
      double *cu = &o->cu[6 * sid];
      for (int a = 0; a < 3; a++) cu[a] += m[a];
      cu[3] += r[1] * m[2] - r[2] * m[1];
      cu[4] += r[2] * m[0] - r[0] * m[2];
      cu[5] += r[0] * m[1] - r[1] * m[0];
    }
  for (long n = 0; n < N; n++) {
    if (!(old[n] && !o->excl[n])) continue;
    int x, y, z;
    coords_of(o, n, &x, &y, &z);
    double rs = 0.0;
    int cnt = 0;
    for (int i = 1; i < o->Q; i++) {
      long nb = cell_of(o, x + o->e[i][0], y + o->e[i][1], z + o->e[i][2]);
      if (old[nb] || o->excl[nb]) continue;
      double r = 0.0;
      for (int k = 0; k < o->Q; k++) r += o->f[(long)k * N + nb];
      rs += r;
      cnt++;
    }
    /* mean density of those neighbours (literal form; the deviation form
     * sums h, the mean density minus 1); rho0 = 1 when there is none */
    double drb = cnt ? rs / cnt : (o->literal ? 1.0 : 0.0);
    /* the solid that covered the node at t; its wall velocity at t+1 */
    int sid = old_owner[n];
    double uw[3] = {0.0, 0.0, 0.0}, feq[QMAX];
    if (sid >= 0) {
      double r[3];
      lever(o, &o->sol[sid], (double)x, (double)y, (double)z, r);
      wall_velocity(&o->sol[sid], r, uw);
    }
    if (o->literal) feq_all(o, drb, uw, feq);
    else heq_all(o, drb, uw, feq);
    for (int i = 0; i < o->Q; i++) o->f[(long)i * N + n] = feq[i];
    /* uncovering (R38): the refilled node's momentum rho_bar u_w comes out of
     * the solid that left it */
    if (o->cover && sid >= 0) {
      const double rb = o->literal ? drb : 1.0 + drb;
      double r[3], m[3];
      lever(o, &o->sol[sid], (double)x, (double)y, (double)z, r);
      for (int a = 0; a < 3; a++) m[a] = rb * uw[a];
      double *cu = &o->cu[6 * sid];
      for (int a = 0; a < 3; a++) cu[a] -= m[a];
      cu[3] -= r[1] * m[2] - r[2] * m[1];
      cu[4] -= r[2] * m[0] - r[0] * m[2];
      cu[5] -= r[0] * m[1] - r[1] * m[0];
    }
  }
  free(old);
  free(old_owner);
  build_links(o);
}

static void one_step(orc *o) {
  int Q = o->Q;
  long N = o->N;
  double *drho = (double *)malloc(sizeof(double) * N);
  double *rho = (double *)malloc(sizeof(double) * N);
  double *j = (double *)calloc(3 * N, sizeof(double));
  double *Ft = (double *)calloc(3 * N, sizeof(double));
  /* density and momentum (sums over i of f_i and f_i e_i; the deviation
   * form sums h_i, whose density sum is rho - 1 and whose momentum sum is j,
   * since sum w_i = 1 and sum w_i e_i = 0) */
#pragma omp parallel for num_threads(o->nthreads) schedule(static)
  for (long n = 0; n < N; n++) {
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    if (!o->excl[n])
      for (int i = 0; i < Q; i++) {
        double v = o->f[(long)i * N + n];
        r += v;
        jx += v * o->e[i][0];
        jy += v * o->e[i][1];
        jz += v * o->e[i][2];
      }
    if (o->literal) {
      rho[n] = o->excl[n] ? 1.0 : r;
      drho[n] = rho[n] - 1.0;
    } else {
      drho[n] = r;
      rho[n] = 1.0 + r;
    }
    j[n] = jx;
    j[N + n] = jy;
    j[2 * N + n] = jz;
    int forced = !o->g_fluid_only || !o->inside[n];
    for (int a = 0; a < 3; a++) Ft[a * N + n] = forced ? o->g[a] : 0.0;
  }
  for (int k = 0; k < 6 * o->nsolid; k++) o->FT[k] = 0.0;
  if (o->method == M_IBM && o->nlag > 0) {
    ibm_force(o, rho, j, Ft);
    for (long n = 0; n < 3 * N; n++) Ft[n] += o->fibm[n];
  }
  collide(o, rho, drho, j, Ft);
  solid_node_output(o);
  if (o->method == M_IBM && o->inner == 1)
    for (int k = 0; k < o->nsolid; k++) {
      solid_t *s = &o->sol[k];
      if (!s->free) continue;
      kempe_integrals(o, s, s->Ik);
      if (s->kfirst) {  /* the solid moved steadily before: no change of its inner momentum yet */
        for (int a = 0; a < 6; a++) s->Ikp[a] = s->Ik[a];
        s->kfirst = 0;
      }
    }
  /* streaming (push); every target slot (i, x + e_i) has one source.  At the
   * domain boundaries of Sec. 3.4 (bounded axes only):
   *  - velocity inlet, a plane halfway before x = 0: a population that would
   *    leave through it returns to its node reversed, with the wall term of
   *    Eq. 10 for the inflow velocity (u_w = (Uin, 0, 0), rho0 = 1);
   *  - outflow past the last x layer: the population leaves the domain (the
   *    ones entering there are set by the convective condition below);
   *  - stress-free planes halfway outside the first and last layers of y or z
   *    (or x): specular reflection, the normal component reversed and the
   *    population kept in its layer (zero normal velocity, zero normal
   *    derivative of the tangential velocity). */
  const int nb[3] = {o->nx, o->ny, o->nz};
#pragma omp parallel for num_threads(o->nthreads) schedule(static)
  for (long n = 0; n < N; n++) {
    if (o->excl[n]) continue;
    int x, y, z;
    coords_of(o, n, &x, &y, &z);
    const int c0[3] = {x, y, z};
    for (int i = 0; i < Q; i++) {
      int t[3], j = i;
      for (int a = 0; a < 3; a++) t[a] = c0[a] + o->e[i][a];
      if (o->bc[0] == BC_OPEN && t[0] < 0) {
        const int ib = o->opp[i];
        const double eu = (double)o->e[ib][0] * o->Uin;
        o->fnew[(long)ib * N + n] = o->fpost[(long)i * N + n] + 6.0 * o->w[ib] * eu; /* 2 rho0 w e.u_w / c_s^2 */
        continue;
      }
      if (o->bc[0] == BC_OPEN && t[0] >= o->nx) continue;
      for (int a = 0; a < 3; a++)
        if (o->bc[a] == BC_SLIP && (t[a] < 0 || t[a] >= nb[a])) {
          t[a] = c0[a];
          j = o->mir[a][j];
        }
      const long m = cell_of(o, t[0], t[1], t[2]);
      if (!o->excl[m]) o->fnew[(long)j * N + m] = o->fpost[(long)i * N + n];
    }
  }
  /* interpolated bounce-back and momentum exchange (Eq. 10, 11, 12-14, 16, 17) */
  acc_t *lacc = (acc_t *)calloc(6 * (o->nsolid > 0 ? o->nsolid : 1), sizeof(acc_t));
  double *plain = (double *)calloc(6 * (o->nsolid > 0 ? o->nsolid : 1), sizeof(double));
  for (long l = 0; l < o->nlink; l++) {
    const link_t *lk = &o->links[l];
    int i = lk->dir, ib = o->opp[i];
    long n = lk->cell;
    int x, y, z;
    coords_of(o, n, &x, &y, &z);
    long ff = cell_of(o, x + o->e[i][0], y + o->e[i][1], z + o->e[i][2]);
    long fff = cell_of(o, x + 2 * o->e[i][0], y + 2 * o->e[i][1], z + 2 * o->e[i][2]);
    const solid_t *s = &o->sol[lk->sid];
    double xw[3] = {(double)x - lk->q * o->e[i][0], (double)y - lk->q * o->e[i][1],
                    (double)z - lk->q * o->e[i][2]};
    double r[3], uw[3];
    lever(o, s, xw[0], xw[1], xw[2], r);
    wall_velocity(s, r, uw);
    double eu = o->e[i][0] * uw[0] + o->e[i][1] * uw[1] + o->e[i][2] * uw[2];
    double B = 2.0 * 1.0 * o->w[i] * eu * 3.0; /* 2 rho0 w_i e_i.u_w / c_s^2, rho0 = 1 */
    /* post-collision values at time t that the schemes may use */
    double fb_f = o->fpost[(long)ib * N + n];                          /* f*_ibar(x_f)   */
    double fb_ff = lk->ff_ok ? o->fpost[(long)ib * N + ff] : 0.0;     /* f*_ibar(x_ff)  */
    double fb_fff = lk->fff_ok ? o->fpost[(long)ib * N + fff] : 0.0;  /* f*_ibar(x_fff) */
    double fs_f = o->fpost[(long)i * N + n];                           /* f*_i(x_f)      */
    double fs_ff = lk->ff_ok ? o->fpost[(long)i * N + ff] : 0.0;      /* f*_i(x_ff)     */
    /* Eq. 11b uses f_i(x_ff, t+1) and f_i(x_fff, t+1); with x_ff, x_fff fluid
     * both are streamed values, f*_i(x_f, t) and f*_i(x_ff, t). */
    double fnew;
    if (o->method == M_ZHAO_YONG)  /* f_ibar(x_f, t) before the collision: o->f until step 7 */
      fnew = orc_zhao_yong_value(lk->q, fs_f, o->f[(long)ib * N + n], B);
    else
      fnew = orc_ibb_value(o->method, lk->q, lk->ff_ok, lk->fff_ok, fb_f, fb_ff, fb_fff, fs_f, fs_f, fs_ff, B);
    o->fnew[(long)i * N + n] = fnew;
    /* Eq. 17: F dt = sum [f*_ibar (e_ibar - u_w) - f_i(t+1) (e_i - u_w)].  In
     * the deviation form f = w + h, and with w_ibar = w_i the rest-state part
     * is w_i (e_ibar - e_i) = -2 w_i e_i, the wall velocity cancelling out of
     * it. */
    double dF[3];
    for (int a = 0; a < 3; a++) {
      dF[a] = fb_f * ((double)o->e[ib][a] - uw[a]) - fnew * ((double)o->e[i][a] - uw[a]);
      if (!o->literal) dF[a] -= 2.0 * o->w[i] * (double)o->e[i][a];
    }
    const double dT[3] = {r[1] * dF[2] - r[2] * dF[1], r[2] * dF[0] - r[0] * dF[2], r[0] * dF[1] - r[1] * dF[0]};
    if (o->literal) {
      double *P = &plain[6 * lk->sid];
      for (int a = 0; a < 3; a++) {
        P[a] += dF[a];
        P[3 + a] += dT[a];
      }
    } else {
      acc_t *A = &lacc[6 * lk->sid];
      for (int a = 0; a < 3; a++) {
        acc_add(&A[a], dF[a]);
        acc_add(&A[3 + a], dT[a]);
      }
    }
  }
  if (o->nlink > 0)
    for (int k = 0; k < 6 * o->nsolid; k++) o->FT[k] = o->literal ? plain[k] : acc_get(&lacc[k]);
  free(lacc);
  free(plain);
  /* the momentum the last move of the solids took from and gave to the fluid
   * (nodes covered and uncovered), part of this step's force and torque */
  if (o->cover && o->cu)
    for (int k = 0; k < 6 * o->nsolid; k++) {
      o->FT[k] += o->cu[k];
      o->cu[k] = 0.0;
    }
  /* convective outflow (Sec. 3.4): d(rho0 u)/dt + U_o d(rho0 u)/dx = 0 taken
   * for the populations that enter the last layer from outside, first-order
   * implicit in time and upwind in x:
   *   f_i(N, t+1) = [f_i(N, t) + U_o f_i(N-1, t+1)] / (1 + U_o),
   * U_o the streamwise velocity of the collision at (N, y, z) (not below 0) */
  if (o->bc[0] == BC_OPEN) {
    const int X = o->nx - 1;
    for (int z = 0; z < o->nz; z++)
      for (int y = 0; y < o->ny; y++) {
        const long n = cell_of(o, X, y, z), m = cell_of(o, X - 1, y, z);
        if (o->excl[n]) continue;
        double Uo = o->u_out[n];
        if (Uo < 0.0) Uo = 0.0;
        for (int i = 0; i < Q; i++)
          if (o->e[i][0] < 0)
            o->fnew[(long)i * N + n] = (o->f[(long)i * N + n] + Uo * o->fnew[(long)i * N + m]) / (1.0 + Uo);
      }
  }
#pragma omp parallel for num_threads(o->nthreads) schedule(static)
  for (long n = 0; n < N; n++)
    if (!o->excl[n])
      for (int i = 0; i < Q; i++) o->f[(long)i * N + n] = o->fnew[(long)i * N + n];
  push_history(o);
  move_solids(o);
  o->t++;
  o->stepped = 1;
  free(drho);
  free(rho);
  free(j);
  free(Ft);
}

int orc_step(orc *o, long nsteps) {
  for (long s = 0; s < nsteps; s++) one_step(o);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* accessors                                                                 */
/* ------------------------------------------------------------------------ */
long orc_cells(const orc *o) { return o->N; }
int orc_q(const orc *o) { return o->Q; }
long orc_time(const orc *o) { return o->t; }
/* offset between the stored value and f_i: 0 (literal) or w_i (deviation) */
static double stored_base(const orc *o, int i) { return o->literal ? 0.0 : o->w[i]; }
void orc_get_f(const orc *o, double *f) {
  for (int i = 0; i < o->Q; i++)
    for (long n = 0; n < o->N; n++) f[(long)i * o->N + n] = stored_base(o, i) + o->f[(long)i * o->N + n];
}
void orc_set_f(orc *o, const double *f) {
  for (int i = 0; i < o->Q; i++)
    for (long n = 0; n < o->N; n++) o->f[(long)i * o->N + n] = f[(long)i * o->N + n] - stored_base(o, i);
}
/* the deviations h = f - w */
void orc_get_h(const orc *o, double *h) {
  for (int i = 0; i < o->Q; i++)
    for (long n = 0; n < o->N; n++)
      h[(long)i * o->N + n] = o->literal ? o->f[(long)i * o->N + n] - o->w[i] : o->f[(long)i * o->N + n];
}
void orc_set_h(orc *o, const double *h) {
  for (int i = 0; i < o->Q; i++)
    for (long n = 0; n < o->N; n++)
      o->f[(long)i * o->N + n] = o->literal ? h[(long)i * o->N + n] + o->w[i] : h[(long)i * o->N + n];
}
/* Representation of the stored populations: literal = 1 stores f_i, 0 the
 * deviation h_i = f_i - w_i; the current state is converted. */
void orc_set_form(orc *o, int literal) {
  literal = literal ? 1 : 0;
  if (literal == o->literal) return;
  for (int i = 0; i < o->Q; i++)
    for (long n = 0; n < o->N; n++) o->f[(long)i * o->N + n] += literal ? o->w[i] : -o->w[i];
  o->literal = literal;
}
int orc_form(const orc *o) { return o->literal; }
void orc_set_threads(orc *o, int n) { o->nthreads = n > 0 ? n : 1; }
/* Domain boundaries (Sec. 3.4): per axis 0 periodic, 1 stress-free planes,
 * 2 (x only) velocity inlet Uin before x = 0 and convective outflow at the
 * last layer.  D2Q9 keeps z periodic.  Returns -1 for an invalid set. */
/* Covering / uncovering momentum of moving IBB solids (R38) on (1) or off. */
void orc_set_cover(orc *o, int on) { o->cover = on ? 1 : 0; }
int orc_set_boundaries(orc *o, int bcx, int bcy, int bcz, double Uin) {
  const int b[3] = {bcx, bcy, bcz};
  for (int a = 0; a < 3; a++) {
    if (b[a] < BC_PERIODIC || b[a] > BC_OPEN) return -1;
    if (b[a] == BC_OPEN && a != 0) return -1;
  }
  if (o->D == 2 && bcz != BC_PERIODIC) return -1;
  if (bcx == BC_OPEN && o->nx < 2) return -1;
  for (int a = 0; a < 3; a++) o->bc[a] = b[a];
  o->Uin = Uin;
  return 0;
}
void orc_get_rates(const orc *o, double *S) { memcpy(S, o->S, sizeof(double) * o->Q); }
void orc_get_mrt(const orc *o, double *M, double *Minv) {
  for (int r = 0; r < o->Q; r++)
    for (int c = 0; c < o->Q; c++) {
      M[r * o->Q + c] = o->M[r][c];
      Minv[r * o->Q + c] = o->Minv[r][c];
    }
}
void orc_lattice(const orc *o, int *e, double *w, int *opp) {
  for (int i = 0; i < o->Q; i++) {
    for (int a = 0; a < 3; a++) e[3 * i + a] = o->e[i][a];
    w[i] = o->w[i];
    opp[i] = o->opp[i];
  }
}
void orc_feq(const orc *o, double rho, const double *u, double *feq) { feq_all(o, rho, u, feq); }
void orc_forcing(const orc *o, const double *u, const double *F, double *Fi) { guo_all(o, u, F, Fi); }

/* Post-collision populations of one node (for the collision pins). */
void orc_collide_node(const orc *o, const double *fin, const double *F, double *fout) {
  double hin[QMAX], drho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < o->Q; i++) {
    hin[i] = fin[i] - stored_base(o, i);
    drho += hin[i];
    for (int a = 0; a < 3; a++) j[a] += hin[i] * o->e[i][a];
  }
  double rho = o->literal ? drho : 1.0 + drho;
  if (o->literal) drho = rho - 1.0;
  orc tmp = *o;
  tmp.N = 1;
  tmp.nthreads = 1;
  double hpost[QMAX];
  unsigned char ex = 0;
  double rho_o, u_o[3];
  tmp.f = hin;
  tmp.fpost = hpost;
  tmp.excl = &ex;
  tmp.rho_out = &rho_o;
  tmp.u_out = u_o;
  double Ft[3] = {F[0], F[1], F[2]};
  collide(&tmp, &rho, &drho, j, Ft);
  for (int i = 0; i < o->Q; i++) fout[i] = stored_base(o, i) + hpost[i];
}

/* Strain rate [6][N] (xx, yy, zz, xy, yz, xz) and dissipation rate
 * eps = 2 nu s_ab s_ab (Sec. 3.1, nu of Eq. 2) of the most recent collision;
 * 0 at IBB solid nodes.  -6 before the first step. */
int orc_strain(const orc *o, double *S, double *eps) {
  if (!o->stepped) return -6;
  const double nu = (o->tau - 0.5) / 3.0;
  for (long n = 0; n < o->N; n++) {
    double ss = 0.0;
    for (int a = 0; a < 6; a++) {
      const double v = o->strain_out[a * o->N + n];
      if (S) S[a * o->N + n] = v;
      ss += (a < 3 ? 1.0 : 2.0) * v * v;
    }
    if (eps) eps[n] = 2.0 * nu * ss;
  }
  return 0;
}

void orc_macros(const orc *o, double *rho, double *u, unsigned char *type) {
  if (!o->stepped) {
    for (long n = 0; n < o->N; n++) {
      double r = 0.0, jj[3] = {0.0, 0.0, 0.0};
      for (int i = 0; i < o->Q; i++) {
        double v = o->f[(long)i * o->N + n];
        r += v;
        for (int a = 0; a < 3; a++) jj[a] += v * o->e[i][a];
      }
      const double rr = o->literal ? r : 1.0 + r;
      if (rho) rho[n] = o->excl[n] ? o->rho_out[n] : rr;
      if (u)
        for (int a = 0; a < 3; a++) u[a * o->N + n] = o->excl[n] ? o->u_out[a * o->N + n] : jj[a] / rr;
    }
  } else {
    if (rho) memcpy(rho, o->rho_out, sizeof(double) * o->N);
    if (u) memcpy(u, o->u_out, sizeof(double) * 3 * o->N);
  }
  if (type) memcpy(type, o->type_out, o->N);
}

void orc_force_torque(const orc *o, double *FT) { memcpy(FT, o->FT, sizeof(double) * 6 * o->nsolid); }
long orc_history_len(const orc *o) { return o->hist_len; }
void orc_history(const orc *o, double *out) {
  memcpy(out, o->hist, sizeof(double) * 6 * o->nsolid * o->hist_len);
}
long orc_link_count(const orc *o) { return o->nlink; }
void orc_links(const orc *o, long *cell, int *dir, int *sid, double *q, int *ff_ok, int *fff_ok) {
  for (long l = 0; l < o->nlink; l++) {
    cell[l] = o->links[l].cell;
    dir[l] = o->links[l].dir;
    sid[l] = o->links[l].sid;
    q[l] = o->links[l].q;
    ff_ok[l] = o->links[l].ff_ok;
    fff_ok[l] = o->links[l].fff_ok;
  }
}
void orc_node_flags(const orc *o, unsigned char *excl, unsigned char *inside, int *owner) {
  if (excl) memcpy(excl, o->excl, o->N);
  if (inside) memcpy(inside, o->inside, o->N);
  if (owner) memcpy(owner, o->owner, sizeof(int) * o->N);
}
void orc_ibm_force_field(const orc *o, double *fibm) { memcpy(fibm, o->fibm, sizeof(double) * 3 * o->N); }
void orc_lagrangian_force(const orc *o, double *F) { memcpy(F, o->Flag, sizeof(double) * 3 * o->nlag); }

/* IBM pieces exposed for the interpolation / spreading pins. */
void orc_interpolate(const orc *o, const double *u, double *Ut) { interpolate(o, u, Ut); }
void orc_spread(const orc *o, const double *F, double *f) {
  memset(f, 0, sizeof(double) * 3 * o->N);
  spread(o, F, f);
}
