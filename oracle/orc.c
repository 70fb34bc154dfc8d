/*
 * orc.c -- plain FP64 CPU oracle of the hybrid free-energy lattice Boltzmann
 * timestep of Tiribocchi, Stella, Gonnella and Lamura, "Hybrid lattice
 * Boltzmann model for binary fluid mixtures" (arXiv:0902.3921).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library neither includes nor links it, and it includes nothing of the
 * GPU library.
 *
 * Style: every array is double precision, every loop visits sites in index
 * order idx = x + nx*(y + ny*z), every operation is written the way the paper
 * states it (no fusion, no reordering), and each pass writes a separate
 * output array.  Build with -O2 -ffp-contract=off -fno-fast-math so that no
 * FMA contraction or reassociation changes the rounding.  OpenMP is used only
 * to split the site loops across threads; each site's result does not depend
 * on the thread count, and every reduction is a serial loop.
 *
 * Paper sections referenced below:
 *   Sec. 2            free energy, chemical potential, pressure (Eqs. freenergy, chempot, diagpress)
 *   Sec. 2.1          LB scheme with forcing term (Eqs. evoleqn, espdistrfunc, forceevoleqn,
 *                     newvel, forceterm, coeff, forza, latticeforceterm)
 *   Sec. 2.2          stencils for the force derivatives (Eqs. xstencil, laplstencil)
 *   Sec. 2.3          finite-difference convection-diffusion step (Eqs. adv, centrdiff,
 *                     backdiff, fordiff, diff)
 *
 * Readings where the paper is silent (each one is also a documented choice of
 * the GPU library, so both sides compute the same method):
 *   - one timestep advances both sub-solvers from the state at time t: the
 *     force and u* come from (f_t, phi_t); the LB collide-and-stream gives
 *     f_{t+1}; the m convection-diffusion substeps take phi_t and u*_t (held
 *     fixed over the substeps) to phi_{t+1};
 *   - the lattice is periodic in every direction;
 *   - initial populations are the equilibrium f^eq(n0, u0);
 *   - the three-dimensional case uses the D3Q19 lattice and the 3x3x3
 *     generalisation of the two stencils (faces and edges only);
 *   - the force defaults to the expanded form of phi*grad(mu) that the paper
 *     analyses in Sec. 3, (a phi + 3 b phi^3) grad phi - kappa phi grad(lap phi),
 *     with the mu-first form -phi grad(a phi + b phi^3 - kappa lap phi) as an
 *     option;
 *   - an upwind tie (u = 0) takes the forward difference (the product with u
 *     is zero either way);
 *   - an opt-in flux-form advection conserves sum(phi) exactly;
 *   - the D2Q5 alternative that Sec. 2 mentions (the convection-diffusion
 *     equation on its own five-velocity lattice, the full-LB variant of the
 *     memory comparison) is an option of the D2Q9 case: populations h_i on
 *     c_0 = 0 and the four axis vectors, weights 1/3 and 1/6, with
 *     phi = sum h_i, sum h^eq c = phi u* and sum h^eq c c = Gamma_h mu I,
 *     relaxed with tau_phi and streamed like f; its mobility is
 *     Gamma = Gamma_h (tau_phi - 1/2), so Gamma_h = Gamma / (tau_phi - 1/2).
 */
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Lattices (Sec. 2.1, Fig. 1 and the text around Eq. espdistrfunc).         */
/* D2Q9: e_0 = 0; e_1..e_4 along the axes with |e| = c; e_5..e_8 diagonal   */
/* with |e| = sqrt(2) c; weights 4/9, 1/9, 1/36; c_s^2 = c^2/3 with c = 1.   */
/* D3Q19 (three-dimensional reading): rest 1/3, six faces 1/18, twelve edges */
/* 1/36.                                                                     */
/* ------------------------------------------------------------------------ */
static const int E2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W2[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int E3[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W3[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2 = c^2 / 3 */

/* Number of velocities, velocity table and weights for dimension d. */
int orc_lattice(int d, int *q, int *e_out, double *w_out) {
  int i, k, nq;
  if (d != 2 && d != 3) return -1;
  nq = (d == 2) ? 9 : 19;
  if (q) *q = nq;
  for (i = 0; i < nq; i++) {
    for (k = 0; k < 3; k++)
      if (e_out) e_out[3 * i + k] = (d == 2) ? E2[i][k] : E3[i][k];
    if (w_out) w_out[i] = (d == 2) ? W2[i] : W3[i];
  }
  return 0;
}

static int nvel(int d) { return d == 2 ? 9 : 19; }
static const int *vel(int d, int i) { return d == 2 ? E2[i] : E3[i]; }
static double wgt(int d, int i) { return d == 2 ? W2[i] : W3[i]; }

/* ------------------------------------------------------------------------ */
/* Periodic grid.                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int d, nx, ny, nz;
  long ns;
} grid;

static grid mkgrid(int d, int nx, int ny, int nz) {
  grid g;
  g.d = d;
  g.nx = nx;
  g.ny = ny;
  g.nz = (d == 2) ? 1 : nz;
  g.ns = (long)g.nx * g.ny * g.nz;
  return g;
}

/* periodic wrap of a coordinate that is at most one lattice length outside */
static int wrap(int v, int n) {
  if (v < 0) return v + n;
  if (v >= n) return v - n;
  return v;
}

/* index of the site (x+dx, y+dy, z+dz) on the periodic lattice */
static long site(const grid *g, int x, int y, int z, int dx, int dy, int dz) {
  return (long)wrap(x + dx, g->nx) +
         (long)g->nx * ((long)wrap(y + dy, g->ny) + (long)g->ny * wrap(z + dz, g->nz));
}

/* ------------------------------------------------------------------------ */
/* Stencils (Sec. 2.2, Eqs. xstencil and laplstencil).                      */
/*                                                                          */
/* Gradient along axis a: the weight of neighbour offset o is              */
/* sign(o_a) * N when o has no transverse component and sign(o_a) * M when  */
/* it has exactly one; 2N + 4M = 1 in 2D.  The 3x3 matrix of Eq. xstencil   */
/* is this rule for a = x; the y derivative is its transpose.  In 3D the    */
/* same rule over the 3x3x3 neighbourhood (corners excluded) gives          */
/* consistency 2N + 8M = 1.                                                 */
/*                                                                          */
/* Laplacian: weight Q for the axis neighbours, R for the diagonal          */
/* neighbours, and -(sum of the others) at the centre, i.e. -4(Q+R) in 2D  */
/* as in Eq. laplstencil, with Q + 2R = 1; in 3D, Q for the 6 faces, R for  */
/* the 12 edges, centre -(6Q+12R), Q + 4R = 1.                              */
/* ------------------------------------------------------------------------ */
static double stencil_M(int d, double N) { return d == 2 ? (1.0 - 2.0 * N) / 4.0 : (1.0 - 2.0 * N) / 8.0; }
static double stencil_R(int d, double Q) { return d == 2 ? (1.0 - Q) / 2.0 : (1.0 - Q) / 4.0; }

static double grad_weight(int d, double N, int axis, const int o[3]) {
  int k, transverse = 0;
  double c;
  if (o[axis] == 0) return 0.0;
  for (k = 0; k < 3; k++)
    if (k != axis) transverse += abs(o[k]);
  if (transverse == 0)
    c = N;
  else if (transverse == 1)
    c = stencil_M(d, N);
  else
    c = 0.0;
  return o[axis] > 0 ? c : -c;
}

static double lap_weight(int d, double Q, const int o[3]) {
  int nz = abs(o[0]) + abs(o[1]) + abs(o[2]);
  double R = stencil_R(d, Q);
  if (nz == 1) return Q;
  if (nz == 2) return R;
  if (nz == 3) return 0.0;
  /* centre: minus the sum of the neighbour weights */
  return d == 2 ? -4.0 * (Q + R) : -(6.0 * Q + 12.0 * R);
}

/* Weights of the 3x3(x3) neighbourhood, offset (dx,dy,dz) stored at
 * (dx+1) + 3(dy+1) + 9(dz+1). */
static void grad_table(int d, double N, int axis, double tab[27]) {
  int dx, dy, dz, o[3];
  for (dz = -1; dz <= 1; dz++)
    for (dy = -1; dy <= 1; dy++)
      for (dx = -1; dx <= 1; dx++) {
        o[0] = dx;
        o[1] = dy;
        o[2] = dz;
        tab[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] = (d == 2 && dz != 0) ? 0.0 : grad_weight(d, N, axis, o);
      }
}

static void lap_table(int d, double Q, double tab[27]) {
  int dx, dy, dz, o[3];
  for (dz = -1; dz <= 1; dz++)
    for (dy = -1; dy <= 1; dy++)
      for (dx = -1; dx <= 1; dx++) {
        o[0] = dx;
        o[1] = dy;
        o[2] = dz;
        tab[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] = (d == 2 && dz != 0) ? 0.0 : lap_weight(d, Q, o);
      }
}

/* out = sum over the neighbourhood of tab[offset] * field[r + offset]; offsets
 * with zero weight are skipped.  Terms are added in the order dz, dy, dx. */
static void apply_stencil(const grid *g, const double tab[27], const double *field, double *out) {
  long r;
  int zlo = (g->d == 3) ? -1 : 0, zhi = (g->d == 3) ? 1 : 0;
#pragma omp parallel for schedule(static)
  for (r = 0; r < (long)g->ny * g->nz; r++) {
    int x, dx, dy, dz;
    int y = (int)(r % g->ny), z = (int)(r / g->ny);
    for (x = 0; x < g->nx; x++) {
      double s = 0.0;
      for (dz = zlo; dz <= zhi; dz++)
        for (dy = -1; dy <= 1; dy++)
          for (dx = -1; dx <= 1; dx++) {
            double wv = tab[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)];
            if (wv != 0.0) s += wv * field[site(g, x, y, z, dx, dy, dz)];
          }
      out[site(g, x, y, z, 0, 0, 0)] = s;
    }
  }
}

/* out[axis*ns + idx] = (grad_D field)_axis, axis = 0..d-1 */
static void apply_grad(const grid *g, double N, const double *field, double *out) {
  int a;
  double tab[27];
  for (a = 0; a < g->d; a++) {
    grad_table(g->d, N, a, tab);
    apply_stencil(g, tab, field, out + a * g->ns);
  }
}

static void apply_lap(const grid *g, double Q, const double *field, double *out) {
  double tab[27];
  lap_table(g->d, Q, tab);
  apply_stencil(g, tab, field, out);
}

/* Public stencil entry points (used by the tests' pins). */
int orc_grad(int d, int nx, int ny, int nz, double N, const double *field, double *out) {
  grid g;
  if (d != 2 && d != 3) return -1;
  g = mkgrid(d, nx, ny, nz);
  apply_grad(&g, N, field, out);
  return 0;
}

int orc_lap(int d, int nx, int ny, int nz, double Q, const double *field, double *out) {
  grid g;
  if (d != 2 && d != 3) return -1;
  g = mkgrid(d, nx, ny, nz);
  apply_lap(&g, Q, field, out);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Local equilibrium, Eq. espdistrfunc (u replaced by u* per Sec. 2.1):     */
/*   f_i^eq = w_i n [1 + e_i.u/c_s^2 + u u:(e_i e_i - c_s^2 I)/(2 c_s^4)]   */
/* where u u:(e e - c_s^2 I) = (e.u)^2 - c_s^2 |u|^2.                       */
/* ------------------------------------------------------------------------ */
int orc_feq(int d, double n, const double *u, double *feq) {
  int i, k, nq;
  if (d != 2 && d != 3) return -1;
  nq = nvel(d);
  for (i = 0; i < nq; i++) {
    const int *e = vel(d, i);
    double eu = 0.0, uu = 0.0;
    for (k = 0; k < d; k++) {
      eu += e[k] * u[k];
      uu += u[k] * u[k];
    }
    feq[i] = wgt(d, i) * n * (1.0 + eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2));
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Lattice forcing term, Eq. latticeforceterm (with Delta t_LB = 1):        */
/*   F_i = (1 - 1/(2 tau)) w_i [ (e_i - u*)/c_s^2 + (e_i.u*) e_i / c_s^4 ].F */
/* This is Eq. forceterm with the coefficients A, B, C of Eq. coeff.        */
/* ------------------------------------------------------------------------ */
int orc_source(int d, double tau, const double *u, const double *F, double *S) {
  int i, k, nq;
  if (d != 2 && d != 3) return -1;
  nq = nvel(d);
  for (i = 0; i < nq; i++) {
    const int *e = vel(d, i);
    double eu = 0.0, s = 0.0;
    for (k = 0; k < d; k++) eu += e[k] * u[k];
    for (k = 0; k < d; k++) s += ((e[k] - u[k]) / CS2 + eu * e[k] / (CS2 * CS2)) * F[k];
    S[i] = (1.0 - 1.0 / (2.0 * tau)) * wgt(d, i) * s;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* D2Q5 lattice Boltzmann for the convection-diffusion equation (the        */
/* alternative named in Sec. 2; the paper solves Eq. convdiffeqn by finite  */
/* differences instead).  Velocities c_0 = 0, c_1..c_4 along +x, +y, -x, -y; */
/* weights 1/3 and 1/6, so that sum w c c = c_s^2 I with c_s^2 = 1/3.       */
/* ------------------------------------------------------------------------ */
static const int E5[5][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}};
static const double W5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};

/* Equilibrium whose moments are sum h^eq = phi, sum h^eq c = phi u and
 * sum h^eq c c = Gamma_h mu I (what Eq. convdiffeqn needs at first order):
 *   h_i^eq = w_i (Gamma_h mu + phi c_i.u) / c_s^2   (i = 1..4),
 *   h_0^eq = phi - sum_{i>0} h_i^eq. */
int orc_feq5(double phi, double mu, const double *u, double gamma_h, double *heq) {
  int i;
  double rest = phi;
  for (i = 1; i < 5; i++) {
    double cu = E5[i][0] * u[0] + E5[i][1] * u[1];
    heq[i] = W5[i] * (gamma_h * mu + phi * cu) / CS2;
    rest -= heq[i];
  }
  heq[0] = rest;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Convection-diffusion substeps (Sec. 2.3).                                */
/* ------------------------------------------------------------------------ */

/* Advection half-step, Eq. adv with the differences of Eqs. centrdiff,
 * backdiff and fordiff, applied along every axis:
 *   h = phi - dt [ phi sum_a D_c u_a + sum_a u_a D^up_a phi ]
 *   D_c u_a(r)   = (u_a(r + 1_a) - u_a(r - 1_a)) / 2
 *   D^up_a phi(r) = phi(r) - phi(r - 1_a)  if u_a(r) > 0
 *                 = phi(r + 1_a) - phi(r)  otherwise
 * mode 1 (opt-in, not the paper's): conservative upwind face fluxes
 *   h = phi - dt sum_a (P_a(r + 1/2) - P_a(r - 1/2)),
 *   P_a(r + 1/2) = v phi(r) if v > 0 else v phi(r + 1_a),
 *   v = (u_a(r) + u_a(r + 1_a)) / 2.
 * u holds d components, component a at u[a*ns + idx]. */
static void ch_advect(const grid *g, double dt, int mode, const double *phi, const double *u,
                      double *h) {
  long r;
#pragma omp parallel for schedule(static)
  for (r = 0; r < (long)g->ny * g->nz; r++) {
    int x, a;
    int y = (int)(r % g->ny), z = (int)(r / g->ny);
    for (x = 0; x < g->nx; x++) {
      long idx = site(g, x, y, z, 0, 0, 0);
      double rhs = 0.0;
      for (a = 0; a < g->d; a++) {
        int o[3] = {0, 0, 0};
        long ip, im;
        const double *ua = u + a * g->ns;
        o[a] = 1;
        ip = site(g, x, y, z, o[0], o[1], o[2]);
        im = site(g, x, y, z, -o[0], -o[1], -o[2]);
        if (mode == 0) {
          double dcu = (ua[ip] - ua[im]) / 2.0;
          double dup = (ua[idx] > 0.0) ? (phi[idx] - phi[im]) : (phi[ip] - phi[idx]);
          rhs += phi[idx] * dcu + ua[idx] * dup;
        } else {
          double vp = (ua[idx] + ua[ip]) / 2.0;
          double vm = (ua[im] + ua[idx]) / 2.0;
          double Pp = (vp > 0.0) ? vp * phi[idx] : vp * phi[ip];
          double Pm = (vm > 0.0) ? vm * phi[im] : vm * phi[idx];
          rhs += Pp - Pm;
        }
      }
      h[idx] = phi[idx] - dt * rhs;
    }
  }
}

/* Diffusion step, Eq. diff:
 *   phi' = h + dt Gamma [ a L h + b L (phi^3) - kappa L (L h) ]
 * with phi the value before the advection half-step (f^n = (phi^n)^3) and L
 * the Laplacian stencil with parameter cdQ (cdQ = 1: the standard 5-point /
 * 7-point operator the paper uses). */
static void ch_diffuse(const grid *g, double dt, double gamma, double a, double b, double kappa,
                       double cdQ, const double *h, const double *phi, double *out) {
  long i;
  double *Lh = (double *)malloc(sizeof(double) * g->ns);
  double *cube = (double *)malloc(sizeof(double) * g->ns);
  double *Lcube = (double *)malloc(sizeof(double) * g->ns);
  double *LLh = (double *)malloc(sizeof(double) * g->ns);
#pragma omp parallel for schedule(static)
  for (i = 0; i < g->ns; i++) cube[i] = phi[i] * phi[i] * phi[i];
  apply_lap(g, cdQ, h, Lh);
  apply_lap(g, cdQ, cube, Lcube);
  apply_lap(g, cdQ, Lh, LLh);
#pragma omp parallel for schedule(static)
  for (i = 0; i < g->ns; i++) out[i] = h[i] + dt * gamma * (a * Lh[i] + b * Lcube[i] - kappa * LLh[i]);
  free(Lh);
  free(cube);
  free(Lcube);
  free(LLh);
}

int orc_ch_advect(int d, int nx, int ny, int nz, double dt, int mode, const double *phi,
                  const double *u, double *h) {
  grid g;
  if (d != 2 && d != 3) return -1;
  g = mkgrid(d, nx, ny, nz);
  ch_advect(&g, dt, mode, phi, u, h);
  return 0;
}

int orc_ch_diffuse(int d, int nx, int ny, int nz, double dt, double gamma, double a, double b,
                   double kappa, double cdQ, const double *h, const double *phi, double *out) {
  grid g;
  if (d != 2 && d != 3) return -1;
  g = mkgrid(d, nx, ny, nz);
  ch_diffuse(&g, dt, gamma, a, b, kappa, cdQ, h, phi, out);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Simulation state.                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
  double a, b, kappa, tau, gamma; /* free energy (Eq. freenergy), BGK tau, mobility */
  double N, Q;                    /* force stencil parameters (Eqs. xstencil, laplstencil) */
  double cd_Q;                    /* Laplacian parameter of the convection-diffusion step */
  int m;                          /* FD substeps per LB step, Delta t_LB = m Delta t_FD */
  int force_form;                 /* 1: expanded (a phi + 3 b phi^3) grad phi - kappa phi grad lap phi; 0: phi grad mu */
  int advection;                  /* 0: the paper's Eq. adv; 1: conservative flux form */
  double g[3];                    /* uniform body acceleration: G = n g added to F */
  int cd_model;                   /* 0: finite differences (Sec. 2.3); 1: D2Q5 lattice Boltzmann */
  double tau_phi;                 /* relaxation time of the D2Q5 populations (cd_model 1) */
} orc_params;

typedef struct {
  grid g;
  orc_params p;
  int q;
  double *f;   /* f[i*ns + idx], populations at time t after streaming */
  double *phi; /* order parameter at time t (cd_model 1: sum of h) */
  double *h;   /* cd_model 1: h[i*ns + idx], D2Q5 populations at time t after streaming */
  long long step;
} orc_ctx;

void orc_destroy(orc_ctx *c);

orc_ctx *orc_create(int d, int nx, int ny, int nz, const orc_params *p) {
  orc_ctx *c;
  if ((d != 2 && d != 3) || nx < 1 || ny < 1 || (d == 3 && nz < 1) || !p) return NULL;
  if (p->m < 1) return NULL;
  c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  c->g = mkgrid(d, nx, ny, nz);
  c->p = *p;
  c->q = nvel(d);
  c->f = (double *)calloc((size_t)c->q * c->g.ns, sizeof(double));
  c->phi = (double *)calloc((size_t)c->g.ns, sizeof(double));
  c->h = (double *)calloc((size_t)5 * c->g.ns, sizeof(double));
  if (p->cd_model == 1 && (d != 2 || !(p->tau_phi > 0.5))) {
    orc_destroy(c);
    return NULL;
  }
  return c;
}

void orc_destroy(orc_ctx *c) {
  if (!c) return;
  free(c->f);
  free(c->phi);
  free(c->h);
  free(c);
}

int orc_set_params(orc_ctx *c, const orc_params *p) {
  if (!c || !p || p->m < 1) return -1;
  if (p->cd_model == 1 && (c->g.d != 2 || !(p->tau_phi > 0.5))) return -1;
  c->p = *p;
  return 0;
}

static void d2q5_init(orc_ctx *c, const double *u);

/* f_i = f_i^eq(n0, u0) at every site (initial populations); with the D2Q5
 * convection-diffusion model also h_i = h_i^eq(phi0, mu0, u0). */
int orc_init(orc_ctx *c, const double *phi, const double *n, const double *u) {
  long idx;
  int i, k;
  for (idx = 0; idx < c->g.ns; idx++) {
    double uu[3] = {0, 0, 0}, feq[19];
    for (k = 0; k < c->g.d; k++) uu[k] = u[k * c->g.ns + idx];
    orc_feq(c->g.d, n[idx], uu, feq);
    for (i = 0; i < c->q; i++) c->f[i * c->g.ns + idx] = feq[i];
    c->phi[idx] = phi[idx];
  }
  if (c->p.cd_model == 1) d2q5_init(c, u);
  c->step = 0;
  return 0;
}

int orc_set_state(orc_ctx *c, const double *f, const double *phi) {
  memcpy(c->f, f, sizeof(double) * c->q * c->g.ns);
  memcpy(c->phi, phi, sizeof(double) * c->g.ns);
  return 0;
}

int orc_get_state(const orc_ctx *c, double *f, double *phi) {
  if (f) memcpy(f, c->f, sizeof(double) * c->q * c->g.ns);
  if (phi) memcpy(phi, c->phi, sizeof(double) * c->g.ns);
  return 0;
}

/* Chemical potential with the force stencil, Eq. chempot:
 *   mu = a phi + b phi^3 - kappa lap_D phi.  lap receives lap_D phi. */
static void chem_pot(const grid *g, const orc_params *p, const double *phi, double *lap, double *mu) {
  long i;
  apply_lap(g, p->Q, phi, lap);
#pragma omp parallel for schedule(static)
  for (i = 0; i < g->ns; i++) mu[i] = p->a * phi[i] + p->b * phi[i] * phi[i] * phi[i] - p->kappa * lap[i];
}

/* Density n = sum_i f_i and momentum sum_i f_i e_i at every site (Sec. 2.1). */
static void moments(const orc_ctx *c, double *n, double *j) {
  const grid *g = &c->g;
  long idx;
#pragma omp parallel for schedule(static)
  for (idx = 0; idx < g->ns; idx++) {
    int i, k;
    double s = 0.0, m[3] = {0, 0, 0};
    for (i = 0; i < c->q; i++) {
      double fi = c->f[i * g->ns + idx];
      s += fi;
      for (k = 0; k < g->d; k++) m[k] += fi * vel(g->d, i)[k];
    }
    n[idx] = s;
    for (k = 0; k < g->d; k++) j[k * g->ns + idx] = m[k];
  }
}

/* Force density, Eq. forza: F = -phi grad mu (plus the optional body force
 * G = n g).  Expanded form (default):
 *   F = -[ (a phi + 3 b phi^3) grad_D phi - kappa phi grad_D(lap_D phi) ].
 * mu-first form: F = -phi grad_D mu with mu from chem_pot. */
static void force_density(const orc_ctx *c, const double *n, double *F) {
  const grid *g = &c->g;
  const orc_params *p = &c->p;
  long ns = g->ns, i;
  double *lap = (double *)malloc(sizeof(double) * ns);
  double *mu = (double *)malloc(sizeof(double) * ns);
  double *gphi = (double *)malloc(sizeof(double) * ns * 3);
  double *glap = (double *)malloc(sizeof(double) * ns * 3);
  chem_pot(g, p, c->phi, lap, mu);
  if (p->force_form == 1) {
    apply_grad(g, p->N, c->phi, gphi);
    apply_grad(g, p->N, lap, glap);
#pragma omp parallel for schedule(static)
    for (i = 0; i < ns; i++) {
      int k;
      double ph = c->phi[i];
      double bulk = p->a * ph + 3.0 * p->b * ph * ph * ph;
      for (k = 0; k < g->d; k++) F[k * ns + i] = -(bulk * gphi[k * ns + i] - p->kappa * ph * glap[k * ns + i]);
    }
  } else {
    apply_grad(g, p->N, mu, gphi);
#pragma omp parallel for schedule(static)
    for (i = 0; i < ns; i++) {
      int k;
      for (k = 0; k < g->d; k++) F[k * ns + i] = -c->phi[i] * gphi[k * ns + i];
    }
  }
#pragma omp parallel for schedule(static)
  for (i = 0; i < ns; i++) {
    int k;
    for (k = 0; k < g->d; k++) F[k * ns + i] += n[i] * p->g[k];
  }
  free(lap);
  free(mu);
  free(gphi);
  free(glap);
}

/* Physical velocity, Eq. newvel: n u* = sum_i f_i e_i + F/2 (Delta t_LB = 1). */
static void velocity(const grid *g, const double *n, const double *j, const double *F, double *u) {
  long i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < g->ns; i++) {
    int k;
    for (k = 0; k < g->d; k++) u[k * g->ns + i] = (j[k * g->ns + i] + 0.5 * F[k * g->ns + i]) / n[i];
  }
}

/* Chemical potential of the D2Q5 model: mu = a phi + b phi^3 - kappa L phi
 * with the Laplacian of the convection-diffusion step (cd_Q), as in
 * Eq. diff, so that the two models share their equilibria. */
static void d2q5_mu(const orc_ctx *c, double *mu) {
  const grid *g = &c->g;
  const orc_params *p = &c->p;
  long i;
  double *lap = (double *)malloc(sizeof(double) * g->ns);
  apply_lap(g, p->cd_Q, c->phi, lap);
  for (i = 0; i < g->ns; i++)
    mu[i] = p->a * c->phi[i] + p->b * c->phi[i] * c->phi[i] * c->phi[i] - p->kappa * lap[i];
  free(lap);
}

/* phi = sum_i h_i, summed in the order i = 0..4. */
static void d2q5_phi(orc_ctx *c) {
  long idx;
  int i;
  for (idx = 0; idx < c->g.ns; idx++) {
    double s = 0.0;
    for (i = 0; i < 5; i++) s += c->h[i * c->g.ns + idx];
    c->phi[idx] = s;
  }
}

static void d2q5_init(orc_ctx *c, const double *u) {
  const grid *g = &c->g;
  long idx;
  int i;
  double gamma_h = c->p.gamma / (c->p.tau_phi - 0.5);
  double *mu = (double *)malloc(sizeof(double) * g->ns);
  d2q5_mu(c, mu);
  for (idx = 0; idx < g->ns; idx++) {
    double uu[2] = {u[idx], u[g->ns + idx]}, heq[5];
    orc_feq5(c->phi[idx], mu[idx], uu, gamma_h, heq);
    for (i = 0; i < 5; i++) c->h[i * g->ns + idx] = heq[i];
  }
  free(mu);
  d2q5_phi(c);
}

/* One D2Q5 step with u* of this step: BGK relaxation with tau_phi towards
 * h^eq(phi, mu, u*), then streaming h_i(r + c_i, t + 1) = h_i^post(r). */
static void d2q5_step(orc_ctx *c, const double *u) {
  const grid *g = &c->g;
  const orc_params *p = &c->p;
  long ns = g->ns, idx;
  double gamma_h = p->gamma / (p->tau_phi - 0.5);
  double *mu = (double *)malloc(sizeof(double) * ns);
  double *hnew = (double *)malloc(sizeof(double) * ns * 5);
  d2q5_mu(c, mu);
  for (idx = 0; idx < ns; idx++) {
    int x = (int)(idx % g->nx), y = (int)(idx / g->nx), i;
    double uu[2] = {u[idx], u[ns + idx]}, heq[5];
    orc_feq5(c->phi[idx], mu[idx], uu, gamma_h, heq);
    for (i = 0; i < 5; i++) {
      double hi = c->h[i * ns + idx];
      double post = hi - (hi - heq[i]) / p->tau_phi;
      hnew[i * ns + site(g, x, y, 0, E5[i][0], E5[i][1], 0)] = post;
    }
  }
  memcpy(c->h, hnew, sizeof(double) * ns * 5);
  d2q5_phi(c);
  free(mu);
  free(hnew);
}

int orc_get_h(const orc_ctx *c, double *h) {
  if (!c || c->p.cd_model != 1) return -1;
  memcpy(h, c->h, sizeof(double) * 5 * c->g.ns);
  return 0;
}

/* Sets the D2Q5 populations and phi = sum h. */
int orc_set_h(orc_ctx *c, const double *h) {
  if (!c || c->p.cd_model != 1) return -1;
  memcpy(c->h, h, sizeof(double) * 5 * c->g.ns);
  d2q5_phi(c);
  return 0;
}

/* One timestep t -> t+1. */
static void one_step(orc_ctx *c) {
  const grid *g = &c->g;
  const orc_params *p = &c->p;
  long ns = g->ns, idx;
  int i, k, s;
  double *n = (double *)malloc(sizeof(double) * ns);
  double *j = (double *)malloc(sizeof(double) * ns * 3);
  double *F = (double *)malloc(sizeof(double) * ns * 3);
  double *u = (double *)malloc(sizeof(double) * ns * 3);
  double *fnew = (double *)malloc(sizeof(double) * ns * c->q);
  double *phis = (double *)malloc(sizeof(double) * ns);
  double *h = (double *)malloc(sizeof(double) * ns);
  double *phin = (double *)malloc(sizeof(double) * ns);
  double dt = 1.0 / (double)p->m;

  /* force from phi_t, then n and u* from f_t and F_t */
  moments(c, n, j);
  force_density(c, n, F);
  velocity(g, n, j, F, u);

  /* BGK collision with forcing (Eq. forceevoleqn, f^eq at u*, source from
   * Eq. latticeforceterm), then streaming f_i(r + e_i, t + 1) = f_i^post(r). */
#pragma omp parallel for schedule(static)
  for (idx = 0; idx < ns; idx++) {
    double uu[3] = {0, 0, 0}, FF[3] = {0, 0, 0}, feq[19], S[19];
    int x = (int)(idx % g->nx), y = (int)((idx / g->nx) % g->ny), z = (int)(idx / ((long)g->nx * g->ny));
    int ii, kk;
    for (kk = 0; kk < g->d; kk++) {
      uu[kk] = u[kk * ns + idx];
      FF[kk] = F[kk * ns + idx];
    }
    orc_feq(g->d, n[idx], uu, feq);
    orc_source(g->d, p->tau, uu, FF, S);
    for (ii = 0; ii < c->q; ii++) {
      const int *e = vel(g->d, ii);
      double fi = c->f[ii * ns + idx];
      double post = fi - (fi - feq[ii]) / p->tau + S[ii];
      fnew[ii * ns + site(g, x, y, z, e[0], e[1], e[2])] = post;
    }
  }

  if (p->cd_model == 1) {
    /* the D2Q5 alternative: one lattice Boltzmann step of phi with u*_t */
    d2q5_step(c, u);
  } else {
    /* m convection-diffusion substeps with u*_t held fixed (Sec. 2.3). */
    memcpy(phis, c->phi, sizeof(double) * ns);
    for (s = 0; s < p->m; s++) {
      ch_advect(g, dt, p->advection, phis, u, h);
      ch_diffuse(g, dt, p->gamma, p->a, p->b, p->kappa, p->cd_Q, h, phis, phin);
      memcpy(phis, phin, sizeof(double) * ns);
    }
    memcpy(c->phi, phis, sizeof(double) * ns);
  }

  memcpy(c->f, fnew, sizeof(double) * ns * c->q);
  c->step++;
  (void)i;
  (void)k;
  free(n);
  free(j);
  free(F);
  free(u);
  free(fnew);
  free(phis);
  free(h);
  free(phin);
}

int orc_step(orc_ctx *c, long long nsteps) {
  long long t;
  if (!c || nsteps < 0) return -1;
  for (t = 0; t < nsteps; t++) one_step(c);
  return 0;
}

/* Readout at time t: n = sum f_i, u* from Eq. newvel with F_t, phi, and
 * mu from Eq. chempot with the force stencil.  Any output may be NULL. */
int orc_fields(const orc_ctx *c, double *n_out, double *u_out, double *phi_out, double *mu_out) {
  const grid *g = &c->g;
  long ns = g->ns;
  double *n = (double *)malloc(sizeof(double) * ns);
  double *j = (double *)malloc(sizeof(double) * ns * 3);
  double *F = (double *)malloc(sizeof(double) * ns * 3);
  double *u = (double *)malloc(sizeof(double) * ns * 3);
  double *lap = (double *)malloc(sizeof(double) * ns);
  double *mu = (double *)malloc(sizeof(double) * ns);
  moments(c, n, j);
  force_density(c, n, F);
  velocity(g, n, j, F, u);
  chem_pot(g, &c->p, c->phi, lap, mu);
  if (n_out) memcpy(n_out, n, sizeof(double) * ns);
  if (u_out) memcpy(u_out, u, sizeof(double) * ns * g->d);
  if (phi_out) memcpy(phi_out, c->phi, sizeof(double) * ns);
  if (mu_out) memcpy(mu_out, mu, sizeof(double) * ns);
  free(n);
  free(j);
  free(F);
  free(u);
  free(lap);
  free(mu);
  return 0;
}

/* Global diagnostics at time t, summed serially in index order:
 *   out[0] = sum n, out[1] = sum phi, out[2] = sum n |u*|^2 / 2,
 *   out[3] = max |u*|, out[4..6] = sum n u*_a,
 *   out[7] = 1 if every population and phi is finite, else 0. */
int orc_reduce(const orc_ctx *c, double *out) {
  const grid *g = &c->g;
  long ns = g->ns, i;
  int k;
  double *n = (double *)malloc(sizeof(double) * ns);
  double *u = (double *)malloc(sizeof(double) * ns * 3);
  double mass = 0.0, ps = 0.0, ke = 0.0, umax = 0.0, mom[3] = {0, 0, 0}, finite = 1.0;
  orc_fields(c, n, u, NULL, NULL);
  for (i = 0; i < ns * c->q; i++)
    if (!isfinite(c->f[i])) finite = 0.0;
  for (i = 0; i < ns; i++)
    if (!isfinite(c->phi[i])) finite = 0.0;
  for (i = 0; i < ns; i++) {
    double u2 = 0.0, um;
    for (k = 0; k < g->d; k++) u2 += u[k * ns + i] * u[k * ns + i];
    mass += n[i];
    ps += c->phi[i];
    ke += 0.5 * n[i] * u2;
    um = sqrt(u2);
    if (um > umax) umax = um;
    for (k = 0; k < g->d; k++) mom[k] += n[i] * u[k * ns + i];
  }
  out[0] = mass;
  out[1] = ps;
  out[2] = ke;
  out[3] = umax;
  out[4] = mom[0];
  out[5] = mom[1];
  out[6] = mom[2];
  out[7] = finite;
  free(n);
  free(u);
  return 0;
}

/* Bulk quantities of a drop for Laplace's law (Sec. 2, Eq. surftens):
 * over the sites whose minimum-image distance from `centre` (x, y[, z]) is
 * below r_in (the inside) and above r_out (the outside), the mean density,
 * the mean phi and the mean bulk pressure of Eq. diagpress without its
 * gradient terms, p0 = n c_s^2 + a phi^2 / 2 + 3 b phi^4 / 4; and the
 * equimolar radius, from the volume V = (sum phi - phi_out N) /
 * (phi_in - phi_out) of the phase with phi = phi_in: R = sqrt(V / pi) in
 * 2D, (3 V / (4 pi))^(1/3) in 3D.
 * out[0..2] = p, phi, n inside; out[3..5] = the same outside;
 * out[6] = sum phi; out[7] = R; out[8], out[9] = the site counts. */
int orc_drop_stats(const orc_ctx *c, const double *centre, double r_in, double r_out, double *out) {
  const grid *g = &c->g;
  const orc_params *p = &c->p;
  long ns = g->ns, idx;
  int k;
  double *n = (double *)malloc(sizeof(double) * ns);
  double s_in[3] = {0, 0, 0}, s_out[3] = {0, 0, 0}, phisum = 0.0, c_in = 0.0, c_out = 0.0, V;
  orc_fields(c, n, NULL, NULL, NULL);
  for (idx = 0; idx < ns; idx++) {
    int xyz[3];
    double r2 = 0.0, ph = c->phi[idx], p0;
    xyz[0] = (int)(idx % g->nx);
    xyz[1] = (int)((idx / g->nx) % g->ny);
    xyz[2] = (int)(idx / ((long)g->nx * g->ny));
    for (k = 0; k < g->d; k++) {
      int len = k == 0 ? g->nx : (k == 1 ? g->ny : g->nz);
      double dx = xyz[k] - centre[k];
      dx -= len * floor(dx / len + 0.5); /* minimum image */
      r2 += dx * dx;
    }
    p0 = n[idx] * CS2 + p->a * ph * ph / 2.0 + 3.0 * p->b * ph * ph * ph * ph / 4.0;
    phisum += ph;
    if (r2 < r_in * r_in) {
      s_in[0] += p0;
      s_in[1] += ph;
      s_in[2] += n[idx];
      c_in += 1.0;
    } else if (r2 > r_out * r_out) {
      s_out[0] += p0;
      s_out[1] += ph;
      s_out[2] += n[idx];
      c_out += 1.0;
    }
  }
  for (k = 0; k < 3; k++) {
    out[k] = c_in > 0 ? s_in[k] / c_in : 0.0;
    out[3 + k] = c_out > 0 ? s_out[k] / c_out : 0.0;
  }
  out[6] = phisum;
  V = (phisum - out[4] * (double)ns) / (out[1] - out[4]);
  out[7] = g->d == 2 ? sqrt(V / M_PI) : cbrt(3.0 * V / (4.0 * M_PI));
  out[8] = c_in;
  out[9] = c_out;
  free(n);
  return 0;
}

long long orc_step_count(const orc_ctx *c) { return c->step; }

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
