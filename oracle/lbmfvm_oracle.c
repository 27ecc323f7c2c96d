/*
 * lbmfvm_oracle.c -- plain FP64 CPU oracle for the hybrid lattice-Boltzmann /
 * finite-volume natural-convection method of Li, Yang & Zhang, "Hybrid
 * LBM-FVM and LBM-MCM methods for fluid flow and heat transfer simulation"
 * (arXiv:1908.08386).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table or constant generator with the HIP library: every
 * table below is written out here from the paper.
 *
 * Mode H ("variable split", Sec. 5.1): the LBM gives the velocity on the whole
 * cavity, the FVM gives the temperature on the whole cavity (grid setting 1:
 * one LBM node at the centre of each control volume).  One time step is three
 * plain sweeps over the grid, in the coupling order of Sec. 6.2 (LBM velocity
 * first, then the temperature from that velocity, then the temperature acts
 * on the LBM through the buoyancy force):
 *
 *   1. streaming (Eq 5, left-hand side, in pull form) with half-way
 *      bounce-back at the walls, then the moments rho = sum f (Eq 16) and
 *      rho V = sum e f (Eq 17);
 *   2. explicit conservative finite-volume energy balance of every control
 *      volume (Eq 24 with Phi = T, i.e. Eq 76 / Eq 89), QUICK convection,
 *      central diffusion, on the fresh LBM velocity;
 *   3. BGK collision (Eq 5 relaxing toward Eq 8, relaxation sign as in
 *      Eq 19) plus the buoyancy force of Eq 18 with G from Eq 81 evaluated
 *      with the fresh temperature.
 *
 * Readings where the paper is silent or garbled (they are listed with their
 * reasons in the design notes of the repository):
 *   - relaxation sign of Eq 5 taken from Eq 19: f* = f - (f - f_eq)/tau + F;
 *   - Eq 18 with p = rho c_s^2 and Delta t = 1; no half-force velocity shift;
 *   - G uses a reference temperature T_ref (mid-wall value by default)
 *     instead of the cold-wall value of Eq 81 (the two differ only by a
 *     hydrostatic pressure in the incompressible limit);
 *   - walls are half-way bounce-back, moving walls in the Ladd form with
 *     wall density 1; a link that leaves through a corner takes the south /
 *     north wall's velocity;
 *   - explicit Euler in time, Delta t_FV = Delta t_LBM = 1 (lock-step);
 *   - QUICK uses ghost cells 2 T_w - T_edge (fixed T) or T_edge (adiabatic)
 *     for its far upstream point; u_f >= 0 takes the "from the left" branch;
 *   - wall faces carry no convective flux; a fixed-temperature wall carries
 *     the diffusive flux -alpha (T_edge - T_w) / (1/2).
 *
 * Storage: every field is row-major [j][i], j = 0 the bottom row, i = 0 the
 * west column; distributions are [q][j][i].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- D2Q9 lattice, Eq 4 and Eq 9 (c = 1, c_s^2 = 1/3, Eq 33) ------------
 * direction order used here: 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW,
 * 8 SE.                                                                      */
#define NQ 9
static const int OC_EX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int OC_EY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double OC_W[NQ] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                                1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                                1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OC_OPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* ---- D2Q5 thermal lattice, Eq 22: 0 rest, 1 E, 2 N, 3 W, 4 S ------------- */
#define NQ5 5
static const int OC_EX5[NQ5] = {0, 1, 0, -1, 0};
static const int OC_EY5[NQ5] = {0, 0, 1, 0, -1};
static const double OC_W5[NQ5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0,
                                  1.0 / 6.0};
static const int OC_OPP5[NQ5] = {0, 3, 4, 1, 2};

enum { OC_W_SIDE = 0, OC_E_SIDE = 1, OC_S_SIDE = 2, OC_N_SIDE = 3 };
enum { OC_VEL_NOSLIP = 0, OC_VEL_PERIODIC = 1 };
enum { OC_T_FIXED = 0, OC_T_ADIABATIC = 1, OC_T_PERIODIC = 2 };
enum { OC_CONV_QUICK = 0, OC_CONV_CENTRAL = 1, OC_CONV_UPWIND = 2 };
enum { OC_FIELD_U = 0, OC_FIELD_V = 1, OC_FIELD_T = 2, OC_FIELD_RHO = 3 };

typedef struct {
  int vel;       /* OC_VEL_NOSLIP (wall, may slide tangentially) or periodic */
  double u_wall; /* tangential wall speed (lattice units)                     */
  int thermal;   /* OC_T_FIXED, OC_T_ADIABATIC or OC_T_PERIODIC              */
  double T_wall; /* wall temperature of a fixed-temperature wall            */
} oc_wall;

typedef struct oc_case {
  int nx, ny;
  double nu, tau, alpha, gbeta, T_ref, gx, gy;
  int conv;
  oc_wall wall[4];
  double *f;      /* post-collision populations f*, [q][j][i]           */
  double *f_pre;  /* streamed populations of the current step            */
  double *T;      /* temperature of the last completed step              */
  double *T_new;  /* temperature being computed                          */
  double *rho, *ux, *uy; /* moments of the last streamed state           */
  double *Fx;     /* x-face fluxes, [j][0..nx]                           */
  double *Fy;     /* y-face fluxes, [0..ny][i]                           */
  double *snap_u, *snap_v, *snap_T;
  long steps;
} oc_case;

#define AT(c, a, j, i) ((a)[(size_t)(j) * (size_t)(c)->nx + (size_t)(i)])
#define FQ(c, a, q, j, i)                                                      \
  ((a)[((size_t)(q) * (size_t)(c)->ny + (size_t)(j)) * (size_t)(c)->nx +     \
       (size_t)(i)])

/* ------------------------------------------------------------------------ */
/* pointwise building blocks                                                 */
/* ------------------------------------------------------------------------ */

/* Eq 8 with c_s^2 = 1/3: f_eq_i = rho w_i [1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u] */
void oc_feq(double rho, double ux, double uy, double out[NQ]) {
  double usq = ux * ux + uy * uy;
  for (int q = 0; q < NQ; ++q) {
    double eu = OC_EX[q] * ux + OC_EY[q] * uy;
    out[q] = rho * OC_W[q] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
  }
}

/* Eq 18 with p = rho c_s^2 and Delta t = 1:
 * F_i = G.(e_i - V) f_eq_i / (rho c_s^2)                                     */
void oc_force(double rho, double ux, double uy, double Gx, double Gy,
              double out[NQ]) {
  double feq[NQ];
  oc_feq(rho, ux, uy, feq);
  for (int q = 0; q < NQ; ++q)
    out[q] = 3.0 * ((OC_EX[q] - ux) * Gx + (OC_EY[q] - uy) * Gy) * feq[q] / rho;
}

/* Collision of one node (Eq 5 with the relaxation sign of Eq 19, Eq 8,
 * Eq 18, Eq 81): f_pre are the streamed populations, T the node's fresh
 * temperature; writes the post-collision populations.                       */
void oc_collide_node(const double f_pre[NQ], double T, double tau,
                     double gbeta, double T_ref, double gx, double gy,
                     double f_out[NQ]) {
  double rho = 0.0, mx = 0.0, my = 0.0;
  for (int q = 0; q < NQ; ++q) {
    rho += f_pre[q];
    mx += OC_EX[q] * f_pre[q];
    my += OC_EY[q] * f_pre[q];
  }
  double ux = mx / rho, uy = my / rho;
  double feq[NQ], F[NQ];
  oc_feq(rho, ux, uy, feq);
  /* Eq 81: the buoyancy acceleration points against gravity (-y) and is
   * proportional to the temperature excess over the reference value.      */
  double Gx = gx, Gy = gbeta * (T - T_ref) + gy;
  oc_force(rho, ux, uy, Gx, Gy, F);
  for (int q = 0; q < NQ; ++q)
    f_out[q] = f_pre[q] - (f_pre[q] - feq[q]) / tau + F[q];
}

/* QUICK face value (Leonard's quadratic upstream interpolation): for a face
 * between cells L and R the value is interpolated from the two neighbouring
 * cells and the next cell upstream.                                         */
static double oc_face_value(int conv, double uf, double Tll, double Tl,
                            double Tr, double Trr) {
  if (conv == OC_CONV_CENTRAL) return 0.5 * (Tl + Tr);
  if (conv == OC_CONV_UPWIND) return uf >= 0.0 ? Tl : Tr;
  if (uf >= 0.0) return (6.0 * Tl + 3.0 * Tr - Tll) / 8.0;
  return (6.0 * Tr + 3.0 * Tl - Trr) / 8.0;
}

/* ------------------------------------------------------------------------ */
/* case object                                                               */
/* ------------------------------------------------------------------------ */

static int oc_xper(const oc_case* c) {
  return c->wall[OC_W_SIDE].vel == OC_VEL_PERIODIC;
}
static int oc_yper(const oc_case* c) {
  return c->wall[OC_S_SIDE].vel == OC_VEL_PERIODIC;
}

oc_case* oc_create(int nx, int ny) {
  if (nx < 4 || ny < 4) return NULL;
  oc_case* c = (oc_case*)calloc(1, sizeof(oc_case));
  if (!c) return NULL;
  size_t n = (size_t)nx * (size_t)ny;
  c->nx = nx;
  c->ny = ny;
  c->f = (double*)calloc(NQ * n, sizeof(double));
  c->f_pre = (double*)calloc(NQ * n, sizeof(double));
  c->T = (double*)calloc(n, sizeof(double));
  c->T_new = (double*)calloc(n, sizeof(double));
  c->rho = (double*)calloc(n, sizeof(double));
  c->ux = (double*)calloc(n, sizeof(double));
  c->uy = (double*)calloc(n, sizeof(double));
  c->Fx = (double*)calloc((size_t)ny * (size_t)(nx + 1), sizeof(double));
  c->Fy = (double*)calloc((size_t)(ny + 1) * (size_t)nx, sizeof(double));
  c->snap_u = (double*)calloc(n, sizeof(double));
  c->snap_v = (double*)calloc(n, sizeof(double));
  c->snap_T = (double*)calloc(n, sizeof(double));
  c->tau = 1.0;
  c->conv = OC_CONV_QUICK;
  for (int s = 0; s < 4; ++s) {
    c->wall[s].vel = OC_VEL_NOSLIP;
    c->wall[s].thermal = OC_T_ADIABATIC;
  }
  if (!c->f || !c->f_pre || !c->T || !c->T_new || !c->rho || !c->ux ||
      !c->uy || !c->Fx || !c->Fy || !c->snap_u || !c->snap_v || !c->snap_T) {
    free(c->f); free(c->f_pre); free(c->T); free(c->T_new); free(c->rho);
    free(c->ux); free(c->uy); free(c->Fx); free(c->Fy); free(c->snap_u);
    free(c->snap_v); free(c->snap_T); free(c);
    return NULL;
  }
  return c;
}

void oc_destroy(oc_case* c) {
  if (!c) return;
  free(c->f); free(c->f_pre); free(c->T); free(c->T_new); free(c->rho);
  free(c->ux); free(c->uy); free(c->Fx); free(c->Fy); free(c->snap_u);
  free(c->snap_v); free(c->snap_T); free(c);
}

/* Lattice parameters directly: nu (Eq 15 gives tau = 3 nu + 1/2, Eq 42),
 * alpha, g*beta, reference temperature, extra body force (gx, gy) and the
 * convection scheme.                                                         */
int oc_set_lattice(oc_case* c, double nu, double alpha, double gbeta,
                   double T_ref, double gx, double gy, int conv) {
  if (!(nu > 0.0) || alpha < 0.0) return -1;
  c->nu = nu;
  c->tau = 3.0 * nu + 0.5;
  c->alpha = alpha;
  c->gbeta = gbeta;
  c->T_ref = T_ref;
  c->gx = gx;
  c->gy = gy;
  c->conv = conv;
  return 0;
}

int oc_set_wall(oc_case* c, int side, int vel, double u_wall, int thermal,
                double T_wall) {
  if (side < 0 || side > 3) return -1;
  c->wall[side].vel = vel;
  c->wall[side].u_wall = u_wall;
  c->wall[side].thermal = thermal;
  c->wall[side].T_wall = T_wall;
  return 0;
}

/* Initial state: rho = 1, V = (u0, v0), f* = f_eq(1, V) and T = T0 (NULL
 * means zero).  The residual snapshot starts from this state.               */
int oc_init(oc_case* c, const double* T0, const double* u0, const double* v0) {
  int nx = c->nx, ny = c->ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double u = u0 ? AT(c, u0, j, i) : 0.0;
      double v = v0 ? AT(c, v0, j, i) : 0.0;
      double feq[NQ];
      oc_feq(1.0, u, v, feq);
      for (int q = 0; q < NQ; ++q) FQ(c, c->f, q, j, i) = feq[q];
      AT(c, c->T, j, i) = T0 ? AT(c, T0, j, i) : 0.0;
      AT(c, c->rho, j, i) = 1.0;
      AT(c, c->ux, j, i) = u;
      AT(c, c->uy, j, i) = v;
      AT(c, c->snap_u, j, i) = u;
      AT(c, c->snap_v, j, i) = v;
      AT(c, c->snap_T, j, i) = AT(c, c->T, j, i);
    }
  c->steps = 0;
  return 0;
}

/* ---- sweep 1: pull streaming, bounce-back walls, moments (Eq 5, 16, 17) - */
static void oc_stream_and_moments(oc_case* c) {
  int nx = c->nx, ny = c->ny, xper = oc_xper(c), yper = oc_yper(c);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      double rho = 0.0, mx = 0.0, my = 0.0;
      for (int q = 0; q < NQ; ++q) {
        int si = i - OC_EX[q], sj = j - OC_EY[q];
        if (xper) si = (si + nx) % nx;
        if (yper) sj = (sj + ny) % ny;
        double fq;
        if (si >= 0 && si < nx && sj >= 0 && sj < ny) {
          fq = FQ(c, c->f, q, sj, si);
        } else {
          /* the link crossed a wall half-way: the population that left this
           * node towards the wall comes back reversed; a sliding wall adds
           * 6 w_q (e_q . u_w) (Ladd's form with wall density 1).            */
          int side = sj < 0 ? OC_S_SIDE
                   : sj >= ny ? OC_N_SIDE
                   : si < 0 ? OC_W_SIDE
                            : OC_E_SIDE;
          double uwx = 0.0, uwy = 0.0;
          if (side == OC_S_SIDE || side == OC_N_SIDE)
            uwx = c->wall[side].u_wall;
          else
            uwy = c->wall[side].u_wall;
          fq = FQ(c, c->f, OC_OPP[q], j, i) +
               6.0 * OC_W[q] * (OC_EX[q] * uwx + OC_EY[q] * uwy);
        }
        FQ(c, c->f_pre, q, j, i) = fq;
        rho += fq;
        mx += OC_EX[q] * fq;
        my += OC_EY[q] * fq;
      }
      AT(c, c->rho, j, i) = rho;
      AT(c, c->ux, j, i) = mx / rho;
      AT(c, c->uy, j, i) = my / rho;
    }
  }
}

/* temperature of cell (i, j) where i may lie one cell outside [0, nx):
 * periodic wrap, or the ghost value of the wall's thermal condition         */
static double oc_T_xext(const oc_case* c, const double* T, int i, int j) {
  int nx = c->nx;
  if (oc_xper(c)) return AT(c, T, j, (i + nx) % nx);
  if (i < 0) {
    double te = AT(c, T, j, 0);
    return c->wall[OC_W_SIDE].thermal == OC_T_FIXED
               ? 2.0 * c->wall[OC_W_SIDE].T_wall - te
               : te;
  }
  if (i >= nx) {
    double te = AT(c, T, j, nx - 1);
    return c->wall[OC_E_SIDE].thermal == OC_T_FIXED
               ? 2.0 * c->wall[OC_E_SIDE].T_wall - te
               : te;
  }
  return AT(c, T, j, i);
}

static double oc_T_yext(const oc_case* c, const double* T, int i, int j) {
  int ny = c->ny;
  if (oc_yper(c)) return AT(c, T, (j + ny) % ny, i);
  if (j < 0) {
    double te = AT(c, T, 0, i);
    return c->wall[OC_S_SIDE].thermal == OC_T_FIXED
               ? 2.0 * c->wall[OC_S_SIDE].T_wall - te
               : te;
  }
  if (j >= ny) {
    double te = AT(c, T, ny - 1, i);
    return c->wall[OC_N_SIDE].thermal == OC_T_FIXED
               ? 2.0 * c->wall[OC_N_SIDE].T_wall - te
               : te;
  }
  return AT(c, T, j, i);
}

/* ---- sweep 2: finite-volume energy balance (Eq 24 / Eq 76) -------------
 * Flux through the face between cells L and R (positive from L to R):
 *   F = u_f T_f - alpha (T_R - T_L),
 * u_f = mean of the two cell-centred LBM velocities (grid setting 1 takes
 * face velocities by interpolating the LBM result), T_f by QUICK.  Then
 *   T_new = T - (F_east - F_west) - (F_north - F_south)   (Delta t = 1).    */
static void oc_energy_update(oc_case* c) {
  int nx = c->nx, ny = c->ny, xper = oc_xper(c), yper = oc_yper(c);
  double a = c->alpha;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int fi = 0; fi <= nx; ++fi) {
      double F;
      if (!xper && (fi == 0 || fi == nx)) {
        /* a wall face: no flow through it; a fixed-temperature wall
         * conducts over the half cell between the wall and the centre   */
        int side = fi == 0 ? OC_W_SIDE : OC_E_SIDE;
        F = 0.0;
        if (c->wall[side].thermal == OC_T_FIXED) {
          double Tw = c->wall[side].T_wall;
          F = fi == 0 ? -a * (AT(c, c->T, j, 0) - Tw) / 0.5
                      : -a * (Tw - AT(c, c->T, j, nx - 1)) / 0.5;
        }
      } else {
        int L = fi - 1, R = fi;
        int Lw = (L + nx) % nx, Rw = R % nx;
        double uf = 0.5 * (AT(c, c->ux, j, Lw) + AT(c, c->ux, j, Rw));
        double Tll = oc_T_xext(c, c->T, L - 1, j);
        double Tl = oc_T_xext(c, c->T, L, j);
        double Tr = oc_T_xext(c, c->T, R, j);
        double Trr = oc_T_xext(c, c->T, R + 1, j);
        F = uf * oc_face_value(c->conv, uf, Tll, Tl, Tr, Trr) - a * (Tr - Tl);
      }
      c->Fx[(size_t)j * (size_t)(nx + 1) + (size_t)fi] = F;
    }
  }
#pragma omp parallel for schedule(static)
  for (int fj = 0; fj <= ny; ++fj) {
    for (int i = 0; i < nx; ++i) {
      double F;
      if (!yper && (fj == 0 || fj == ny)) {
        int side = fj == 0 ? OC_S_SIDE : OC_N_SIDE;
        F = 0.0;
        if (c->wall[side].thermal == OC_T_FIXED) {
          double Tw = c->wall[side].T_wall;
          F = fj == 0 ? -a * (AT(c, c->T, 0, i) - Tw) / 0.5
                      : -a * (Tw - AT(c, c->T, ny - 1, i)) / 0.5;
        }
      } else {
        int L = fj - 1, R = fj;
        int Lw = (L + ny) % ny, Rw = R % ny;
        double vf = 0.5 * (AT(c, c->uy, Lw, i) + AT(c, c->uy, Rw, i));
        double Tll = oc_T_yext(c, c->T, i, L - 1);
        double Tl = oc_T_yext(c, c->T, i, L);
        double Tr = oc_T_yext(c, c->T, i, R);
        double Trr = oc_T_yext(c, c->T, i, R + 1);
        F = vf * oc_face_value(c->conv, vf, Tll, Tl, Tr, Trr) - a * (Tr - Tl);
      }
      c->Fy[(size_t)fj * (size_t)nx + (size_t)i] = F;
    }
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double fe = c->Fx[(size_t)j * (size_t)(nx + 1) + (size_t)(i + 1)];
      double fw = c->Fx[(size_t)j * (size_t)(nx + 1) + (size_t)i];
      double fn = c->Fy[(size_t)(j + 1) * (size_t)nx + (size_t)i];
      double fs = c->Fy[(size_t)j * (size_t)nx + (size_t)i];
      AT(c, c->T_new, j, i) = AT(c, c->T, j, i) - (fe - fw) - (fn - fs);
    }
}

/* ---- sweep 3: collision with buoyancy from the fresh temperature -------- */
static void oc_collide(oc_case* c) {
  int nx = c->nx, ny = c->ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double fp[NQ], fo[NQ];
      for (int q = 0; q < NQ; ++q) fp[q] = FQ(c, c->f_pre, q, j, i);
      oc_collide_node(fp, AT(c, c->T_new, j, i), c->tau, c->gbeta, c->T_ref,
                      c->gx, c->gy, fo);
      for (int q = 0; q < NQ; ++q) FQ(c, c->f, q, j, i) = fo[q];
    }
}

int oc_step(oc_case* c, long n) {
  for (long s = 0; s < n; ++s) {
    oc_stream_and_moments(c);
    oc_energy_update(c);
    oc_collide(c);
    double* t = c->T;
    c->T = c->T_new;
    c->T_new = t;
    c->steps++;
  }
  return 0;
}

long oc_steps(const oc_case* c) { return c->steps; }

/* fields after the last step: u, v, rho are the moments of the streamed
 * state (before collision), T the last temperature                          */
int oc_fetch(const oc_case* c, int field, double* out) {
  const double* src = field == OC_FIELD_U   ? c->ux
                    : field == OC_FIELD_V   ? c->uy
                    : field == OC_FIELD_T   ? c->T
                    : field == OC_FIELD_RHO ? c->rho
                                            : NULL;
  if (!src) return -1;
  memcpy(out, src, (size_t)c->nx * (size_t)c->ny * sizeof(double));
  return 0;
}

/* post-collision populations, [q][j][i] */
int oc_fetch_f(const oc_case* c, double* out) {
  memcpy(out, c->f, (size_t)NQ * c->nx * c->ny * sizeof(double));
  return 0;
}

/* relative change since the last snapshot, r = ||phi - phi_snap||_2 /
 * ||phi||_2 for phi = u, v, T (absolute when ||phi|| < 1e-300); the
 * snapshot is then replaced by the current fields                           */
int oc_residual(oc_case* c, double r[3]) {
  const double* cur[3] = {c->ux, c->uy, c->T};
  double* snap[3] = {c->snap_u, c->snap_v, c->snap_T};
  size_t n = (size_t)c->nx * c->ny;
  for (int k = 0; k < 3; ++k) {
    double num = 0.0, den = 0.0;
    for (size_t p = 0; p < n; ++p) {
      double d = cur[k][p] - snap[k][p];
      num += d * d;
      den += cur[k][p] * cur[k][p];
    }
    double norm = sqrt(den);
    r[k] = norm < 1e-300 ? sqrt(num) : sqrt(num) / norm;
    memcpy(snap[k], cur[k], n * sizeof(double));
  }
  return 0;
}

/* Nusselt numbers of the two x-walls (Eq 90 with X = x / H, H = ny):
 * out = {Nu_hot_avg, Nu_cold_avg, Nu_hot_max, Y_hot_max, Nu_cold_max,
 *        Y_cold_max, Nu2_hot_avg, Nu2_cold_avg}.
 * Nu(j) is the conductive flux through the wall face over the half cell,
 * 2 H (T_w - T_edge) / Delta T; Nu2 the second-order one-sided gradient
 * through the wall value and the first two cell centres.  Delta T is the
 * difference of the two wall temperatures (1 when they are equal).         */
int oc_nusselt(const oc_case* c, double out[8]) {
  int nx = c->nx, ny = c->ny;
  double Th = c->wall[OC_W_SIDE].T_wall, Tc = c->wall[OC_E_SIDE].T_wall;
  double dT = Th - Tc;
  if (dT == 0.0) dT = 1.0;
  double H = (double)ny;
  double sh = 0.0, sc = 0.0, sh2 = 0.0, sc2 = 0.0;
  double mh = -INFINITY, mc = -INFINITY;
  int jh = 0, jc = 0;
  for (int j = 0; j < ny; ++j) {
    double t0 = AT(c, c->T, j, 0), t1 = AT(c, c->T, j, 1);
    double tn = AT(c, c->T, j, nx - 1), tm = AT(c, c->T, j, nx - 2);
    double nh = 2.0 * H * (Th - t0) / dT;
    double nc = 2.0 * H * (tn - Tc) / dT;
    double nh2 = H * (8.0 * Th - 9.0 * t0 + t1) / (3.0 * dT);
    double nc2 = H * (9.0 * tn - 8.0 * Tc - tm) / (3.0 * dT);
    sh += nh;
    sc += nc;
    sh2 += nh2;
    sc2 += nc2;
    if (nh > mh) { mh = nh; jh = j; }
    if (nc > mc) { mc = nc; jc = j; }
  }
  out[0] = sh / ny;
  out[1] = sc / ny;
  out[2] = mh;
  out[3] = (jh + 0.5) / ny;
  out[4] = mc;
  out[5] = (jc + 0.5) / ny;
  out[6] = sh2 / ny;
  out[7] = sc2 / ny;
  return 0;
}

/* invariants: total of all post-collision populations, total of T          */
int oc_mass(const oc_case* c, double* sum_f, double* sum_T) {
  size_t n = (size_t)c->nx * c->ny;
  double sf = 0.0, st = 0.0;
  for (size_t p = 0; p < (size_t)NQ * n; ++p) sf += c->f[p];
  for (size_t p = 0; p < n; ++p) st += c->T[p];
  *sum_f = sf;
  *sum_T = st;
  return 0;
}

/* Lattice parameters from the physical groups (Eq 82-89 with Pr = nu /
 * alpha, lattice units Delta x = Delta t = 1, H = ny cells, Delta T = 1):
 *   U_c = characteristic buoyancy velocity in lattice units,
 *   nu = U_c H sqrt(Pr / Ra), alpha = nu / Pr, tau = 3 nu + 1/2 (Eq 15/42),
 *   tau_T = 3 alpha + 1/2 (Eq 20), g beta = U_c^2 / (H Delta T), Ma = U_c/c_s.
 * U_char <= 0 selects the default: 0.1, lowered where the explicit
 * temperature update needs it (alpha <= 0.2, U_c^2 <= 2 alpha) and, when
 * split != 0 (the domain-decomposed mode), where the explicit
 * artificial-compressibility momentum update needs it: its linear
 * amplification stays <= 1 only for nu <= 1/12 (with beta = c_s^2), so
 * nu <= 0.08 is used.
 * out = {U_c, nu, tau, alpha, tau_T, g beta, T_ref, Ma}                      */
int oc_physics_params(double Ra, double Pr, int H, double U_char, int split,
                      double out[8]) {
  if (!(Ra > 0.0) || !(Pr > 0.0) || H < 1) return -1;
  double U = U_char;
  if (!(U > 0.0)) {
    U = 0.1;
    double a = 0.2 * sqrt(Ra * Pr) / H;
    if (a < U) U = a;
    if (split) {
      double b = 0.08 * sqrt(Ra / Pr) / H;
      if (b < U) U = b;
    }
    double d = 2.0 * H / sqrt(Ra * Pr);
    if (d < U) U = d;
  }
  double nu = U * H * sqrt(Pr / Ra);
  double alpha = nu / Pr;
  out[0] = U;
  out[1] = nu;
  out[2] = 3.0 * nu + 0.5;
  out[3] = alpha;
  out[4] = 3.0 * alpha + 0.5;
  out[5] = U * U / (double)H;
  out[6] = 0.0;
  out[7] = U * sqrt(3.0);
  return 0;
}

int oc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* D2Q5 pointwise pieces (Eq 21, Eq 22), used by the domain-decomposed mode */
void oc_geq5(double T, double ux, double uy, double out[NQ5]) {
  for (int q = 0; q < NQ5; ++q)
    out[q] = T * OC_W5[q] * (1.0 + 3.0 * (OC_EX5[q] * ux + OC_EY5[q] * uy));
}

/* keep the D2Q5 tables referenced when the split mode is compiled out */
int oc_d2q5_opp(int q) { return OC_OPP5[q]; }
