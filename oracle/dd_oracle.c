/*
 * dd_oracle.c -- plain FP64 CPU oracle for the domain-decomposed LBM|FVM
 * natural-convection method (Sec. 4 of Li, Yang & Zhang, arXiv:1908.08386),
 * and for the two single-method cavities it is compared against there
 * (pure FVM, pure thermal LBM).
 *
 * TEST INFRASTRUCTURE ONLY; shares no code with the HIP library.
 *
 * Geometry of the split mode (vertical split, Fig 17a): nx even, s = nx/2.
 *   LBM nodes      i = 0 .. ib,      ib = s + 1 (artificial boundary x_b)
 *   FV cells       i = i0 .. nx-1,   i0 = s - 1 (its west face is the FV
 *                                     artificial boundary)
 *   shared columns i0, i0+1, i0+2 = ib (three, as in Sec. 3.2.2 / 4.1.2)
 * One LBM node sits at the centre of each FV cell.
 *
 * LBM zone: D2Q9 BGK flow with buoyancy force (Eq 5, 8, 18, 81) and D2Q5
 * BGK heat (Eq 19-23); half-way bounce-back (f), anti-bounce-back at fixed
 * temperature walls and bounce-back at adiabatic walls (g).
 * FV zone: the incompressible equations of Eq 73-76 on a staggered (MAC)
 * grid (u on x-faces, v on y-faces, p and T at centres), advanced
 * explicitly with the LBM time step (lock-step, Eq 52): momentum with QUICK
 * convection and central diffusion, then an artificial-compressibility
 * pressure update p <- p - c_s^2 div u* (which keeps p comparable with the
 * LBM pressure c_s^2 rho, Eq 91-93), then the energy balance on u*.
 *
 * One step of the split mode (Gauss-Seidel order of the procedure listed at
 * the end of Sec. 3.2.2):
 *   1. FV ghost columns i0-2, i0-1 from the LBM state of the previous step
 *      (face velocities by two-point averages, the analogue of Eq 55-56;
 *      temperatures at coincident centres);
 *   2. FV step;
 *   3. rho0 = mean LBM density (previous step) and p_bar = mean FV pressure
 *      (new) over the three shared columns (Sec. 4.1.2);
 *   4. LBM streaming on nodes 0 .. ib-1; the boundary node x_b gets
 *      rho_b from Eq 93 (its level shifted so that the LBM zone keeps its
 *      mass, see iface_boundary_node), u_b, v_b, T_b from the FV zone and
 *      its populations from non-equilibrium extrapolation (Eq 60 /
 *      Eq 94-95) or from the finite-difference velocity-gradient closure
 *      (Eq 70-72);
 *   5. collision of all LBM nodes.
 * The north wall may slide along +x (the lid-driven cavity of Sec. 3.3,
 * Fig. 5): half-way bounce-back with the moving-wall term in the LBM zone,
 * the ghost u = 2 u_lid - u_edge in the FV zone.
 * Output: LBM values on columns < s, FV values (face velocities averaged
 * to centres) on columns >= s.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q9 9
#define Q5 5
static const int DX9[Q9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int DY9[Q9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9D[Q9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                               1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP9[Q9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const int DX5[Q5] = {0, 1, 0, -1, 0};
static const int DY5[Q5] = {0, 0, 1, 0, -1};
static const double W5D[Q5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0,
                               1.0 / 6.0};
static const int OPP5[Q5] = {0, 3, 4, 1, 2};
static const double CS2D = 1.0 / 3.0;

enum { DD_SPLIT = 0, DD_PURE_FV = 1, DD_PURE_LBM = 2 };
enum { DD_NEQ = 0, DD_FDGRAD = 1 };
enum { SW = 0, SE = 1, SS = 2, SN = 3 };
enum { DD_WALL = 0, DD_PERIODIC = 1 };

typedef struct dd_case {
  int nx, ny, mode, iface;
  int s, i0, ib; /* split column, first FV cell, LBM boundary column */
  int nl;        /* LBM columns 0 .. nl-1                           */
  int c0;        /* first real FV cell                               */
  int nf;        /* stored FV columns c0-2 .. nx (x-face nx included) */
  int xper, yper;
  double nu, alpha, gbeta, T_ref, tau, tauT, gx;
  int tfix[4];
  double Tw[4];
  int gdir; /* buoyancy along +y (0, gravity -y) or along +x (1, gravity -x):
               the horizontally divided cavity of Fig. 17b, stored transposed */
  int conv;
  double ulid;  /* tangential velocity of the north wall (0: at rest)     */
  double excess0; /* split mode: mass of the LBM nodes 0 .. ib-1 over one
                     per node, at init                                    */
  double kp, ki;  /* gains of the level of Eq 93 on the zone's mass deficit
                     and on its running sum                              */
  double integ;   /* running sum of the deficit over the steps           */
  /* LBM zone, [q][j][i] / [j][i] with nl columns */
  double *f, *fpre, *g, *gpre;
  double *rho, *ux, *uy, *TL; /* moments of the last LBM step (pre-collision) */
  /* FV zone: column c is stored at index c - (c0 - 2) for c in c0-2 .. nx;
   * u face x = c at the same index; v face y = jf of column c at [jf][idx]
   * (ny + 1 rows)                                                          */
  double *u, *v, *p, *T, *us, *vs, *Tn;
  double rho0, pbar;
  double *snap[3];
  long steps;
} dd_case;

/* ------------------------------------------------------------------------ */
static double face_val(int conv, double uf, double ll, double l, double r,
                       double rr) {
  if (conv == 1) return 0.5 * (l + r);
  if (conv == 2) return uf >= 0.0 ? l : r;
  if (uf >= 0.0) return (6.0 * l + 3.0 * r - ll) / 8.0;
  return (6.0 * r + 3.0 * l - rr) / 8.0;
}

static void feq9(double rho, double ux, double uy, double out[Q9]) {
  double usq = ux * ux + uy * uy;
  for (int q = 0; q < Q9; ++q) {
    double eu = DX9[q] * ux + DY9[q] * uy;
    out[q] = rho * W9D[q] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
  }
}

/* Eq 21 */
static void geq5(double T, double ux, double uy, double out[Q5]) {
  for (int q = 0; q < Q5; ++q)
    out[q] = T * W5D[q] * (1.0 + 3.0 * (DX5[q] * ux + DY5[q] * uy));
}

/* Eq 93: density of the LBM boundary node from the FV pressure,
 * rho_L = rho0 ((p_S - p_bar) / (rho0 c_s^2) + 1)                          */
double dd_boundary_density(double rho0, double pS, double pbar) {
  return rho0 * ((pS - pbar) / (rho0 * CS2D) + 1.0);
}

/* Populations of the LBM boundary node (kind DD_NEQ or DD_FDGRAD).
 *   NEE (Eq 60 / Eq 94): f_b = f_eq(rho_b, u_b) + f_f - f_eq(rho_f, u_f),
 *     with f_f the streamed populations of the neighbour node x_f;
 *   FD gradient (Eq 70 with rho kept from Eq 69):
 *     f_b = f_eq(rho_b, u_b) - (tau w_i rho_b / c_s^2) Q_i : S,
 *     Q_i = e_i e_i - c_s^2 I, S = sym grad u given as (dudx, dudy, dvdx)
 *     with dv/dy = -du/dx (Eq 72).                                         */
void dd_reconstruct_node(int kind, const double f_f[Q9], double rho_b,
                         double ub, double vb, double tau, double dudx,
                         double dudy, double dvdx, double out[Q9]) {
  double fb[Q9];
  feq9(rho_b, ub, vb, fb);
  if (kind == DD_NEQ) {
    double rf = 0.0, mx = 0.0, my = 0.0;
    for (int q = 0; q < Q9; ++q) {
      rf += f_f[q];
      mx += DX9[q] * f_f[q];
      my += DY9[q] * f_f[q];
    }
    double ff[Q9];
    feq9(rf, mx / rf, my / rf, ff);
    for (int q = 0; q < Q9; ++q) out[q] = fb[q] + f_f[q] - ff[q];
  } else {
    double Sxx = dudx, Syy = -dudx, Sxy = 0.5 * (dudy + dvdx);
    for (int q = 0; q < Q9; ++q) {
      double QS = (DX9[q] * DX9[q] - CS2D) * Sxx + 2.0 * DX9[q] * DY9[q] * Sxy +
                  (DY9[q] * DY9[q] - CS2D) * Syy;
      out[q] = fb[q] - tau * W9D[q] * rho_b / CS2D * QS;
    }
  }
}

/* ------------------------------------------------------------------------ */
#define LIDX(c, j) ((size_t)(j) * (size_t)(c)->nl)
#define FL(c, a, q, j, i) \
  ((a)[((size_t)(q) * (size_t)(c)->ny + (size_t)(j)) * (size_t)(c)->nl + (size_t)(i)])
#define LN(c, a, j, i) ((a)[(size_t)(j) * (size_t)(c)->nl + (size_t)(i)])
/* FV stored column index of real column x */
#define FX(c, x) ((x) - ((c)->c0 - 2))
#define FC(c, a, j, x) ((a)[(size_t)(j) * (size_t)(c)->nf + (size_t)FX(c, x)])
#define FVF(c, a, jf, x) ((a)[(size_t)(jf) * (size_t)(c)->nf + (size_t)FX(c, x)])

dd_case* dd_create(int nx, int ny, int mode) {
  if (nx < 8 || ny < 4) return NULL;
  if (mode == DD_SPLIT && (nx % 2 || nx < 12)) return NULL;
  dd_case* c = (dd_case*)calloc(1, sizeof(dd_case));
  if (!c) return NULL;
  c->nx = nx;
  c->ny = ny;
  c->mode = mode;
  c->s = nx / 2;
  c->i0 = c->s - 1;
  c->ib = c->s + 1;
  c->nl = mode == DD_SPLIT ? c->ib + 1 : mode == DD_PURE_LBM ? nx : 0;
  c->c0 = mode == DD_SPLIT ? c->i0 : 0;
  c->nf = mode == DD_PURE_LBM ? 0 : nx - c->c0 + 3;
  c->tau = c->tauT = 1.0;
  c->kp = 0.25;
  c->ki = 1.0 / 64.0;
  c->tfix[SW] = c->tfix[SE] = 1;
  c->Tw[SW] = 0.5;
  c->Tw[SE] = -0.5;
  size_t nl = (size_t)c->nl * ny, nf = (size_t)c->nf * (ny + 1);
  int ok = 1;
  if (nl) {
    ok &= !!(c->f = calloc(Q9 * nl, sizeof(double)));
    ok &= !!(c->fpre = calloc(Q9 * nl, sizeof(double)));
    ok &= !!(c->g = calloc(Q5 * nl, sizeof(double)));
    ok &= !!(c->gpre = calloc(Q5 * nl, sizeof(double)));
    ok &= !!(c->rho = calloc(nl, sizeof(double)));
    ok &= !!(c->ux = calloc(nl, sizeof(double)));
    ok &= !!(c->uy = calloc(nl, sizeof(double)));
    ok &= !!(c->TL = calloc(nl, sizeof(double)));
  }
  if (nf) {
    ok &= !!(c->u = calloc(nf, sizeof(double)));
    ok &= !!(c->v = calloc(nf, sizeof(double)));
    ok &= !!(c->p = calloc(nf, sizeof(double)));
    ok &= !!(c->T = calloc(nf, sizeof(double)));
    ok &= !!(c->us = calloc(nf, sizeof(double)));
    ok &= !!(c->vs = calloc(nf, sizeof(double)));
    ok &= !!(c->Tn = calloc(nf, sizeof(double)));
  }
  for (int k = 0; k < 3; ++k)
    ok &= !!(c->snap[k] = calloc((size_t)nx * ny, sizeof(double)));
  if (!ok) {
    /* dd_destroy frees what was allocated */
    extern void dd_destroy(dd_case*);
    dd_destroy(c);
    return NULL;
  }
  return c;
}

void dd_destroy(dd_case* c) {
  if (!c) return;
  free(c->f); free(c->fpre); free(c->g); free(c->gpre); free(c->rho);
  free(c->ux); free(c->uy); free(c->TL); free(c->u); free(c->v); free(c->p);
  free(c->T); free(c->us); free(c->vs); free(c->Tn);
  for (int k = 0; k < 3; ++k) free(c->snap[k]);
  free(c);
}

/* nu, alpha (tau = 3 nu + 1/2, tau_T = 3 alpha + 1/2, Eq 15 / Eq 20),
 * g beta, T_ref, body acceleration along x, convection scheme            */
int dd_set_lattice(dd_case* c, double nu, double alpha, double gbeta,
                   double T_ref, double gx, int conv) {
  if (!(nu > 0.0) || !(alpha > 0.0)) return -1;
  c->nu = nu;
  c->alpha = alpha;
  c->tau = 3.0 * nu + 0.5;
  c->tauT = 3.0 * alpha + 0.5;
  c->gbeta = gbeta;
  c->T_ref = T_ref;
  c->gx = gx;
  c->conv = conv;
  return 0;
}

/* side: 0 W, 1 E, 2 S, 3 N; kind DD_WALL (no slip, at rest) or
 * DD_PERIODIC (pure modes only, both sides of the axis); thermal 1 = fixed
 * T_wall, 0 = adiabatic                                                     */
int dd_set_wall(dd_case* c, int side, double unused, int kind_thermal,
                double T_wall) {
  (void)unused;
  if (side < 0 || side > 3) return -1;
  int kind = kind_thermal >> 4, thermal = kind_thermal & 15;
  if (kind == DD_PERIODIC) {
    if (c->mode == DD_SPLIT) return -1;
    if (side < 2) c->xper = 1; else c->yper = 1;
    return 0;
  }
  c->tfix[side] = thermal;
  c->Tw[side] = T_wall;
  return 0;
}

/* ---- FV zone accessors with ghost rules -------------------------------- */
static int fv_has_west_wall(const dd_case* c) {
  return c->mode == DD_PURE_FV && !c->xper;
}

/* u on x-face x (row j may be -2 .. ny+1) */
static double U_at(const dd_case* c, const double* u, int x, int j) {
  int nx = c->nx, ny = c->ny;
  if (c->yper) j = (j + ny) % ny;
  else if (j < 0) return -U_at(c, u, x, -1 - j);       /* no-slip mirror */
  else if (j >= ny) return 2.0 * c->ulid - U_at(c, u, x, 2 * ny - 1 - j);
  if (c->xper) x = ((x % nx) + nx) % nx;
  else if (x > nx) return -U_at(c, u, 2 * nx - x, j); /* through the wall face */
  else if (x < 0 && fv_has_west_wall(c)) return -U_at(c, u, -x, j);
  return FC(c, u, j, x);
}

/* v on y-face jf of column x (jf may be -1 .. ny+1) */
static double V_at(const dd_case* c, const double* v, int x, int jf) {
  int nx = c->nx, ny = c->ny;
  if (c->yper) jf = ((jf % ny) + ny) % ny;
  else if (jf < 0) return -V_at(c, v, x, -jf);
  else if (jf > ny) return -V_at(c, v, x, 2 * ny - jf);
  if (c->xper) x = ((x % nx) + nx) % nx;
  else if (x >= nx) return -V_at(c, v, 2 * nx - 1 - x, jf); /* no-slip mirror */
  else if (x < 0 && fv_has_west_wall(c)) return -V_at(c, v, -1 - x, jf);
  return FVF(c, v, jf, x);
}

/* T at cell (x, j), one ghost layer past walls by the thermal rule */
static double T_at(const dd_case* c, const double* T, int x, int j) {
  int nx = c->nx, ny = c->ny;
  if (c->yper) j = ((j % ny) + ny) % ny;
  else if (j < 0) {
    double te = T_at(c, T, x, 0);
    return c->tfix[SS] ? 2.0 * c->Tw[SS] - te : te;
  } else if (j >= ny) {
    double te = T_at(c, T, x, ny - 1);
    return c->tfix[SN] ? 2.0 * c->Tw[SN] - te : te;
  }
  if (c->xper) x = ((x % nx) + nx) % nx;
  else if (x >= nx) {
    double te = FC(c, T, j, nx - 1);
    return c->tfix[SE] ? 2.0 * c->Tw[SE] - te : te;
  } else if (x < 0 && fv_has_west_wall(c)) {
    double te = FC(c, T, j, 0);
    return c->tfix[SW] ? 2.0 * c->Tw[SW] - te : te;
  }
  return FC(c, T, j, x);
}

static double P_at(const dd_case* c, const double* p, int x, int j) {
  int nx = c->nx, ny = c->ny;
  if (c->yper) j = ((j % ny) + ny) % ny;
  if (c->xper) x = ((x % nx) + nx) % nx;
  return FC(c, p, j, x);
}

/* first and last u face updated by the momentum equation */
static void fv_u_face_range(const dd_case* c, int* lo, int* hi) {
  if (c->xper) { *lo = 0; *hi = c->nx - 1; return; }
  *lo = c->c0 + 1; /* west face is the wall (pure) or prescribed (split) */
  *hi = c->nx - 1;
}

/* ---- FV zone step ------------------------------------------------------ */
static void fv_step(dd_case* c) {
  const int nx = c->nx, ny = c->ny, conv = c->conv;
  const double nu = c->nu, al = c->alpha;
  int ulo, uhi;
  fv_u_face_range(c, &ulo, &uhi);
  const int vlo = c->yper ? 0 : 1, vhi = c->yper ? ny - 1 : ny - 1;
  const int xlo = c->xper ? 0 : c->c0;

  /* u*: momentum on x-faces */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int x = ulo; x <= uhi; ++x) {
      /* x-convection: cell-centre fluxes of cells x-1 and x */
      double Fc[2];
      for (int k = 0; k < 2; ++k) {
        int m = x - 1 + k; /* cell m between faces m and m+1 */
        double ub = 0.5 * (U_at(c, c->u, m, j) + U_at(c, c->u, m + 1, j));
        double uh = face_val(conv, ub, U_at(c, c->u, m - 1, j), U_at(c, c->u, m, j),
                             U_at(c, c->u, m + 1, j), U_at(c, c->u, m + 2, j));
        Fc[k] = ub * uh;
      }
      /* y-convection: corner fluxes at (x, j) and (x, j+1) */
      double Gc[2];
      for (int k = 0; k < 2; ++k) {
        int jf = j + k;
        double vb = 0.5 * (V_at(c, c->v, x - 1, jf) + V_at(c, c->v, x, jf));
        double uh = face_val(conv, vb, U_at(c, c->u, x, jf - 2), U_at(c, c->u, x, jf - 1),
                             U_at(c, c->u, x, jf), U_at(c, c->u, x, jf + 1));
        Gc[k] = vb * uh;
      }
      double uc = U_at(c, c->u, x, j);
      double lap = U_at(c, c->u, x + 1, j) + U_at(c, c->u, x - 1, j) +
                   U_at(c, c->u, x, j + 1) + U_at(c, c->u, x, j - 1) - 4.0 * uc;
      double dp = P_at(c, c->p, x, j) - P_at(c, c->p, x - 1, j);
      FC(c, c->us, j, x) = uc - (Fc[1] - Fc[0]) - (Gc[1] - Gc[0]) + nu * lap - dp + c->gx;
      if (c->gdir) { /* buoyancy on the x-face from the two adjacent cells */
        double Tfx = 0.5 * (T_at(c, c->T, x - 1, j) + T_at(c, c->T, x, j));
        FC(c, c->us, j, x) += c->gbeta * (Tfx - c->T_ref);
      }
    }
    if (!c->xper) {
      FC(c, c->us, j, c->c0) = FC(c, c->u, j, c->c0); /* wall 0 or prescribed */
      FC(c, c->us, j, nx) = 0.0;                      /* stored? see below   */
    }
  }
  /* v*: momentum on y-faces */
#pragma omp parallel for schedule(static)
  for (int jf = vlo; jf <= vhi; ++jf) {
    for (int x = xlo; x < nx; ++x) {
      double Fc[2];
      for (int k = 0; k < 2; ++k) {
        int m = jf - 1 + k; /* cell row m between faces m and m+1 */
        double vb = 0.5 * (V_at(c, c->v, x, m) + V_at(c, c->v, x, m + 1));
        double vh = face_val(conv, vb, V_at(c, c->v, x, m - 1), V_at(c, c->v, x, m),
                             V_at(c, c->v, x, m + 1), V_at(c, c->v, x, m + 2));
        Fc[k] = vb * vh;
      }
      double Gc[2];
      for (int k = 0; k < 2; ++k) {
        int xc = x + k; /* corner at x = xc */
        double ub = 0.5 * (U_at(c, c->u, xc, jf - 1) + U_at(c, c->u, xc, jf));
        double vh = face_val(conv, ub, V_at(c, c->v, xc - 2, jf), V_at(c, c->v, xc - 1, jf),
                             V_at(c, c->v, xc, jf), V_at(c, c->v, xc + 1, jf));
        Gc[k] = ub * vh;
      }
      double vc = V_at(c, c->v, x, jf);
      double lap = V_at(c, c->v, x + 1, jf) + V_at(c, c->v, x - 1, jf) +
                   V_at(c, c->v, x, jf + 1) + V_at(c, c->v, x, jf - 1) - 4.0 * vc;
      double dp = P_at(c, c->p, x, jf) - P_at(c, c->p, x, jf - 1);
      double Tf = 0.5 * (T_at(c, c->T, x, jf - 1) + T_at(c, c->T, x, jf));
      FVF(c, c->vs, jf, x) = vc - (Gc[1] - Gc[0]) - (Fc[1] - Fc[0]) + nu * lap - dp;
      if (!c->gdir) FVF(c, c->vs, jf, x) += c->gbeta * (Tf - c->T_ref);
    }
  }
  if (!c->yper)
    for (int x = xlo; x < nx; ++x) {
      FVF(c, c->vs, 0, x) = 0.0;
      FVF(c, c->vs, ny, x) = 0.0;
    }
  /* pressure: p <- p - c_s^2 div u* (artificial compressibility) */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int x = xlo; x < nx; ++x) {
      double ue = (!c->xper && x == nx - 1) ? 0.0 : U_at(c, c->us, x + 1, j);
      double uw = U_at(c, c->us, x, j);
      double vn = V_at(c, c->vs, x, j + 1), vs = V_at(c, c->vs, x, j);
      FC(c, c->p, j, x) -= CS2D * ((ue - uw) + (vn - vs));
    }
  /* energy on u*, v* (conservative QUICK + central diffusion) */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int x = xlo; x < nx; ++x) {
      double F[2], G[2];
      for (int k = 0; k < 2; ++k) {
        int xf = x + k; /* face between cells xf-1 and xf */
        if (!c->xper && xf == nx) {
          F[k] = c->tfix[SE] ? -al * (c->Tw[SE] - FC(c, c->T, j, nx - 1)) / 0.5 : 0.0;
        } else if (fv_has_west_wall(c) && xf == 0) {
          F[k] = c->tfix[SW] ? -al * (FC(c, c->T, j, 0) - c->Tw[SW]) / 0.5 : 0.0;
        } else {
          double uf = U_at(c, c->us, xf, j);
          double th = face_val(conv, uf, T_at(c, c->T, xf - 2, j), T_at(c, c->T, xf - 1, j),
                               T_at(c, c->T, xf, j), T_at(c, c->T, xf + 1, j));
          F[k] = uf * th - al * (T_at(c, c->T, xf, j) - T_at(c, c->T, xf - 1, j));
        }
        int jf = j + k;
        if (!c->yper && jf == 0) {
          G[k] = c->tfix[SS] ? -al * (FC(c, c->T, 0, x) - c->Tw[SS]) / 0.5 : 0.0;
        } else if (!c->yper && jf == ny) {
          G[k] = c->tfix[SN] ? -al * (c->Tw[SN] - FC(c, c->T, ny - 1, x)) / 0.5 : 0.0;
        } else {
          double vf = V_at(c, c->vs, x, jf);
          double th = face_val(conv, vf, T_at(c, c->T, x, jf - 2), T_at(c, c->T, x, jf - 1),
                               T_at(c, c->T, x, jf), T_at(c, c->T, x, jf + 1));
          G[k] = vf * th - al * (T_at(c, c->T, x, jf) - T_at(c, c->T, x, jf - 1));
        }
      }
      FC(c, c->Tn, j, x) = FC(c, c->T, j, x) - (F[1] - F[0]) - (G[1] - G[0]);
    }
  /* commit: u <- u*, v <- v*, T <- T_new on the zone's own cells/faces */
  for (int j = 0; j < ny; ++j)
    for (int x = xlo; x < nx; ++x) FC(c, c->T, j, x) = FC(c, c->Tn, j, x);
  for (int j = 0; j < ny; ++j)
    for (int x = ulo; x <= uhi; ++x) FC(c, c->u, j, x) = FC(c, c->us, j, x);
  for (int jf = 0; jf <= ny; ++jf)
    for (int x = xlo; x < nx; ++x) FVF(c, c->v, jf, x) = FVF(c, c->vs, jf, x);
}

/* ---- LBM zone step (nodes 0 .. nstream-1 streamed) ---------------------- */
static void lbm_stream(dd_case* c, int nstream) {
  const int nl = c->nl, ny = c->ny;
  const int east_wall = c->mode == DD_PURE_LBM && !c->xper;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nstream; ++i) {
      double r = 0.0, mx = 0.0, my = 0.0, t = 0.0;
      for (int q = 0; q < Q9; ++q) {
        int si = i - DX9[q], sj = j - DY9[q];
        if (c->xper) si = (si + nl) % nl;
        if (c->yper) sj = (sj + ny) % ny;
        int out = sj < 0 || sj >= ny || si < 0 || (east_wall && si >= nl);
        double fq = out ? FL(c, c->f, OPP9[q], j, i) : FL(c, c->f, q, sj, si);
        /* half-way bounce-back from the sliding north wall: the returning
         * population gains 6 w_q (e_q . u_w); a source beyond the north
         * wall counts as that wall also at the two top corners           */
        if (out && !c->yper && sj >= ny) fq += 6.0 * W9D[q] * DX9[q] * c->ulid;
        FL(c, c->fpre, q, j, i) = fq;
        r += fq;
        mx += DX9[q] * fq;
        my += DY9[q] * fq;
      }
      for (int q = 0; q < Q5; ++q) {
        int si = i - DX5[q], sj = j - DY5[q];
        if (c->xper) si = (si + nl) % nl;
        if (c->yper) sj = (sj + ny) % ny;
        int side = sj < 0 ? SS : sj >= ny ? SN : si < 0 ? SW : (east_wall && si >= nl) ? SE : -1;
        double gq;
        if (side < 0) gq = FL(c, c->g, q, sj, si);
        else if (c->tfix[side]) /* anti-bounce-back: fixed temperature */
          gq = -FL(c, c->g, OPP5[q], j, i) + 2.0 * W5D[q] * c->Tw[side];
        else /* bounce-back: zero heat flux */
          gq = FL(c, c->g, OPP5[q], j, i);
        FL(c, c->gpre, q, j, i) = gq;
        t += gq;
      }
      LN(c, c->rho, j, i) = r;
      LN(c, c->ux, j, i) = mx / r;
      LN(c, c->uy, j, i) = my / r;
      LN(c, c->TL, j, i) = t;
    }
}

static void lbm_collide(dd_case* c) {
  const int nl = c->nl, ny = c->ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nl; ++i) {
      double r = LN(c, c->rho, j, i), ux = LN(c, c->ux, j, i), uy = LN(c, c->uy, j, i);
      double t = LN(c, c->TL, j, i);
      double fe[Q9], ge[Q5];
      feq9(r, ux, uy, fe);
      geq5(t, ux, uy, ge);
      double Gx = c->gx, Gy = c->gbeta * (t - c->T_ref);
      if (c->gdir) {
        Gx = c->gx + c->gbeta * (t - c->T_ref);
        Gy = 0.0;
      }
      for (int q = 0; q < Q9; ++q) {
        double F = 3.0 * ((DX9[q] - ux) * Gx + (DY9[q] - uy) * Gy) * fe[q] / r;
        double fp = FL(c, c->fpre, q, j, i);
        FL(c, c->f, q, j, i) = fp - (fp - fe[q]) / c->tau + F;
      }
      for (int q = 0; q < Q5; ++q) {
        double gp = FL(c, c->gpre, q, j, i);
        FL(c, c->g, q, j, i) = gp - (gp - ge[q]) / c->tauT;
      }
    }
}

/* ---- interface ---------------------------------------------------------- */
static void iface_fill_ghosts(dd_case* c) {
  const int ny = c->ny, c0 = c->c0;
  for (int j = 0; j < ny; ++j) {
    /* u faces x = c0-1 and x = c0 from the LBM nodes on either side */
    for (int x = c0 - 1; x <= c0; ++x)
      FC(c, c->u, j, x) = 0.5 * (LN(c, c->ux, j, x - 1) + LN(c, c->ux, j, x));
    /* temperatures of the ghost cells = LBM T at the same centres */
    for (int x = c0 - 2; x <= c0 - 1; ++x) FC(c, c->T, j, x) = LN(c, c->TL, j, x);
  }
  /* global continuity of the FV zone: it is closed on its other three sides,
   * so the prescribed inflow through its artificial boundary must sum to
   * zero; the small net flux of the LBM velocities (which conserve rho u,
   * not u) is removed from that face                                      */
  {
    double m = 0.0;
    for (int j = 0; j < ny; ++j) m += FC(c, c->u, j, c0);
    m /= ny;
    for (int j = 0; j < ny; ++j) FC(c, c->u, j, c0) -= m;
  }
  for (int x = c0 - 2; x <= c0 - 1; ++x) {
    FVF(c, c->v, 0, x) = 0.0;
    FVF(c, c->v, ny, x) = 0.0;
    for (int jf = 1; jf < ny; ++jf)
      FVF(c, c->v, jf, x) = 0.5 * (LN(c, c->uy, jf - 1, x) + LN(c, c->uy, jf, x));
  }
}

/* mean LBM density (previous step) over the three shared columns */
static double iface_rho0(const dd_case* c) {
  double s = 0.0;
  for (int j = 0; j < c->ny; ++j)
    for (int x = c->i0; x <= c->ib; ++x) s += LN(c, c->rho, j, x);
  return s / (3.0 * c->ny);
}

/* mean FV pressure (new) over the three shared columns */
static double iface_pbar(const dd_case* c) {
  double s = 0.0;
  for (int j = 0; j < c->ny; ++j)
    for (int x = c->i0; x <= c->ib; ++x) s += FC(c, c->p, j, x);
  return s / (3.0 * c->ny);
}

static void iface_boundary_node(dd_case* c) {
  const int ny = c->ny, ib = c->ib, xf = ib - 1;
  /* The level of Eq 93.  rho0, the mean LBM density over the shared
   * columns, follows the LBM zone's own level, so nothing holds the zone's
   * mass: the walls conserve it and it changes only through the links to
   * x_b, by whatever small net flux the coupling leaves.  The boundary
   * density is therefore shifted, uniformly over the rows, by kp times the
   * amount e that -- carried by the rest weights of the populations x_b
   * sends into the zone (W, NW, SW; one diagonal fewer on the two wall
   * rows) -- would return the zone's mass (nodes 0 .. ib-1, just streamed)
   * to its value at init, plus ki times the running sum of e over the
   * steps.  The sum can only settle where e = 0, so every steady state
   * holds the zone's mass at its value at init whatever the gains (with
   * kp alone the steady mass would sit off by an amount inversely
   * proportional to kp, and the fields with it).  A whole correction each
   * step overshoots with the finite-difference closure: its boundary
   * populations answer the FV pressure, which answers the shift one step
   * later.  The mass is summed as its excess over one per node: each
   * rho - 1 is exact, so the small deficit does not drown in the rounding
   * of a sum of ones.                                                     */
  double m = 0.0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < ib; ++i) m += LN(c, c->rho, j, i) - 1.0;
  const double wsum = ny * (W9D[3] + W9D[6] + W9D[7]) - W9D[6] - W9D[7];
  const double e = c->excess0 - m;
  c->integ += e;
  const double delta = (c->kp * e + c->ki * c->integ) / wsum;
  for (int j = 0; j < ny; ++j) {
    double ub = 0.5 * (FC(c, c->u, j, ib) + FC(c, c->u, j, ib + 1));
    double vb = 0.5 * (FVF(c, c->v, j, ib) + FVF(c, c->v, j + 1, ib));
    double Tb = FC(c, c->T, j, ib);
    double rb = dd_boundary_density(c->rho0, FC(c, c->p, j, ib), c->pbar) + delta;
    double ff[Q9], fo[Q9];
    for (int q = 0; q < Q9; ++q) ff[q] = FL(c, c->fpre, q, j, xf);
    double dudx = FC(c, c->u, j, ib + 1) - FC(c, c->u, j, ib);
    /* cell-centred u of column ib at rows j-1 and j+1 (no-slip mirror at
     * the walls) and cell-centred v of columns ib-1 and ib+1              */
    double um = j > 0 ? 0.5 * (FC(c, c->u, j - 1, ib) + FC(c, c->u, j - 1, ib + 1)) : -ub;
    double up = j < ny - 1 ? 0.5 * (FC(c, c->u, j + 1, ib) + FC(c, c->u, j + 1, ib + 1))
                           : 2.0 * c->ulid - ub;
    double vw = 0.5 * (FVF(c, c->v, j, ib - 1) + FVF(c, c->v, j + 1, ib - 1));
    double ve = 0.5 * (FVF(c, c->v, j, ib + 1) + FVF(c, c->v, j + 1, ib + 1));
    dd_reconstruct_node(c->iface, ff, rb, ub, vb, c->tau, dudx, 0.5 * (up - um),
                        0.5 * (ve - vw), fo);
    double r = 0.0, mx = 0.0, my = 0.0;
    for (int q = 0; q < Q9; ++q) {
      FL(c, c->fpre, q, j, ib) = fo[q];
      r += fo[q];
      mx += DX9[q] * fo[q];
      my += DY9[q] * fo[q];
    }
    /* g by non-equilibrium extrapolation (Eq 95) */
    double uf = LN(c, c->ux, j, xf), vf = LN(c, c->uy, j, xf), Tf = LN(c, c->TL, j, xf);
    double gb[Q5], gf[Q5];
    geq5(Tb, ub, vb, gb);
    geq5(Tf, uf, vf, gf);
    double t = 0.0;
    for (int q = 0; q < Q5; ++q) {
      double gq = gb[q] + FL(c, c->gpre, q, j, xf) - gf[q];
      FL(c, c->gpre, q, j, ib) = gq;
      t += gq;
    }
    LN(c, c->rho, j, ib) = r;
    LN(c, c->ux, j, ib) = mx / r;
    LN(c, c->uy, j, ib) = my / r;
    LN(c, c->TL, j, ib) = t;
  }
}

/* ------------------------------------------------------------------------ */
/* output fields: LBM on columns < s (all columns in the pure LBM mode), FV
 * elsewhere, velocities at the cell centres                               */
static void dd_output(const dd_case* c, int field, double* out) {
  int nx = c->nx, ny = c->ny;
  int lbm_cols = c->mode == DD_PURE_LBM ? nx : c->mode == DD_PURE_FV ? 0 : c->s;
  for (int j = 0; j < ny; ++j)
    for (int x = 0; x < nx; ++x) {
      double v;
      if (x < lbm_cols) {
        v = field == 0 ? LN(c, c->ux, j, x) : field == 1 ? LN(c, c->uy, j, x)
          : field == 2 ? LN(c, c->TL, j, x) : LN(c, c->rho, j, x);
      } else {
        double ue = (!c->xper && x == nx - 1) ? 0.0 : U_at(c, c->u, x + 1, j);
        v = field == 0 ? 0.5 * (U_at(c, c->u, x, j) + ue)
          : field == 1 ? 0.5 * (V_at(c, c->v, x, j) + V_at(c, c->v, x, j + 1))
          : field == 2 ? FC(c, c->T, j, x) : 1.0 + FC(c, c->p, j, x) / CS2D;
      }
      out[(size_t)j * nx + x] = v;
    }
}

/* mass of the LBM nodes 0 .. ib-1 (split mode) over one per node, from
 * the post-collision populations (summed per node in the streaming's
 * order)                                                                 */
static double zone_excess(const dd_case* c) {
  if (c->mode != DD_SPLIT) return 0.0;
  double m = 0.0;
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->ib; ++i) {
      double r = 0.0;
      for (int q = 0; q < Q9; ++q) r += FL(c, c->f, q, j, i);
      m += r - 1.0;
    }
  return m;
}

/* mass of the LBM nodes 0 .. ib-1 (split mode)                          */
double dd_zone_mass(const dd_case* c) {
  return c->mode == DD_SPLIT ? (double)c->ib * c->ny + zone_excess(c) : 0.0;
}

int dd_init(dd_case* c, const double* T0) {
  int ny = c->ny;
  for (int j = 0; j < ny; ++j)
    for (int x = 0; x < c->nl; ++x) {
      double t = T0 ? T0[(size_t)j * c->nx + x] : 0.0;
      for (int q = 0; q < Q9; ++q) FL(c, c->f, q, j, x) = W9D[q];
      for (int q = 0; q < Q5; ++q) FL(c, c->g, q, j, x) = W5D[q] * t;
      LN(c, c->rho, j, x) = 1.0;
      LN(c, c->ux, j, x) = 0.0;
      LN(c, c->uy, j, x) = 0.0;
      LN(c, c->TL, j, x) = t;
    }
  if (c->nf) {
    size_t nf = (size_t)c->nf * (ny + 1);
    memset(c->u, 0, nf * sizeof(double));
    memset(c->v, 0, nf * sizeof(double));
    memset(c->p, 0, nf * sizeof(double));
    memset(c->T, 0, nf * sizeof(double));
    for (int j = 0; j < ny; ++j)
      for (int x = c->c0 - 2; x < c->nx; ++x)
        if (x >= 0) FC(c, c->T, j, x) = T0 ? T0[(size_t)j * c->nx + x] : 0.0;
  }
  for (int k = 0; k < 3; ++k) dd_output(c, k, c->snap[k]);
  c->excess0 = zone_excess(c);
  c->integ = 0.0;
  c->steps = 0;
  return 0;
}

int dd_step(dd_case* c, long n) {
  for (long k = 0; k < n; ++k) {
    if (c->mode == DD_PURE_FV) {
      fv_step(c);
    } else if (c->mode == DD_PURE_LBM) {
      lbm_stream(c, c->nl);
      lbm_collide(c);
    } else {
      iface_fill_ghosts(c);
      fv_step(c);
      c->rho0 = iface_rho0(c);
      c->pbar = iface_pbar(c);
      lbm_stream(c, c->ib);
      iface_boundary_node(c);
      lbm_collide(c);
    }
    c->steps++;
  }
  return 0;
}

/* field: 0 u, 1 v, 2 T, 3 rho (FV: 1 + p / c_s^2), 4 raw FV p (cells),
 * 5 raw FV u faces ([ny][nx+1]), 6 raw FV v faces ([ny+1][nx])            */
int dd_fetch(const dd_case* c, int field, double* out) {
  int nx = c->nx, ny = c->ny;
  if (field <= 3) {
    dd_output(c, field, out);
    return 0;
  }
  if (!c->nf) return -1;
  int xlo = c->mode == DD_SPLIT ? c->c0 : 0;
  if (field == 4) {
    for (int j = 0; j < ny; ++j)
      for (int x = 0; x < nx; ++x) out[(size_t)j * nx + x] = x >= xlo ? FC(c, c->p, j, x) : 0.0;
  } else if (field == 5) {
    for (int j = 0; j < ny; ++j)
      for (int x = 0; x <= nx; ++x)
        out[(size_t)j * (nx + 1) + x] = (x >= xlo && x < nx) ? FC(c, c->u, j, x) : 0.0;
  } else if (field == 6) {
    for (int jf = 0; jf <= ny; ++jf)
      for (int x = 0; x < nx; ++x) out[(size_t)jf * nx + x] = x >= xlo ? FVF(c, c->v, jf, x) : 0.0;
  } else {
    return -1;
  }
  return 0;
}

int dd_residual(dd_case* c, double r[3]) {
  size_t n = (size_t)c->nx * c->ny;
  double* cur = (double*)malloc(n * sizeof(double));
  if (!cur) return -1;
  for (int k = 0; k < 3; ++k) {
    dd_output(c, k, cur);
    double num = 0.0, den = 0.0;
    for (size_t i = 0; i < n; ++i) {
      double d = cur[i] - c->snap[k][i];
      num += d * d;
      den += cur[i] * cur[i];
    }
    double norm = sqrt(den);
    r[k] = norm < 1e-300 ? sqrt(num) : sqrt(num) / norm;
    memcpy(c->snap[k], cur, n * sizeof(double));
  }
  free(cur);
  return 0;
}

/* Nusselt numbers from the output temperature field (same formulas as the
 * single-cavity oracle): {avg hot, avg cold, max hot, y, max cold, y,
 * 2nd-order hot, 2nd-order cold}                                          */
int dd_nusselt(const dd_case* c, double out[8]) {
  int nx = c->nx, ny = c->ny;
  double* T = (double*)malloc((size_t)nx * ny * sizeof(double));
  if (!T) return -1;
  dd_output(c, 2, T);
  double Th = c->Tw[SW], Tc = c->Tw[SE], dT = Th - Tc;
  if (dT == 0.0) dT = 1.0;
  double H = ny, sh = 0, sc = 0, sh2 = 0, sc2 = 0, mh = -INFINITY, mc = -INFINITY;
  int jh = 0, jc = 0;
  for (int j = 0; j < ny; ++j) {
    double t0 = T[(size_t)j * nx], t1 = T[(size_t)j * nx + 1];
    double tn = T[(size_t)j * nx + nx - 1], tm = T[(size_t)j * nx + nx - 2];
    double nh = 2.0 * H * (Th - t0) / dT, nc = 2.0 * H * (tn - Tc) / dT;
    sh += nh;
    sc += nc;
    sh2 += H * (8.0 * Th - 9.0 * t0 + t1) / (3.0 * dT);
    sc2 += H * (9.0 * tn - 8.0 * Tc - tm) / (3.0 * dT);
    if (nh > mh) { mh = nh; jh = j; }
    if (nc > mc) { mc = nc; jc = j; }
  }
  free(T);
  out[0] = sh / ny; out[1] = sc / ny; out[2] = mh; out[3] = (jh + 0.5) / ny;
  out[4] = mc; out[5] = (jc + 0.5) / ny; out[6] = sh2 / ny; out[7] = sc2 / ny;
  return 0;
}

/* uniform initial velocity for the periodic pure-mode pins */
int dd_init_uniform_flow(dd_case* c, const double* T0, double U, double V) {
  dd_init(c, T0);
  for (int j = 0; j < c->ny; ++j)
    for (int x = 0; x < c->nl; ++x) {
      double fe[Q9];
      feq9(1.0, U, V, fe);
      for (int q = 0; q < Q9; ++q) FL(c, c->f, q, j, x) = fe[q];
      double t = LN(c, c->TL, j, x), ge[Q5];
      geq5(t, U, V, ge);
      for (int q = 0; q < Q5; ++q) FL(c, c->g, q, j, x) = ge[q];
      LN(c, c->ux, j, x) = U;
      LN(c, c->uy, j, x) = V;
    }
  c->excess0 = zone_excess(c);
  c->integ = 0.0;
  return 0;
}

/* set the raw FV state (pins): arrays as in dd_fetch fields 4, 5, 6     */
int dd_set_fv(dd_case* c, const double* p, const double* u, const double* v) {
  if (!c->nf) return -1;
  int nx = c->nx, ny = c->ny, xlo = c->mode == DD_SPLIT ? c->c0 : 0;
  for (int j = 0; j < ny; ++j)
    for (int x = xlo; x < nx; ++x) {
      if (p) FC(c, c->p, j, x) = p[(size_t)j * nx + x];
      if (u) FC(c, c->u, j, x) = u[(size_t)j * (nx + 1) + x];
    }
  if (v)
    for (int jf = 0; jf <= ny; ++jf)
      for (int x = xlo; x < nx; ++x) FVF(c, c->v, jf, x) = v[(size_t)jf * nx + x];
  return 0;
}

int dd_set_iface(dd_case* c, int kind) {
  if (kind != DD_NEQ && kind != DD_FDGRAD) return -1;
  c->iface = kind;
  return 0;
}

int dd_set_gdir(dd_case* c, int gdir) {
  if (gdir < 0 || gdir > 1) return -1;
  c->gdir = gdir;
  return 0;
}

/* tangential velocity of the north wall (lid-driven cavity, Sec. 3.3) */
int dd_set_lid(dd_case* c, double u) {
  if (c->yper) return -1;
  c->ulid = u;
  return 0;
}

long dd_steps(const dd_case* c) { return c->steps; }

int dd_set_level(dd_case* c, double kp, double ki) {
  if (!(kp >= 0.0) || !(ki >= 0.0)) return 1;
  c->kp = kp;
  c->ki = ki;
  return 0;
}
