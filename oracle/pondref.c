/*
 * pondref.c -- FP64 CPU oracle of the Particles-on-Demand (PonD) finite-volume
 * time step, after Kallikounis & Karlin, arXiv 2302.00310.
 *
 * TEST INFRASTRUCTURE ONLY: this file is the reference the GPU library is
 * checked against.  It is deliberately plain: dense Q x Q transform matrices
 * built by solving the moment system, loops over faces and cells in the order
 * of the paper's algorithm summary (Sec. IV A 3), everything in double.  It
 * shares no code with the GPU library.
 *
 * Readings of points the paper leaves open are marked "reading:".
 */
#include "pondref.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static char g_err[256] = "";
static int fail(const char* msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return -1;
}
const char* pondref_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* Lattices: Table I (Gauss--Hermite nodes and weights, T_L = 1).            */
/* ------------------------------------------------------------------------ */
typedef struct {
  int q;
  double c[5];
  double w[5];
} lat1;

static void lattice_d1q4(lat1* L) {
  const double s6 = sqrt(6.0);
  const double a = sqrt(3.0 - s6), b = sqrt(3.0 + s6);
  L->q = 4;
  L->c[0] = -b; L->c[1] = -a; L->c[2] = a; L->c[3] = b;
  L->w[0] = (3.0 - s6) / 12.0;
  L->w[1] = (3.0 + s6) / 12.0;
  L->w[2] = (3.0 + s6) / 12.0;
  L->w[3] = (3.0 - s6) / 12.0;
}

static void lattice_d1q3(lat1* L) {
  const double r3 = sqrt(3.0);
  L->q = 3;
  L->c[0] = -r3; L->c[1] = 0.0; L->c[2] = r3; L->c[3] = 0.0;
  L->w[0] = 1.0 / 6.0; L->w[1] = 2.0 / 3.0; L->w[2] = 1.0 / 6.0; L->w[3] = 0.0;
}

/* D1Q5: the five-point Gauss--Hermite rule, nodes 0, +-sqrt(5 -+ sqrt 10),
   weights 8/15 and (7 +- 2 sqrt 10)/60 (the 1D factor of D2Q25, Table I). */
static void lattice_d1q5(lat1* L) {
  const double s10 = sqrt(10.0);
  const double a = sqrt(5.0 - s10), b = sqrt(5.0 + s10);
  L->q = 5;
  L->c[0] = -b; L->c[1] = -a; L->c[2] = 0.0; L->c[3] = a; L->c[4] = b;
  L->w[0] = (7.0 - 2.0 * s10) / 60.0;
  L->w[1] = (7.0 + 2.0 * s10) / 60.0;
  L->w[2] = 8.0 / 15.0;
  L->w[3] = (7.0 + 2.0 * s10) / 60.0;
  L->w[4] = (7.0 - 2.0 * s10) / 60.0;
}

/* 0: D1Q4, 1: D1Q3, 2: D1Q5 */
static void lattice_get(int which, lat1* L) {
  if (which == 0) lattice_d1q4(L);
  else if (which == 1) lattice_d1q3(L);
  else lattice_d1q5(L);
}

/* lattice_get index of the 1D rule with q nodes */
static int lat_of_q(int q) { return q == 4 ? 0 : (q == 3 ? 1 : 2); }

int pondref_lattice(int lattice, double* c, double* w) {
  if (lattice < 0 || lattice > 2) return fail("lattice must be 0 (D1Q4), 1 (D1Q3) or 2 (D1Q5)");
  lat1 L;
  lattice_get(lattice, &L);
  for (int k = 0; k < L.q; k++) { c[k] = L.c[k]; w[k] = L.w[k]; }
  return L.q;
}

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra.                                               */
/* ------------------------------------------------------------------------ */
static double ipow(double x, int n) {
  double r = 1.0;
  for (int k = 0; k < n; k++) r *= x;
  return r;
}

/* Solve A X = B in place (B becomes X); A is n x n, B is n x m, row-major.
   Gaussian elimination with partial pivoting. */
static int solve_dense(int n, double* A, double* B, int m) {
  for (int col = 0; col < n; col++) {
    int piv = col;
    for (int r = col + 1; r < n; r++)
      if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
    if (A[piv * n + col] == 0.0) return -1;
    if (piv != col) {
      for (int k = 0; k < n; k++) { double t = A[col * n + k]; A[col * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
      for (int k = 0; k < m; k++) { double t = B[col * m + k]; B[col * m + k] = B[piv * m + k]; B[piv * m + k] = t; }
    }
    for (int r = col + 1; r < n; r++) {
      const double fct = A[r * n + col] / A[col * n + col];
      if (fct == 0.0) continue;
      for (int k = col; k < n; k++) A[r * n + k] -= fct * A[col * n + k];
      for (int k = 0; k < m; k++) B[r * m + k] -= fct * B[col * m + k];
    }
  }
  for (int col = n - 1; col >= 0; col--) {
    for (int k = 0; k < m; k++) {
      double acc = B[col * m + k];
      for (int j = col + 1; j < n; j++) acc -= A[col * n + j] * B[j * m + k];
      B[col * m + k] = acc / A[col * n + col];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Reference-frame transformation G_{lambda}^{lambda'} (Sec. II B, App. B).  */
/*                                                                          */
/* Particle velocities in frame lambda = {u, T}: v_i = sqrt(T) c_i + u       */
/* (eq. veli, T_L = 1).  The Lagrange (moment-matching) transform is the    */
/* square map G = [M^{lambda'}]^{-1} M^{lambda} of App. B: the transformed  */
/* populations reproduce every moment sum_i f_i p(v_i) for p in the span of  */
/* the tensor monomials v_x^a v_y^b, a, b < q (orders 0..3 for D2Q16, 0..2   */
/* for D2Q9, eq. Mcondition).  The moment basis is written in the target     */
/* frame's centred, scaled coordinates xi = (v - u')/sqrt(T') -- a change of */
/* basis of the same polynomial space, which leaves G unchanged and keeps    */
/* the moment matrices well conditioned at high Mach number.                */
/* ------------------------------------------------------------------------ */

/* 1D factor: G1 (q x q, row k = target node, column m = source node) with
   sum_k c_k^a G1[k][m] = xi_m^a, a = 0..q-1, xi_m = s c_m + d. */
static int tf1_lagrange(const lat1* L, double s, double d, double* G1) {
  const int q = L->q;
  double V[25], X[25];
  for (int a = 0; a < q; a++)
    for (int k = 0; k < q; k++) {
      V[a * q + k] = ipow(L->c[k], a);
      X[a * q + k] = ipow(s * L->c[k] + d, a);
    }
  if (solve_dense(q, V, X, q)) return -1;
  memcpy(G1, X, sizeof(double) * q * q);
  return 0;
}

/* Probabilists' Hermite polynomials He_n(x), i.e. the paper's H^(n) with
   T_L = 1 in one dimension (App. A). */
static double hermite(int n, double x) {
  switch (n) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return x * x - 1.0;
    case 3: return x * x * x - 3.0 * x;
    case 4: return x * x * x * x - 6.0 * x * x + 3.0;
  }
  return 0.0;
}

static const double factorial[5] = {1.0, 1.0, 2.0, 6.0, 24.0};

static void frame_shift(const double src[3], const double dst[3], double* s, double* dx,
                        double* dy) {
  const double rt = sqrt(dst[2]);
  *s = sqrt(src[2] / dst[2]);
  *dx = (src[0] - dst[0]) / rt;
  *dy = (src[1] - dst[1]) / rt;
}

/* Dense transform matrix for the tensor lattice (Q = q^dim). */
static int transform_matrix(int dim, const lat1* L, int transform, const double src[3],
                            const double dst[3], double* G) {
  const int q = L->q;
  double s, dx, dy;
  frame_shift(src, dst, &s, &dx, &dy);
  if (transform == PONDREF_TF_LAGRANGE) {
    double Gx[25], Gy[25];
    if (tf1_lagrange(L, s, dx, Gx)) return -1;
    if (dim == 1) {
      memcpy(G, Gx, sizeof(double) * q * q);
      return 0;
    }
    if (tf1_lagrange(L, s, dy, Gy)) return -1;
    /* The tensor moment system factorizes: G = G_x (x) G_y, population index
       i = i_x + q i_y. */
    const int Q = q * q;
    for (int ky = 0; ky < q; ky++)
      for (int kx = 0; kx < q; kx++)
        for (int my = 0; my < q; my++)
          for (int mx = 0; mx < q; mx++)
            G[(kx + q * ky) * Q + (mx + q * my)] = Gx[kx * q + mx] * Gy[ky * q + my];
    return 0;
  }
  /* Grad's projection of order K = q-1 (eq. GradsProjection):
       f'_k = W_k sum_{|n| <= K} alpha^(n) H^(n)(c_k) / n!,
     with alpha^(n) the Hermite moments of the source populations in the
     target frame's centred, scaled velocities (App. A); in 2D the sum runs
     over a + b <= K. */
  const int K = q - 1;
  if (dim == 1) {
    for (int k = 0; k < q; k++)
      for (int m = 0; m < q; m++) {
        const double xm = s * L->c[m] + dx;
        double acc = 0.0;
        for (int a = 0; a <= K; a++) acc += hermite(a, L->c[k]) * hermite(a, xm) / factorial[a];
        G[k * q + m] = L->w[k] * acc;
      }
    return 0;
  }
  const int Q = q * q;
  /* the Hermite values at the target nodes and at the shifted source nodes,
     tabulated once (the same numbers the sum below would evaluate) */
  double hc[5][5], hx[5][5], hy[5][5];
  for (int a = 0; a <= K; a++)
    for (int k = 0; k < q; k++) {
      hc[a][k] = hermite(a, L->c[k]);
      hx[a][k] = hermite(a, s * L->c[k] + dx);
      hy[a][k] = hermite(a, s * L->c[k] + dy);
    }
  for (int ky = 0; ky < q; ky++)
    for (int kx = 0; kx < q; kx++)
      for (int my = 0; my < q; my++)
        for (int mx = 0; mx < q; mx++) {
          double acc = 0.0;
          for (int a = 0; a <= K; a++)
            for (int b = 0; a + b <= K; b++)
              acc += hc[a][kx] * hc[b][ky] * hx[a][mx] * hy[b][my] / (factorial[a] * factorial[b]);
          G[(kx + q * ky) * Q + (mx + q * my)] = L->w[kx] * L->w[ky] * acc;
        }
  return 0;
}

int pondref_transform_matrix(int dim, int lattice, int transform, const double src[3],
                             const double dst[3], double* G) {
  if (dim != 1 && dim != 2) return fail("dim must be 1 or 2");
  if (lattice < 0 || lattice > 2) return fail("lattice must be 0, 1 or 2");
  if (src[2] <= 0.0 || dst[2] <= 0.0) return fail("frame temperature must be positive");
  lat1 L;
  lattice_get(lattice, &L);
  if (transform_matrix(dim, &L, transform, src, dst, G)) return fail("singular moment system");
  return 0;
}

int pondref_transform_matrix_full(int dim, int lattice, const double src[3],
                                  const double dst[3], double* G) {
  if (dim != 1 && dim != 2) return fail("dim must be 1 or 2");
  lat1 L;
  lattice_get(lattice, &L);
  const int q = L.q, Q = dim == 1 ? q : q * q;
  double s, dx, dy;
  frame_shift(src, dst, &s, &dx, &dy);
  double* V = (double*)malloc(sizeof(double) * Q * Q);
  double* X = (double*)malloc(sizeof(double) * Q * Q);
  /* row (a, b) of the moment matrix: monomial xi_x^a xi_y^b; column: population */
  for (int r = 0; r < Q; r++) {
    const int a = r % q, b = r / q;
    for (int k = 0; k < Q; k++) {
      const int kx = k % q, ky = k / q;
      if (dim == 1) {
        V[r * Q + k] = ipow(L.c[k], r);
        X[r * Q + k] = ipow(s * L.c[k] + dx, r);
      } else {
        V[r * Q + k] = ipow(L.c[kx], a) * ipow(L.c[ky], b);
        X[r * Q + k] = ipow(s * L.c[kx] + dx, a) * ipow(s * L.c[ky] + dy, b);
      }
    }
  }
  const int rc = solve_dense(Q, V, X, Q);
  if (!rc) memcpy(G, X, sizeof(double) * Q * Q);
  free(V);
  free(X);
  return rc ? fail("singular moment system") : 0;
}

/* ------------------------------------------------------------------------ */
/* Multiscale frame transformation (Sec. III C, eqs. lifting1, projection1). */
/*                                                                          */
/* Between a source lattice with q1s nodes per axis and a target with q1t,  */
/* both Hermite-Grad expansions (eq. GradsProjection):                       */
/*  - same lattice: Grad's projection of order q1 - 1 (the map above);      */
/*  - lifting (D2Q9 -> D2Q16): the moments the D2Q9 populations carry       */
/*    (Hermite moments of total order <= 2) are kept and the missing         */
/*    third-order ones take their equilibrium value.  reading: equilibrium  */
/*    in the source's comoving frame, where the Maxwellian's third Hermite  */
/*    moments vanish (a Galilean-invariant choice); the lifted D2Q16 set is */
/*    built there and then mapped to the target frame by Grad's projection; */
/*  - projection (D2Q16 -> D2Q9): Grad's expansion of order 2 in the target */
/*    frame from the Hermite moments of the D2Q16 populations.               */
/* ------------------------------------------------------------------------ */
static int ms_matrix(int transform, int q1s, const double src[3], int q1t, const double dst[3],
                     double* G) {
  lat1 Ls, Lt;
  lattice_get(lat_of_q(q1s), &Ls);
  lattice_get(lat_of_q(q1t), &Lt);
  if (q1s == q1t) return transform_matrix(2, &Ls, transform, src, dst, G);
  if (q1s == 3) {
    /* lifting: own-frame D2Q16 expansion with alpha_ab (a + b <= 2) from the
       D2Q9 populations and alpha_ab = 0 for a + b = 3 */
    double lift[16 * 9], Gt[256];
    for (int ky = 0; ky < 4; ky++)
      for (int kx = 0; kx < 4; kx++)
        for (int my = 0; my < 3; my++)
          for (int mx = 0; mx < 3; mx++) {
            double acc = 0.0;
            for (int a = 0; a <= 2; a++)
              for (int b = 0; a + b <= 2; b++)
                acc += hermite(a, Lt.c[kx]) * hermite(b, Lt.c[ky]) * hermite(a, Ls.c[mx]) *
                       hermite(b, Ls.c[my]) / (factorial[a] * factorial[b]);
            lift[(kx + 4 * ky) * 9 + (mx + 3 * my)] = Lt.w[kx] * Lt.w[ky] * acc;
          }
    if (transform_matrix(2, &Lt, PONDREF_TF_GRAD, src, dst, Gt)) return -1;
    for (int k = 0; k < 16; k++)
      for (int m = 0; m < 9; m++) {
        double acc = 0.0;
        for (int j = 0; j < 16; j++) acc += Gt[k * 16 + j] * lift[j * 9 + m];
        G[k * 9 + m] = acc;
      }
    return 0;
  }
  /* projection */
  double sc, dx, dy;
  frame_shift(src, dst, &sc, &dx, &dy);
  for (int ky = 0; ky < 3; ky++)
    for (int kx = 0; kx < 3; kx++)
      for (int my = 0; my < 4; my++)
        for (int mx = 0; mx < 4; mx++) {
          const double xm = sc * Ls.c[mx] + dx, ym = sc * Ls.c[my] + dy;
          double acc = 0.0;
          for (int a = 0; a <= 2; a++)
            for (int b = 0; a + b <= 2; b++)
              acc += hermite(a, Lt.c[kx]) * hermite(b, Lt.c[ky]) * hermite(a, xm) *
                     hermite(b, ym) / (factorial[a] * factorial[b]);
          G[(kx + 3 * ky) * 16 + (mx + 4 * my)] = Lt.w[kx] * Lt.w[ky] * acc;
        }
  return 0;
}

int pondref_ms_matrix(int q1s, const double src[3], int q1t, const double dst[3], double* G) {
  if ((q1s != 3 && q1s != 4) || (q1t != 3 && q1t != 4)) return fail("q1 must be 3 or 4");
  if (src[2] <= 0.0 || dst[2] <= 0.0) return fail("frame temperature must be positive");
  if (ms_matrix(PONDREF_TF_GRAD, q1s, src, q1t, dst, G)) return fail("singular moment system");
  return 0;
}

/* rectangular: out (Qt) = G (Qt x Qs) in (Qs) */
static void matvec_r(int Qt, int Qs, const double* G, const double* in, double* out) {
  for (int k = 0; k < Qt; k++) {
    double acc = 0.0;
    for (int m = 0; m < Qs; m++) acc += G[k * Qs + m] * in[m];
    out[k] = acc;
  }
}

static void matvec(int Q, const double* G, const double* in, double* out) {
  for (int k = 0; k < Q; k++) {
    double acc = 0.0;
    for (int m = 0; m < Q; m++) acc += G[k * Q + m] * in[m];
    out[k] = acc;
  }
}

/* ------------------------------------------------------------------------ */
/* State.                                                                    */
/* ------------------------------------------------------------------------ */
#define NG 2 /* ghost layers */
#define TIE_BAND 1e-11 /* |v_n| <= TIE_BAND sqrt(T_F) is an upwind tie */
#define QMAX 25

struct pondref_state {
  pondref_config cfg;
  int D;
  lat1 Lf, Lg;       /* D1Q4 (D1Q5 for the D2Q25 f-lattice) for f, D1Q3 for g */
  int Qf, Qg;
  double Wf[QMAX], Wg[9];
  double cfx[QMAX], cfy[QMAX], cgx[9], cgy[9]; /* lattice velocity components */
  int nxp, nyp;      /* padded extents */
  double* f;         /* [cell][Qf], populations f~ in the cell's frame */
  double* g;         /* [cell][Qg] */
  double* fr;        /* [cell][3]  frame (u_x, u_y, T) */
  double* fbp;       /* [cell][Qf] phi-bar-plus of f */
  double* gbp;       /* [cell][Qg] */
  double* ffx; double* gfx; double* lfx; /* x-faces */
  double* ffy; double* gfy; double* lfy; /* y-faces */
  /* f-lattice per cell, as the 1D node count q1 (4: D2Q16 / D1Q4, 3: D2Q9),
     and per face; the multiscale switch indicator of the last step */
  unsigned char* lat;
  unsigned char* latfx; unsigned char* latfy;
  unsigned char* flag;
  double* theta;
  /* per-lattice tables, index 0: q1 = 4, index 1: q1 = 3 (2D tensor or 1D) */
  int Qq[2];
  double Wq[2][QMAX], cxq[2][QMAX], cyq[2][QMAX];
  double dt, dx, tau1, tau2, cv;
  int dt_fixed;
  long nstep;
};

static inline int cidx(const pondref_state* s, int x, int y) {
  return (x + NG) + s->nxp * (s->D == 2 ? (y + NG) : 0);
}

int pondref_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
int pondref_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int check_config(const pondref_config* c) {
  if (c->dim != 1 && c->dim != 2) return fail("dim must be 1 or 2");
  if (c->nx < 1 || c->ny < 1 || (c->dim == 1 && c->ny != 1)) return fail("bad grid size");
  if (c->transform != PONDREF_TF_LAGRANGE && c->transform != PONDREF_TF_GRAD)
    return fail("unknown transform");
  if (!(c->gamma > 1.0)) return fail("gamma must exceed 1");
  if (!(c->tau > 0.0)) return fail("tau must be positive");
  if (!(c->prandtl > 0.0 && c->prandtl <= 1.0)) return fail("Pr must lie in (0, 1]");
  if (!(c->cfl > 0.0)) return fail("cfl must be positive");
  if (c->limiter != PONDREF_LIM_VANLEER && c->limiter != PONDREF_LIM_MINMOD)
    return fail("unknown limiter");
  if (c->n_corr < 0) return fail("n_corr must be >= 0");
  if (c->flat < 0 || c->flat > 3) return fail("unknown f-lattice");
  if (c->flat == PONDREF_F_D2Q25 && c->transform != PONDREF_TF_GRAD)
    return fail("the D2Q25 f-lattice uses the fourth-order Grad projection");
  if (c->flat != PONDREF_F_D2Q16 && c->dim != 2) return fail("the D2Q9, multiscale and D2Q25 f-lattices are 2D");
  if (c->flat == PONDREF_F_MULTISCALE && c->transform != PONDREF_TF_GRAD)
    return fail("the multiscale deployment uses Grad's projection");
  if (c->flat == PONDREF_F_MULTISCALE && !(c->ms_threshold >= 0.0))
    return fail("the multiscale threshold must be >= 0");
  const int nside = c->dim == 2 ? 4 : 2;
  for (int k = 0; k < nside; k++)
    if (c->bc[k] < 0 || c->bc[k] > 3) return fail("unknown boundary condition");
  for (int k = 0; k < nside; k++) {
    if (c->bc[k] != PONDREF_BC_WALL) continue;
    if (c->dim != 2 || c->flat != PONDREF_F_D2Q16) return fail("walls need 2D and the D2Q16 f-lattice");
    if ((k < 2 ? c->nx : c->ny) < 3) return fail("a wall needs three cells along its normal");
    if (!(c->wall[k][2] > 0.0) || !isfinite(c->wall[k][0]) || !isfinite(c->wall[k][1]))
      return fail("a wall needs a positive temperature and a finite velocity");
    if (c->wall[k][k < 2 ? 0 : 1] != 0.0) return fail("a wall cannot move along its normal");
  }
  if (!isfinite(c->accel[0]) || !isfinite(c->accel[1])) return fail("the body force must be finite");
  if ((c->accel[0] != 0.0 || c->accel[1] != 0.0) && (c->dim != 2 || c->flat != PONDREF_F_D2Q16))
    return fail("a body force needs 2D and the D2Q16 f-lattice");
  for (int a = 0; a < nside; a += 2)
    if ((c->bc[a] == PONDREF_BC_PERIODIC) != (c->bc[a + 1] == PONDREF_BC_PERIODIC))
      return fail("a periodic axis needs periodic conditions on both sides");
  for (int k = 0; k < nside; k++)
    if (c->bc[k] == PONDREF_BC_INFLOW && !(c->inflow[k][0] > 0.0 && c->inflow[k][3] > 0.0))
      return fail("inflow state needs positive density and pressure");
  return 0;
}

int pondref_create(const pondref_config* cfg, pondref_state** out) {
  if (!cfg || !out) return fail("null argument");
  if (check_config(cfg)) return -1;
  pondref_state* s = (pondref_state*)calloc(1, sizeof(pondref_state));
  s->cfg = *cfg;
  s->D = cfg->dim;
  if (cfg->dim == 2 && cfg->flat == PONDREF_F_D2Q25) lattice_d1q5(&s->Lf);
  else lattice_d1q4(&s->Lf);
  lattice_d1q3(&s->Lg);
  if (s->D == 1) {
    s->Qf = 4; s->Qg = 3;
    for (int i = 0; i < 4; i++) { s->Wf[i] = s->Lf.w[i]; s->cfx[i] = s->Lf.c[i]; s->cfy[i] = 0.0; }
    for (int i = 0; i < 3; i++) { s->Wg[i] = s->Lg.w[i]; s->cgx[i] = s->Lg.c[i]; s->cgy[i] = 0.0; }
  } else {
    const int q = s->Lf.q;
    s->Qf = q * q; s->Qg = 9;
    /* eq. (wi): W_i = w_ix w_iy, c_i = (c_ix, c_iy), i = i_x + q i_y */
    for (int iy = 0; iy < q; iy++)
      for (int ix = 0; ix < q; ix++) {
        const int i = ix + q * iy;
        s->Wf[i] = s->Lf.w[ix] * s->Lf.w[iy];
        s->cfx[i] = s->Lf.c[ix];
        s->cfy[i] = s->Lf.c[iy];
      }
    for (int iy = 0; iy < 3; iy++)
      for (int ix = 0; ix < 3; ix++) {
        const int i = ix + 3 * iy;
        s->Wg[i] = s->Lg.w[ix] * s->Lg.w[iy];
        s->cgx[i] = s->Lg.c[ix];
        s->cgy[i] = s->Lg.c[iy];
      }
  }
  /* per-lattice tables: the solve's f-lattice D2Q16 / D2Q25 / D1Q4 (index
     0) and the D2Q9 f-lattice (index 1, tensor D1Q3, i = i_x + 3 i_y) */
  s->Qq[0] = s->Qf;
  for (int i = 0; i < s->Qf; i++) { s->Wq[0][i] = s->Wf[i]; s->cxq[0][i] = s->cfx[i]; s->cyq[0][i] = s->cfy[i]; }
  s->Qq[1] = s->Qg;
  for (int i = 0; i < s->Qg; i++) { s->Wq[1][i] = s->Wg[i]; s->cxq[1][i] = s->cgx[i]; s->cyq[1][i] = s->cgy[i]; }
  s->nxp = cfg->nx + 2 * NG;
  s->nyp = s->D == 2 ? cfg->ny + 2 * NG : 1;
  const size_t nc = (size_t)s->nxp * s->nyp;
  s->lat = (unsigned char*)malloc(nc);
  s->flag = (unsigned char*)calloc(nc, 1);
  memset(s->lat, cfg->flat == PONDREF_F_D2Q9 ? 3 : s->Lf.q, nc);
  s->theta = (double*)calloc((size_t)cfg->nx * cfg->ny, sizeof(double));
  s->f = (double*)calloc(nc * s->Qf, sizeof(double));
  s->g = (double*)calloc(nc * s->Qg, sizeof(double));
  s->fr = (double*)calloc(nc * 3, sizeof(double));
  s->fbp = (double*)calloc(nc * s->Qf, sizeof(double));
  s->gbp = (double*)calloc(nc * s->Qg, sizeof(double));
  const size_t nfx = (size_t)(cfg->nx + 1) * cfg->ny;
  const size_t nfy = s->D == 2 ? (size_t)cfg->nx * (cfg->ny + 1) : 0;
  s->ffx = (double*)calloc(nfx * s->Qf, sizeof(double));
  s->gfx = (double*)calloc(nfx * s->Qg, sizeof(double));
  s->lfx = (double*)calloc(nfx * 3, sizeof(double));
  s->latfx = (unsigned char*)calloc(nfx, 1);
  s->latfy = (unsigned char*)calloc(nfy ? nfy : 1, 1);
  if (nfy) {
    s->ffy = (double*)calloc(nfy * s->Qf, sizeof(double));
    s->gfy = (double*)calloc(nfy * s->Qg, sizeof(double));
    s->lfy = (double*)calloc(nfy * 3, sizeof(double));
  }
  s->dx = cfg->dx > 0.0 ? cfg->dx : 1.0 / cfg->nx;
  s->cv = 1.0 / (cfg->gamma - 1.0); /* C_p = C_v + 1 (Sec. III A) */
  *out = s;
  return 0;
}

void pondref_destroy(pondref_state* s) {
  if (!s) return;
  free(s->f); free(s->g); free(s->fr); free(s->fbp); free(s->gbp);
  free(s->ffx); free(s->gfx); free(s->lfx);
  free(s->ffy); free(s->gfy); free(s->lfy);
  free(s->lat); free(s->latfx); free(s->latfy); free(s->flag); free(s->theta);
  free(s);
}

/* ------------------------------------------------------------------------ */
/* Equilibria and moments (Sec. III A).                                      */
/* ------------------------------------------------------------------------ */

/* Comoving equilibria: f^eq = rho W_i (eq. feqPond), g^eq = (C_v - D/2) T rho W_i
   (eq. geqPond), written in the comoving frame lambda = {u, T}. */
static void comoving_eq(const pondref_state* s, int q1, double rho, double T, double* feq,
                        double* geq) {
  const int l = q1 == 3 ? 1 : 0;
  for (int i = 0; i < s->Qq[l]; i++) feq[i] = rho * s->Wq[l][i];
  const double e = (s->cv - 0.5 * s->D) * T * rho;
  for (int i = 0; i < s->Qg; i++) geq[i] = e * s->Wg[i];
}

/* Conservation laws (eq. ConservationLaws and eq. E): density, velocity and
   temperature from f and g written in frame fr, v_i = sqrt(T) c_i + u. */
static void moments(const pondref_state* s, int q1, const double* f, const double* g,
                    const double fr[3], double* rho, double* ux, double* uy, double* T,
                    double* rhoE) {
  const int l = q1 == 3 ? 1 : 0;
  const double rt = sqrt(fr[2]);
  double m0 = 0.0, mx = 0.0, my = 0.0, e = 0.0;
  for (int i = 0; i < s->Qq[l]; i++) {
    const double vx = rt * s->cxq[l][i] + fr[0];
    const double vy = s->D == 2 ? rt * s->cyq[l][i] + fr[1] : 0.0;
    m0 += f[i];
    mx += vx * f[i];
    my += vy * f[i];
    e += 0.5 * (vx * vx + vy * vy) * f[i];
  }
  for (int i = 0; i < s->Qg; i++) e += g[i];
  *rho = m0;
  *ux = mx / m0;
  *uy = my / m0;
  if (rhoE) *rhoE = e;
  /* rho E = C_v rho T + rho u^2 / 2 */
  *T = (e - 0.5 * m0 * ((*ux) * (*ux) + (*uy) * (*uy))) / (s->cv * m0);
}

/* ------------------------------------------------------------------------ */
/* Initial data (Sec. IV A 3, item 1): comoving equilibrium, T = p / rho.    */
/* ------------------------------------------------------------------------ */
static double cfl_dt(const pondref_config* c, const double* rho, const double* ux,
                     const double* uy, const double* p) {
  /* CFL = max|v_ia| dt / dx = 0.2 (Sec. V); the max runs over cells,
     populations and axes of |sqrt(T) c_ia + u_a|, at t = 0 (reading). */
  /* the largest node of the f-lattice in use (D2Q9 alone: sqrt 3) */
  double cmax = sqrt(3.0 + sqrt(6.0));
  if (c->dim == 2 && c->flat == PONDREF_F_D2Q9) cmax = sqrt(3.0);
  if (c->dim == 2 && c->flat == PONDREF_F_D2Q25) cmax = sqrt(5.0 + sqrt(10.0));
  const double dx = c->dx > 0.0 ? c->dx : 1.0 / c->nx;
  double vmax = 0.0;
  const size_t n = (size_t)c->nx * c->ny;
  for (size_t k = 0; k < n; k++) {
    const double rt = sqrt(p[k] / rho[k]);
    double vx = fabs(ux[k]) + rt * cmax;
    double vy = c->dim == 2 ? fabs(uy[k]) + rt * cmax : 0.0;
    if (vx > vmax) vmax = vx;
    if (vy > vmax) vmax = vy;
  }
  return c->cfl * dx / vmax;
}

double pondref_cfl_dt(const pondref_config* c, const double* rho, const double* ux,
                      const double* uy, const double* p) {
  if (check_config(c)) return -1.0;
  return cfl_dt(c, rho, ux, uy, p);
}

static void set_times(pondref_state* s) {
  s->tau1 = s->cfg.tau * s->dt;          /* reading: tau is tau1 in units of dt */
  s->tau2 = s->tau1 / s->cfg.prandtl;    /* Pr = tau1 / tau2 */
}

int pondref_init_fields(pondref_state* s, const double* rho, const double* ux, const double* uy,
                        const double* p) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  for (int k = 0; k < nx * ny; k++)
    if (!(rho[k] > 0.0) || !(p[k] > 0.0) || !isfinite(ux[k]) || (s->D == 2 && !isfinite(uy[k])))
      return fail("initial density and pressure must be positive and finite");
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const int k = x + nx * y, c = cidx(s, x, y);
      double* fr = s->fr + 3 * c;
      fr[0] = ux[k];
      fr[1] = s->D == 2 ? uy[k] : 0.0;
      fr[2] = p[k] / rho[k];
      comoving_eq(s, s->lat[c], rho[k], fr[2], s->f + (size_t)c * s->Qf, s->g + (size_t)c * s->Qg);
    }
  if (!s->dt_fixed) s->dt = cfl_dt(&s->cfg, rho, ux, uy, p);
  set_times(s);
  s->nstep = 0;
  return 0;
}

int pondref_set_dt(pondref_state* s, double dt) {
  if (!(dt > 0.0)) return fail("dt must be positive");
  s->dt = dt;
  s->dt_fixed = 1;
  set_times(s);
  return 0;
}
double pondref_get_dt(const pondref_state* s) { return s->dt; }

/* ------------------------------------------------------------------------ */
/* Ghost cells (Sec. IV D): two layers.                                      */
/* reading: periodic wraps; zero gradient copies the populations and frame   */
/* of the nearest interior cell; inflow is the comoving equilibrium of the   */
/* fixed state.  A ghost's x coordinate is resolved first, then y, so a      */
/* corner ghost next to an inflow x side takes that side's state.            */
/* ------------------------------------------------------------------------ */
static int resolve_axis(int v, int n, int bc_lo, int bc_hi, int* side_inflow, int lo_side) {
  if (v < 0) {
    if (bc_lo == PONDREF_BC_PERIODIC) return ((v % n) + n) % n;
    if (bc_lo == PONDREF_BC_ZERO_GRADIENT) return 0;
    *side_inflow = lo_side;
    return 0;
  }
  if (v >= n) {
    if (bc_hi == PONDREF_BC_PERIODIC) return v % n;
    if (bc_hi == PONDREF_BC_ZERO_GRADIENT) return n - 1;
    *side_inflow = lo_side + 1;
    return n - 1;
  }
  return v;
}

/* ------------------------------------------------------------------------ */
/* Wall ghosts (Sec. IV D: ghost-node approach with the Chapman-Enskog      */
/* non-equilibrium of the first order).                                     */
/* reading: ghost layer k mirrors the k-th cell from the wall: density      */
/* keeps its value (zero normal gradient), velocity and temperature are     */
/* reflected about the wall's values (u_G = 2 u_w - u_B, T_G = 2 T_w - T_B). */
/* The hydrodynamic gradients at a ghost are second-order central           */
/* differences of this mirror-extended field at the start of the step;      */
/* along the wall, past the domain, the field wraps on a periodic axis and  */
/* takes the nearest cell otherwise.                                        */
/* ------------------------------------------------------------------------ */

/* (rho, u_x, u_y, T) of the extended field at normal index m (m >= 0: the
   interior cell m rows in from wall `side`; m < 0: ghost layer -m) and
   coordinate t along the wall */
static void wall_field(const pondref_state* s, int side, int m, int t, double out[4]) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const int nt = side < 2 ? ny : nx;
  const int bt = side < 2 ? s->cfg.bc[2] : s->cfg.bc[0];
  if (t < 0 || t >= nt)
    t = bt == PONDREF_BC_PERIODIC ? ((t % nt) + nt) % nt : (t < 0 ? 0 : nt - 1);
  const int mm = m >= 0 ? m : -m - 1;
  int x, y;
  switch (side) {
    case 0: x = mm; y = t; break;
    case 1: x = nx - 1 - mm; y = t; break;
    case 2: x = t; y = mm; break;
    default: x = t; y = ny - 1 - mm; break;
  }
  const int c = cidx(s, x, y);
  const double* f = s->f + (size_t)c * s->Qf;
  double rho = 0.0;
  for (int i = 0; i < s->Qf; i++) rho += f[i];
  out[0] = rho;
  out[1] = s->fr[3 * c + 0];
  out[2] = s->fr[3 * c + 1];
  out[3] = s->fr[3 * c + 2];
  if (m < 0) {
    const double* w = s->cfg.wall[side];
    out[1] = 2.0 * w[0] - out[1];
    out[2] = 2.0 * w[1] - out[2];
    out[3] = 2.0 * w[2] - out[3];
  }
}

/* Ghost populations: the comoving equilibrium plus the non-equilibrium
   part whose moments are the Chapman-Enskog ones (Sec. IV D), expanded in
   Hermite polynomials of c = (v - u_G)/sqrt(T_G) (Grad's projection: order
   3 for f on D2Q16, order 2 for g on D2Q9).  With p = rho T,
   S = grad u + (grad u)^T and d = div u:
     f: P1 = -tau1 p (S - (d / C_v) I), central third moment
        -tau2 p [dT/dx_a delta_bc]_cyc;
     g: zeroth moment tau1 (C_v - D/2) p d / C_v, central first moment
        -tau2 (C_v - D/2) p grad T, central second moment
        -tau1 (C_v - D/2) p T (S - (2 d / C_v) I).
   reading: the g moments are re-derived from the first Chapman-Enskog
   order with g^eq = (C_v - D/2) T rho W (eq. geqPond) and written about
   the ghost's own velocity (the printed ones carry a factor 2 and a sign
   of a different normalisation of g).  Then the non-equilibrium parts
   carry no mass, momentum or energy, the total heat flux is
   -tau2 C_p p grad T (kappa of Sec. IV) and the stress is that of mu and
   varsigma.  The stored variable is f~ = f^eq + (1 + dt / (2 tau1)) f^neq
   (eq. variableTransform with the BGK time of the streaming part). */
static void wall_ghost(const pondref_state* s, int side, int k, int t, double* f, double* g,
                       double fr[3]) {
  double G[4], pn[4], mn[4], pt[4], mt[4];
  wall_field(s, side, -k, t, G);
  wall_field(s, side, -k + 1, t, pn);   /* one cell further in */
  wall_field(s, side, -k - 1, t, mn);   /* one cell further out */
  wall_field(s, side, -k, t + 1, pt);
  wall_field(s, side, -k, t - 1, mt);
  const double h = 0.5 / s->dx;
  /* m grows inward: along +x or +y on the low sides, against it on the high */
  const double sn = (side == 0 || side == 2) ? 1.0 : -1.0;
  /* d/dx_a of (u_x, u_y, T): row a = derivative direction */
  double A[2][3];
  for (int q = 0; q < 3; q++) {
    const double dn = sn * (pn[q + 1] - mn[q + 1]) * h;
    const double dtg = (pt[q + 1] - mt[q + 1]) * h;
    if (side < 2) { A[0][q] = dn; A[1][q] = dtg; }
    else { A[0][q] = dtg; A[1][q] = dn; }
  }
  const double rho = G[0], ux = G[1], uy = G[2], T = G[3], p = rho * T;
  const double Sxx = 2.0 * A[0][0], Syy = 2.0 * A[1][1], Sxy = A[0][1] + A[1][0];
  const double d = A[0][0] + A[1][1], Tx = A[0][2], Ty = A[1][2];
  const double cv = s->cv, ce = s->cv - 1.0; /* C_v - D/2, D = 2 */
  const double t1 = s->tau1, t2 = s->tau2;
  /* f: Hermite coefficients alpha_ab (a x-indices, b y-indices) */
  const double Pxx = -t1 * p * (Sxx - d / cv), Pyy = -t1 * p * (Syy - d / cv), Pxy = -t1 * p * Sxy;
  const double a20 = Pxx / T, a11 = Pxy / T, a02 = Pyy / T;
  const double T32 = T * sqrt(T);
  const double a30 = -3.0 * t2 * p * Tx / T32, a21 = -t2 * p * Ty / T32;
  const double a12 = -t2 * p * Tx / T32, a03 = -3.0 * t2 * p * Ty / T32;
  /* g: Hermite coefficients */
  const double b0 = t1 * ce * p * d / cv;
  const double b1x = -t2 * ce * p * Tx / sqrt(T), b1y = -t2 * ce * p * Ty / sqrt(T);
  const double M2xx = -t1 * ce * p * T * (Sxx - 2.0 * d / cv);
  const double M2yy = -t1 * ce * p * T * (Syy - 2.0 * d / cv);
  const double M2xy = -t1 * ce * p * T * Sxy;
  const double b20 = M2xx / T - b0, b11 = M2xy / T, b02 = M2yy / T - b0;
  const double kf = 1.0 + s->dt / (2.0 * t1);
  for (int i = 0; i < 16; i++) {
    const double cx = s->cfx[i], cy = s->cfy[i];
    const double neq = a20 * hermite(2, cx) / 2.0 + a11 * cx * cy + a02 * hermite(2, cy) / 2.0 +
                       a30 * hermite(3, cx) / 6.0 + a21 * hermite(2, cx) * cy / 2.0 +
                       a12 * cx * hermite(2, cy) / 2.0 + a03 * hermite(3, cy) / 6.0;
    f[i] = rho * s->Wf[i] + kf * s->Wf[i] * neq;
  }
  for (int i = 0; i < 9; i++) {
    const double cx = s->cgx[i], cy = s->cgy[i];
    const double neq = b0 + b1x * cx + b1y * cy + b20 * hermite(2, cx) / 2.0 + b11 * cx * cy +
                       b02 * hermite(2, cy) / 2.0;
    g[i] = ce * T * rho * s->Wg[i] + kf * s->Wg[i] * neq;
  }
  fr[0] = ux;
  fr[1] = uy;
  fr[2] = T;
}

int pondref_wall_ghost(const pondref_state* s, int side, int layer, int t, double* f, double* g,
                       double frame[3]) {
  if (!s || !f || !g || !frame) return fail("null argument");
  if (s->D != 2 || side < 0 || side > 3 || s->cfg.bc[side] != PONDREF_BC_WALL)
    return fail("not a wall side");
  if (layer < 1 || layer > NG) return fail("ghost layer must be 1 or 2");
  if (t < 0 || t >= (side < 2 ? s->cfg.ny : s->cfg.nx)) return fail("t out of range");
  wall_ghost(s, side, layer, t, f, g, frame);
  return 0;
}

static void fill_ghosts(pondref_state* s) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const int ylo = s->D == 2 ? -NG : 0, yhi = s->D == 2 ? ny + NG : 1;
  for (int y = ylo; y < yhi; y++)
    for (int x = -NG; x < nx + NG; x++) {
      if (x >= 0 && x < nx && y >= 0 && y < ny) continue;
      int side = -1;
      const int sx = resolve_axis(x, nx, s->cfg.bc[0], s->cfg.bc[1], &side, 0);
      int sy = y;
      if (side < 0 && s->D == 2) sy = resolve_axis(y, ny, s->cfg.bc[2], s->cfg.bc[3], &side, 2);
      const int c = cidx(s, x, y);
      double* fr = s->fr + 3 * c;
      if (side >= 0 && s->cfg.bc[side] == PONDREF_BC_WALL) {
        /* wall ghost: layer from the distance to the wall, coordinate along
           the wall resolved as above (x first) */
        const int v = side < 2 ? x : y, n = side < 2 ? nx : ny;
        const int k = v < 0 ? -v : v - n + 1;
        int t = side < 2 ? y : sx;
        if (side < 2 && (t < 0 || t >= ny))
          t = s->cfg.bc[2] == PONDREF_BC_PERIODIC ? ((t % ny) + ny) % ny : (t < 0 ? 0 : ny - 1);
        s->lat[c] = 4;
        wall_ghost(s, side, k, t, s->f + (size_t)c * s->Qf, s->g + (size_t)c * s->Qg, fr);
      } else if (side >= 0) {
        /* reading: an inflow ghost takes the f-lattice of the interior cell
           next to it */
        const int bx = sx, by = s->D == 2 ? (y < 0 ? 0 : (y >= ny ? ny - 1 : y)) : 0;
        s->lat[c] = s->lat[cidx(s, bx, by)];
        const double* st = s->cfg.inflow[side];
        fr[0] = st[1];
        fr[1] = s->D == 2 ? st[2] : 0.0;
        fr[2] = st[3] / st[0];
        comoving_eq(s, s->lat[c], st[0], fr[2], s->f + (size_t)c * s->Qf, s->g + (size_t)c * s->Qg);
      } else {
        const int src = cidx(s, sx, sy);
        s->lat[c] = s->lat[src];
        memcpy(fr, s->fr + 3 * src, 3 * sizeof(double));
        memcpy(s->f + (size_t)c * s->Qf, s->f + (size_t)src * s->Qf, s->Qf * sizeof(double));
        memcpy(s->g + (size_t)c * s->Qg, s->g + (size_t)src * s->Qg, s->Qg * sizeof(double));
      }
    }
}

/* ------------------------------------------------------------------------ */
/* Multiscale switch (Sec. IV C, Sec. V multiscale framework): D2Q16 where   */
/* the flow velocity and temperature gradients are steep, D2Q9 elsewhere.    */
/* reading (threshold and stencil are not given): central differences of    */
/* the cell frames, indicator theta = dx (|grad u| / sqrt(gamma T) +          */
/* |grad T| / T) with Frobenius / Euclidean norms, D2Q16 within two cells    */
/* (Chebyshev distance) of a cell with theta >= ms_threshold.  Ghost flags   */
/* follow the ghost rule of the populations (inflow: the next interior      */
/* cell).  Cells whose lattice changes have their populations lifted or     */
/* projected in their own frame.  Needs the ghost frames filled.            */
/* ------------------------------------------------------------------------ */
static void switch_lattices(pondref_state* s) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const double thr = s->cfg.ms_threshold, gam = s->cfg.gamma;
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const double* xp = s->fr + 3 * cidx(s, x + 1, y);
      const double* xm = s->fr + 3 * cidx(s, x - 1, y);
      const double* yp = s->fr + 3 * cidx(s, x, y + 1);
      const double* ym = s->fr + 3 * cidx(s, x, y - 1);
      const double T = s->fr[3 * cidx(s, x, y) + 2];
      const double uxx = 0.5 * (xp[0] - xm[0]), uyx = 0.5 * (xp[1] - xm[1]);
      const double uxy = 0.5 * (yp[0] - ym[0]), uyy = 0.5 * (yp[1] - ym[1]);
      const double Tx = 0.5 * (xp[2] - xm[2]), Ty = 0.5 * (yp[2] - ym[2]);
      const double gu = sqrt(uxx * uxx + uyx * uyx + uxy * uxy + uyy * uyy);
      const double gT = sqrt(Tx * Tx + Ty * Ty);
      const double th = gu / sqrt(gam * T) + gT / T;
      s->theta[x + nx * y] = th;
      s->flag[cidx(s, x, y)] = th >= thr;
    }
  for (int y = -NG; y < ny + NG; y++)
    for (int x = -NG; x < nx + NG; x++) {
      if (x >= 0 && x < nx && y >= 0 && y < ny) continue;
      int side = -1;
      const int sx = resolve_axis(x, nx, s->cfg.bc[0], s->cfg.bc[1], &side, 0);
      int sy = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
      if (side < 0) sy = resolve_axis(y, ny, s->cfg.bc[2], s->cfg.bc[3], &side, 2);
      s->flag[cidx(s, x, y)] = s->flag[cidx(s, sx, sy)];
    }
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      int hi = 0;
      for (int j = -2; j <= 2; j++)
        for (int i = -2; i <= 2; i++) hi |= s->flag[cidx(s, x + i, y + j)];
      const int c = cidx(s, x, y);
      const int q1 = hi ? 4 : 3;
      if (q1 != s->lat[c]) {
        const int qo = s->lat[c];
        double G[256], tmp[QMAX];
        double* f = s->f + (size_t)c * s->Qf;
        ms_matrix(PONDREF_TF_GRAD, qo, s->fr + 3 * c, q1, s->fr + 3 * c, G);
        matvec_r(q1 * q1, qo * qo, G, f, tmp);
        for (int i = 0; i < s->Qf; i++) f[i] = i < q1 * q1 ? tmp[i] : 0.0;
        s->lat[c] = (unsigned char)q1;
      }
    }
}

/* ------------------------------------------------------------------------ */
/* Quasi-equilibrium half step (Sec. IV B, eq. QE_relaxation, eq. quasi_f).  */
/* In the comoving frame e_i = sqrt(T) c_i, so                               */
/*   f* - f^eq = W_i alpha3 : H^(3)(c_i) / 6,  alpha3 = sum_i f_i H^(3)(c_i), */
/*   g* - g^eq = W_i (sum_j g_j c_j) . c_i,                                   */
/* and the half step adds (dt/2)(1/tau1 - 1/tau2) times these.  Applied to   */
/* the stored f~ (reading: the QE term is linear in the third Hermite        */
/* moment, which the variable transform only rescales).                      */
/* ------------------------------------------------------------------------ */
static void qe_half_step(const pondref_state* s, int q1, double* f, double* g) {
  const double kappa = 0.5 * s->dt * (1.0 / s->tau1 - 1.0 / s->tau2);
  if (kappa == 0.0) return;
  if (s->D == 2 && q1 == 3) {
    /* reading: the D2Q9 f-lattice carries no third-order moments, so only
       the g part of the quasi-equilibrium relaxation acts on it */
    double agx = 0.0, agy = 0.0;
    for (int i = 0; i < 9; i++) { agx += g[i] * s->cgx[i]; agy += g[i] * s->cgy[i]; }
    for (int i = 0; i < 9; i++) g[i] += kappa * s->Wg[i] * (agx * s->cgx[i] + agy * s->cgy[i]);
    return;
  }
  if (s->D == 1) {
    double a3 = 0.0, ag = 0.0;
    for (int i = 0; i < 4; i++) a3 += f[i] * hermite(3, s->cfx[i]);
    for (int i = 0; i < 3; i++) ag += g[i] * s->cgx[i];
    for (int i = 0; i < 4; i++) f[i] += kappa * s->Wf[i] * a3 * hermite(3, s->cfx[i]) / 6.0;
    for (int i = 0; i < 3; i++) g[i] += kappa * s->Wg[i] * ag * s->cgx[i];
    return;
  }
  /* H^(3)_{abc}(c) = c_a c_b c_c - [c_a delta_bc]_cyc (App. A) */
  double axxx = 0.0, axxy = 0.0, axyy = 0.0, ayyy = 0.0, agx = 0.0, agy = 0.0;
  for (int i = 0; i < s->Qf; i++) {
    const double cx = s->cfx[i], cy = s->cfy[i];
    axxx += f[i] * (cx * cx * cx - 3.0 * cx);
    axxy += f[i] * (cx * cx * cy - cy);
    axyy += f[i] * (cx * cy * cy - cx);
    ayyy += f[i] * (cy * cy * cy - 3.0 * cy);
  }
  for (int i = 0; i < 9; i++) { agx += g[i] * s->cgx[i]; agy += g[i] * s->cgy[i]; }
  for (int i = 0; i < s->Qf; i++) {
    const double cx = s->cfx[i], cy = s->cfy[i];
    const double contr = axxx * (cx * cx * cx - 3.0 * cx) + 3.0 * axxy * (cx * cx * cy - cy) +
                         3.0 * axyy * (cx * cy * cy - cx) + ayyy * (cy * cy * cy - 3.0 * cy);
    f[i] += kappa * s->Wf[i] * contr / 6.0;
  }
  for (int i = 0; i < 9; i++) g[i] += kappa * s->Wg[i] * (agx * s->cgx[i] + agy * s->cgy[i]);
}

/* ------------------------------------------------------------------------ */
/* Slope limiters (Sec. IV A 2).                                             */
/* reading: van Leer as (a|b| + |a|b)/(|a| + |b|), 0 when both vanish;      */
/* minmod as 0 when ab <= 0, else sign(a) min(|a|, |b|).                     */
/* ------------------------------------------------------------------------ */
static double limiter(int kind, double a, double b) {
  if (kind == PONDREF_LIM_MINMOD) {
    if (a * b <= 0.0) return 0.0;
    return a > 0.0 ? fmin(a, b) : fmax(a, b);
  }
  const double den = fabs(a) + fabs(b);
  if (den == 0.0) return 0.0;
  return (a * fabs(b) + fabs(a) * b) / den;
}

/* f populations from lattice q1s in frame src to lattice q1t in frame dst
   (1D: the D1Q4 map of the configured transform). */
static void xf_f(const pondref_state* s, int q1s, const double src[3], int q1t,
                 const double dst[3], const double* in, double* out) {
  double G[QMAX * QMAX];
  if (s->D == 1) {
    transform_matrix(1, &s->Lf, s->cfg.transform, src, dst, G);
    matvec(4, G, in, out);
    return;
  }
  ms_matrix(s->cfg.transform, q1s, src, q1t, dst, G);
  matvec_r(q1t * q1t, q1s * q1s, G, in, out);
}

/* ------------------------------------------------------------------------ */
/* Flux evaluation at one face (Sec. IV A 2).                                */
/* ------------------------------------------------------------------------ */
typedef struct {
  int L, R, LL, RR, Lp, Lm, Rp, Rm; /* padded cell indices of the stencil */
  int axis;                         /* 0: normal along x, 1: along y */
} face_stencil;

/* One reconstruction of a population at the face from upwind cell U:
   phi(x') = phi(x_U) + (x' - x_U) . sigma (MUSCL), x' = x_b - v dt/2.  In
   cell units: the normal offset is +-1/2 - v_n dt/(2 dx), the transverse one
   -v_t dt/(2 dx). */
static double reconstruct(int lim, double PU, double Pm, double Pp, double Ptm, double Ptp,
                          double dn, double dtv, int twod) {
  double val = PU + dn * limiter(lim, PU - Pm, Pp - PU);
  if (twod) val += dtv * limiter(lim, PU - Ptm, Ptp - PU);
  return val;
}

static void face_flux(const pondref_state* s, const face_stencil* st, double* fout, double* gout,
                      double* lout, unsigned char* qout) {
  const int D = s->D, Qf = s->Qf, Qg = s->Qg;
  /* reading: a face uses the higher-order f-lattice of its two cells, so
     D2Q16 regions extend to their boundary faces (the stencil's other
     cells are lifted or projected into it) */
  const int qF = s->lat[st->L] > s->lat[st->R] ? s->lat[st->L] : s->lat[st->R];
  const int lq = qF == 3 ? 1 : 0;
  const int QF = s->Qq[lq];
  const double* fcx = s->cxq[lq];
  const double* fcy = s->cyq[lq];
  const int twod = D == 2;
  const double lam = s->dt / s->dx;
  const int ncell = twod ? 8 : 4;
  const int cells[8] = {st->L, st->R, st->LL, st->RR, st->Lp, st->Lm, st->Rp, st->Rm};
  double Pf[8][QMAX], Pg[8][QMAX];
  double Gg[81];
  double fbar[QMAX], gbar[9];
  const double* frL = s->fr + 3 * st->L;
  const double* frR = s->fr + 3 * st->R;
  /* eq. AvgFrame: the face frame is the average of the adjacent cell frames */
  double lF[3] = {0.5 * (frL[0] + frR[0]), 0.5 * (frL[1] + frR[1]), 0.5 * (frL[2] + frR[2])};
  double rho_b = 0.0, u_b[2] = {0.0, 0.0}, T_b = 0.0;
  const int a = st->axis, t = 1 - st->axis;

  for (int pass = 0; pass <= s->cfg.n_corr; pass++) {
    /* transform the stencil's phi-bar-plus into the face frame */
    for (int k = 0; k < ncell; k++) {
      const int c = cells[k];
      xf_f(s, s->lat[c], s->fr + 3 * c, qF, lF, s->fbp + (size_t)c * Qf, Pf[k]);
      transform_matrix(D, &s->Lg, s->cfg.transform, s->fr + 3 * c, lF, Gg);
      matvec(Qg, Gg, s->gbp + (size_t)c * Qg, Pg[k]);
    }
    /* eq. InterfacePop with MUSCL at the departure point */
    const double rt = sqrt(lF[2]);
    for (int pop = 0; pop < 2; pop++) {
      const int Q = pop == 0 ? QF : Qg;
      const double* cx = pop == 0 ? fcx : s->cgx;
      const double* cy = pop == 0 ? fcy : s->cgy;
      double (*P)[QMAX] = pop == 0 ? Pf : Pg;
      double* out = pop == 0 ? fbar : gbar;
      for (int i = 0; i < Q; i++) {
        const double v[2] = {rt * cx[i] + lF[0], twod ? rt * cy[i] + lF[1] : 0.0};
        const double vn = v[a], vt = v[t];
        const double dtv = -0.5 * lam * vt;
        /* stencil slots: 0 L, 1 R, 2 L-e_a, 3 R+e_a, 4 L+e_t, 5 L-e_t, 6 R+e_t, 7 R-e_t */
        const double recL = reconstruct(s->cfg.limiter, P[0][i], P[2][i], P[1][i],
                                        twod ? P[5][i] : 0.0, twod ? P[4][i] : 0.0,
                                        0.5 - 0.5 * lam * vn, dtv, twod);
        const double recR = reconstruct(s->cfg.limiter, P[1][i], P[0][i], P[3][i],
                                        twod ? P[7][i] : 0.0, twod ? P[6][i] : 0.0,
                                        -0.5 - 0.5 * lam * vn, dtv, twod);
        /* upwind by the sign of the normal velocity.  reading: a normal
           velocity within TIE_BAND of the face thermal speed counts as zero
           (rounding noise around a fluid at rest must not pick a side), and
           a tie takes the mean of both reconstructions */
        const double band = TIE_BAND * rt;
        out[i] = vn > band ? recL : (vn < -band ? recR : 0.5 * (recL + recR));
      }
    }
    /* macroscopic fields at the face from f-bar and g-bar in lambda_F */
    double m0 = 0.0, m1[2] = {0.0, 0.0}, e = 0.0;
    for (int i = 0; i < QF; i++) {
      const double vx = rt * fcx[i] + lF[0];
      const double vy = twod ? rt * fcy[i] + lF[1] : 0.0;
      m0 += fbar[i];
      m1[0] += vx * fbar[i];
      m1[1] += vy * fbar[i];
      e += 0.5 * (vx * vx + vy * vy) * fbar[i];
    }
    for (int i = 0; i < Qg; i++) e += gbar[i];
    rho_b = m0;
    u_b[0] = m1[0] / m0;
    u_b[1] = m1[1] / m0;
    T_b = (e - 0.5 * m0 * (u_b[0] * u_b[0] + u_b[1] * u_b[1])) / (s->cv * m0);
    /* predictor-corrector: the next pass evaluates the face in the frame
       of the face moments just found */
    if (pass < s->cfg.n_corr) {
      lF[0] = u_b[0];
      lF[1] = u_b[1];
      lF[2] = T_b;
    }
  }
  /* face equilibrium in lambda_F: phi^eq = rho G_{u,T}^{lambda_F} W
     (eq. NonComovingEq) */
  const double lb[3] = {u_b[0], u_b[1], T_b};
  double feqc[QMAX], geqc[9], feq[QMAX], geq[9];
  comoving_eq(s, qF, rho_b, T_b, feqc, geqc);
  xf_f(s, qF, lb, qF, lF, feqc, feq);
  transform_matrix(D, &s->Lg, s->cfg.transform, lb, lF, Gg);
  matvec(Qg, Gg, geqc, geq);
  /* invert eq. FluxTransf: phi-bar = phi - (dt/4) Omega with BGK Omega */
  const double tau = s->tau1, dt = s->dt;
  for (int i = 0; i < Qf; i++)
    fout[i] = i < QF ? (4.0 * tau * fbar[i] + dt * feq[i]) / (4.0 * tau + dt) : 0.0;
  *qout = (unsigned char)qF;
  for (int i = 0; i < Qg; i++) gout[i] = (4.0 * tau * gbar[i] + dt * geq[i]) / (4.0 * tau + dt);
  lout[0] = lF[0];
  lout[1] = lF[1];
  lout[2] = lF[2];
}

/* ------------------------------------------------------------------------ */
/* Body force (App. D): Strang half step of d f_i / dt = F_i with           */
/* F_i = a . (v_i - u) / T f^eq_i, one explicit Euler step of dt / 2:        */
/* f* = f + (dt/2) F, which moves the velocity to u* = u + (dt/2) a.          */
/* reading: the printed F carries a minus sign that would decelerate the     */
/* flow while u* accelerates it; the sign is taken so that the force adds    */
/* (dt/2) rho a of momentum, as u* states.  In the comoving frame            */
/* (v - u)/T = c / sqrt(T) and f^eq = rho W.  Applied to the stored f~ (its  */
/* moments are those of f); g is not forced.  The cell then takes the       */
/* comoving frame of its new moments (u*, and T from the energy, which the   */
/* Euler step changes by (dt/2) rho a.u), re-gauged as after the update.    */
/* ------------------------------------------------------------------------ */
static void force_half_step(pondref_state* s, int c) {
  double* f = s->f + (size_t)c * s->Qf;
  double* g = s->g + (size_t)c * s->Qg;
  double* fr = s->fr + 3 * c;
  const double ax = s->cfg.accel[0], ay = s->cfg.accel[1];
  double rho = 0.0;
  for (int i = 0; i < 16; i++) rho += f[i];
  const double rt = sqrt(fr[2]);
  for (int i = 0; i < 16; i++)
    f[i] += 0.5 * s->dt * rho * s->Wf[i] * (ax * s->cfx[i] + ay * s->cfy[i]) / rt;
  double r2, ux, uy, T, Gg[81], tf[QMAX], tg[9];
  moments(s, 4, f, g, fr, &r2, &ux, &uy, &T, NULL);
  const double nfr[3] = {ux, uy, T};
  xf_f(s, 4, fr, 4, nfr, f, tf);
  transform_matrix(2, &s->Lg, s->cfg.transform, fr, nfr, Gg);
  matvec(9, Gg, g, tg);
  memcpy(f, tf, sizeof(double) * 16);
  memcpy(g, tg, sizeof(double) * 9);
  memcpy(fr, nfr, sizeof nfr);
}

/* ------------------------------------------------------------------------ */
/* One time step t_n -> t_{n+1}.                                             */
/* ------------------------------------------------------------------------ */
static void one_step(pondref_state* s) {
  const int nx = s->cfg.nx, ny = s->cfg.ny, D = s->D, Qf = s->Qf, Qg = s->Qg;
  const int twod = D == 2;
  const double tau = s->tau1, dt = s->dt, lam = dt / s->dx;

  const int forced = s->cfg.accel[0] != 0.0 || s->cfg.accel[1] != 0.0;
  /* body force, first half step (App. D) */
  if (forced) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) force_half_step(s, cidx(s, x, y));
  }

  /* multiscale: choose each cell's f-lattice for this step (Sec. IV C) */
  if (twod && s->cfg.flat == PONDREF_F_MULTISCALE) {
    fill_ghosts(s);
    switch_lattices(s);
  }

  /* Strang splitting, first quasi-equilibrium half step (Sec. IV B) */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const int c = cidx(s, x, y);
      qe_half_step(s, s->lat[c], s->f + (size_t)c * Qf, s->g + (size_t)c * Qg);
    }

  fill_ghosts(s);

  /* phi-bar-plus = phi + (dt/4) Omega (eq. Fbarplus), from the stored
     phi~ = phi - (dt/2) Omega (eq. variableTransform):
       phi-bar-plus = [(2 tau - dt/2) phi~ + (3 dt / 2) phi^eq] / (2 tau + dt) */
  const int ylo = twod ? -NG : 0, yhi = twod ? ny + NG : 1;
#pragma omp parallel for schedule(static)
  for (int y = ylo; y < yhi; y++)
    for (int x = -NG; x < nx + NG; x++) {
      const int c = cidx(s, x, y);
      const double* f = s->f + (size_t)c * Qf;
      const double* g = s->g + (size_t)c * Qg;
      const int Qc = s->Qq[s->lat[c] == 3 ? 1 : 0];
      double rho = 0.0;
      for (int i = 0; i < Qc; i++) rho += f[i];
      double feq[QMAX] = {0}, geq[9];
      comoving_eq(s, s->lat[c], rho, s->fr[3 * c + 2], feq, geq);
      for (int i = 0; i < Qf; i++)
        s->fbp[(size_t)c * Qf + i] = ((2.0 * tau - 0.5 * dt) * f[i] + 1.5 * dt * feq[i]) / (2.0 * tau + dt);
      for (int i = 0; i < Qg; i++)
        s->gbp[(size_t)c * Qg + i] = ((2.0 * tau - 0.5 * dt) * g[i] + 1.5 * dt * geq[i]) / (2.0 * tau + dt);
    }

  /* loop over faces: x-faces (face i sits between cells i-1 and i) */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; y++)
    for (int i = 0; i <= nx; i++) {
      face_stencil st;
      st.axis = 0;
      st.L = cidx(s, i - 1, y); st.R = cidx(s, i, y);
      st.LL = cidx(s, i - 2, y); st.RR = cidx(s, i + 1, y);
      if (twod) {
        st.Lp = cidx(s, i - 1, y + 1); st.Lm = cidx(s, i - 1, y - 1);
        st.Rp = cidx(s, i, y + 1); st.Rm = cidx(s, i, y - 1);
      } else {
        st.Lp = st.Lm = st.Rp = st.Rm = 0;
      }
      const size_t fi = (size_t)i + (size_t)(nx + 1) * y;
      face_flux(s, &st, s->ffx + fi * Qf, s->gfx + fi * Qg, s->lfx + fi * 3, s->latfx + fi);
    }
  if (twod) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; j++)
      for (int x = 0; x < nx; x++) {
        face_stencil st;
        st.axis = 1;
        st.L = cidx(s, x, j - 1); st.R = cidx(s, x, j);
        st.LL = cidx(s, x, j - 2); st.RR = cidx(s, x, j + 1);
        st.Lp = cidx(s, x + 1, j - 1); st.Lm = cidx(s, x - 1, j - 1);
        st.Rp = cidx(s, x + 1, j); st.Rm = cidx(s, x - 1, j);
        const size_t fi = (size_t)x + (size_t)nx * j;
        face_flux(s, &st, s->ffy + fi * Qf, s->gfy + fi * Qg, s->lfy + fi * 3, s->latfy + fi);
      }
  }

  /* loop over cells: fluxes into the cell frame (eq. fluxEq), DUGKS update
     (eq. FinalUpdateDUGKS), then the new comoving frame */
  const double b = (2.0 * tau - dt) / (2.0 * tau + dt), c_eq = 2.0 * dt / (2.0 * tau + dt);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const int c = cidx(s, x, y);
      double* f = s->f + (size_t)c * Qf;
      double* g = s->g + (size_t)c * Qg;
      double* fr = s->fr + 3 * c;
      double Gg[81];
      double flf[QMAX] = {0}, flg[9] = {0}, tf[QMAX] = {0}, tg[9];
      const double rt = sqrt(fr[2]);
      const int qc = s->lat[c], lc = qc == 3 ? 1 : 0, Qc = s->Qq[lc];
      const int nface = twod ? 4 : 2;
      for (int k = 0; k < nface; k++) {
        /* faces: west (-x), east (+x), south (-y), north (+y) */
        const double* pf; const double* pg; const double* lf;
        double sign;
        int axis, qf;
        if (k < 2) {
          const size_t fi = (size_t)(x + k) + (size_t)(nx + 1) * y;
          pf = s->ffx + fi * Qf; pg = s->gfx + fi * Qg; lf = s->lfx + fi * 3;
          qf = s->latfx[fi];
          sign = k == 0 ? -1.0 : 1.0;
          axis = 0;
        } else {
          const size_t fi = (size_t)x + (size_t)nx * (y + (k - 2));
          pf = s->ffy + fi * Qf; pg = s->gfy + fi * Qg; lf = s->lfy + fi * 3;
          qf = s->latfy[fi];
          sign = k == 2 ? -1.0 : 1.0;
          axis = 1;
        }
        /* face populations into the cell's frame and f-lattice */
        xf_f(s, qf, lf, qc, fr, pf, tf);
        transform_matrix(D, &s->Lg, s->cfg.transform, lf, fr, Gg);
        matvec(Qg, Gg, pg, tg);
        /* (v_i^lambda . n_c) in the cell frame */
        for (int i = 0; i < Qc; i++) {
          const double vn = axis == 0 ? rt * s->cxq[lc][i] + fr[0] : rt * s->cyq[lc][i] + fr[1];
          flf[i] += sign * vn * tf[i];
        }
        for (int i = 0; i < Qg; i++) {
          const double vn = axis == 0 ? rt * s->cgx[i] + fr[0] : rt * s->cgy[i] + fr[1];
          flg[i] += sign * vn * tg[i];
        }
      }
      double rho = 0.0;
      for (int i = 0; i < Qc; i++) rho += f[i];
      double feq[QMAX], geq[9];
      comoving_eq(s, qc, rho, fr[2], feq, geq);
      for (int i = 0; i < Qc; i++) f[i] = b * f[i] + c_eq * feq[i] - lam * flf[i];
      for (int i = 0; i < Qg; i++) g[i] = b * g[i] + c_eq * geq[i] - lam * flg[i];
      /* reading: the step ends in the comoving frame of the updated
         moments (the frame of t_{n+1}, Sec. IV A 1) */
      double r2, ux, uy, T;
      moments(s, qc, f, g, fr, &r2, &ux, &uy, &T, NULL);
      const double nfr[3] = {ux, twod ? uy : 0.0, T};
      xf_f(s, qc, fr, qc, nfr, f, tf);
      transform_matrix(D, &s->Lg, s->cfg.transform, fr, nfr, Gg);
      matvec(Qg, Gg, g, tg);
      memcpy(f, tf, sizeof(double) * Qc);
      memcpy(g, tg, sizeof(double) * Qg);
      memcpy(fr, nfr, sizeof nfr);
      /* second quasi-equilibrium half step */
      qe_half_step(s, qc, f, g);
      /* body force, second half step */
      if (forced) force_half_step(s, c);
    }
  s->nstep++;
}

int pondref_qe_half_step(int dim, double kappa, double* f, double* g) {
  /* kappa = (dt/2)(1/tau1 - 1/tau2); a throwaway state carries the lattice */
  pondref_config c;
  memset(&c, 0, sizeof c);
  c.dim = dim; c.nx = 1; c.ny = 1; c.gamma = 1.4; c.tau = 1.0; c.prandtl = 1.0; c.cfl = 0.2;
  c.bc[0] = c.bc[1] = c.bc[2] = c.bc[3] = PONDREF_BC_PERIODIC;
  pondref_state* s;
  if (pondref_create(&c, &s)) return -1;
  s->dt = 1.0;
  s->tau1 = 1.0;
  s->tau2 = 1.0 / (1.0 - 2.0 * kappa); /* so that (dt/2)(1/tau1 - 1/tau2) = kappa */
  qe_half_step(s, 4, f, g);
  pondref_destroy(s);
  return 0;
}

int pondref_step(pondref_state* s, int nsteps) {
  if (!(s->dt > 0.0)) return fail("fields not initialised");
  for (int k = 0; k < nsteps; k++) one_step(s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Observables and state access.                                             */
/* ------------------------------------------------------------------------ */
int pondref_moments(const pondref_state* s, double* rho, double* ux, double* uy, double* T) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const int c = cidx(s, x, y), k = x + nx * y;
      double r, a, b, t;
      moments(s, s->lat[c], s->f + (size_t)c * s->Qf, s->g + (size_t)c * s->Qg, s->fr + 3 * c, &r, &a, &b, &t, NULL);
      if (rho) rho[k] = r;
      if (ux) ux[k] = a;
      if (uy) uy[k] = b;
      if (T) T[k] = t;
    }
  return 0;
}

int pondref_totals(const pondref_state* s, double out[4]) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  double tot[4] = {0, 0, 0, 0};
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const int c = cidx(s, x, y);
      double r, a, b, t, e;
      moments(s, s->lat[c], s->f + (size_t)c * s->Qf, s->g + (size_t)c * s->Qg, s->fr + 3 * c, &r, &a, &b, &t, &e);
      tot[0] += r; tot[1] += r * a; tot[2] += r * b; tot[3] += e;
    }
  memcpy(out, tot, sizeof tot);
  return 0;
}

int pondref_get_state(const pondref_state* s, double* f, double* g, double* frame) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const size_t n = (size_t)nx * ny;
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const int c = cidx(s, x, y);
      const size_t k = (size_t)x + (size_t)nx * y;
      if (f) for (int i = 0; i < s->Qf; i++) f[i * n + k] = s->f[(size_t)c * s->Qf + i];
      if (g) for (int i = 0; i < s->Qg; i++) g[i * n + k] = s->g[(size_t)c * s->Qg + i];
      if (frame) for (int i = 0; i < 3; i++) frame[i * n + k] = s->fr[3 * c + i];
    }
  return 0;
}

int pondref_set_state(pondref_state* s, const double* f, const double* g, const double* frame) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const size_t n = (size_t)nx * ny;
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const int c = cidx(s, x, y);
      const size_t k = (size_t)x + (size_t)nx * y;
      for (int i = 0; i < s->Qf; i++) s->f[(size_t)c * s->Qf + i] = f[i * n + k];
      for (int i = 0; i < s->Qg; i++) s->g[(size_t)c * s->Qg + i] = g[i * n + k];
      for (int i = 0; i < 3; i++) s->fr[3 * c + i] = frame[i * n + k];
      if (!(s->fr[3 * c + 2] > 0.0)) return fail("frame temperature must be positive");
    }
  return 0;
}

int pondref_get_lattice(const pondref_state* s, int* q, double* theta) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      const size_t k = (size_t)x + (size_t)nx * y;
      const int q1 = s->lat[cidx(s, x, y)];
      if (q) q[k] = s->D == 2 ? q1 * q1 : q1;
      if (theta) theta[k] = s->theta[k];
    }
  return 0;
}

int pondref_get_faces(const pondref_state* s, double* fx, double* gx, double* lx, double* fy,
                      double* gy, double* ly) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const size_t nfx = (size_t)(nx + 1) * ny;
  if (fx) memcpy(fx, s->ffx, sizeof(double) * nfx * s->Qf);
  if (gx) memcpy(gx, s->gfx, sizeof(double) * nfx * s->Qg);
  if (lx) memcpy(lx, s->lfx, sizeof(double) * nfx * 3);
  if (s->D == 2) {
    const size_t nfy = (size_t)nx * (ny + 1);
    if (fy) memcpy(fy, s->ffy, sizeof(double) * nfy * s->Qf);
    if (gy) memcpy(gy, s->gfy, sizeof(double) * nfy * s->Qg);
    if (ly) memcpy(ly, s->lfy, sizeof(double) * nfy * 3);
  }
  return 0;
}
