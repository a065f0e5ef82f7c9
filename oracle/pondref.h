/*
 * pondref.h -- FP64 CPU oracle of the Particles-on-Demand finite-volume step
 * (Kallikounis & Karlin, "Particles on Demand method: theoretical analysis,
 * simplification techniques and model extensions", arXiv 2302.00310).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct implementation written straight
 * from the paper.  It shares no code, header or table with the GPU library.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Layouts (all host memory, owned by the caller):
 *   fields   : row-major [ny][nx], x fastest.
 *   f states : [Qf][ny][nx]  population planes, i = ix + q1*iy, nodes ascending.
 *   g states : [Qg][ny][nx].
 *   frame    : [3][ny][nx]   (u_x, u_y, T) of the frame each cell's populations
 *                            are written in.
 * Return codes: 0 success, negative on error (message via pondref_last_error).
 */
#ifndef PONDREF_H
#define PONDREF_H
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { PONDREF_TF_LAGRANGE = 0, PONDREF_TF_GRAD = 1 };
/* Walls (Sec. IV D, 2D with the D2Q16 f-lattice): ghost cells mirror the
   cells next to the wall -- density even, velocity and temperature odd
   about the wall's values -- and carry the Chapman-Enskog non-equilibrium
   of the mirrored gradients. */
enum { PONDREF_BC_PERIODIC = 0, PONDREF_BC_ZERO_GRADIENT = 1, PONDREF_BC_INFLOW = 2,
       PONDREF_BC_WALL = 3 };
enum { PONDREF_LIM_VANLEER = 0, PONDREF_LIM_MINMOD = 1 };
/* 2D f-lattice (Sec. III C): D2Q16 everywhere, D2Q9 everywhere, the
   multiscale D2Q9/D2Q16 deployment chosen cell by cell (Sec. IV C), or
   D2Q25 everywhere with the fourth-order Grad projection (Sec. III B, the
   full invariant moment system; Sec. V shock structure). */
enum { PONDREF_F_D2Q16 = 0, PONDREF_F_D2Q9 = 1, PONDREF_F_MULTISCALE = 2, PONDREF_F_D2Q25 = 3 };

typedef struct {
  int dim, nx, ny;          /* ny = 1 when dim = 1 */
  int transform;            /* PONDREF_TF_* */
  double gamma;             /* C_v = 1/(gamma-1) */
  double tau;               /* tau1 / dt */
  double prandtl;           /* tau1 / tau2, in (0, 1] */
  double cfl;               /* dt = cfl*dx/max|v_ia| at t = 0 */
  double dx;                /* 0 -> 1/nx */
  int bc[4];                /* -x, +x, -y, +y */
  double inflow[4][4];      /* rho, u_x, u_y, p per side */
  int limiter;              /* PONDREF_LIM_* */
  int n_corr;               /* face-frame corrector passes */
  int flat;                 /* PONDREF_F_* (2D only; 0 in 1D) */
  double ms_threshold;      /* multiscale switch: D2Q16 where the gradient
                               indicator reaches this value (dilated by two
                               cells), D2Q9 elsewhere */
  double wall[4][3];        /* u_x, u_y, T of the wall per side (used if WALL;
                               T > 0, no velocity normal to the wall) */
  double accel[2];          /* body-force acceleration a (App. D; 2D, D2Q16);
                               0 = no force */
} pondref_config;

typedef struct pondref_state pondref_state;

const char* pondref_last_error(void);
int pondref_create(const pondref_config* cfg, pondref_state** out);
void pondref_destroy(pondref_state* s);
/* Comoving equilibrium from primitive fields; fixes dt unless set_dt was called. */
int pondref_init_fields(pondref_state* s, const double* rho, const double* ux,
                        const double* uy, const double* p);
/* dt the CFL rule gives for these fields (no state needed). */
double pondref_cfl_dt(const pondref_config* cfg, const double* rho, const double* ux,
                      const double* uy, const double* p);
int pondref_set_dt(pondref_state* s, double dt);
double pondref_get_dt(const pondref_state* s);
int pondref_step(pondref_state* s, int nsteps);
int pondref_moments(const pondref_state* s, double* rho, double* ux, double* uy, double* T);
int pondref_totals(const pondref_state* s, double out[4]);
int pondref_get_state(const pondref_state* s, double* f, double* g, double* frame);
int pondref_set_state(pondref_state* s, const double* f, const double* g, const double* frame);
/* Face data of the last step: populations phi^{lambda_F}(x_b, t+1/2) and the
   face frame.  x-faces: [(nx+1)*ny] (face i between cells i-1 and i of row
   j at index i + (nx+1)*j); y-faces: [nx*(ny+1)].  Pops are [face][Q]. */
int pondref_get_faces(const pondref_state* s, double* fx, double* gx, double* lx,
                      double* fy, double* gy, double* ly);
int pondref_set_threads(int n);
int pondref_get_threads(void);

/* Building blocks exposed for pin tests.
   lattice: 0 = D1Q4 (f), 1 = D1Q3 (g), 2 = D1Q5 (f of D2Q25).  Nodes and
   weights in ascending order. */
int pondref_lattice(int lattice, double* c, double* w);
/* Dense transform matrix G (Q x Q, row = target population) mapping
   populations written in frame src = (u_x, u_y, T) to frame dst, for the
   tensor lattice of dimension dim.  transform: PONDREF_TF_*. */
int pondref_transform_matrix(int dim, int lattice, int transform, const double src[3],
                             const double dst[3], double* G);
/* Same map for the Lagrange (moment-matching) transform, built by solving the
   full Q x Q moment system of App. B without using the tensor structure. */
int pondref_transform_matrix_full(int dim, int lattice, const double src[3],
                                  const double dst[3], double* G);

/* Multiscale frame transformation of a 2D f-lattice (Sec. III C): q1s, q1t
   are the 1D node counts of the source and target lattices (4: D2Q16,
   3: D2Q9).  Same lattice: Grad's projection of order q1 - 1.  q1s = 3,
   q1t = 4 (lifting): the D2Q16 expansion whose moments of total order <= 2
   are those of the D2Q9 populations and whose third-order Hermite moments
   take their equilibrium value (zero) in the source's comoving frame.
   q1s = 4, q1t = 3 (projection): Grad's expansion of order 2 from the D2Q16
   moments.  G is (q1t^2) x (q1s^2), row = target population. */
int pondref_ms_matrix(int q1s, const double src[3], int q1t, const double dst[3], double* G);
/* Per cell (row-major [ny][nx]): the f-lattice's population count (16 or 9)
   and the switch indicator of the last step
   theta = dx (|grad u| / sqrt(gamma T) + |grad T| / T) (0 when not
   multiscale).  Either pointer may be NULL. */
int pondref_get_lattice(const pondref_state* s, int* q, double* theta);

/* Ghost cell `layer` (1 or 2) of wall side `side` (0 -x, 1 +x, 2 -y, 3 +y)
   at coordinate t along the wall, built from the current state: f~ (16),
   g~ (9) in the ghost's comoving frame (u_x, u_y, T). */
int pondref_wall_ghost(const pondref_state* s, int side, int layer, int t, double* f,
                       double* g, double frame[3]);

/* One quasi-equilibrium half step on a single cell's f (Qf) and g (Qg),
   written in their comoving frame; kappa = (dt/2)(1/tau1 - 1/tau2). */
int pondref_qe_half_step(int dim, double kappa, double* f, double* g);

#ifdef __cplusplus
}
#endif
#endif
