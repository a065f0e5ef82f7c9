/*
 * pond.h -- C interface of libpond.so, an MI355X (gfx950) implementation of
 * the Particles-on-Demand (PonD) finite-volume time step of Kallikounis &
 * Karlin, "Particles on Demand method: theoretical analysis, simplification
 * techniques and model extensions" (arXiv 2302.00310).
 *
 * State of a solve (Sec. II A, III A, IV A 1): on every cell j of a 1D or 2D
 * Cartesian grid, populations f~ (D1Q4 / D2Q16, Table I) and g~ (D1Q3 /
 * D2Q9) written in the cell's comoving frame lambda_j = {u_j, T_j}, with
 * particle velocities v_i = sqrt(T_j) c_i + u_j (eq. veli, T_L = 1).  The
 * library keeps, per cell, the conserved moments (rho, rho u, rho E) of eq.
 * ConservationLaws as 64-bit fixed-point integers (the frame is derived from
 * them) and the non-equilibrium parts f~ - rho W and g~ - (C_v - D/2) T rho W
 * (eqs. feqPond, geqPond) as planes of FP64 (POND_FP64) or FP32 (POND_MIXED).
 *
 * One step (pond_step) is the scheme of Sec. IV A-B: quasi-equilibrium half
 * step (eq. QE_relaxation), ghost cells (Sec. IV D), face frame by averaging
 * (eq. AvgFrame) plus n_corr corrector passes, moment-matching transforms of
 * the stencil into the face frame (Sec. II B, App. B), MUSCL half-step
 * reconstruction (eq. InterfacePop), face equilibrium (eq. NonComovingEq),
 * fluxes back into the cell frames (eq. fluxEq), DUGKS update (eq.
 * FinalUpdateDUGKS), new comoving frame, second quasi-equilibrium half step.
 *
 * Conventions
 *  - Every call returns an int status: 0 (POND_OK), 1 (POND_PENDING) or a
 *    negative POND_ERR_* code; pond_last_error() gives the message of the
 *    last failure on the calling thread.
 *  - Host arrays are owned by the caller and are only read or written during
 *    the call.  Fields are row-major [ny][nx], x fastest, FP64.
 *  - The device arena (dev_arena, arena_bytes) and the HIP stream are owned
 *    by the caller, must outlive the state, and the library places all of the
 *    state's device buffers inside the arena.  Work is enqueued on the stream.
 *  - A pond_state is not thread-safe; server calls are.
 *  - The library requires a gfx950 device; it has no CPU fallback.
 */
#ifndef POND_H
#define POND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  POND_OK = 0,
  POND_PENDING = 1,
  POND_ERR_INVALID = -1,     /* bad config or argument */
  POND_ERR_NOMEM = -2,       /* arena smaller than pond_state_bytes() */
  POND_ERR_DEVICE = -3,      /* HIP runtime error */
  POND_ERR_UNSTABLE = -4,    /* rho <= 0, T <= 0, non-finite value or ledger overflow */
  POND_ERR_REJECTED = -5,    /* serving: footprint larger than the whole arena */
  POND_ERR_UNSUPPORTED = -6  /* valid request the library does not implement */
};

/* f-lattice (the g-lattice is D1Q3 / D2Q9), Table I */
enum { POND_D1Q4 = 1, POND_D2Q16 = 2, POND_D2Q9 = 3, POND_D2Q9_D2Q16 = 4, POND_D2Q25 = 5 };
/* POND_D2Q25: the fourth-order f-lattice (tensor of the 5-point
   Gauss-Hermite rule, Table I) with the fourth-order Grad projection
   (Sec. III B, full invariant moment system): needs POND_TF_GRAD and dim 2;
   no walls or body force.  Runs as four plain kernel launches per step
   (cell pass, x- and y-face passes, update) with the face data in the
   arena (not fused like D2Q16). */
/* POND_D2Q9: the second-order f-lattice everywhere.  POND_D2Q9_D2Q16: the
   multiscale deployment (Sec. III C, Sec. IV C) -- each step, D2Q16 within
   two cells of a cell whose gradient indicator
   dx (|grad u| / sqrt(gamma T) + |grad T| / T) reaches ms_threshold, D2Q9
   elsewhere, with the lifting / projection maps between them.  Both need
   POND_TF_GRAD and dim 2.  With the D2Q9 f-lattice the update does not
   conserve energy exactly (App. C): a D2Q9 cell takes the energy of its
   populations. */
/* POND_MIXED: FP32 populations, transforms and collision; FP64 gauge,
   temperature recovery and conservative flux sums. */
enum { POND_FP64 = 0, POND_MIXED = 1 };
/* Frame transformation: POND_TF_LAGRANGE is the square moment-matching map
   G = [M^{lambda'}]^{-1} M^{lambda} of App. B (tensor Lagrange
   interpolation); POND_TF_GRAD is Grad's projection of eq. GradsProjection
   truncated at total order q-1. */
enum { POND_TF_LAGRANGE = 0, POND_TF_GRAD = 1 };
/* Boundary conditions (Sec. IV D).  ZERO_GRADIENT copies the nearest cell;
   INFLOW imposes the comoving equilibrium of a fixed state.  WALL (2D,
   POND_D2Q16 only): the two ghost layers mirror the cells next to the wall
   -- density kept, velocity and temperature reflected about the wall's
   values -- in their comoving frame, plus the first-order Chapman-Enskog
   non-equilibrium of the mirrored gradients (central differences of the
   state at the start of the step).  A ghost off the end of a wall takes
   the coordinate along the wall the x-then-y ghost rule gives it.  Mass
   is not exactly conserved through a wall (the ghosts are not exact
   reflections of the populations). */
enum { POND_BC_PERIODIC = 0, POND_BC_ZERO_GRADIENT = 1, POND_BC_INFLOW = 2, POND_BC_WALL = 3 };
enum { POND_LIM_VANLEER = 0, POND_LIM_MINMOD = 1 };

typedef struct {
  int dim, nx, ny;           /* dim 1 or 2; ny = 1 when dim = 1; nx, ny >= 4 (2D), nx >= 4 (1D) */
  int lattice;               /* POND_D1Q4 (dim 1); POND_D2Q16, POND_D2Q9, POND_D2Q9_D2Q16 or
                                POND_D2Q25 (dim 2) */
  int transform;             /* POND_TF_* */
  int precision;             /* POND_FP64 or POND_MIXED */
  double gamma;              /* adiabatic exponent, > 1; C_v = 1/(gamma - 1) */
  double tau;                /* tau1 / dt, > 0 (BGK relaxation time in time steps) */
  double prandtl;            /* Pr = tau1 / tau2, in (0, 1] */
  double cfl;                /* dt = cfl dx / max|sqrt(T) c_ia + u_a| at t = 0 (Sec. V) */
  double dx;                 /* cell size; 0 -> 1/nx */
  int bc[4];                 /* POND_BC_* on the -x, +x, -y, +y sides */
  double inflow[4][4];       /* per side (rho, u_x, u_y, p), used where bc = INFLOW */
  int limiter;               /* POND_LIM_* (slopes of the MUSCL reconstruction) */
  int n_corr;                /* face-frame corrector passes, 0..4; 0 = the explicit scheme */
  double ms_threshold;       /* POND_D2Q9_D2Q16 switch threshold, >= 0 (0.05 is typical) */
  double wall[4][3];         /* per side (u_x, u_y, T) of the wall, used where bc = WALL:
                                T > 0 and no velocity along the wall's normal */
  double accel[2];           /* body-force acceleration a (App. D), 0 = none; dim 2 and
                                POND_D2Q16 only.  Each step is wrapped in two half steps
                                f~ += (dt/2) rho W a.c / sqrt(T) (comoving frame, explicit
                                Euler), each followed by the move to the new comoving
                                frame: momentum gains (dt/2) rho a per half step */
} pond_config;

typedef struct pond_state pond_state;

/* Copies the message of the calling thread's last failure into buf
   (NUL-terminated, at most n bytes).  Returns POND_OK. */
int pond_last_error(char* buf, size_t n);

/* Device bytes a solve with this configuration needs (0 if invalid). */
size_t pond_state_bytes(const pond_config* cfg);

/* Validates cfg, places the state in [dev_arena, dev_arena + arena_bytes)
   (device memory, 256-byte aligned), records hip_stream (a hipStream_t; NULL
   = default stream) and returns a handle in *out.  Errors: POND_ERR_INVALID,
   POND_ERR_NOMEM, POND_ERR_DEVICE (no gfx950 device). */
int pond_create(const pond_config* cfg, void* dev_arena, size_t arena_bytes, void* hip_stream,
                pond_state** out);

/* Initial data (Sec. IV A 3, item 1): the comoving equilibrium of the
   primitive fields rho, u_x, u_y (ignored in 1D, may be NULL) and p, host
   arrays of nx*ny doubles; T = p / rho.  Fixes dt by the CFL rule and the
   fixed-point scale of the conserved moments.  Blocks until the copy is
   done.  Errors: POND_ERR_INVALID (non-positive rho or p, non-finite input). */
int pond_init_fields(pond_state* s, const double* rho, const double* ux, const double* uy,
                     const double* p);

/* Enqueues nsteps >= 0 time steps on the stream and returns without waiting. */
int pond_step(pond_state* s, int nsteps);

/* Waits for the stream, then writes rho, u_x, u_y, T (host arrays of nx*ny
   doubles; any may be NULL) from the conserved moments.  Returns
   POND_ERR_UNSTABLE if a step met rho <= 0, T <= 0, a non-finite value or a
   ledger overflow since creation. */
int pond_moments(pond_state* s, double* rho, double* ux, double* uy, double* T);

/* Waits for the stream, then sums the conserved moments over all cells
   exactly (integer sum of the fixed-point ledger) and returns the totals of
   rho, rho u_x, rho u_y, rho E, each rounded once to double, times the cell
   volume dx^dim. */
int pond_totals(pond_state* s, double out[4]);

/* The same exact totals as 128-bit integers in units of 2^-scale_bits (before
   the volume factor): out[2k] = high 64 bits (signed), out[2k+1] = low 64
   bits, k = rho, rho u_x, rho u_y, rho E.  Bitwise comparison of two calls
   checks exact conservation. */
int pond_totals_fixed(pond_state* s, int64_t out[8], int* scale_bits);

/* Waits for the stream and writes the populations f~ (Qf planes of nx*ny
   doubles, i = i_x + q i_y, nodes ascending), g~ (Qg planes) and the frame
   (u_x, u_y, T planes) they are written in.  Any pointer may be NULL.
   Qf = 25 for POND_D2Q25 solves (i = i_x + 5 i_y). */
int pond_export_state(pond_state* s, double* f, double* g, double* frame);

/* Per cell (row-major [ny][nx], host arrays, either may be NULL): the
   f-lattice's population count the state is written in (16 or 9) and the
   switch indicator of the last step (zeros unless POND_D2Q9_D2Q16).  Waits
   for the stream. */
int pond_lattice_map(pond_state* s, int* q, double* theta);

/* dt in use and the number of steps taken. */
int pond_get_time(pond_state* s, double* dt, int64_t* nsteps);

/* Checkpoint: the raw device state (conserved-moment ledger, non-equilibrium
   planes, dt, step count and configuration) to / from a file.  pond_load
   requires a state created with an identical configuration. */
int pond_save(pond_state* s, const char* path);
int pond_load(pond_state* s, const char* path);

/* Waits for the stream and releases the handle (the arena stays the caller's). */
int pond_destroy(pond_state* s);

/* Gauss--Hermite constants compiled into the kernels (Table I), for checks
   without a GPU: out[0..3] D1Q4 nodes, out[4..7] weights, out[8..10] D1Q3
   nodes, out[11..13] weights. */
int pond_lattice_constants(double out[14]);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of independent solves.                      */
/* ------------------------------------------------------------------------ */
typedef struct pond_server pond_server;

typedef struct {
  pond_config cfg;                   /* any configuration pond_create accepts */
  const double *rho, *ux, *uy, *p;   /* initial fields, copied by pond_submit */
  int nsteps;
  uint64_t tag;                      /* caller's label, echoed in the result */
} pond_request;

typedef struct {
  int status;                        /* POND_OK, POND_PENDING or POND_ERR_* */
  double *rho, *ux, *uy, *T;         /* caller-provided nx*ny arrays, filled when done (may be NULL) */
  double t_submit, t_admit, t_done;  /* seconds on the server's clock */
  uint64_t tag;
} pond_result;

/* Starts a server thread that owns [dev_arena, dev_arena + bytes) and the
   stream, and keeps at most max_active solves resident. */
int pond_server_create(void* dev_arena, size_t bytes, void* hip_stream, int max_active,
                       pond_server** out);
/* Copies the request's inputs and queues it; never waits for the GPU.
   POND_ERR_REJECTED if its footprint exceeds the whole arena; the error of
   validation for a configuration pond_create would reject.  Mixed-precision
   2D solves on the D2Q16, D2Q9 and multiscale f-lattices share one batched
   step kernel per step; FP64, 1D and D2Q25 solves run their own step
   kernels in the same per-chunk graph.  A result equals the same solve run
   alone through pond_step, bit for bit. */
int pond_submit(pond_server* srv, const pond_request* req, uint64_t* id);
/* POND_PENDING while the solve is queued or running; otherwise copies the
   moments into res' arrays, fills the times and returns the solve's status
   (once: the result is released after a non-pending poll). */
int pond_poll(pond_server* srv, uint64_t id, pond_result* res);
/* Counters since pond_server_create (seconds on the server's clock):
   out[0] elapsed, out[1] cell-updates advanced, out[2] batched chunks
   launched, out[3] changes of the resident set, and host time spent in
   out[4] admissions (state set-up and initial fields), out[5] retirements
   (moments to host, including the wait for the GPU), out[6] batch-table
   uploads, out[7] graph captures; out[8] GPU time of the step chunks
   finished so far (HIP events around each chunk).  Serving metrics only;
   not on the step path. */
int pond_server_stats(pond_server* srv, double out[9]);
/* Stops admitting, finishes or drops queued work, joins the thread. */
int pond_server_destroy(pond_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* POND_H */
