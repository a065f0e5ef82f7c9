// Internal declarations shared by the HIP kernels and the host side of
// libpond.so.  Not part of the public interface (include/pond.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pond {

// Gauss--Hermite constants of Table I (T_L = 1), correctly rounded from the
// closed forms.  D1Q4 nodes in ascending order: -B, -A, A, B with weights
// WB, WA, WA, WB; D1Q3 nodes -R3, 0, R3 with weights 1/6, 2/3, 1/6.
constexpr double kA = 0.7419637843027258;     // sqrt(3 - sqrt 6)
constexpr double kB = 2.3344142183389773;     // sqrt(3 + sqrt 6)
constexpr double kA2 = 0.5505102572168219;    // 3 - sqrt 6
constexpr double kB2 = 5.449489742783178;     // 3 + sqrt 6
constexpr double kWA = 0.4541241452319315;    // (3 + sqrt 6) / 12
constexpr double kWB = 0.04587585476806849;   // (3 - sqrt 6) / 12
constexpr double kKA = -0.13755667699048205;  // 1 / (2A (A^2 - B^2))
constexpr double kKB = 0.04372063527294086;   // 1 / (2B (B^2 - A^2))
constexpr double kR3 = 1.7320508075688772;    // sqrt 3
// D1Q5 (the 1D factor of D2Q25): nodes -B5, -A5, 0, A5, B5, weights
// W5B, W5A, 8/15, W5A, W5B.
constexpr double kA5 = 1.355626179974266;     // sqrt(5 - sqrt 10)
constexpr double kB5 = 2.8569700138728056;    // sqrt(5 + sqrt 10)
constexpr double kW5A = 0.22207592200561266;  // (7 + 2 sqrt 10) / 60
constexpr double kW5B = 0.01125741132772069;  // (7 - 2 sqrt 10) / 60

// Tile shapes of the fused step kernel.
constexpr int kTX2 = 16, kTY2 = 15;  // 2D: 240 cells, 255 x-faces, 256 y-faces
constexpr int kTX1 = 255;            // 1D: 255 cells, 256 faces
constexpr int kThreads = 256;

// Everything one launch of the step kernel needs (passed by value).
struct StepArgs {
  int nx, ny;
  int bc[4];
  int n_corr, limiter, transform;  // transform: 0 Lagrange (App. B), 1 Grad projection
  int tiles_x, tiles_y;
  double inv_scale;        // 2^-E: fixed-point unit of the conserved-moment ledger
  double scale;            // 2^E
  double cv, icv, geq;     // C_v, 1/C_v, C_v - D/2
  double lam;              // dt / dx
  double a_pre;            // (2 tau - dt/2) / (2 tau + dt)
  double b_upd;            // (2 tau - dt) / (2 tau + dt)
  double c_face1, c_face2; // 4 tau / (4 tau + dt), dt / (4 tau + dt)
  double kappa;            // (dt/2) (1/tau1 - 1/tau2)
  const long long* inflow; // device table [side][q] of the inflow states' fixed-point moments
  size_t cells;            // nx * ny: stride between planes
  const void* n_in;        // Qf + Qg planes of non-equilibrium populations
  void* n_out;
  const long long* U_in;   // 4 planes: rho, rho u_x, rho u_y, rho E (fixed point)
  long long* U_out;
  int* flag;               // bit 1: non-physical state, bit 2: ledger overflow
  // multiscale f-lattices (per cell, 4 = D2Q16, 3 = D2Q9 nodes per axis):
  // the lattice n_in is written in, and the one this step uses and writes
  const unsigned char* lat_in;
  const unsigned char* lat_out;
  int ms;                  // kernel mode: 0 D2Q16, 1 multiscale, 2 D2Q16 with walls or force, 3 D2Q9
  // multiscale: words that are 0 when no cell of lat_in / lat_out is on
  // D2Q16 (null elsewhere); such a step runs in the D2Q9 kernel
  const int* q16_in;
  const int* q16_out;
  // walls: ghost layer k (1, 2) of side s at coordinate t along the wall is
  // entry (2 s + k - 1) wall_len + t of wall_n-long planes, written before
  // each step by the wall-ghost kernel and read by the tile loader
  const long long* wU;     // 4 fixed-point ledger planes
  const void* wN;          // NP non-equilibrium population planes
  int wall_len;
  size_t wall_n;
  double wall[4][3];       // (u_x, u_y, T) of each side's wall
  double idx2;             // 1 / (2 dx)
  double tau1, tau2;       // relaxation times (tau2 = tau1 / Pr)
  double kf;               // 1 + dt / (2 tau1): non-equilibrium scaling of the stored variable
  int force;               // 1: body force (2D, D2Q16)
  double hax, hay;         // (dt/2) a: body-force acceleration times half a step
};

// One solve of a batched step launch: the arguments of its even and odd
// steps (ping-pong buffers swapped) and the first block of its tile range.
struct BatchEntry {
  StepArgs args[2];
  int tile_begin;
  int tiles;
};

// Host-side launchers (defined in pond_kernels.hip).
// Step kernels by kind: transform t (0 Lagrange, 1 Grad) and mode ms (0:
// D2Q16 everywhere; 1: per-cell f-lattices, D2Q9 or multiscale, Grad only;
// 2: D2Q16 with walls or a body force -- their loader and update carry the
// extra work, which the plain kernels leave out; 3: D2Q9 everywhere).
constexpr int kind_of(int transform, int ms) { return transform + 2 * ms; }
// kind_mask: bit kind_of(t, ms) set launches that kernel (a batch may hold
// solves of several kinds; each kernel skips the others' blocks).
hipError_t launch_step_batch(bool fp64, unsigned kind_mask, const BatchEntry* tab, int n,
                             int total_tiles, int parity, hipStream_t st);
// Multiscale switch of one solve: the indicator theta per cell from the
// ledger's frames, then the f-lattice (4 or 3 nodes per axis) per cell.
// q16_out: set to 1 if any cell gets D2Q16 (cleared first).
hipError_t launch_switch(const StepArgs& a, const long long* U, double threshold, double gamma,
                         int* q16_out,
                         double* theta, unsigned char* lat_out, hipStream_t st);
hipError_t launch_step_1d(bool fp64, const StepArgs& a, hipStream_t st);
// One step of a D2Q25 solve (cell pass, x- and y-face passes, update),
// a.n_in/U_in -> a.n_out/U_out, with the intermediate buffers given.
hipError_t launch_q25_step(bool fp64, const StepArgs& a, void* P, double* fr, void* fpx, void* fpy,
                           double* ffx, double* ffy, long long* psx, long long* psy,
                           hipStream_t st);
// Wall ghosts of one 2D solve from the ledger a.U_in, written to wU / wN
// (the buffers a.wU / a.wN point to).
hipError_t launch_wall_ghosts(bool fp64, const StepArgs& a, long long* wU, void* wN,
                              hipStream_t st);
hipError_t launch_init(int dim, bool fp64, const double* fields, size_t cells, size_t first,
                       size_t count, double scale, double cv, void* n, long long* U,
                       hipStream_t st);
hipError_t launch_moments(int dim, const long long* U, size_t cells, size_t first, size_t count,
                          double inv_scale, double icv, double* out, hipStream_t st);
hipError_t launch_export(int dim, bool fp64, const void* n, const long long* U, size_t cells,
                         size_t first, size_t count, double inv_scale, double icv, double geq,
                         double* out, hipStream_t st);
hipError_t launch_totals(const long long* U, size_t cells, int blocks, long long* out,
                         hipStream_t st);

}  // namespace pond
