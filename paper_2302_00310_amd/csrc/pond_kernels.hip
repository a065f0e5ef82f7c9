// HIP kernels of the PonD finite-volume time step for gfx950.
//
// One fused kernel per time step.  A workgroup owns a tile of cells; it
//   0. loads the tile plus a two-cell halo (ghost cells resolved on the fly,
//      Sec. IV D), derives each cell's comoving frame from its conserved
//      moments, applies the first quasi-equilibrium half step (eq.
//      QE_relaxation) and stores phi-bar-plus (eq. Fbarplus) in LDS;
//   1. evaluates every x-face of the tile (face frame eq. AvgFrame plus
//      corrector passes, stencil transforms into the face frame, MUSCL
//      half-step reconstruction eq. InterfacePop, face equilibrium eq.
//      NonComovingEq, inversion of eq. FluxTransf) into LDS;
//   2. transforms the west/east face populations into each cell's frame
//      (eq. fluxEq) and accumulates the flux;
//   3./4. the same for the y-faces;
//   5. applies the DUGKS update (eq. FinalUpdateDUGKS), moves the cell to the
//      comoving frame of its new conserved moments, applies the second
//      quasi-equilibrium half step and writes the cell back.
// The conserved moments of every cell are a 64-bit fixed-point ledger that
// each face updates by one rounded flux, added to one neighbour and
// subtracted from the other, so their totals are conserved exactly.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pond_internal.h"

namespace pond {
namespace {

constexpr int BC_PERIODIC = 0, BC_ZERO_GRADIENT = 1;
constexpr int LIM_MINMOD = 1;
constexpr double kTieBand = 1e-11;  // |v_n| <= kTieBand sqrt(T_F): upwind tie

// --------------------------------------------------------------------------
// Lattice constants (Table I) as compile-time values.
// --------------------------------------------------------------------------
template <int Q1, typename T>
__device__ __forceinline__ constexpr T node(int k) {
  if constexpr (Q1 == 4) {
    return k == 0 ? T(-kB) : k == 1 ? T(-kA) : k == 2 ? T(kA) : T(kB);
  } else {
    return k == 0 ? T(-kR3) : k == 1 ? T(0) : T(kR3);
  }
}
template <int Q1, typename T>
__device__ __forceinline__ constexpr T weight(int k) {
  if constexpr (Q1 == 4) {
    return (k == 0 || k == 3) ? T(kWB) : T(kWA);
  } else {
    return k == 1 ? T(2.0 / 3.0) : T(1.0 / 6.0);
  }
}

// Lagrange basis polynomials on the lattice nodes, out[k] = l_k(x).
template <typename T>
__device__ __forceinline__ void lagrange(T x, T (&out)[4]) {
  // nodes -B, -A, A, B:  l_{+-B} = KB (x^2 - A^2)(B +- x),  l_{+-A} = KA (x^2 - B^2)(A +- x)
  const T x2 = x * x;
  const T p = (x2 - T(kA2)) * T(kKB);
  const T q = (x2 - T(kB2)) * T(kKA);
  out[0] = p * (T(kB) - x);
  out[1] = q * (T(kA) - x);
  out[2] = q * (T(kA) + x);
  out[3] = p * (T(kB) + x);
}
template <typename T>
__device__ __forceinline__ void lagrange(T x, T (&out)[3]) {
  // nodes -R3, 0, R3:  l_{+-R3} = x (x +- R3) / 6,  l_0 = 1 - x^2 / 3
  const T h = x * T(1.0 / 6.0);
  out[0] = h * (x - T(kR3));
  out[1] = T(1) - x * x * T(1.0 / 3.0);
  out[2] = h * (x + T(kR3));
}

// One-dimensional factor of the moment-matching map (App. B): with
// xi_m = s c_m + d the source velocity written in the target frame's
// centred, scaled coordinates, A[k][m] = l_k(xi_m).
template <int Q1, typename T>
__device__ __forceinline__ void tf_factor(T s, T d, T (&A)[Q1][Q1]) {
  T l[Q1];
#pragma unroll
  for (int m = 0; m < Q1; ++m) {
    lagrange(s * node<Q1, T>(m) + d, l);
#pragma unroll
    for (int k = 0; k < Q1; ++k) A[k][m] = l[k];
  }
}

template <int Q1, typename T>
__device__ __forceinline__ void tf_apply1(const T (&A)[Q1][Q1], const T* in, T* out) {
#pragma unroll
  for (int k = 0; k < Q1; ++k) {
    T acc = A[k][0] * in[0];
#pragma unroll
    for (int m = 1; m < Q1; ++m) acc += A[k][m] * in[m];
    out[k] = acc;
  }
}

// Transform populations of one lattice (Q1 nodes per axis) from a frame with
// (sqrt T, u) to the target frame given by (1/sqrt T', u').
template <int D, int Q1, typename T>
__device__ __forceinline__ void transform(double rt_src, double ux_src, double uy_src,
                                          double irt_dst, double ux_dst, double uy_dst,
                                          const T* in, T* out) {
  const T s = T(rt_src * irt_dst);
  if constexpr (D == 1) {
    T Ax[Q1][Q1];
    tf_factor<Q1, T>(s, T((ux_src - ux_dst) * irt_dst), Ax);
    tf_apply1<Q1, T>(Ax, in, out);
  } else {
    // y factor first, then x: keeps one coefficient matrix live at a time
    T Ay[Q1][Q1], Y[Q1][Q1];
    tf_factor<Q1, T>(s, T((uy_src - uy_dst) * irt_dst), Ay);
#pragma unroll
    for (int mx = 0; mx < Q1; ++mx)
#pragma unroll
      for (int ky = 0; ky < Q1; ++ky) {
        T acc = Ay[ky][0] * in[mx];
#pragma unroll
        for (int my = 1; my < Q1; ++my) acc += Ay[ky][my] * in[mx + Q1 * my];
        Y[mx][ky] = acc;
      }
    T Ax[Q1][Q1];
    tf_factor<Q1, T>(s, T((ux_src - ux_dst) * irt_dst), Ax);
#pragma unroll
    for (int kx = 0; kx < Q1; ++kx)
#pragma unroll
      for (int ky = 0; ky < Q1; ++ky) {
        T acc = Ax[kx][0] * Y[0][ky];
#pragma unroll
        for (int mx = 1; mx < Q1; ++mx) acc += Ax[kx][mx] * Y[mx][ky];
        out[kx + Q1 * ky] = acc;
      }
  }
}

// Quadrature of the Lagrange basis against the weights:
// out[k] = sum_m l_k(s c_m + d) w_m, the 1D factor of G W (eq. NonComovingEq).
template <int Q1, typename T>
__device__ __forceinline__ void eq_factor(T s, T d, T (&out)[Q1]) {
#pragma unroll
  for (int k = 0; k < Q1; ++k) out[k] = T(0);
  T l[Q1];
#pragma unroll
  for (int m = 0; m < Q1; ++m) {
    lagrange(s * node<Q1, T>(m) + d, l);
#pragma unroll
    for (int k = 0; k < Q1; ++k) out[k] += l[k] * weight<Q1, T>(m);
  }
}

// Slope limiters (Sec. IV A 2): van Leer (a|b| + |a|b) / (|a| + |b|), minmod.
template <typename T>
__device__ __forceinline__ T limit(int kind, T a, T b) {
  if (kind == LIM_MINMOD) {
    if (a * b <= T(0)) return T(0);
    return a > T(0) ? fmin(a, b) : fmax(a, b);
  }
  const T den = fabs(a) + fabs(b);
  return den > T(0) ? (a * fabs(b) + fabs(a) * b) / den : T(0);
}

// --------------------------------------------------------------------------
// Frame of a cell from its conserved moments (eqs. ConservationLaws, E).
// --------------------------------------------------------------------------
struct Frame {
  double rho, ux, uy, T, rt, irt;
};

__device__ __forceinline__ Frame gauge(const long long (&U)[4], const StepArgs& a) {
  Frame g;
  g.rho = double(U[0]) * a.inv_scale;
  const double mx = double(U[1]) * a.inv_scale;
  const double my = double(U[2]) * a.inv_scale;
  const double e = double(U[3]) * a.inv_scale;
  const double ir = 1.0 / g.rho;
  g.ux = mx * ir;
  g.uy = my * ir;
  // rho E = C_v rho T + rho u^2 / 2
  g.T = (e - 0.5 * (mx * g.ux + my * g.uy)) * ir * a.icv;
  g.rt = sqrt(g.T);
  g.irt = 1.0 / g.rt;
  return g;
}

__device__ __forceinline__ long long to_fixed(double x, double scale, int* bad) {
  const double y = rint(x * scale);
  if (!(fabs(y) < 4.0e18)) {
    *bad = 1;
    return 0;
  }
  return (long long)y;
}

// Quasi-equilibrium half step on the non-equilibrium parts n (f) and m (g),
// written in their comoving frame (e_i = sqrt(T) c_i):
//   f += kappa W_i alpha3 : H3(c_i) / 6,  alpha3 = sum_i f_i H3(c_i);
//   g += kappa W_i (sum_j g_j c_j) . c_i   (eq. quasi_f, eq. QE_relaxation).
template <int D, typename T>
__device__ __forceinline__ void qe_half(T* n, T* m, T kappa) {
  if constexpr (D == 1) {
    T a3 = T(0), ag = T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T c = node<4, T>(i);
      a3 += n[i] * (c * c * c - T(3) * c);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) ag += m[i] * node<3, T>(i);
    a3 *= kappa * T(1.0 / 6.0);
    ag *= kappa;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T c = node<4, T>(i);
      n[i] += weight<4, T>(i) * a3 * (c * c * c - T(3) * c);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) m[i] += weight<3, T>(i) * ag * node<3, T>(i);
  } else {
    T axxx = T(0), axxy = T(0), axyy = T(0), ayyy = T(0), agx = T(0), agy = T(0);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const T cx = node<4, T>(i & 3), cy = node<4, T>(i >> 2);
      axxx += n[i] * (cx * cx * cx - T(3) * cx);
      axxy += n[i] * (cx * cx * cy - cy);
      axyy += n[i] * (cx * cy * cy - cx);
      ayyy += n[i] * (cy * cy * cy - T(3) * cy);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      agx += m[i] * node<3, T>(i % 3);
      agy += m[i] * node<3, T>(i / 3);
    }
    const T k6 = kappa * T(1.0 / 6.0);
    axxx *= k6;
    axxy *= T(3) * k6;
    axyy *= T(3) * k6;
    ayyy *= k6;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const T cx = node<4, T>(i & 3), cy = node<4, T>(i >> 2);
      const T w = weight<4, T>(i & 3) * weight<4, T>(i >> 2);
      n[i] += w * (axxx * (cx * cx * cx - T(3) * cx) + axxy * (cx * cx * cy - cy) +
                   axyy * (cx * cy * cy - cx) + ayyy * (cy * cy * cy - T(3) * cy));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const T w = weight<3, T>(i % 3) * weight<3, T>(i / 3);
      m[i] += kappa * w * (agx * node<3, T>(i % 3) + agy * node<3, T>(i / 3));
    }
  }
}

// Ghost cells: a coordinate outside [0, n) wraps (periodic), clamps to the
// nearest interior cell (zero gradient) or flags the side's inflow state.
// The x coordinate is resolved first, then y.
__device__ __forceinline__ int resolve(int v, int n, int bc_lo, int bc_hi, int* side, int lo_side) {
  if (v < 0) {
    if (bc_lo == BC_PERIODIC) return ((v % n) + n) % n;
    if (bc_lo == BC_ZERO_GRADIENT) return 0;
    *side = lo_side;
    return 0;
  }
  if (v >= n) {
    if (bc_hi == BC_PERIODIC) return v % n;
    if (bc_hi == BC_ZERO_GRADIENT) return n - 1;
    *side = lo_side + 1;
    return n - 1;
  }
  return v;
}

// --------------------------------------------------------------------------
// Tile geometry.
// --------------------------------------------------------------------------
template <int D>
struct Geo {
  static constexpr int TX = D == 2 ? kTX2 : kTX1;
  static constexpr int TY = D == 2 ? kTY2 : 1;
  static constexpr int HX = TX + 4;
  static constexpr int HY = D == 2 ? TY + 4 : 1;
  static constexpr int NH = HX * HY;          // halo tile
  static constexpr int OY = D == 2 ? 2 : 0;   // interior offset in y
  static constexpr int NI = TX * TY;          // interior cells
  static constexpr int QF = D == 2 ? 16 : 4;
  static constexpr int QG = D == 2 ? 9 : 3;
  static constexpr int NP = QF + QG;
  static constexpr int NFX = (TX + 1) * TY;
  static constexpr int NFY = D == 2 ? TX * (TY + 1) : 0;
  static constexpr int NF = NFX > NFY ? NFX : NFY;
  static constexpr int NS = D == 2 ? 8 : 4;   // stencil cells per face
  static_assert(NI <= kThreads && NFX <= kThreads && NFY <= kThreads, "one pass per phase");
};

template <int D, typename T>
struct Smem {
  using G = Geo<D>;
  T P[G::NP * G::NH];          // phi-bar-plus of the halo tile, plane-major
  double U[G::NH], V[G::NH], TT[G::NH], RT[G::NH];  // cell frames (u_x, u_y, T, sqrt T)
  T F[G::NP * G::NF];          // face populations phi^{lambda_F}
  double FU[G::NF], FV[G::NF], FRT[G::NF];          // face frames
  long long Psi[4 * G::NF];    // rounded conserved fluxes of the faces
};

// Halo coordinates of tile slot k: interior slots first (thread k owns
// interior slot k), then the ring.
template <int D>
__device__ __forceinline__ void slot_coords(int k, int* hx, int* hy) {
  using G = Geo<D>;
  if (k < G::NI) {
    *hx = k % G::TX + 2;
    *hy = k / G::TX + G::OY;
    return;
  }
  int r = k - G::NI;
  if constexpr (D == 1) {
    *hy = 0;
    *hx = r < 2 ? r : G::TX + r;
  } else {
    if (r < 2 * G::HX) {
      *hy = r / G::HX;
      *hx = r % G::HX;
    } else if (r < 4 * G::HX) {
      r -= 2 * G::HX;
      *hy = G::HY - 2 + r / G::HX;
      *hx = r % G::HX;
    } else {
      r -= 4 * G::HX;
      *hy = 2 + r / 4;
      const int c = r % 4;
      *hx = c < 2 ? c : G::TX + c;
    }
  }
}

// Tensor weights W_i = w_ix w_iy (eq. wi) of the f- and g-lattices.
template <int D, typename T>
__device__ __forceinline__ constexpr T wf(int i) {
  return D == 2 ? weight<4, T>(i & 3) * weight<4, T>(i >> 2) : weight<4, T>(i);
}
template <int D, typename T>
__device__ __forceinline__ constexpr T wg(int i) {
  return D == 2 ? weight<3, T>(i % 3) * weight<3, T>(i / 3) : weight<3, T>(i);
}

// Conserved moments and non-equilibrium populations of grid cell (gx, gy),
// which may lie outside the grid: ghost cells follow the boundary rules.
template <int D, typename T>
__device__ __forceinline__ void load_cell(const StepArgs& a, int gx, int gy, long long (&U)[4],
                                          T (&n)[Geo<D>::NP]) {
  constexpr int NP = Geo<D>::NP;
  int side = -1;
  const int sx = resolve(gx, a.nx, a.bc[0], a.bc[1], &side, 0);
  int sy = 0;
  if constexpr (D == 2) {
    sy = gy;
    if (side < 0) sy = resolve(gy, a.ny, a.bc[2], a.bc[3], &side, 2);
  }
  if (side >= 0) {
    // select the side's inflow state with constant indices (no indexed copy of the arguments)
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (side == k)
#pragma unroll
        for (int q = 0; q < 4; ++q) U[q] = a.inflow_U[k][q];
#pragma unroll
    for (int i = 0; i < NP; ++i) n[i] = T(0);
    return;
  }
  const T* nin = static_cast<const T*>(a.n_in);
  const size_t cell = size_t(sx) + size_t(a.nx) * size_t(sy);
#pragma unroll
  for (int q = 0; q < 4; ++q) U[q] = a.U_in[q * a.cells + cell];
#pragma unroll
  for (int i = 0; i < NP; ++i) n[i] = nin[i * a.cells + cell];
}

// --------------------------------------------------------------------------
// One face: populations phi^{lambda_F}(x_b, t + dt/2) and the conserved flux.
// Stencil slots: 0 L, 1 R, 2 L-e_a, 3 R+e_a, 4 L+e_t, 5 L-e_t, 6 R+e_t, 7 R-e_t.
// --------------------------------------------------------------------------

// MUSCL reconstruction at the departure point x_b - v dt/2 (eq. InterfacePop)
// of one lattice's populations, from the upwind cell by the sign of the
// normal velocity; an exact tie takes the mean of both upwind values.  The
// stencil is transformed into the face frame one cell at a time and folded
// into the running left- and right-upwind reconstructions.
template <int D, int Q1, typename T, int AXIS>
__device__ __forceinline__ void reconstruct(const StepArgs& a, const Smem<D, T>& sm,
                                            const int (&st)[Geo<D>::NS], int plane0, double rtF,
                                            double irtF, double uF, double vF, T* bar) {
  using G = Geo<D>;
  constexpr int Q = D == 2 ? Q1 * Q1 : Q1;
  auto tfs = [&](int slot, T* out) {
    const int h = st[slot];
    T in[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) in[i] = sm.P[(plane0 + i) * G::NH + h];
    transform<D, Q1, T>(sm.RT[h], sm.U[h], D == 2 ? sm.V[h] : 0.0, irtF, uF, vF, in, out);
    // keep the scheduler from overlapping the stencil cells' transforms
    // (each one holds its own LDS loads and coefficients in registers)
    __builtin_amdgcn_sched_barrier(0);
  };
  // normal / transverse particle velocities in the face frame (FP64)
  auto vnorm = [&](int i) {
    return rtF * node<Q1, double>(AXIS == 0 ? (i % Q1) : (i / Q1)) + (AXIS == 0 ? uF : vF);
  };
  auto dtrans = [&](int i) {
    return T(-0.5 * a.lam * (rtF * node<Q1, double>(AXIS == 0 ? (i / Q1) : (i % Q1)) + (AXIS == 0 ? vF : uF)));
  };
  // upwind weights: 1 on the upwind side, 1/2 on both sides at a tie; a
  // normal velocity within kTieBand of the face thermal speed is a tie, so
  // rounding noise around a fluid at rest cannot pick a side
  const double band = kTieBand * rtF;
  auto wl = [&](int i) { const double v = vnorm(i); return v > band ? T(1) : (v < -band ? T(0) : T(0.5)); };
  auto wr = [&](int i) { const double v = vnorm(i); return v < -band ? T(1) : (v > band ? T(0) : T(0.5)); };
  T PL[Q], PR[Q], rec[Q];
  tfs(0, PL);
  tfs(1, PR);
  {
    T t[Q];
    tfs(2, t);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T w = wl(i);
      rec[i] = w == T(0) ? T(0)
                         : w * (PL[i] + T(0.5 - 0.5 * a.lam * vnorm(i)) * limit(a.limiter, PL[i] - t[i], PR[i] - PL[i]));
    }
    tfs(3, t);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T w = wr(i);
      if (w != T(0))
        rec[i] += w * (PR[i] + T(-0.5 - 0.5 * a.lam * vnorm(i)) * limit(a.limiter, PR[i] - PL[i], t[i] - PR[i]));
    }
  }
  if constexpr (D == 2) {
    T tp[Q], tm[Q];
    tfs(4, tp);
    tfs(5, tm);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T w = wl(i);
      if (w != T(0)) rec[i] += w * dtrans(i) * limit(a.limiter, PL[i] - tm[i], tp[i] - PL[i]);
    }
    tfs(6, tp);
    tfs(7, tm);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T w = wr(i);
      if (w != T(0)) rec[i] += w * dtrans(i) * limit(a.limiter, PR[i] - tm[i], tp[i] - PR[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) bar[i] = rec[i];
}

template <int D, typename T, int AXIS>
__device__ void face_eval(const StepArgs& a, Smem<D, T>& sm, const int (&st)[Geo<D>::NS], int fidx) {
  using G = Geo<D>;
  constexpr int QF = G::QF, QG = G::QG;
  const int hL = st[0], hR = st[1];
  // eq. AvgFrame
  double uF = 0.5 * (sm.U[hL] + sm.U[hR]);
  double vF = D == 2 ? 0.5 * (sm.V[hL] + sm.V[hR]) : 0.0;
  double TF = 0.5 * (sm.TT[hL] + sm.TT[hR]);
  T fbar[QF], gbar[QG];
  double rho_b = 0.0, ub = 0.0, vb = 0.0, Tb = 0.0, rtF = 0.0, irtF = 0.0;
  for (int pass = 0; pass <= a.n_corr; ++pass) {
    rtF = sqrt(TF);
    irtF = 1.0 / rtF;
    reconstruct<D, 4, T, AXIS>(a, sm, st, 0, rtF, irtF, uF, vF, fbar);
    reconstruct<D, 3, T, AXIS>(a, sm, st, QF, rtF, irtF, uF, vF, gbar);
    // macroscopic fields at the face, in FP64
    double m0 = 0.0, mx = 0.0, my = 0.0, e = 0.0;
#pragma unroll
    for (int i = 0; i < QF; ++i) {
      const double vx = rtF * node<4, double>(i & 3) + uF;
      const double vy = D == 2 ? rtF * node<4, double>(i >> 2) + vF : 0.0;
      const double fb = double(fbar[i]);
      m0 += fb;
      mx += vx * fb;
      my += vy * fb;
      e += 0.5 * (vx * vx + vy * vy) * fb;
    }
#pragma unroll
    for (int i = 0; i < QG; ++i) e += double(gbar[i]);
    rho_b = m0;
    ub = mx / m0;
    vb = my / m0;
    Tb = (e - 0.5 * m0 * (ub * ub + vb * vb)) / (a.cv * m0);
    if (pass < a.n_corr) {  // corrector: re-evaluate in the frame just found
      uF = ub;
      vF = vb;
      TF = Tb;
    }
  }
  // face equilibrium rho G_{u_b,T_b}^{lambda_F} W (eq. NonComovingEq), separable
  const T sb = T(sqrt(Tb) * irtF);
  const T c1 = T(a.c_face1), c2 = T(a.c_face2);
  {
    T ex[4], ey[4];
    eq_factor<4, T>(sb, T((ub - uF) * irtF), ex);
    if constexpr (D == 2) eq_factor<4, T>(sb, T((vb - vF) * irtF), ey);
    const T r = T(rho_b);
#pragma unroll
    for (int i = 0; i < QF; ++i) {
      const T feq = D == 2 ? r * ex[i & 3] * ey[i >> 2] : r * ex[i];
      fbar[i] = c1 * fbar[i] + c2 * feq;  // phi from phi-bar: inverts eq. FluxTransf
    }
  }
  {
    T ex[3], ey[3];
    eq_factor<3, T>(sb, T((ub - uF) * irtF), ex);
    if constexpr (D == 2) eq_factor<3, T>(sb, T((vb - vF) * irtF), ey);
    const T r = T(a.geq * Tb * rho_b);
#pragma unroll
    for (int i = 0; i < QG; ++i) {
      const T geq = D == 2 ? r * ex[i % 3] * ey[i / 3] : r * ex[i];
      gbar[i] = c1 * gbar[i] + c2 * geq;
    }
  }
  // conserved fluxes through the face, in FP64, rounded once to the ledger unit
  double Fr = 0.0, Fx = 0.0, Fy = 0.0, FE = 0.0;
#pragma unroll
  for (int i = 0; i < QF; ++i) {
    const double vx = rtF * node<4, double>(i & 3) + uF;
    const double vy = D == 2 ? rtF * node<4, double>(i >> 2) + vF : 0.0;
    const double vn = AXIS == 0 ? vx : vy;
    const double p = double(fbar[i]) * vn;
    Fr += p;
    Fx += vx * p;
    Fy += vy * p;
    FE += 0.5 * (vx * vx + vy * vy) * p;
  }
#pragma unroll
  for (int i = 0; i < QG; ++i) {
    const int in_ = AXIS == 0 ? (i % 3) : (i / 3);
    const double vn = rtF * node<3, double>(in_) + (AXIS == 0 ? uF : vF);
    FE += vn * double(gbar[i]);
  }
  int bad = 0;
  const double sc = a.lam * a.scale;
  sm.Psi[0 * G::NF + fidx] = to_fixed(Fr, sc, &bad);
  sm.Psi[1 * G::NF + fidx] = to_fixed(Fx, sc, &bad);
  sm.Psi[2 * G::NF + fidx] = to_fixed(Fy, sc, &bad);
  sm.Psi[3 * G::NF + fidx] = to_fixed(FE, sc, &bad);
  if (bad || !(rho_b > 0.0) || !(Tb > 0.0)) atomicOr(a.flag, bad ? 2 : 1);
#pragma unroll
  for (int i = 0; i < QF; ++i) sm.F[i * G::NF + fidx] = fbar[i];
#pragma unroll
  for (int i = 0; i < QG; ++i) sm.F[(QF + i) * G::NF + fidx] = gbar[i];
  sm.FU[fidx] = uF;
  sm.FV[fidx] = vF;
  sm.FRT[fidx] = rtF;
}

// Flux of two opposite faces into the cell frame (eq. fluxEq):
// acc += v_a^{lambda_j} (G phi_hi - G phi_lo).
template <int D, typename T, int AXIS>
__device__ __forceinline__ void gather_faces(Smem<D, T>& sm, int flo, int fhi, const Frame& c,
                                             T (&acc)[Geo<D>::NP]) {
  using G = Geo<D>;
  constexpr int QF = G::QF, QG = G::QG;
  T dlt[G::NP];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int fi = side ? fhi : flo;
    const double rtF = sm.FRT[fi], uF = sm.FU[fi], vF = sm.FV[fi];
    T in[QF], out[QF];
#pragma unroll
    for (int i = 0; i < QF; ++i) in[i] = sm.F[i * G::NF + fi];
    transform<D, 4, T>(rtF, uF, vF, c.irt, c.ux, c.uy, in, out);
#pragma unroll
    for (int i = 0; i < QF; ++i) dlt[i] = side ? out[i] - dlt[i] : out[i];
    T ing[QG], outg[QG];
#pragma unroll
    for (int i = 0; i < QG; ++i) ing[i] = sm.F[(QF + i) * G::NF + fi];
    transform<D, 3, T>(rtF, uF, vF, c.irt, c.ux, c.uy, ing, outg);
#pragma unroll
    for (int i = 0; i < QG; ++i) dlt[QF + i] = side ? outg[i] - dlt[QF + i] : outg[i];
  }
  const T rt = T(c.rt), u = T(AXIS == 0 ? c.ux : c.uy);
#pragma unroll
  for (int i = 0; i < QF; ++i) {
    const int k = AXIS == 0 ? (i & 3) : (i >> 2);
    acc[i] += (rt * node<4, T>(k) + u) * dlt[i];
  }
#pragma unroll
  for (int i = 0; i < QG; ++i) {
    const int k = AXIS == 0 ? (i % 3) : (i / 3);
    acc[QF + i] += (rt * node<3, T>(k) + u) * dlt[QF + i];
  }
}

// --------------------------------------------------------------------------
// The fused step kernel.
// --------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(kThreads) step_kernel(StepArgs a) {
  using G = Geo<D>;
  constexpr int QF = G::QF, QG = G::QG, NP = G::NP;
  __shared__ Smem<D, T> sm;
  const int tid = threadIdx.x;
  const int bx = blockIdx.x % a.tiles_x, by = blockIdx.x / a.tiles_x;
  const int x0 = bx * G::TX, y0 = by * G::TY;
  const T kappa = T(a.kappa), apre = T(a.a_pre);

  // ---- 0. halo tile: ghost resolution, frame, first QE half step, phi-bar-plus
  for (int k = tid; k < G::NH; k += kThreads) {
    int hx, hy;
    slot_coords<D>(k, &hx, &hy);
    const int gx = x0 + hx - 2, gy = y0 + hy - G::OY;
    long long U[4];
    T n[NP];
    load_cell<D, T>(a, gx, gy, U, n);
    const Frame fr = gauge(U, a);
    qe_half<D, T>(n, n + QF, kappa);
    const int h = hx + G::HX * hy;
    const T r = T(fr.rho), rg = T(a.geq * fr.T * fr.rho);
#pragma unroll
    for (int i = 0; i < QF; ++i) sm.P[i * G::NH + h] = r * wf<D, T>(i) + apre * n[i];
#pragma unroll
    for (int i = 0; i < QG; ++i) sm.P[(QF + i) * G::NH + h] = rg * wg<D, T>(i) + apre * n[QF + i];
    sm.U[h] = fr.ux;
    sm.V[h] = fr.uy;
    sm.TT[h] = fr.T;
    sm.RT[h] = fr.rt;
  }
  __syncthreads();
  // the thread's own cell (interior slot tid)
  const int cx = tid % G::TX, cy = tid / G::TX;
  const bool own_in = tid < G::NI && x0 + cx < a.nx && (D == 1 || y0 + cy < a.ny);
  Frame ownF{};
  if (tid < G::NI) {
    const int h = cx + 2 + G::HX * (cy + G::OY);
    ownF.ux = sm.U[h];
    ownF.uy = sm.V[h];
    ownF.T = sm.TT[h];
    ownF.rt = sm.RT[h];
    ownF.irt = 1.0 / ownF.rt;
  }

  T acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = T(0);
  long long dU[4] = {0, 0, 0, 0};

  // ---- 1. x-faces
  if (tid < G::NFX) {
    const int fi = tid % (G::TX + 1), fj = tid / (G::TX + 1);
    const int hy = fj + G::OY;
    const int hL = fi + 1 + G::HX * hy;
    int st[G::NS];
    st[0] = hL;
    st[1] = hL + 1;
    st[2] = hL - 1;
    st[3] = hL + 2;
    if constexpr (D == 2) {
      st[4] = hL + G::HX;
      st[5] = hL - G::HX;
      st[6] = hL + 1 + G::HX;
      st[7] = hL + 1 - G::HX;
    }
    face_eval<D, T, 0>(a, sm, st, tid);
  }
  __syncthreads();
  // ---- 2. west/east faces into the cell frame
  if (tid < G::NI) {
    const int fw = cx + (G::TX + 1) * cy;
    gather_faces<D, T, 0>(sm, fw, fw + 1, ownF, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) dU[q] += sm.Psi[q * G::NF + fw + 1] - sm.Psi[q * G::NF + fw];
  }
  if constexpr (D == 2) {
    __syncthreads();
    // ---- 3. y-faces
    if (tid < G::NFY) {
      const int fi = tid % G::TX, fj = tid / G::TX;
      const int hS = (fi + 2) + G::HX * (fj + 1);
      int st[G::NS];
      st[0] = hS;
      st[1] = hS + G::HX;
      st[2] = hS - G::HX;
      st[3] = hS + 2 * G::HX;
      st[4] = hS + 1;
      st[5] = hS - 1;
      st[6] = hS + G::HX + 1;
      st[7] = hS + G::HX - 1;
      face_eval<D, T, 1>(a, sm, st, tid);
    }
    __syncthreads();
    // ---- 4. south/north faces
    if (tid < G::NI) {
      const int fs = cx + G::TX * cy;
      gather_faces<D, T, 1>(sm, fs, fs + G::TX, ownF, acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) dU[q] += sm.Psi[q * G::NF + fs + G::TX] - sm.Psi[q * G::NF + fs];
    }
  }

  // ---- 5. DUGKS update, new comoving frame, second QE half step
  if (own_in) {
    long long U[4];
    T own[NP];
    load_cell<D, T>(a, x0 + cx, y0 + cy, U, own);
    const Frame f0 = gauge(U, a);  // the frame the populations are written in
    qe_half<D, T>(own, own + QF, kappa);
    const T b = T(a.b_upd), lam = T(a.lam);
    const T r = T(f0.rho), rg = T(a.geq * f0.T * f0.rho);
    T ft[QF], gt[QG];
#pragma unroll
    for (int i = 0; i < QF; ++i) ft[i] = r * wf<D, T>(i) + b * own[i] - lam * acc[i];
#pragma unroll
    for (int i = 0; i < QG; ++i) gt[i] = rg * wg<D, T>(i) + b * own[QF + i] - lam * acc[QF + i];
    long long U2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) U2[q] = U[q] - dU[q];
    const Frame nf = gauge(U2, a);
    T n2[NP];
    transform<D, 4, T>(f0.rt, f0.ux, f0.uy, nf.irt, nf.ux, nf.uy, ft, n2);
    transform<D, 3, T>(f0.rt, f0.ux, f0.uy, nf.irt, nf.ux, nf.uy, gt, n2 + QF);
    const T r2 = T(nf.rho), rg2 = T(a.geq * nf.T * nf.rho);
#pragma unroll
    for (int i = 0; i < QF; ++i) n2[i] -= r2 * wf<D, T>(i);
#pragma unroll
    for (int i = 0; i < QG; ++i) n2[QF + i] -= rg2 * wg<D, T>(i);
    qe_half<D, T>(n2, n2 + QF, kappa);
    if (!(nf.rho > 0.0) || !(nf.T > 0.0) || !isfinite(double(n2[0]))) atomicOr(a.flag, 1);
    bool over = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) over |= (U2[q] > (1LL << 62)) || (U2[q] < -(1LL << 62));
    if (over) atomicOr(a.flag, 2);
    const size_t cell = size_t(x0 + cx) + size_t(a.nx) * size_t(D == 2 ? y0 + cy : 0);
    T* nout = static_cast<T*>(a.n_out);
#pragma unroll
    for (int i = 0; i < NP; ++i) nout[i * a.cells + cell] = n2[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) a.U_out[q * a.cells + cell] = U2[q];
  }
}

// --------------------------------------------------------------------------
// Initial data, observables, exact totals.
// --------------------------------------------------------------------------
template <int D, typename T>
__global__ void init_kernel(const double* fields, size_t cells, size_t first, size_t count,
                            double scale, double cv, T* n, long long* U) {
  constexpr int NP = D == 2 ? 25 : 7;
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const size_t c = first + k;
  const double rho = fields[k], ux = fields[count + k], uy = D == 2 ? fields[2 * count + k] : 0.0;
  const double p = fields[3 * count + k];
  // comoving equilibrium: the non-equilibrium parts vanish
#pragma unroll
  for (int i = 0; i < NP; ++i) n[i * cells + c] = T(0);
  U[c] = (long long)rint(rho * scale);
  U[cells + c] = (long long)rint(rho * ux * scale);
  U[2 * cells + c] = (long long)rint(rho * uy * scale);
  U[3 * cells + c] = (long long)rint((cv * p + 0.5 * rho * (ux * ux + uy * uy)) * scale);
}

__global__ void moments_kernel(const long long* U, size_t cells, size_t first, size_t count,
                               double inv_scale, double icv, double* out) {
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const size_t c = first + k;
  const double rho = double(U[c]) * inv_scale;
  const double mx = double(U[cells + c]) * inv_scale, my = double(U[2 * cells + c]) * inv_scale;
  const double e = double(U[3 * cells + c]) * inv_scale;
  const double ux = mx / rho, uy = my / rho;
  out[k] = rho;
  out[count + k] = ux;
  out[2 * count + k] = uy;
  out[3 * count + k] = (e - 0.5 * (mx * ux + my * uy)) / rho * icv;
}

template <int D, typename T>
__global__ void export_kernel(const T* n, const long long* U, size_t cells, size_t first,
                              size_t count, double inv_scale, double icv, double geq, double* out) {
  constexpr int QF = D == 2 ? 16 : 4, QG = D == 2 ? 9 : 3;
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const size_t c = first + k;
  const double rho = double(U[c]) * inv_scale;
  const double mx = double(U[cells + c]) * inv_scale, my = double(U[2 * cells + c]) * inv_scale;
  const double e = double(U[3 * cells + c]) * inv_scale;
  const double ux = mx / rho, uy = my / rho;
  const double T_ = (e - 0.5 * (mx * ux + my * uy)) / rho * icv;
  for (int i = 0; i < QF; ++i) {
    const double w = D == 2 ? weight<4, double>(i & 3) * weight<4, double>(i >> 2) : weight<4, double>(i);
    out[i * count + k] = rho * w + double(n[i * cells + c]);
  }
  for (int i = 0; i < QG; ++i) {
    const double w = D == 2 ? weight<3, double>(i % 3) * weight<3, double>(i / 3) : weight<3, double>(i);
    out[(QF + i) * count + k] = geq * T_ * rho * w + double(n[(QF + i) * cells + c]);
  }
  out[(QF + QG) * count + k] = ux;
  out[(QF + QG + 1) * count + k] = uy;
  out[(QF + QG + 2) * count + k] = T_;
}

// Exact per-block sums of the ledger planes as 128-bit integers.
__global__ void __launch_bounds__(256) totals_kernel(const long long* U, size_t cells,
                                                    long long* out) {
  __shared__ __int128 red[4][256];
  __int128 acc[4] = {0, 0, 0, 0};
  for (size_t c = size_t(blockIdx.x) * 256 + threadIdx.x; c < cells; c += size_t(gridDim.x) * 256)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += (__int128)U[q * cells + c];
#pragma unroll
  for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) {
    const __int128 v = red[threadIdx.x][0];
    out[(blockIdx.x * 4 + threadIdx.x) * 2] = (long long)(v >> 64);
    out[(blockIdx.x * 4 + threadIdx.x) * 2 + 1] = (long long)(unsigned long long)v;
  }
}

}  // namespace

hipError_t launch_step(int dim, bool fp64, const StepArgs& a, hipStream_t st) {
  const dim3 grid(a.tiles_x * a.tiles_y), block(kThreads);
  if (dim == 1) {
    if (fp64) hipLaunchKernelGGL((step_kernel<1, double>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((step_kernel<1, float>), grid, block, 0, st, a);
  } else {
    if (fp64) hipLaunchKernelGGL((step_kernel<2, double>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((step_kernel<2, float>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_init(int dim, bool fp64, const double* fields, size_t cells, size_t first,
                       size_t count, double scale, double cv, void* n, long long* U,
                       hipStream_t st) {
  const dim3 grid((count + 255) / 256), block(256);
  if (dim == 1) {
    if (fp64) hipLaunchKernelGGL((init_kernel<1, double>), grid, block, 0, st, fields, cells, first, count, scale, cv, (double*)n, U);
    else hipLaunchKernelGGL((init_kernel<1, float>), grid, block, 0, st, fields, cells, first, count, scale, cv, (float*)n, U);
  } else {
    if (fp64) hipLaunchKernelGGL((init_kernel<2, double>), grid, block, 0, st, fields, cells, first, count, scale, cv, (double*)n, U);
    else hipLaunchKernelGGL((init_kernel<2, float>), grid, block, 0, st, fields, cells, first, count, scale, cv, (float*)n, U);
  }
  return hipGetLastError();
}

hipError_t launch_moments(int /*dim*/, const long long* U, size_t cells, size_t first, size_t count,
                          double inv_scale, double icv, double* out, hipStream_t st) {
  hipLaunchKernelGGL(moments_kernel, dim3((count + 255) / 256), dim3(256), 0, st, U, cells, first,
                     count, inv_scale, icv, out);
  return hipGetLastError();
}

hipError_t launch_export(int dim, bool fp64, const void* n, const long long* U, size_t cells,
                         size_t first, size_t count, double inv_scale, double icv, double geq,
                         double* out, hipStream_t st) {
  const dim3 grid((count + 255) / 256), block(256);
  if (dim == 1) {
    if (fp64) hipLaunchKernelGGL((export_kernel<1, double>), grid, block, 0, st, (const double*)n, U, cells, first, count, inv_scale, icv, geq, out);
    else hipLaunchKernelGGL((export_kernel<1, float>), grid, block, 0, st, (const float*)n, U, cells, first, count, inv_scale, icv, geq, out);
  } else {
    if (fp64) hipLaunchKernelGGL((export_kernel<2, double>), grid, block, 0, st, (const double*)n, U, cells, first, count, inv_scale, icv, geq, out);
    else hipLaunchKernelGGL((export_kernel<2, float>), grid, block, 0, st, (const float*)n, U, cells, first, count, inv_scale, icv, geq, out);
  }
  return hipGetLastError();
}

hipError_t launch_totals(const long long* U, size_t cells, int blocks, long long* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(totals_kernel, dim3(blocks), dim3(256), 0, st, U, cells, out);
  return hipGetLastError();
}

}  // namespace pond
