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
#include <type_traits>

#include "pond_internal.h"

namespace pond {
namespace {

constexpr int BC_PERIODIC = 0, BC_ZERO_GRADIENT = 1, BC_WALL = 3;
constexpr int LIM_VANLEER = 0, LIM_MINMOD = 1;
constexpr int TF_LAGRANGE = 0, TF_GRAD = 1;
constexpr double kTieBand = 1e-11;  // |v_n| <= kTieBand sqrt(T_F): upwind tie

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    __builtin_amdgcn_sched_barrier(0);
    static_for<B + 1, E>(f);
  }
}

// --------------------------------------------------------------------------
// Lattice constants (Table I) as compile-time values.
// --------------------------------------------------------------------------
template <int Q1, typename T>
__device__ __forceinline__ constexpr T node(int k) {
  if constexpr (Q1 == 5) {
    return k == 0 ? T(-kB5) : k == 1 ? T(-kA5) : k == 2 ? T(0) : k == 3 ? T(kA5) : T(kB5);
  } else if constexpr (Q1 == 4) {
    return k == 0 ? T(-kB) : k == 1 ? T(-kA) : k == 2 ? T(kA) : T(kB);
  } else {
    return k == 0 ? T(-kR3) : k == 1 ? T(0) : T(kR3);
  }
}
template <int Q1, typename T>
__device__ __forceinline__ constexpr T weight(int k) {
  if constexpr (Q1 == 5) {
    return (k == 0 || k == 4) ? T(kW5B) : (k == 1 || k == 3) ? T(kW5A) : T(8.0 / 15.0);
  } else if constexpr (Q1 == 4) {
    return (k == 0 || k == 3) ? T(kWB) : T(kWA);
  } else {
    return k == 1 ? T(2.0 / 3.0) : T(1.0 / 6.0);
  }
}

// Per-point factors of the Lagrange basis on the lattice nodes: l_k(x) is a
// product of a node-pair factor and one linear term, lag_entry<k>().
template <int Q1, typename T>
struct LagPoint {
  T x, p, q;  // D1Q4: p = KB (x^2 - A^2), q = KA (x^2 - B^2); D1Q3: p = x / 6, q = x^2 / 3
};
template <int Q1, typename T>
__device__ __forceinline__ LagPoint<Q1, T> lag_point(T x) {
  LagPoint<Q1, T> r;
  r.x = x;
  const T x2 = x * x;
  if constexpr (Q1 == 4) {
    r.p = (x2 - T(kA2)) * T(kKB);
    r.q = (x2 - T(kB2)) * T(kKA);
  } else {
    r.p = x * T(1.0 / 6.0);
    r.q = x2 * T(1.0 / 3.0);
  }
  return r;
}
template <int Q1, typename T>
__device__ __forceinline__ T lag_entry(int k, const LagPoint<Q1, T>& L) {
  if constexpr (Q1 == 4) {
    return k == 0 ? L.p * (T(kB) - L.x) : k == 1 ? L.q * (T(kA) - L.x)
         : k == 2 ? L.q * (T(kA) + L.x) : L.p * (T(kB) + L.x);
  } else {
    return k == 0 ? L.p * (L.x - T(kR3)) : k == 1 ? T(1) - L.q : L.p * (L.x + T(kR3));
  }
}

// sum_m l_k(x_m) v_m for every node k, through node-pair sums: for D1Q4,
// l_{-+B}(x) = p(x) (B -+ x) and l_{-+A}(x) = q(x) (A -+ x), so the pair's two
// outputs are B sum p v -+ sum p x v (likewise for A); for D1Q3,
// l_{-+R3} = (x^2 -+ R3 x)/6 and l_0 = 1 - x^2/3.
template <int Q1, typename T>
struct PairBasis {
  T c0[Q1], c1[Q1], c2[Q1], c3[Q1];  // D1Q4: p, p x, q, q x; D1Q3: x, x^2
  __device__ __forceinline__ explicit PairBasis(const T* x) {
#pragma unroll
    for (int m = 0; m < Q1; ++m) {
      const T x2 = x[m] * x[m];
      if constexpr (Q1 == 4) {
        c0[m] = x2 * T(kKB) + T(-kA2 * kKB);
        c2[m] = x2 * T(kKA) + T(-kB2 * kKA);
        c1[m] = c0[m] * x[m];
        c3[m] = c2[m] * x[m];
      } else {
        c0[m] = x[m];
        c1[m] = x2;
      }
    }
  }
  // v[m * SV] -> o[k * SO]
  template <int SV, int SO>
  __device__ __forceinline__ void apply(const T* v, T* o) const {
    if constexpr (Q1 == 4) {
      T P0 = c0[0] * v[0], P1 = c1[0] * v[0], Q0 = c2[0] * v[0], Qs = c3[0] * v[0];
#pragma unroll
      for (int m = 1; m < 4; ++m) {
        P0 += c0[m] * v[m * SV];
        P1 += c1[m] * v[m * SV];
        Q0 += c2[m] * v[m * SV];
        Qs += c3[m] * v[m * SV];
      }
      o[0] = T(kB) * P0 - P1;
      o[SO] = T(kA) * Q0 - Qs;
      o[2 * SO] = T(kA) * Q0 + Qs;
      o[3 * SO] = T(kB) * P0 + P1;
    } else {
      T S0 = v[0], S1 = c0[0] * v[0], S2 = c1[0] * v[0];
#pragma unroll
      for (int m = 1; m < 3; ++m) {
        S0 += v[m * SV];
        S1 += c0[m] * v[m * SV];
        S2 += c1[m] * v[m * SV];
      }
      o[0] = (S2 - T(kR3) * S1) * T(1.0 / 6.0);
      o[SO] = S0 - S2 * T(1.0 / 3.0);
      o[2 * SO] = (S2 + T(kR3) * S1) * T(1.0 / 6.0);
    }
  }
};

// Transform of one lattice's populations from a frame with (sqrt T, u) to the
// frame with (1/sqrt T', u').  TF_LAGRANGE: the moment-matching map of App. B,
// on the tensor lattice G = A_x (x) A_y with A[k][m] = l_k(xi_m),
// xi_m = s c_m + d, s = sqrt(T/T'), d = (u - u')/sqrt(T'), applied factor by
// factor.  TF_GRAD: Grad's projection (eq. GradsProjection).  In 1D the two
// coincide.  The 2D maps are xform below.
template <int TF, int Q1, typename T, int AXIS, int K0, int NK>
__device__ __forceinline__ void xform(T s, T dn, T dt, const T* in, T* out);

template <int D, int Q1, typename T, int TF>
__device__ __forceinline__ void transform(double rt_src, double ux_src, double uy_src,
                                          double irt_dst, double ux_dst, double uy_dst,
                                          const T* in, T* out) {
  const T s = T(rt_src * irt_dst);
  const T dx = T((ux_src - ux_dst) * irt_dst);
  if constexpr (D == 1) {
    T x[Q1];
#pragma unroll
    for (int m = 0; m < Q1; ++m) x[m] = s * node<Q1, T>(m) + dx;
    PairBasis<Q1, T>(x).template apply<1, 1>(in, out);
  } else {
    xform<TF, Q1, T, 0, 0, Q1>(s, dx, T((uy_src - uy_dst) * irt_dst), in, out);
  }
}


// The same map restricted to the outputs whose transverse index (i_y for an
// x-face, i_x for a y-face) lies in [K0, K0 + NK), given the 2D frame shift as
// s = sqrt(T/T'), dn / dt = normal / transverse (u - u')/sqrt(T'); out is
// indexed j = n + Q1 t (n: normal index, t = transverse index - K0).  The
// transverse factor is applied first: whole through node-pair sums, or only
// the NK needed rows of it.  The normal factor goes through node-pair sums.
template <int Q1, typename T, int AXIS, int K0, int NK>
__device__ __forceinline__ void transform_part(T s, T dn, T dt, const T* in, T* out) {
  constexpr int SN = AXIS == 0 ? 1 : Q1, ST = AXIS == 0 ? Q1 : 1;
  T Z[NK][Q1];  // Z[t][mn] = sum_mt A_t[K0 + t][mt] in[mn SN + mt ST]
  if constexpr (NK == Q1) {
    T xt[Q1];
#pragma unroll
    for (int m = 0; m < Q1; ++m) xt[m] = s * node<Q1, T>(m) + dt;
    const PairBasis<Q1, T> bt(xt);
#pragma unroll
    for (int mn = 0; mn < Q1; ++mn) bt.template apply<ST, Q1>(in + mn * SN, &Z[0][mn]);
  } else {
    LagPoint<Q1, T> E[Q1];
#pragma unroll
    for (int m = 0; m < Q1; ++m) E[m] = lag_point<Q1, T>(s * node<Q1, T>(m) + dt);
#pragma unroll
    for (int t = 0; t < NK; ++t) {
      T row[Q1];
#pragma unroll
      for (int mt = 0; mt < Q1; ++mt) row[mt] = lag_entry<Q1, T>(K0 + t, E[mt]);
#pragma unroll
      for (int mn = 0; mn < Q1; ++mn) {
        T acc = row[0] * in[mn * SN];
#pragma unroll
        for (int mt = 1; mt < Q1; ++mt) acc += row[mt] * in[mn * SN + mt * ST];
        Z[t][mn] = acc;
      }
    }
  }
  T xi[Q1];
#pragma unroll
  for (int m = 0; m < Q1; ++m) xi[m] = s * node<Q1, T>(m) + dn;
  const PairBasis<Q1, T> bn(xi);
#pragma unroll
  for (int t = 0; t < NK; ++t) bn.template apply<1, 1>(Z[t], out + Q1 * t);
}

// He_a(c_k) / a! on the lattice nodes (probabilists' Hermite polynomials).
template <int Q1>
__host__ __device__ constexpr double hermite_node(int a, int k) {
  const double c = node<Q1, double>(k);
  return a == 0   ? 1.0
         : a == 1 ? c
         : a == 2 ? (c * c - 1.0) / 2.0
         : a == 3 ? (c * c * c - 3.0 * c) / 6.0
                  : (c * c * c * c - 6.0 * c * c + 3.0) / 24.0;
}

// Grad's expansion of order K from a source lattice with QS nodes per axis
// onto a target lattice with QT (eq. GradsProjection; Hermite moments of
// App. A):
//   f'_{kn,kt} = W_kn W_kt sum_{a + b <= K} alpha_ab He_a(c_kn) He_b(c_kt) / (a! b!),
//   alpha_ab = sum_{mn,mt} He_a(x_mn) He_b(y_mt) f_{mn,mt},
// with x = s c + dn (normal axis) and y = s c + dt (transverse axis) the
// source nodes seen from the target frame; in is indexed mn SN + mt ST over
// the source lattice, out as kn + QT kt.  QS = QT, K = QS - 1 is Grad's
// projection of the lattice (keeping a + b <= K drops 6 of the 16 D2Q16
// modes and 3 of the 9 D2Q9 ones, so it is not the identity when the frames
// coincide); QS = 4, QT = 3, K = 2 is the multiscale projection; QS = 3,
// QT = 4, K = 2 with s = 1, d = 0 is the lifting in the source's own frame,
// where the missing third-order moments take their equilibrium value 0.
template <int QS, int QT, int K, typename T, int AXIS>
__device__ __forceinline__ void grad_map(T s, T dn, T dt, const T* in, T* out) {
  constexpr int SN = AXIS == 0 ? 1 : QS, ST = AXIS == 0 ? QS : 1;
  auto herm = [](T x, T (&h)[5]) {  // He_0..He_K at x
    const T x2 = x * x;
    h[0] = T(1);
    h[1] = x;
    h[2] = x2 - T(1);
    if constexpr (K >= 3) h[3] = x * (x2 - T(3));
    if constexpr (K >= 4) h[4] = x2 * (x2 - T(6)) + T(3);
  };
  // beta[mn][b] = sum_mt He_b(y_mt) f[mn][mt], accumulated point by point so
  // that only one point's Hermite values are live
  T beta[QS][K + 1];
#pragma unroll
  for (int mt = 0; mt < QS; ++mt) {
    T h[5];
    herm(s * node<QS, T>(mt) + dt, h);
#pragma unroll
    for (int mn = 0; mn < QS; ++mn) {
      const T f = in[mn * SN + mt * ST];
#pragma unroll
      for (int b = 0; b <= K; ++b) beta[mn][b] = mt == 0 ? h[b] * f : beta[mn][b] + h[b] * f;
    }
  }
  // alpha[a][b] = sum_mn He_a(x_mn) beta[mn][b], a + b <= K
  T alpha[K + 1][K + 1];
#pragma unroll
  for (int mn = 0; mn < QS; ++mn) {
    T h[5];
    herm(s * node<QS, T>(mn) + dn, h);
#pragma unroll
    for (int b = 0; b <= K; ++b) {
#pragma unroll
      for (int a = 0; a + b <= K; ++a)
        alpha[a][b] = mn == 0 ? h[a] * beta[0][b] : alpha[a][b] + h[a] * beta[mn][b];
    }
  }
  // FP32: the Hermite moments are finished before the expansion starts (the
  // empty asm keeps the compiler from interleaving the two stages, which
  // left more values live than the registers hold and spilled)
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int b = 0; b <= K; ++b) {
#pragma unroll
      for (int a = 0; a + b <= K; ++a) asm volatile("" : "+v"(alpha[a][b]));
    }
  }
  // gamma[kn][b] = W_kn sum_{a <= K - b} He_a(c_kn)/a! alpha[a][b];
  // out[kn][kt] = W_kt sum_b He_b(c_kt)/b! gamma[kn][b]
#pragma unroll
  for (int kn = 0; kn < QT; ++kn) {
    T gam[K + 1];
#pragma unroll
    for (int b = 0; b <= K; ++b) {
      T acc = T(hermite_node<QT>(0, kn)) * alpha[0][b];
#pragma unroll
      for (int a = 1; a + b <= K; ++a) acc += T(hermite_node<QT>(a, kn)) * alpha[a][b];
      gam[b] = T(weight<QT, double>(kn)) * acc;
    }
#pragma unroll
    for (int kt = 0; kt < QT; ++kt) {
      T acc = gam[0];
#pragma unroll
      for (int b = 1; b <= K; ++b) acc += T(hermite_node<QT>(b, kt)) * gam[b];
      out[kn + QT * kt] = T(weight<QT, double>(kt)) * acc;
    }
  }
}

// Grad's projection of one lattice into the target frame.
template <int Q1, typename T, int AXIS>
__device__ __forceinline__ void transform_grad(T s, T dn, T dt, const T* in, T* out) {
  grad_map<Q1, Q1, Q1 - 1, T, AXIS>(s, dn, dt, in, out);
}

template <int TF, int Q1, typename T, int AXIS, int K0, int NK>
__device__ __forceinline__ void xform(T s, T dn, T dt, const T* in, T* out) {
  if constexpr (TF == TF_GRAD) {
    if constexpr (NK == Q1) {
      transform_grad<Q1, T, AXIS>(s, dn, dt, in, out);
    } else {
      T all[Q1 * Q1];
      transform_grad<Q1, T, AXIS>(s, dn, dt, in, all);
#pragma unroll
      for (int j = 0; j < Q1 * NK; ++j) out[j] = all[j + Q1 * K0];
    }
  } else {
    transform_part<Q1, T, AXIS, K0, NK>(s, dn, dt, in, out);
  }
}

// Quadrature of the Lagrange basis against the weights:
// out[k] = sum_m l_k(s c_m + d) w_m, the 1D factor of G W (eq. NonComovingEq).
template <int Q1, typename T>
__device__ __forceinline__ void eq_factor(T s, T d, T (&out)[Q1]) {
#pragma unroll
  for (int k = 0; k < Q1; ++k) out[k] = T(0);
#pragma unroll
  for (int m = 0; m < Q1; ++m) {
    const LagPoint<Q1, T> L = lag_point<Q1, T>(s * node<Q1, T>(m) + d);
#pragma unroll
    for (int k = 0; k < Q1; ++k) out[k] += lag_entry<Q1, T>(k, L) * weight<Q1, T>(m);
  }
}

// Slope limiters (Sec. IV A 2): van Leer (a|b| + |a|b) / (|a| + |b|), minmod.
template <int LIM, typename T>
__device__ __forceinline__ T limit(T a, T b) {
  if constexpr (LIM == LIM_MINMOD) {
    if (a * b <= T(0)) return T(0);
    return a > T(0) ? fmin(a, b) : fmax(a, b);
  }
  const T den = fabs(a) + fabs(b);
  if constexpr (sizeof(T) == 4) {
    // FP32: hardware reciprocal (1 ulp) instead of an IEEE division
    return den > T(0) ? (a * fabs(b) + fabs(a) * b) * __builtin_amdgcn_rcpf(den) : T(0);
  } else {
    return den > T(0) ? (a * fabs(b) + fabs(a) * b) / den : T(0);
  }
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
__device__ __forceinline__ void qe_half(T* n, T* m, T kappa, bool with_f = true) {
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
    // a D2Q9 f-lattice carries no third-order moments: only g relaxes
    if (!with_f) axxx = axxy = axyy = ayyy = T(0);
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
  double U[G::NH], V[G::NH], RT[G::NH];  // cell frames (u_x, u_y, sqrt T)
  T F[G::NP * G::NF];          // face populations phi^{lambda_F}
  double FU[G::NF], FV[G::NF], FRT[G::NF];          // face frames
  int skip;                    // the solve has already failed: leave the tile
  // per-cell f-lattice (multiscale kernels): 4 = D2Q16, 3 = D2Q9 (nodes per
  // axis) of the halo slots and of the faces
  unsigned char Lat[G::NH];
  unsigned char FL[G::NF];
};

// Sets `bit` in the solve's status flag if `cond` holds on any active lane of
// the wave, with one atomic per wave: a solve that has gone non-physical
// would otherwise have every cell contend for the one flag word.
__device__ __forceinline__ void raise_flag(int* flag, bool cond, int bit) {
  const unsigned long long m = __ballot(cond);
  if (m && __lane_id() == __ffsll((long long)m) - 1) atomicOr(flag, bit);
}

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
// Returns what the slot holds: a cell of the grid (periodic and
// zero-gradient ghosts are copies of one), an inflow ghost or a wall ghost.
// WALLS = false: the caller never asks for a wall ghost (cells of the grid,
// or solves on per-cell f-lattices, which take no walls).
enum SlotKind { SLOT_CELL = 0, SLOT_INFLOW = 1, SLOT_WALL = 2 };
template <int D, typename T, bool WALLS = true>
__device__ __forceinline__ int load_cell(const StepArgs& a, int gx, int gy, long long (&U)[4],
                                          T (&n)[Geo<D>::NP]) {
  constexpr int NP = Geo<D>::NP;
  int side = -1;
  const int sx = resolve(gx, a.nx, a.bc[0], a.bc[1], &side, 0);
  int sy = 0;
  if constexpr (D == 2) {
    sy = gy;
    if (side < 0) sy = resolve(gy, a.ny, a.bc[2], a.bc[3], &side, 2);
  }
  if constexpr (D == 2 && WALLS) {
    // (select, not an index: a run-time index into the arguments would put
    // them in scratch memory)
    const int bcs = side == 0 ? a.bc[0] : side == 1 ? a.bc[1] : side == 2 ? a.bc[2] : a.bc[3];
    if (side >= 0 && bcs == BC_WALL) {
      // wall ghost of layer k at coordinate t along the wall (x first: off
      // the end of an x wall, y wraps on a periodic axis, else clamps);
      // slots past the second layer (partial tiles) repeat the second
      const int v = side < 2 ? gx : gy, nn = side < 2 ? a.nx : a.ny;
      const int k = min(v < 0 ? -v : v - nn + 1, 2);
      int t = side < 2 ? gy : sx;
      if (side < 2 && (t < 0 || t >= a.ny))
        t = a.bc[2] == BC_PERIODIC ? ((t % a.ny) + a.ny) % a.ny : (t < 0 ? 0 : a.ny - 1);
      const size_t e = size_t(2 * side + k - 1) * size_t(a.wall_len) + size_t(t);
      const T* wn = static_cast<const T*>(a.wN);
#pragma unroll
      for (int q = 0; q < 4; ++q) U[q] = a.wU[q * a.wall_n + e];
#pragma unroll
      for (int i = 0; i < NP; ++i) n[i] = wn[i * a.wall_n + e];
      return SLOT_WALL;
    }
  }
  if (side >= 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) U[q] = a.inflow[4 * side + q];
#pragma unroll
    for (int i = 0; i < NP; ++i) n[i] = T(0);
    return SLOT_INFLOW;
  }
  const T* nin = static_cast<const T*>(a.n_in);
  const size_t cell = size_t(sx) + size_t(a.nx) * size_t(sy);
#pragma unroll
  for (int q = 0; q < 4; ++q) U[q] = a.U_in[q * a.cells + cell];
#pragma unroll
  for (int i = 0; i < NP; ++i) n[i] = nin[i * a.cells + cell];
  return SLOT_CELL;
}

// Body force (App. D), one Strang half step of d f / dt = F with
// F_i = a . (v_i - u) / T f^eq_i by an explicit Euler step of dt/2 (the
// sign that makes the force add (dt/2) rho a of momentum, as u* = u +
// (dt/2) a states).  In the comoving frame (v - u)/T = c / sqrt(T) and
// f^eq = rho W, so the step adds rho W_i (dt/2) a.c_i / sqrt(T) to f~ and
// changes the ledger by (dt/2) rho a (momentum) and (dt/2) a.(rho u)
// (energy); the cell then moves to the comoving frame of its new moments.
// force_ledger: the ledger part only (ha = (dt/2) a).
__device__ __forceinline__ void force_ledger(const StepArgs& a, long long (&U)[4], int* bad) {
  const double rho = double(U[0]) * a.inv_scale;
  const double mx = double(U[1]) * a.inv_scale, my = double(U[2]) * a.inv_scale;
  U[1] += to_fixed(rho * a.hax, a.scale, bad);
  U[2] += to_fixed(rho * a.hay, a.scale, bad);
  U[3] += to_fixed(a.hax * mx + a.hay * my, a.scale, bad);
}

template <typename T, int TF>
__device__ __forceinline__ void force_half(const StepArgs& a, long long (&U)[4], T (&n)[25]) {
  const Frame f0 = gauge(U, a);
  int bad = 0;
  force_ledger(a, U, &bad);
  raise_flag(a.flag, bad != 0, 2);
  const Frame f1 = gauge(U, a);
  const T r = T(f0.rho), kx = T(a.hax * f0.irt), ky = T(a.hay * f0.irt);
  const T rg0 = T(a.geq * f0.T * f0.rho), rg1 = T(a.geq * f1.T * f1.rho);
  T ft[16], gt[9], o[25];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const T w = wf<2, T>(i);
    ft[i] = r * w * (T(1) + kx * node<4, T>(i & 3) + ky * node<4, T>(i >> 2)) + n[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) gt[i] = rg0 * wg<2, T>(i) + n[16 + i];
  transform<2, 4, T, TF>(f0.rt, f0.ux, f0.uy, f1.irt, f1.ux, f1.uy, ft, o);
  transform<2, 3, T, TF>(f0.rt, f0.ux, f0.uy, f1.irt, f1.ux, f1.uy, gt, o + 16);
#pragma unroll
  for (int i = 0; i < 16; ++i) n[i] = o[i] - r * wf<2, T>(i);
#pragma unroll
  for (int i = 0; i < 9; ++i) n[16 + i] = o[16 + i] - rg1 * wg<2, T>(i);
}

// f-lattice of grid cell (gx, gy) for this step (multiscale kernels): the
// lattice the switch chose for the cell the ghost rule resolves to (an
// inflow ghost: the next interior cell), and the lattice its stored
// populations are written in.
__device__ __forceinline__ void cell_lattice(const StepArgs& a, int gx, int gy, int* q_new,
                                             int* q_old) {
  int side = -1;
  const int sx = resolve(gx, a.nx, a.bc[0], a.bc[1], &side, 0);
  int sy = gy < 0 ? 0 : (gy >= a.ny ? a.ny - 1 : gy);
  if (side < 0) sy = resolve(gy, a.ny, a.bc[2], a.bc[3], &side, 2);
  const size_t cell = size_t(sx) + size_t(a.nx) * size_t(sy);
  *q_new = a.lat_out[cell];
  *q_old = side >= 0 ? *q_new : a.lat_in[cell];
}

// Non-equilibrium populations of a cell moved between f-lattices in the
// cell's own frame (multiscale switch): lifting keeps the moments to order
// two and sets the third-order ones to their equilibrium value 0, projection
// keeps the moments to order two.  The comoving equilibrium rho W maps to
// rho W exactly either way, so the non-equilibrium part maps on its own.
template <typename T>
__device__ __forceinline__ void relattice(T* n, int q_old, int q_new) {
  if (q_old == q_new) return;
  T t[16];
  if (q_new == 4) {
    grad_map<3, 4, 2, T, 0>(T(1), T(0), T(0), n, t);
#pragma unroll
    for (int i = 0; i < 16; ++i) n[i] = t[i];
  } else {
    grad_map<4, 3, 2, T, 0>(T(1), T(0), T(0), n, t);
#pragma unroll
    for (int i = 0; i < 9; ++i) n[i] = t[i];
  }
}

// A stencil cell of a multiscale face: the f populations in LDS slot h
// (f-lattice sm.Lat[h]) in the face frame and on the face's f-lattice Q1T --
// Grad's projection when the lattices agree, lifting (own-frame expansion
// onto D2Q16, then D2Q16 Grad) or projection (D2Q16 -> D2Q9) otherwise.
// out is indexed n + Q1T t (n normal, t transverse).
template <int Q1T, typename T, int AXIS, int MODE>
__device__ __forceinline__ void ms_stencil(const Smem<2, T>& sm, int h, T s, T dn, T dt, T* out) {
  using G = Geo<2>;
  if (MODE == 4 || (MODE == 1 && sm.Lat[h] == 4)) {
    T in[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) in[i] = sm.P[i * G::NH + h];
    if constexpr (Q1T == 4) grad_map<4, 4, 3, T, AXIS>(s, dn, dt, in, out);
    else grad_map<4, 3, 2, T, AXIS>(s, dn, dt, in, out);
  } else {
    T in[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) in[i] = sm.P[i * G::NH + h];
    if constexpr (Q1T == 4) {
      T l[16];
      grad_map<3, 4, 2, T, 0>(T(1), T(0), T(0), in, l);
      grad_map<4, 4, 3, T, AXIS>(s, dn, dt, l, out);
    } else {
      grad_map<3, 3, 2, T, AXIS>(s, dn, dt, in, out);
    }
  }
}

// --------------------------------------------------------------------------
// One face: populations phi^{lambda_F}(x_b, t + dt/2) and the conserved flux.
// Stencil slots: 0 L, 1 R, 2 L-e_a, 3 R+e_a, 4 L+e_t, 5 L-e_t, 6 R+e_t, 7 R-e_t.
// --------------------------------------------------------------------------

// MUSCL reconstruction at the departure point x_b - v dt/2 (eq. InterfacePop)
// of the populations of one lattice whose transverse index lies in
// [K0, K0 + NK) (local index j = n + Q1 t), from the upwind cell by the sign
// of the normal velocity.  A normal velocity within kTieBand of the face
// thermal speed is a tie (rounding noise around a fluid at rest cannot pick a
// side), and a tie takes the mean of both upwind reconstructions.  The
// stencil is transformed into the face frame one cell at a time; the upwind
// operands of the two limiters are selected per population, so each
// population costs one normal and one transverse limiter; ties take a second
// pass.
template <int D, int Q1, typename T, int AXIS, int K0, int NK, int LIM, int TF, int MSF = 0>
__device__ __forceinline__ void reconstruct(const StepArgs& a, const Smem<D, T>& sm,
                                            const int (&st)[Geo<D>::NS], int plane0, double rtF,
                                            double irtF, double uF, double vF, T* bar) {
  using G = Geo<D>;
  constexpr int Q = D == 2 ? Q1 * Q1 : Q1;  // populations of the lattice
  constexpr int NQ = D == 2 ? Q1 * NK : Q1; // populations of this part
  // stencil cell `slot` in the face frame
  auto tfs = [&](int slot, T* out) {
    // compiler-only memory fence: the LDS loads of one stencil cell are not
    // hoisted above the work of the previous one
    asm volatile("" ::: "memory");
    const int h = st[slot];
    if constexpr (D == 2 && MSF) {
      // f of a multiscale face: the cell's own f-lattice onto the face's
      const T s = T(sm.RT[h] * irtF);
      const T dn = T(((AXIS == 0 ? sm.U[h] : sm.V[h]) - (AXIS == 0 ? uF : vF)) * irtF);
      const T dt = T(((AXIS == 0 ? sm.V[h] : sm.U[h]) - (AXIS == 0 ? vF : uF)) * irtF);
      T all[Q1 * Q1];
      ms_stencil<Q1, T, AXIS, MSF>(sm, h, s, dn, dt, all);
#pragma unroll
      for (int j = 0; j < Q1 * NK; ++j) out[j] = all[j + Q1 * K0];
    } else {
      T in[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) in[i] = sm.P[(plane0 + i) * G::NH + h];
      if constexpr (D == 2) {
        const T s = T(sm.RT[h] * irtF);
        const T dn = T(((AXIS == 0 ? sm.U[h] : sm.V[h]) - (AXIS == 0 ? uF : vF)) * irtF);
        const T dt = T(((AXIS == 0 ? sm.V[h] : sm.U[h]) - (AXIS == 0 ? vF : uF)) * irtF);
        xform<TF, Q1, T, AXIS, K0, NK>(s, dn, dt, in, out);
      } else {
        transform<1, Q1, T, TF>(sm.RT[h], sm.U[h], 0.0, irtF, uF, 0.0, in, out);
      }
    }
    // keep the scheduler from overlapping the stencil cells' transforms
    // (each one holds its own LDS loads and coefficients in registers)
    __builtin_amdgcn_sched_barrier(0);
  };
  auto nidx = [](int j) { return j % Q1; };                     // normal node index
  auto tidx = [](int j) { return D == 2 ? K0 + j / Q1 : 0; };   // transverse node index
  // upwind side decided in FP64 (bit j: population j upwinded from L / tied)
  const double band = kTieBand * rtF;
  unsigned left = 0, tie = 0;
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    const double v = rtF * node<Q1, double>(nidx(j)) + (AXIS == 0 ? uF : vF);
    const unsigned l = !(v < -band), t = l & unsigned(!(v > band));
    left |= l << j;
    tie |= t << j;
  }
  // departure-point offsets in cell units: normal -v_n dt/(2 dx) (+-1/2 from
  // the upwind centre), transverse -v_t dt/(2 dx)
  const T rtT = T(rtF), unT = T(AXIS == 0 ? uF : vF), utT = T(AXIS == 0 ? vF : uF);
  const T hl = T(0.5 * a.lam);
  auto vnorm = [&](int j) { return rtT * node<Q1, T>(nidx(j)) + unT; };
  auto dtrans = [&](int j) { return -hl * (rtT * node<Q1, T>(tidx(j)) + utT); };
  auto isl = [&](int j) { return (left >> j) & 1u; };
  T PL[NQ], PR[NQ], X[NQ], rec[NQ];
  tfs(0, PL);
  tfs(1, PR);
  {
    // normal slope: L side limits (PL - P_{L-e}, PR - PL), R side (PR - PL, P_{R+e} - PR)
    T t[NQ];
    tfs(2, t);
#pragma unroll
    for (int j = 0; j < NQ; ++j) X[j] = PL[j] - t[j];
    tfs(3, t);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const bool l = isl(j);
      const T mid = PR[j] - PL[j];
      const T sa = l ? X[j] : mid, sb = l ? mid : t[j] - PR[j];
      const T dn = (l ? T(0.5) : T(-0.5)) - hl * vnorm(j);
      rec[j] = (l ? PL[j] : PR[j]) + dn * limit<LIM>(sa, sb);
    }
  }
  if constexpr (D == 2) {
    // transverse slope at the upwind cell
    T ta[NQ], tb[NQ];
    {
      T t[NQ];
      tfs(4, t);
#pragma unroll
      for (int j = 0; j < NQ; ++j) tb[j] = t[j] - PL[j];
      tfs(5, t);
#pragma unroll
      for (int j = 0; j < NQ; ++j) ta[j] = PL[j] - t[j];
      tfs(6, t);
#pragma unroll
      for (int j = 0; j < NQ; ++j) tb[j] = isl(j) ? tb[j] : t[j] - PR[j];
      tfs(7, t);
#pragma unroll
      for (int j = 0; j < NQ; ++j) ta[j] = isl(j) ? ta[j] : PR[j] - t[j];
    }
#pragma unroll
    for (int j = 0; j < NQ; ++j) rec[j] += dtrans(j) * limit<LIM>(ta[j], tb[j]);
  }
  if (tie) {
    // ties: the right-upwind reconstruction, then the mean of both
    T t[NQ], rr[NQ];
    tfs(3, t);
#pragma unroll
    for (int j = 0; j < NQ; ++j)
      rr[j] = PR[j] + (T(-0.5) - hl * vnorm(j)) * limit<LIM>(PR[j] - PL[j], t[j] - PR[j]);
    if constexpr (D == 2) {
      T tp[NQ];
      tfs(6, tp);
      tfs(7, t);
#pragma unroll
      for (int j = 0; j < NQ; ++j) rr[j] += dtrans(j) * limit<LIM>(PR[j] - t[j], tp[j] - PR[j]);
    }
#pragma unroll
    for (int j = 0; j < NQ; ++j)
      if ((tie >> j) & 1u) rec[j] = T(0.5) * (rec[j] + rr[j]);
  }
#pragma unroll
  for (int j = 0; j < NQ; ++j) bar[j] = rec[j];
}

// Whether a population's normal velocity at the face lies in the tie band.
template <int Q1, int AXIS>
__device__ __forceinline__ bool tied(double rtF, double uF, double vF) {
  const double band = kTieBand * rtF;
  bool t = false;
#pragma unroll
  for (int n = 0; n < Q1; ++n) t |= fabs(rtF * node<Q1, double>(n) + (AXIS == 0 ? uF : vF)) <= band;
  return t;
}

// The same reconstruction for all Q1 x Q1 populations of one 2D lattice at
// once (out indexed j = n + Q1 t), walking the stencil one cell at a time:
// each cell is transformed into the face frame whole and folded into the
// running limiter operands, so the frame-dependent coefficients of a cell are
// formed once per face rather than once per transverse row.  Faces where a
// population's normal velocity falls in the tie band take the row-wise path.
template <int Q1, typename T, int AXIS, int LIM, int TF, int MSF = 0>
__device__ __forceinline__ void reconstruct_full(const StepArgs& a, Smem<2, T>& sm,
                                                 const int (&st)[Geo<2>::NS], int plane0,
                                                 int fidx, double rtF, double irtF, double uF,
                                                 double vF, T* out) {
  using G = Geo<2>;
  constexpr int Q = Q1 * Q1;
  auto tfs = [&](int slot, T* o) {
    // compiler-only memory fence: the LDS loads of one stencil cell are not
    // hoisted above the work of the previous one
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
    const int h = st[slot];
    const T s = T(sm.RT[h] * irtF);
    const T dn = T(((AXIS == 0 ? sm.U[h] : sm.V[h]) - (AXIS == 0 ? uF : vF)) * irtF);
    const T dt = T(((AXIS == 0 ? sm.V[h] : sm.U[h]) - (AXIS == 0 ? vF : uF)) * irtF);
    if constexpr (MSF) {
      ms_stencil<Q1, T, AXIS, MSF>(sm, h, s, dn, dt, o);  // f of a multiscale face
    } else {
      T in[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) in[i] = sm.P[(plane0 + i) * G::NH + h];
      xform<TF, Q1, T, AXIS, 0, Q1>(s, dn, dt, in, o);
    }
    // the empty asm pins the finished outputs: without it the compiler sinks
    // parts of the transform into the consumers and keeps its operands live
    // across the next cells (spills)
#pragma unroll
    for (int i = 0; i < Q; ++i) asm volatile("" : "+v"(o[i]));
    __builtin_amdgcn_sched_barrier(0);
  };
  // the upwind side depends on the normal node only (bit n), decided in FP64;
  // the caller has ruled out ties
  unsigned left = 0;
#pragma unroll
  for (int n = 0; n < Q1; ++n)
    left |= unsigned(rtF * node<Q1, double>(n) + (AXIS == 0 ? uF : vF) > 0.0) << n;
  const T rtT = T(rtF), unT = T(AXIS == 0 ? uF : vF), utT = T(AXIS == 0 ? vF : uF);
  const T hl = T(0.5 * a.lam);
  auto isl = [&](int j) { return (left >> (j % Q1)) & 1u; };
  auto vnorm = [&](int j) { return rtT * node<Q1, T>(j % Q1) + unT; };
  auto dtrans = [&](int j) { return -hl * (rtT * node<Q1, T>(j / Q1) + utT); };
  // the partial reconstruction waits in this face's slot of the face buffer
  // (indexed by j) while the transverse neighbours are transformed
  auto park = [&](int j) -> T& { return sm.F[(plane0 + j) * G::NF + fidx]; };
  T PL[Q], PR[Q], S[Q], TB[Q];
  tfs(0, PL);
  tfs(1, PR);
  {
    T t[Q];
    tfs(2, t);  // first normal-limiter operand
#pragma unroll
    for (int j = 0; j < Q; ++j) S[j] = isl(j) ? PL[j] - t[j] : PR[j] - PL[j];
    tfs(3, t);  // second operand, then the normal slope term at the upwind cell
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const bool l = isl(j);
      const T sb = l ? PR[j] - PL[j] : t[j] - PR[j];
      const T dn = (l ? T(0.5) : T(-0.5)) - hl * vnorm(j);
      park(j) = (l ? PL[j] : PR[j]) + dn * limit<LIM>(S[j], sb);
    }
    // transverse slope term: left-upwind populations from L's neighbours
    // (4, 5), added to the parked value, then right-upwind ones from R's (6, 7)
    tfs(4, t);
#pragma unroll
    for (int j = 0; j < Q; ++j) TB[j] = t[j] - PL[j];
    tfs(5, t);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const T d = dtrans(j) * limit<LIM>(PL[j] - t[j], TB[j]);
      park(j) += isl(j) ? d : T(0);
    }
    tfs(6, t);
#pragma unroll
    for (int j = 0; j < Q; ++j) TB[j] = t[j] - PR[j];
    tfs(7, t);
#pragma unroll
    for (int j = 0; j < Q; ++j) S[j] = isl(j) ? T(0) : dtrans(j) * limit<LIM>(PR[j] - t[j], TB[j]);
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) out[j] = park(j) + S[j];
}

// MS: 0 one f-lattice (D2Q16); 1 per-cell f-lattices; 3 / 4 a tile whose
// cells are all D2Q9 / all D2Q16 in a solve with per-cell lattices.
template <int D, typename T, int AXIS, int LIM, int TF, int MS = 0>
__device__ __forceinline__ void face_eval(const StepArgs& a, Smem<D, T>& sm, const int (&st)[Geo<D>::NS], int fidx) {
  using G = Geo<D>;
  constexpr int QF = G::QF, QG = G::QG;
  // each lattice is reconstructed whole unless a tie needs the row-wise path
  constexpr bool kWhole = true;
  const int hL = st[0], hR = st[1];
  // f-lattice of the face: the higher one of its two cells (multiscale)
  bool f16 = true;
  if constexpr (MS == 3) f16 = false;
  if constexpr (MS == 1) f16 = max(sm.Lat[hL], sm.Lat[hR]) == 4;
  // eq. AvgFrame
  double uF = 0.5 * (sm.U[hL] + sm.U[hR]);
  double vF = D == 2 ? 0.5 * (sm.V[hL] + sm.V[hR]) : 0.0;
  double TFc = 0.5 * (sm.RT[hL] * sm.RT[hL] + sm.RT[hR] * sm.RT[hR]);  // face temperature
  double rho_b = 0.0, ub = 0.0, vb = 0.0, Tb = 0.0, rtF = 0.0, irtF = 0.0;
#pragma unroll 1
  for (int pass = 0; pass <= a.n_corr; ++pass) {
    rtF = sqrt(TFc);
    irtF = 1.0 / rtF;
    // macroscopic fields at the face, in FP64; f-bar is parked in the face
    // slot of LDS while g is reconstructed
    double m0 = 0.0, mx = 0.0, my = 0.0, e = 0.0;
    // f in parts by transverse index (two halves in 2D); g whole
    auto take_f = [&](const T* bar, int k0, int nk) {
      for (int j = 0; j < (D == 2 ? 4 * nk : 4); ++j) {
        const int n = j % 4, t = k0 + j / 4;
        const int i = D == 1 ? n : (AXIS == 0 ? n + 4 * t : t + 4 * n);
        const double vx = rtF * node<4, double>(i & 3) + uF;
        const double vy = D == 2 ? rtF * node<4, double>(i >> 2) + vF : 0.0;
        const double fb = double(bar[j]);
        m0 += fb;
        mx += vx * fb;
        my += vy * fb;
        e += 0.5 * (vx * vx + vy * vy) * fb;
        sm.F[i * G::NF + fidx] = bar[j];
      }
    };
    if constexpr (D == 2 && MS) {
      if (!f16) {
        // D2Q9 f-lattice at this face: 3 x 3 populations in planes 0..8
        T bar[9];
        if (!tied<3, AXIS>(rtF, uF, vF)) {
          reconstruct_full<3, T, AXIS, LIM, TF, MS>(a, sm, st, 0, fidx, rtF, irtF, uF, vF, bar);
        } else {
          static_for<0, 3>([&](auto part) {
            constexpr int K0 = decltype(part)::value;
            reconstruct<D, 3, T, AXIS, K0, 1, LIM, TF, MS>(a, sm, st, 0, rtF, irtF, uF, vF,
                                                             bar + 3 * K0);
          });
        }
        const double un = AXIS == 0 ? uF : vF, ut = AXIS == 0 ? vF : uF;
        double C[3] = {0.0, 0.0, 0.0}, mn = 0.0, mt = 0.0, e2 = 0.0;
#pragma unroll
        for (int n = 0; n < 3; ++n) {
          double R = 0.0;
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            const double fb = double(bar[n + 3 * t]);
            R += fb;
            C[t] += fb;
            sm.F[(AXIS == 0 ? n + 3 * t : t + 3 * n) * G::NF + fidx] = bar[n + 3 * t];
          }
          const double vn = rtF * node<3, double>(n) + un;
          m0 += R;
          mn += vn * R;
          e2 += vn * vn * R;
        }
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const double vt = rtF * node<3, double>(t) + ut;
          mt += vt * C[t];
          e2 += vt * vt * C[t];
        }
        mx += AXIS == 0 ? mn : mt;
        my += AXIS == 0 ? mt : mn;
        e += 0.5 * e2;
      }
    }
    if constexpr (D == 2) {
      if (!f16) {
      } else if (kWhole && !tied<4, AXIS>(rtF, uF, vF)) {
        T bar[QF];
        reconstruct_full<4, T, AXIS, LIM, TF, MS>(a, sm, st, 0, fidx, rtF, irtF, uF, vF, bar);
        // moments through row sums R_n (over t) and column sums C_t (over n)
        const double un = AXIS == 0 ? uF : vF, ut = AXIS == 0 ? vF : uF;
        double C[4] = {0.0, 0.0, 0.0, 0.0}, mn = 0.0, mt = 0.0, e2 = 0.0;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          double R = 0.0;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const double fb = double(bar[n + 4 * t]);
            R += fb;
            C[t] += fb;
            sm.F[(AXIS == 0 ? n + 4 * t : t + 4 * n) * G::NF + fidx] = bar[n + 4 * t];
          }
          const double vn = rtF * node<4, double>(n) + un;
          m0 += R;
          mn += vn * R;
          e2 += vn * vn * R;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double vt = rtF * node<4, double>(t) + ut;
          mt += vt * C[t];
          e2 += vt * vt * C[t];
        }
        mx += AXIS == 0 ? mn : mt;
        my += AXIS == 0 ? mt : mn;
        e += 0.5 * e2;
      } else {
        // one row of the transverse index at a time, resolving ties
        static_for<0, 4>([&](auto part) {
          constexpr int K0 = decltype(part)::value;
          T bar[4];
          reconstruct<D, 4, T, AXIS, K0, 1, LIM, TF, MS>(a, sm, st, 0, rtF, irtF, uF, vF, bar);
          take_f(bar, K0, 1);
        });
      }
    } else {
      T bar[4];
      reconstruct<D, 4, T, AXIS, 0, 1, LIM, TF>(a, sm, st, 0, rtF, irtF, uF, vF, bar);
      take_f(bar, 0, 1);
    }
    auto g_rows = [&]() {
      static_for<0, (D == 2 ? 3 : 1)>([&](auto part) {
        constexpr int K0 = decltype(part)::value;
        T gbar[3];
        reconstruct<D, 3, T, AXIS, K0, 1, LIM, TF>(a, sm, st, QF, rtF, irtF, uF, vF, gbar);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const int i = D == 1 ? j : (AXIS == 0 ? j + 3 * K0 : K0 + 3 * j);
          e += double(gbar[j]);
          sm.F[(QF + i) * G::NF + fidx] = gbar[j];
        }
      });
    };
    if constexpr (D == 2) {
      if (kWhole && !tied<3, AXIS>(rtF, uF, vF)) {
        T gbar[QG];
        reconstruct_full<3, T, AXIS, LIM, TF>(a, sm, st, QF, fidx, rtF, irtF, uF, vF, gbar);
#pragma unroll
        for (int j = 0; j < QG; ++j) {
          const int n = j % 3, t = j / 3;
          const int i = AXIS == 0 ? n + 3 * t : t + 3 * n;
          e += double(gbar[j]);
          sm.F[(QF + i) * G::NF + fidx] = gbar[j];
        }
      } else {
        g_rows();
      }
    } else {
      g_rows();
    }
    rho_b = m0;
    ub = mx / m0;
    vb = my / m0;
    Tb = (e - 0.5 * m0 * (ub * ub + vb * vb)) / (a.cv * m0);
    if (pass < a.n_corr) {  // corrector: re-evaluate in the frame just found
      uF = ub;
      vF = vb;
      TFc = Tb;
    }
  }
  // face equilibrium rho G_{u_b,T_b}^{lambda_F} W (eq. NonComovingEq), separable;
  // phi = c1 phi-bar + c2 phi^eq inverts eq. FluxTransf
  const T sb = T(sqrt(Tb) * irtF);
  const T c1 = T(a.c_face1), c2 = T(a.c_face2);
  if constexpr (D == 2 && TF == TF_GRAD) {
    // not separable: the map applied to the comoving rho W (and g's)
    const T dn = T(((AXIS == 0 ? ub : vb) - (AXIS == 0 ? uF : vF)) * irtF);
    const T dt = T(((AXIS == 0 ? vb : ub) - (AXIS == 0 ? vF : uF)) * irtF);
    if (f16) {
      T w[QF], eq[QF];
      const T r = T(rho_b);
#pragma unroll
      for (int i = 0; i < QF; ++i) w[i] = r * wf<D, T>(i);
      transform_grad<4, T, AXIS>(sb, dn, dt, w, eq);
#pragma unroll
      for (int j = 0; j < QF; ++j) {
        const int n = j % 4, t = j / 4;
        T& slot = sm.F[(AXIS == 0 ? n + 4 * t : t + 4 * n) * G::NF + fidx];
        slot = c1 * slot + c2 * eq[j];
      }
    } else {
      T w[9], eq[9];
      const T r = T(rho_b);
#pragma unroll
      for (int i = 0; i < 9; ++i) w[i] = r * wg<D, T>(i);
      transform_grad<3, T, AXIS>(sb, dn, dt, w, eq);
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const int n = j % 3, t = j / 3;
        T& slot = sm.F[(AXIS == 0 ? n + 3 * t : t + 3 * n) * G::NF + fidx];
        slot = c1 * slot + c2 * eq[j];
      }
    }
    {
      T w[QG], eq[QG];
      const T r = T(a.geq * Tb * rho_b);
#pragma unroll
      for (int i = 0; i < QG; ++i) w[i] = r * wg<D, T>(i);
      transform_grad<3, T, AXIS>(sb, dn, dt, w, eq);
#pragma unroll
      for (int j = 0; j < QG; ++j) {
        const int n = j % 3, t = j / 3;
        T& slot = sm.F[(QF + (AXIS == 0 ? n + 3 * t : t + 3 * n)) * G::NF + fidx];
        slot = c1 * slot + c2 * eq[j];
      }
    }
  } else {
    {
      T ex[4], ey[4];
      eq_factor<4, T>(sb, T((ub - uF) * irtF), ex);
      if constexpr (D == 2) eq_factor<4, T>(sb, T((vb - vF) * irtF), ey);
      const T r = T(rho_b);
#pragma unroll
      for (int i = 0; i < QF; ++i) {
        const T feq = D == 2 ? r * ex[i & 3] * ey[i >> 2] : r * ex[i];
        T& slot = sm.F[i * G::NF + fidx];
        slot = c1 * slot + c2 * feq;
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
        T& slot = sm.F[(QF + i) * G::NF + fidx];
        slot = c1 * slot + c2 * geq;
      }
    }
  }
  raise_flag(a.flag, !(rho_b > 0.0) || !(Tb > 0.0), 1);
  if constexpr (MS == 1) sm.FL[fidx] = f16 ? 4 : 3;
  sm.FU[fidx] = uF;
  sm.FV[fidx] = vF;
  sm.FRT[fidx] = rtF;
}

// Conserved fluxes through a face (mass, momentum, energy of phi^{lambda_F}
// times the normal particle velocity in the face frame, App. C), in FP64,
// times dt/dx and rounded once to the ledger unit.  Both cells next to a face
// evaluate it from the same LDS data, so they apply the same integer.
template <int D, typename T, int AXIS, int MS = 0>
__device__ __forceinline__ void face_flux(const StepArgs& a, const Smem<D, T>& sm, int fi,
                                          long long (&psi)[4]) {
  using G = Geo<D>;
  constexpr int QF = G::QF, QG = G::QG;
  const double rtF = sm.FRT[fi], uF = sm.FU[fi], vF = sm.FV[fi];
  double Fr = 0.0, Fx = 0.0, Fy = 0.0, FE = 0.0;
  if constexpr (D == 2) {
    // sums over the transverse index first: with n the normal and t the
    // transverse node, v_n and v_t are per-node and the moments factor as
    // sums over n of v_n {1, v_n, ., v_n^2/2} times row sums over t
    const double un = AXIS == 0 ? uF : vF, ut = AXIS == 0 ? vF : uF;
    double vt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) vt[k] = rtF * node<4, double>(k) + ut;
    double Fn = 0.0, Ft = 0.0;
    // f on a D2Q9 face (multiscale): nodes of D1Q3, three rows
    bool f9 = false;
    if constexpr (MS == 3) f9 = true;
    if constexpr (MS == 1) f9 = sm.FL[fi] == 3;
    if (f9) {
      double vt3[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) vt3[k] = rtF * node<3, double>(k) + ut;
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        const double vn = rtF * node<3, double>(n) + un;
        double R = 0.0, Y = 0.0, Y2 = 0.0;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const double f = double(sm.F[(AXIS == 0 ? n + 3 * t : t + 3 * n) * G::NF + fi]);
          R += f;
          Y += vt3[t] * f;
          Y2 += vt3[t] * vt3[t] * f;
        }
        Fr += vn * R;
        Fn += vn * vn * R;
        Ft += vn * Y;
        FE += 0.5 * vn * (vn * vn * R + Y2);
      }
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const double vn = rtF * node<4, double>(n) + un;
      double R = 0.0, Y = 0.0, Y2 = 0.0;
      if (!f9) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = AXIS == 0 ? n + 4 * t : t + 4 * n;
          const double f = double(sm.F[i * G::NF + fi]);
          R += f;
          Y += vt[t] * f;
          Y2 += vt[t] * vt[t] * f;
        }
      }
      double Rg = 0.0;
      if (n < 3) {
        const double vg = rtF * node<3, double>(n) + un;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const int i = AXIS == 0 ? n + 3 * t : t + 3 * n;
          Rg += double(sm.F[(QF + i) * G::NF + fi]);
        }
        FE += vg * Rg;
      }
      Fr += vn * R;
      Fn += vn * vn * R;
      Ft += vn * Y;
      FE += 0.5 * vn * (vn * vn * R + Y2);
    }
    Fx = AXIS == 0 ? Fn : Ft;
    Fy = AXIS == 0 ? Ft : Fn;
  } else {
#pragma unroll
    for (int i = 0; i < QF; ++i) {
      const double vx = rtF * node<4, double>(i) + uF;
      const double p = double(sm.F[i * G::NF + fi]) * vx;
      Fr += p;
      Fx += vx * p;
      FE += 0.5 * vx * vx * p;
    }
#pragma unroll
    for (int i = 0; i < QG; ++i)
      FE += (rtF * node<3, double>(i) + uF) * double(sm.F[(QF + i) * G::NF + fi]);
  }
  int bad = 0;
  const double sc = a.lam * a.scale;
  psi[0] = to_fixed(Fr, sc, &bad);
  psi[1] = to_fixed(Fx, sc, &bad);
  psi[2] = to_fixed(Fy, sc, &bad);
  psi[3] = to_fixed(FE, sc, &bad);
  raise_flag(a.flag, bad != 0, 2);
}

// Flux of two opposite faces into the cell frame (eq. fluxEq):
// acc += v_a^{lambda_j} (G phi_hi - G phi_lo).
template <int D, typename T, int AXIS, int TF>
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
    transform<D, 4, T, TF>(rtF, uF, vF, c.irt, c.ux, c.uy, in, out);
#pragma unroll
    for (int i = 0; i < QF; ++i) dlt[i] = side ? out[i] - dlt[i] : out[i];
    __builtin_amdgcn_sched_barrier(0);
    T ing[QG], outg[QG];
#pragma unroll
    for (int i = 0; i < QG; ++i) ing[i] = sm.F[(QF + i) * G::NF + fi];
    transform<D, 3, T, TF>(rtF, uF, vF, c.irt, c.ux, c.uy, ing, outg);
#pragma unroll
    for (int i = 0; i < QG; ++i) dlt[QF + i] = side ? outg[i] - dlt[QF + i] : outg[i];
    __builtin_amdgcn_sched_barrier(0);
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

// gather_faces for a cell of a multiscale solve whose f-lattice is qc: each
// face's f populations (f-lattice sm.FL) go into the cell frame and onto the
// cell's lattice -- Grad's projection of the lattice, or the D2Q16 -> D2Q9
// projection where a D2Q16 face borders a D2Q9 cell (a D2Q16 cell only
// borders D2Q16 faces).  A D2Q9 cell uses f entries 0..8 of acc.
template <typename T, int AXIS, int TF, int MODE>
__device__ __forceinline__ void gather_faces_ms(Smem<2, T>& sm, int flo, int fhi, const Frame& c,
                                                int qc_dyn, T (&acc)[Geo<2>::NP]) {
  const int qc = MODE == 1 ? qc_dyn : MODE;
  using G = Geo<2>;
  constexpr int QF = G::QF, QG = G::QG;
  T dlt[G::NP];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int fi = side ? fhi : flo;
    const double rtF = sm.FRT[fi], uF = sm.FU[fi], vF = sm.FV[fi];
    T out[QF];
    if (qc == 4) {
      T in[QF];
#pragma unroll
      for (int i = 0; i < QF; ++i) in[i] = sm.F[i * G::NF + fi];
      transform<2, 4, T, TF>(rtF, uF, vF, c.irt, c.ux, c.uy, in, out);
    } else if (MODE == 1 && sm.FL[fi] == 4) {
      T in[QF];
#pragma unroll
      for (int i = 0; i < QF; ++i) in[i] = sm.F[i * G::NF + fi];
      const T s = T(rtF * c.irt), dx = T((uF - c.ux) * c.irt), dy = T((vF - c.uy) * c.irt);
      grad_map<4, 3, 2, T, 0>(s, dx, dy, in, out);
    } else {
      T in[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) in[i] = sm.F[i * G::NF + fi];
      transform<2, 3, T, TF>(rtF, uF, vF, c.irt, c.ux, c.uy, in, out);
    }
#pragma unroll
    for (int i = 0; i < QF; ++i) dlt[i] = side ? out[i] - dlt[i] : out[i];
    __builtin_amdgcn_sched_barrier(0);
    T ing[QG], outg[QG];
#pragma unroll
    for (int i = 0; i < QG; ++i) ing[i] = sm.F[(QF + i) * G::NF + fi];
    transform<2, 3, T, TF>(rtF, uF, vF, c.irt, c.ux, c.uy, ing, outg);
#pragma unroll
    for (int i = 0; i < QG; ++i) dlt[QF + i] = side ? outg[i] - dlt[QF + i] : outg[i];
    __builtin_amdgcn_sched_barrier(0);
  }
  const T rt = T(c.rt), u = T(AXIS == 0 ? c.ux : c.uy);
  if (qc == 4) {
#pragma unroll
    for (int i = 0; i < QF; ++i) {
      const int k = AXIS == 0 ? (i & 3) : (i >> 2);
      acc[i] += (rt * node<4, T>(k) + u) * dlt[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int k = AXIS == 0 ? (i % 3) : (i / 3);
      acc[i] += (rt * node<3, T>(k) + u) * dlt[i];
    }
  }
#pragma unroll
  for (int i = 0; i < QG; ++i) {
    const int k = AXIS == 0 ? (i % 3) : (i / 3);
    acc[QF + i] += (rt * node<3, T>(k) + u) * dlt[QF + i];
  }
}

// Phase 5 for a cell of a multiscale solve: the same DUGKS update on the
// cell's own f-lattice q (D2Q9: entries 0..8).  A D2Q9 cell's energy is the
// energy moment of its updated populations (with the second-order f-lattice
// the update does not carry the conserved flux of energy exactly, App. C),
// its mass and momentum stay the ledger's.
template <typename T, int TF, int MODE>
__device__ __forceinline__ void step_update_ms(const StepArgs& a, int x, int y,
                                               const T (&acc)[Geo<2>::NP], const long long (&dU)[4],
                                               T kappa) {
  using G = Geo<2>;
  constexpr int QF = G::QF, QG = G::QG, NP = G::NP;
  long long U[4];
  T own[NP];
  load_cell<2, T, false>(a, x, y, U, own);
  int q, qo;
  cell_lattice(a, x, y, &q, &qo);
  relattice(own, qo, q);
  if constexpr (MODE != 1) q = MODE;  // the same value: the tile is uniform
  const Frame f0 = gauge(U, a);  // the frame the populations are written in
  qe_half<2, T>(own, own + QF, kappa, q == 4);
  const T b = T(a.b_upd), lam = T(a.lam);
  const T r = T(f0.rho), rg = T(a.geq * f0.T * f0.rho);
  T ft[QF], gt[QG];
  if (q == 4) {
#pragma unroll
    for (int i = 0; i < QF; ++i) ft[i] = r * wf<2, T>(i) + b * own[i] - lam * acc[i];
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) ft[i] = r * wg<2, T>(i) + b * own[i] - lam * acc[i];
  }
#pragma unroll
  for (int i = 0; i < QG; ++i) gt[i] = rg * wg<2, T>(i) + b * own[QF + i] - lam * acc[QF + i];
  long long U2[4];
#pragma unroll
  for (int q2 = 0; q2 < 4; ++q2) U2[q2] = U[q2] - dU[q2];
  if (q == 3) {
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const double vx = f0.rt * node<3, double>(i % 3) + f0.ux;
      const double vy = f0.rt * node<3, double>(i / 3) + f0.uy;
      e += 0.5 * (vx * vx + vy * vy) * double(ft[i]) + double(gt[i]);
    }
    int bad = 0;
    U2[3] = to_fixed(e, a.scale, &bad);
    raise_flag(a.flag, bad != 0, 2);
  }
  const Frame nf = gauge(U2, a);
  T n2[NP];
  __builtin_amdgcn_sched_barrier(0);
  if (q == 4) transform<2, 4, T, TF>(f0.rt, f0.ux, f0.uy, nf.irt, nf.ux, nf.uy, ft, n2);
  else transform<2, 3, T, TF>(f0.rt, f0.ux, f0.uy, nf.irt, nf.ux, nf.uy, ft, n2);
  __builtin_amdgcn_sched_barrier(0);
  transform<2, 3, T, TF>(f0.rt, f0.ux, f0.uy, nf.irt, nf.ux, nf.uy, gt, n2 + QF);
  __builtin_amdgcn_sched_barrier(0);
  const T r2 = T(nf.rho), rg2 = T(a.geq * nf.T * nf.rho);
  if (q == 4) {
#pragma unroll
    for (int i = 0; i < QF; ++i) n2[i] -= r2 * wf<2, T>(i);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) n2[i] -= r2 * wg<2, T>(i);
#pragma unroll
    for (int i = 9; i < QF; ++i) n2[i] = T(0);
  }
#pragma unroll
  for (int i = 0; i < QG; ++i) n2[QF + i] -= rg2 * wg<2, T>(i);
  qe_half<2, T>(n2, n2 + QF, kappa, q == 4);
  raise_flag(a.flag, !(nf.rho > 0.0) || !(nf.T > 0.0) || !isfinite(double(n2[0])), 1);
  bool over = false;
#pragma unroll
  for (int q2 = 0; q2 < 4; ++q2) over |= (U2[q2] > (1LL << 62)) || (U2[q2] < -(1LL << 62));
  raise_flag(a.flag, over, 2);
  const size_t cell = size_t(x) + size_t(a.nx) * size_t(y);
  T* nout = static_cast<T*>(a.n_out);
#pragma unroll
  for (int i = 0; i < NP; ++i) nout[i * a.cells + cell] = n2[i];
#pragma unroll
  for (int q2 = 0; q2 < 4; ++q2) a.U_out[q2 * a.cells + cell] = U2[q2];
}

// --------------------------------------------------------------------------
// The fused step kernel.
// --------------------------------------------------------------------------
// Phases 1-5 of a tile (faces, gathers, update) after its halo is loaded.
// M: the f-lattice mode of the faces (see face_eval).  EXT: the solve may
// carry a body force (D2Q16 solves with walls or a force run this variant).
template <int D, typename T, int LIM, int TF, int M, bool EXT = false>
__device__ __forceinline__ void step_body(const StepArgs& a, Smem<D, T>& sm, int tid, int x0, int y0,
                                          T kappa) {
  using G = Geo<D>;
  constexpr int QF = G::QF, QG = G::QG, NP = G::NP;
  // the thread's own cell (interior slot tid); its frame is read from LDS
  // where it is needed, so that nothing of it is held through the face phases
  const int cx = tid % G::TX, cy = tid / G::TX;
  const bool own_in = tid < G::NI && x0 + cx < a.nx && (D == 1 || y0 + cy < a.ny);
  const int own_slot = cx + 2 + G::HX * (cy + G::OY);
  auto own_frame = [&]() {
    Frame f{};
    const int h = own_slot;
    f.ux = sm.U[h];
    f.uy = sm.V[h];
    f.T = sm.RT[h] * sm.RT[h];
    f.rt = sm.RT[h];
    f.irt = 1.0 / f.rt;
    return f;
  };

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
    face_eval<D, T, 0, LIM, TF, M>(a, sm, st, tid);
  }
  __syncthreads();
  // ---- 2. west/east faces into the cell frame
  T acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = T(0);
  long long dU[4] = {0, 0, 0, 0};
  if (tid < G::NI) {
    const int fw = cx + (G::TX + 1) * cy;
    if constexpr (D == 2 && M != 0)
      gather_faces_ms<T, 0, TF, M>(sm, fw, fw + 1, own_frame(), sm.Lat[own_slot], acc);
    else
      gather_faces<D, T, 0, TF>(sm, fw, fw + 1, own_frame(), acc);
    long long pw[4], pe[4];
    __builtin_amdgcn_sched_barrier(0);
    face_flux<D, T, 0, M>(a, sm, fw, pw);
    __builtin_amdgcn_sched_barrier(0);
    face_flux<D, T, 0, M>(a, sm, fw + 1, pe);
#pragma unroll
    for (int q = 0; q < 4; ++q) dU[q] += pe[q] - pw[q];
  }
  if constexpr (D == 2) {
    // park the x-flux in the cell's own output slot (written only by this
    // thread, read by nobody else this step) while the y-faces use the registers
    T* nout = static_cast<T*>(a.n_out);
    const size_t ocell = size_t(x0 + cx) + size_t(a.nx) * size_t(y0 + cy);
    if (own_in) {
#pragma unroll
      for (int i = 0; i < NP; ++i) nout[i * a.cells + ocell] = acc[i];
    }
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
      face_eval<D, T, 1, LIM, TF, M>(a, sm, st, tid);
    }
    __syncthreads();
    // ---- 4. south/north faces
    if (own_in) {
#pragma unroll
      for (int i = 0; i < NP; ++i) acc[i] = nout[i * a.cells + ocell];
    }
    if (tid < G::NI) {
      const int fs = cx + G::TX * cy;
      if constexpr (M != 0)
        gather_faces_ms<T, 1, TF, M>(sm, fs, fs + G::TX, own_frame(), sm.Lat[own_slot], acc);
      else
        gather_faces<D, T, 1, TF>(sm, fs, fs + G::TX, own_frame(), acc);
      long long ps[4], pn[4];
      __builtin_amdgcn_sched_barrier(0);
      face_flux<D, T, 1, M>(a, sm, fs, ps);
      __builtin_amdgcn_sched_barrier(0);
      face_flux<D, T, 1, M>(a, sm, fs + G::TX, pn);
#pragma unroll
      for (int q = 0; q < 4; ++q) dU[q] += pn[q] - ps[q];
    }
  }

  // ---- 5. DUGKS update, new comoving frame, second QE half step
  if constexpr (D == 2 && M != 0) {
    if (own_in) step_update_ms<T, TF, M>(a, x0 + cx, y0 + cy, acc, dU, kappa);
    return;
  }
  if (own_in) {
    long long U[4];
    T own[NP];
    load_cell<D, T, false>(a, x0 + cx, y0 + cy, U, own);
    if constexpr (D == 2 && EXT)
      if (a.force) force_half<T, TF>(a, U, own);  // as in the loader
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
    __builtin_amdgcn_sched_barrier(0);
    transform<D, 4, T, TF>(f0.rt, f0.ux, f0.uy, nf.irt, nf.ux, nf.uy, ft, n2);
    __builtin_amdgcn_sched_barrier(0);
    transform<D, 3, T, TF>(f0.rt, f0.ux, f0.uy, nf.irt, nf.ux, nf.uy, gt, n2 + QF);
    __builtin_amdgcn_sched_barrier(0);
    const T r2 = T(nf.rho), rg2 = T(a.geq * nf.T * nf.rho);
#pragma unroll
    for (int i = 0; i < QF; ++i) n2[i] -= r2 * wf<D, T>(i);
#pragma unroll
    for (int i = 0; i < QG; ++i) n2[QF + i] -= rg2 * wg<D, T>(i);
    qe_half<D, T>(n2, n2 + QF, kappa);
    // second body-force half step
    if constexpr (D == 2 && EXT)
      if (a.force) force_half<T, TF>(a, U2, n2);
    raise_flag(a.flag, !(nf.rho > 0.0) || !(nf.T > 0.0) || !isfinite(double(n2[0])), 1);
    bool over = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) over |= (U2[q] > (1LL << 62)) || (U2[q] < -(1LL << 62));
    raise_flag(a.flag, over, 2);
    const size_t cell = size_t(x0 + cx) + size_t(a.nx) * size_t(D == 2 ? y0 + cy : 0);
    T* nout = static_cast<T*>(a.n_out);
#pragma unroll
    for (int i = 0; i < NP; ++i) nout[i * a.cells + cell] = n2[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) a.U_out[q * a.cells + cell] = U2[q];
  }
}

// MS: 0 D2Q16; 1 per-cell f-lattices (multiscale); 2 D2Q16 with walls or a
// body force; 3 D2Q9 everywhere (the D2Q9 body alone, with its own register
// allocation).
template <int D, typename T, int LIM, int TF, int MS = 0>
__device__ __forceinline__ void step_tile(const StepArgs& a, int tile, Smem<D, T>& sm) {
  using G = Geo<D>;
  constexpr int QF = G::QF, QG = G::QG, NP = G::NP;
  const int tid = threadIdx.x;
  const int bx = tile % a.tiles_x, by = tile / a.tiles_x;
  const int x0 = bx * G::TX, y0 = by * G::TY;
  const T kappa = T(a.kappa), apre = T(a.a_pre);
  // a solve whose status flag is already raised has failed: its state is no
  // longer used, so its tiles do no work (one read per workgroup, shared
  // through LDS so that the whole workgroup takes the same branch)
  if (tid == 0) sm.skip = *static_cast<volatile int*>(a.flag);
  __syncthreads();
  if (sm.skip) return;

  // ---- 0. halo tile: ghost resolution, frame, first QE half step, phi-bar-plus
#pragma unroll 1
  for (int k = tid; k < G::NH; k += kThreads) {
    int hx, hy;
    slot_coords<D>(k, &hx, &hy);
    const int gx = x0 + hx - 2, gy = y0 + hy - G::OY;
    long long U[4];
    T n[NP];
    // a wall ghost is built at the start of the step with its relaxed
    // non-equilibrium: the first QE half step does not act on it.  The
    // first body-force half step acts on the cells of the grid (the ghosts
    // of walls and inflow sides are built from the forced state or fixed).
    const int kind = load_cell<D, T, MS == 2>(a, gx, gy, U, n);
    if constexpr (D == 2 && MS == 2)
      if (a.force && kind == SLOT_CELL) force_half<T, TF>(a, U, n);
    const T kap = kind == SLOT_WALL ? T(0) : kappa;
    const Frame fr = gauge(U, a);
    const int h = hx + G::HX * hy;
    const T r = T(fr.rho), rg = T(a.geq * fr.T * fr.rho);
    if constexpr (D == 2 && MS == 1) {
      // multiscale: the slot's f-lattice for this step; populations stored
      // on another lattice are lifted or projected first
      int qn, qo;
      cell_lattice(a, gx, gy, &qn, &qo);
      relattice(n, qo, qn);
      sm.Lat[h] = (unsigned char)qn;
      qe_half<D, T>(n, n + QF, kap, qn == 4);
      if (qn == 4) {
#pragma unroll
        for (int i = 0; i < QF; ++i) sm.P[i * G::NH + h] = r * wf<D, T>(i) + apre * n[i];
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) sm.P[i * G::NH + h] = r * wg<D, T>(i) + apre * n[i];
      }
    } else if constexpr (D == 2 && MS == 3) {
      // D2Q9 everywhere: every slot on D2Q9, no switch
      sm.Lat[h] = 3;
      qe_half<D, T>(n, n + QF, kap, false);
#pragma unroll
      for (int i = 0; i < 9; ++i) sm.P[i * G::NH + h] = r * wg<D, T>(i) + apre * n[i];
    } else {
      qe_half<D, T>(n, n + QF, kap);
#pragma unroll
      for (int i = 0; i < QF; ++i) sm.P[i * G::NH + h] = r * wf<D, T>(i) + apre * n[i];
    }
#pragma unroll
    for (int i = 0; i < QG; ++i) sm.P[(QF + i) * G::NH + h] = rg * wg<D, T>(i) + apre * n[QF + i];
    sm.U[h] = fr.ux;
    sm.V[h] = fr.uy;
    sm.RT[h] = fr.rt;
  }
  __syncthreads();
  // phases 1-5; with per-cell f-lattices a tile whose halo is all D2Q9 or
  // all D2Q16 runs a body specialised to that lattice
  if constexpr (D == 2 && MS == 1) {
    bool has16 = false, has9 = false;
    for (int k = tid; k < G::NH; k += kThreads) {
      has16 |= sm.Lat[k] == 4;
      has9 |= sm.Lat[k] == 3;
    }
    const int any16 = __syncthreads_or(has16), any9 = __syncthreads_or(has9);
    if (!any9) step_body<D, T, LIM, TF, 4>(a, sm, tid, x0, y0, kappa);
    else if (!any16) step_body<D, T, LIM, TF, 3>(a, sm, tid, x0, y0, kappa);
    else step_body<D, T, LIM, TF, 1>(a, sm, tid, x0, y0, kappa);
  } else if constexpr (D == 2 && MS == 3) {
    step_body<D, T, LIM, TF, 3>(a, sm, tid, x0, y0, kappa);
  } else {
    step_body<D, T, LIM, TF, 0, MS == 2>(a, sm, tid, x0, y0, kappa);
  }
}

// One 1D solve: block b advances tile b.
template <int D, typename T>
__global__ void __launch_bounds__(kThreads, (D == 2 && sizeof(T) == 4) ? 2 : 1) step_kernel(StepArgs a) {
  __shared__ Smem<D, T> sm;
  // the limiter is uniform over a launch: one straight-line body per kind
  // (in 1D both transforms are the same map)
  if (a.limiter == LIM_MINMOD) step_tile<D, T, LIM_MINMOD, TF_LAGRANGE>(a, blockIdx.x, sm);
  else step_tile<D, T, LIM_VANLEER, TF_LAGRANGE>(a, blockIdx.x, sm);
}

// Workgroups are dealt to the 8 XCDs round-robin (block b to XCD b mod 8),
// and each XCD has its own L2.  Renumbering so that XCD x works through one
// contiguous run of tiles makes neighbouring tiles, which share halo cache
// lines, meet in the same L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, k = b / kXcd;
  const int q = nb / kXcd, r = nb % kXcd;
  return x * q + min(x, r) + k;
}

// A ragged batch of independent solves in one launch: block b advances tile
// b - tile_begin of the entry whose tile range holds b.  Each entry carries
// the arguments of both step parities; step `parity` uses args[parity].
template <int D, typename T, int TF, int MS>
__global__ void __launch_bounds__(kThreads, (D == 2 && sizeof(T) == 4) ? 2 : 1)
    step_batch_kernel(const BatchEntry* tab, int n, int parity) {
  __shared__ Smem<D, T> sm;
  int lo = 0, hi = n - 1;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  while (lo < hi) {  // last entry with tile_begin <= b
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].tile_begin <= b) lo = mid; else hi = mid - 1;
  }
  // copied before the first store, so the uniform loads stay scalar
  const StepArgs a = tab[lo].args[parity];
  const int tile = b - tab[lo].tile_begin;
  // one kernel per transform and f-lattice mode (each keeps its own
  // register allocation); blocks of solves of another kind leave at once
  if (a.transform != TF) return;
  if constexpr (MS == 1 || MS == 3) {
    // a multiscale step whose f-lattice maps before and after it are all
    // D2Q9 (no cell stored on or moving to D2Q16) runs in the D2Q9 kernel
    const bool all9 = a.ms == 1 && a.q16_in && *a.q16_in == 0 && *a.q16_out == 0;
    if (MS == 1 ? (a.ms != 1 || all9) : (a.ms != 3 && !all9)) return;
  } else {
    if (a.ms != MS) return;
  }
  // the limiter is uniform over a solve: one straight-line body per kind
  if (a.limiter == LIM_MINMOD) step_tile<D, T, LIM_MINMOD, TF, MS>(a, tile, sm);
  else step_tile<D, T, LIM_VANLEER, TF, MS>(a, tile, sm);
}

// --------------------------------------------------------------------------
// Multiscale switch (Sec. IV C): D2Q16 where the velocity and temperature
// gradients are steep, D2Q9 elsewhere.  Indicator per cell, from central
// differences of the frames (ghosts by the boundary rules, an inflow ghost
// has the inflow state's frame):
//   theta = dx (|grad u| / sqrt(gamma T) + |grad T| / T),
// then D2Q16 within two cells (Chebyshev distance) of a cell with
// theta >= threshold; off the grid a periodic axis wraps and the other
// sides take the nearest interior cell.
// --------------------------------------------------------------------------
__device__ __forceinline__ Frame frame_at(const StepArgs& a, const long long* U, int gx, int gy) {
  int side = -1;
  const int sx = resolve(gx, a.nx, a.bc[0], a.bc[1], &side, 0);
  int sy = gy;
  if (side < 0) sy = resolve(gy, a.ny, a.bc[2], a.bc[3], &side, 2);
  long long u[4];
  if (side >= 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = a.inflow[4 * side + q];
  } else {
    const size_t cell = size_t(sx) + size_t(a.nx) * size_t(sy);
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = U[q * a.cells + cell];
  }
  return gauge(u, a);
}

__global__ void switch_theta_kernel(StepArgs a, const long long* U, double gamma, double* theta,
                                    int* q16_out) {
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  // clears the "some cell on D2Q16" word the lattice kernel sets next
  if (k == 0) *q16_out = 0;
  if (k >= a.cells) return;
  const int x = int(k % size_t(a.nx)), y = int(k / size_t(a.nx));
  const Frame xp = frame_at(a, U, x + 1, y), xm = frame_at(a, U, x - 1, y);
  const Frame yp = frame_at(a, U, x, y + 1), ym = frame_at(a, U, x, y - 1);
  const Frame c = frame_at(a, U, x, y);
  const double uxx = 0.5 * (xp.ux - xm.ux), uyx = 0.5 * (xp.uy - xm.uy);
  const double uxy = 0.5 * (yp.ux - ym.ux), uyy = 0.5 * (yp.uy - ym.uy);
  const double Tx = 0.5 * (xp.T - xm.T), Ty = 0.5 * (yp.T - ym.T);
  const double gu = sqrt(uxx * uxx + uyx * uyx + uxy * uxy + uyy * uyy);
  const double gT = sqrt(Tx * Tx + Ty * Ty);
  theta[k] = gu / sqrt(gamma * c.T) + gT / c.T;
}

__global__ void switch_lattice_kernel(StepArgs a, const double* theta, double threshold,
                                      unsigned char* lat, int* q16_out) {
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool in = k < a.cells;
  const int x = in ? int(k % size_t(a.nx)) : 0, y = in ? int(k / size_t(a.nx)) : 0;
  bool hi = false;
  for (int j = in ? -2 : 3; j <= 2; ++j) {
    for (int i = -2; i <= 2; ++i) {
      // the ghost rule of the populations: x first; past an inflow side
      // the nearest interior cell, without wrapping y
      int side = -1;
      const int sx = resolve(x + i, a.nx, a.bc[0], a.bc[1], &side, 0);
      int sy = y + j < 0 ? 0 : (y + j >= a.ny ? a.ny - 1 : y + j);
      if (side < 0) sy = resolve(y + j, a.ny, a.bc[2], a.bc[3], &side, 2);
      hi |= theta[size_t(sx) + size_t(a.nx) * size_t(sy)] >= threshold;
    }
  }
  if (in) lat[k] = hi ? 4 : 3;
  // "some cell on D2Q16": one vote per block, and no atomic once it is set
  // (a word every wave raised would serialise thousands of atomics)
  const int any = __syncthreads_or(hi);
  if (threadIdx.x == 0 && any && *static_cast<volatile int*>(q16_out) == 0) atomicOr(q16_out, 1);
}

// --------------------------------------------------------------------------
// Wall ghosts (Sec. IV D).  Ghost layer k of a wall mirrors the k-th cell in
// from the wall: same density, velocity and temperature reflected about the
// wall's values.  Its populations are the comoving equilibrium plus the
// first-order Chapman-Enskog non-equilibrium, expanded on Hermite
// polynomials of c = (v - u_G) / sqrt(T_G) (order 3 on D2Q16 for f, order
// 2 on D2Q9 for g), from the gradients of the mirror-extended field by
// central differences (along the wall, past the grid, a periodic axis wraps
// and the others take the nearest cell).  With p = rho T, S = grad u +
// (grad u)^T, d = div u and c_e = C_v - 1:
//   f: second moments -tau1 p (S - (d / C_v) I), third central moments
//      -tau2 p [dT/dx_a delta_bc]_cyc;
//   g: zeroth moment tau1 c_e p d / C_v, first central -tau2 c_e p grad T,
//      second central -tau1 c_e p T (S - (2 d / C_v) I),
// so the non-equilibrium carries no mass, momentum or energy.  Stored as
// n = (1 + dt / (2 tau1)) f^neq with the ghost's ledger moments.
// --------------------------------------------------------------------------
struct Prim {
  double rho, ux, uy, T;
};

// Extended field next to wall `side`: m >= 0 the interior cell m rows in,
// m < 0 ghost layer -m.
__device__ __forceinline__ Prim wall_field(const StepArgs& a, int side, int m, int t) {
  const int nt = side < 2 ? a.ny : a.nx;
  const int bt = side < 2 ? a.bc[2] : a.bc[0];
  if (t < 0 || t >= nt) t = bt == BC_PERIODIC ? ((t % nt) + nt) % nt : (t < 0 ? 0 : nt - 1);
  const int mm = m >= 0 ? m : -m - 1;
  const int x = side == 0 ? mm : side == 1 ? a.nx - 1 - mm : t;
  const int y = side == 2 ? mm : side == 3 ? a.ny - 1 - mm : t;
  const size_t cell = size_t(x) + size_t(a.nx) * size_t(y);
  long long u[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) u[q] = a.U_in[q * a.cells + cell];
  // the ghosts follow the cells after the first body-force half step (an
  // overflow of these increments is flagged where the step kernel applies
  // the same ones to the cell)
  int bad = 0;
  if (a.force) force_ledger(a, u, &bad);
  const Frame f = gauge(u, a);
  Prim p{f.rho, f.ux, f.uy, f.T};
  if (m < 0) {
    p.ux = 2.0 * a.wall[side][0] - p.ux;
    p.uy = 2.0 * a.wall[side][1] - p.uy;
    p.T = 2.0 * a.wall[side][2] - p.T;
  }
  return p;
}

// Writes the ghost entries to wu (4 ledger planes) and wn (NP population
// planes); the step kernel reads the same buffer through a.wU / a.wN.
template <typename T>
__global__ void wall_ghost_kernel(StepArgs a, long long* wu, T* wn) {
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= a.wall_n) return;
  const int L = a.wall_len;
  const int side = int(e / size_t(2 * L)), k = int((e / size_t(L)) % 2) + 1, t = int(e % size_t(L));
  if (a.bc[side] != BC_WALL || t >= (side < 2 ? a.ny : a.nx)) return;
  const Prim g = wall_field(a, side, -k, t);
  const Prim in = wall_field(a, side, -k + 1, t), out = wall_field(a, side, -k - 1, t);
  const Prim tp = wall_field(a, side, -k, t + 1), tm = wall_field(a, side, -k, t - 1);
  // derivatives along the inward normal and along the wall
  const double sn = (side == 0 || side == 2) ? a.idx2 : -a.idx2;
  const double nux = sn * (in.ux - out.ux), nuy = sn * (in.uy - out.uy), nT = sn * (in.T - out.T);
  const double tux = a.idx2 * (tp.ux - tm.ux), tuy = a.idx2 * (tp.uy - tm.uy), tT = a.idx2 * (tp.T - tm.T);
  const bool xw = side < 2;
  const double dxux = xw ? nux : tux, dxuy = xw ? nuy : tuy, dxT = xw ? nT : tT;
  const double dyux = xw ? tux : nux, dyuy = xw ? tuy : nuy, dyT = xw ? tT : nT;
  const double p = g.rho * g.T, icv = a.icv, ce = a.cv - 1.0;
  const double d = dxux + dyuy;
  const double sxx = 2.0 * dxux, syy = 2.0 * dyuy, sxy = dxuy + dyux;
  const double iT = 1.0 / g.T, irt = sqrt(iT), i32 = iT * irt;
  // f Hermite coefficients (a, b) = (x order, y order)
  const double v = -a.tau1 * p * iT;
  const double f20 = v * (sxx - d * icv), f02 = v * (syy - d * icv), f11 = v * sxy;
  const double w = -a.tau2 * p * i32;
  const double f30 = 3.0 * w * dxT, f21 = w * dyT, f12 = w * dxT, f03 = 3.0 * w * dyT;
  // g Hermite coefficients
  const double g00 = a.tau1 * ce * p * d * icv;
  const double g10 = -a.tau2 * ce * p * dxT * irt, g01 = -a.tau2 * ce * p * dyT * irt;
  const double u2 = -a.tau1 * ce * p;
  const double g20 = u2 * (sxx - 2.0 * d * icv) - g00, g02 = u2 * (syy - 2.0 * d * icv) - g00;
  const double g11 = u2 * sxy;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const double cx = node<4, double>(i & 3), cy = node<4, double>(i >> 2);
    const double hx2 = cx * cx - 1.0, hy2 = cy * cy - 1.0;
    const double hx3 = cx * (cx * cx - 3.0), hy3 = cy * (cy * cy - 3.0);
    const double s2 = 0.5 * (f20 * hx2 + f02 * hy2) + f11 * cx * cy;
    const double s3 = (f30 * hx3 + f03 * hy3) * (1.0 / 6.0) + 0.5 * (f21 * hx2 * cy + f12 * cx * hy2);
    wn[i * a.wall_n + e] = T(a.kf * weight<4, double>(i & 3) * weight<4, double>(i >> 2) * (s2 + s3));
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double cx = node<3, double>(i % 3), cy = node<3, double>(i / 3);
    const double s = g00 + g10 * cx + g01 * cy + 0.5 * (g20 * (cx * cx - 1.0) + g02 * (cy * cy - 1.0)) +
                     g11 * cx * cy;
    wn[(16 + i) * a.wall_n + e] = T(a.kf * weight<3, double>(i % 3) * weight<3, double>(i / 3) * s);
  }
  int bad = 0;
  wu[e] = to_fixed(g.rho, a.scale, &bad);
  wu[a.wall_n + e] = to_fixed(g.rho * g.ux, a.scale, &bad);
  wu[2 * a.wall_n + e] = to_fixed(g.rho * g.uy, a.scale, &bad);
  wu[3 * a.wall_n + e] =
      to_fixed(a.cv * p + 0.5 * g.rho * (g.ux * g.ux + g.uy * g.uy), a.scale, &bad);
  raise_flag(a.flag, !(g.rho > 0.0) || !(g.T > 0.0), 1);
  raise_flag(a.flag, bad != 0, 2);
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

// --------------------------------------------------------------------------
// D2Q25 f-lattice with the fourth-order Grad projection (Sec. III B, the
// full invariant moment system; g stays on D2Q9 with Grad's order 2).  Three
// plain kernels per step, with the face data in HBM: a cell pass (first QE
// half step, phi-bar-plus, frames), a face pass per axis (face frame and
// corrector passes, the stencil in the face frame, MUSCL, face moments, face
// equilibrium, inversion of eq. FluxTransf, the ledger flux), and a cell
// update (fluxes into the cell frame, DUGKS update, new frame from the
// ledger, re-gauge, second QE half step).  Population planes: f 0..24
// (i = i_x + 5 i_y), g 25..33.
// --------------------------------------------------------------------------
constexpr int kQ25 = 25, kNP25 = 34;

template <typename T>
__device__ __forceinline__ T w25(int i) {
  return weight<5, T>(i % 5) * weight<5, T>(i / 5);
}
template <typename T>
__device__ __forceinline__ T w9(int i) {
  return weight<3, T>(i % 3) * weight<3, T>(i / 3);
}

// QE half step on D2Q25 (same form as on D2Q16: the third Hermite moments
// relax, eq. quasi_f) and on the D2Q9 g (first moment).
template <typename T>
__device__ __forceinline__ void qe_half25(T* n, T* m, T kappa) {
  T axxx = T(0), axxy = T(0), axyy = T(0), ayyy = T(0);
#pragma unroll
  for (int i = 0; i < kQ25; ++i) {
    const T cx = node<5, T>(i % 5), cy = node<5, T>(i / 5);
    axxx += n[i] * (cx * cx * cx - T(3) * cx);
    axxy += n[i] * (cx * cx * cy - cy);
    axyy += n[i] * (cx * cy * cy - cx);
    ayyy += n[i] * (cy * cy * cy - T(3) * cy);
  }
  T agx = T(0), agy = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    agx += m[i] * node<3, T>(i % 3);
    agy += m[i] * node<3, T>(i / 3);
  }
  const T k6 = kappa * T(1.0 / 6.0);
#pragma unroll
  for (int i = 0; i < kQ25; ++i) {
    const T cx = node<5, T>(i % 5), cy = node<5, T>(i / 5);
    const T c = axxx * (cx * cx * cx - T(3) * cx) + T(3) * axxy * (cx * cx * cy - cy) +
                T(3) * axyy * (cx * cy * cy - cx) + ayyy * (cy * cy * cy - T(3) * cy);
    n[i] += k6 * w25<T>(i) * c;
  }
#pragma unroll
  for (int i = 0; i < 9; ++i)
    m[i] += kappa * w9<T>(i) * (agx * node<3, T>(i % 3) + agy * node<3, T>(i / 3));
}

// f (25) and g (9) between frames by Grad's projection (orders 4 and 2).
template <typename T>
__device__ __forceinline__ void xform25(double rt_src, double ux_src, double uy_src, double irt_dst,
                                        double ux_dst, double uy_dst, const T* in, T* out) {
  const T s = T(rt_src * irt_dst);
  const T dx = T((ux_src - ux_dst) * irt_dst), dy = T((uy_src - uy_dst) * irt_dst);
  grad_map<5, 5, 4, T, 0>(s, dx, dy, in, out);
  grad_map<3, 3, 2, T, 0>(s, dx, dy, in + kQ25, out + kQ25);
}

struct Q25Bufs {
  void* P;           // kNP25 planes of phi-bar-plus per grid cell
  double* fr;        // 3 planes: u_x, u_y, T of each grid cell
  void* fp[2];       // face populations phi^{lambda_F}: [axis] kNP25 planes per face
  double* ff[2];     // face frames: [axis] 3 planes
  long long* psi[2]; // face ledger fluxes: [axis] 4 planes
};

// 256-thread blocks: without the bound the compiler keeps each thread to 128
// VGPRs (room for 1024-thread blocks) and the face and cell passes, which
// hold eight projected stencil cells or four face sets, spill to scratch.
template <typename T>
__global__ void __launch_bounds__(256) q25_prep_kernel(StepArgs a, Q25Bufs b) {
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= a.cells) return;
  long long U[4];
  T n[kNP25];
  const T* nin = static_cast<const T*>(a.n_in);
#pragma unroll
  for (int q = 0; q < 4; ++q) U[q] = a.U_in[q * a.cells + k];
#pragma unroll
  for (int i = 0; i < kNP25; ++i) n[i] = nin[i * a.cells + k];
  const Frame f = gauge(U, a);
  qe_half25<T>(n, n + kQ25, T(a.kappa));
  const T r = T(f.rho), rg = T(a.geq * f.T * f.rho), ap = T(a.a_pre);
  T* P = static_cast<T*>(b.P);
#pragma unroll
  for (int i = 0; i < kQ25; ++i) P[i * a.cells + k] = r * w25<T>(i) + ap * n[i];
#pragma unroll
  for (int i = 0; i < 9; ++i) P[(kQ25 + i) * a.cells + k] = rg * w9<T>(i) + ap * n[kQ25 + i];
  b.fr[k] = f.ux;
  b.fr[a.cells + k] = f.uy;
  b.fr[2 * a.cells + k] = f.T;
}

// phi-bar-plus planes [P0, P0 + NQ) and frame of grid cell (gx, gy), which
// may be a ghost: the boundary rules of the step kernels (x first; periodic
// wraps, zero gradient takes the nearest cell, inflow is the comoving
// equilibrium of the fixed state).
template <typename T, int P0, int NQ>
__device__ __forceinline__ void q25_slot(const StepArgs& a, const Q25Bufs& b, int gx, int gy, T* P,
                                         double* fr) {
  int side = -1;
  const int sx = resolve(gx, a.nx, a.bc[0], a.bc[1], &side, 0);
  int sy = gy;
  if (side < 0) sy = resolve(gy, a.ny, a.bc[2], a.bc[3], &side, 2);
  if (side >= 0) {
    long long U[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) U[q] = a.inflow[4 * side + q];
    const Frame f = gauge(U, a);
    const T r = P0 == 0 ? T(f.rho) : T(a.geq * f.T * f.rho);
#pragma unroll
    for (int i = 0; i < NQ; ++i) P[i] = r * (P0 == 0 ? w25<T>(i) : w9<T>(i));
    fr[0] = f.ux;
    fr[1] = f.uy;
    fr[2] = f.T;
    return;
  }
  const size_t c = size_t(sx) + size_t(a.nx) * size_t(sy);
  const T* Pin = static_cast<const T*>(b.P);
#pragma unroll
  for (int i = 0; i < NQ; ++i) P[i] = Pin[(P0 + i) * a.cells + c];
  fr[0] = b.fr[c];
  fr[1] = b.fr[a.cells + c];
  fr[2] = b.fr[2 * a.cells + c];
}

// The face reconstruction of one lattice: f (Q1 = 5, planes 0..24) or g
// (Q1 = 3, planes 25..33).  The eight stencil cells are projected into the
// face frame by Grad's expansion of order Q1 - 1 and kept in registers
// through the MUSCL step; doing the lattices one after the other halves the
// values held at once.
template <typename T, int LIM, int AXIS, int Q1, int P0>
__device__ __forceinline__ void q25_part(const StepArgs& a, const Q25Bufs& b, const int (&cxs)[8],
                                         const int (&cys)[8], double uF, double vF, double TF,
                                         T* bar) {
  constexpr int NQ = Q1 * Q1;
  const double rtF = sqrt(TF), irtF = 1.0 / rtF;
  T P[8][NQ];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    T src[NQ];
    double fr[3];
    q25_slot<T, P0, NQ>(a, b, cxs[k], cys[k], src, fr);
    const T s = T(sqrt(fr[2]) * irtF);
    const T dx = T((fr[0] - uF) * irtF), dy = T((fr[1] - vF) * irtF);
    grad_map<Q1, Q1, Q1 - 1, T, 0>(s, dx, dy, src, P[k]);
    // one stencil cell at a time: its projection finished and pinned before
    // the next cell's loads (the compiler would otherwise hoist all loads
    // and hold them with the results)
#pragma unroll
    for (int i = 0; i < NQ; ++i) asm volatile("" : "+v"(P[k][i]));
    __builtin_amdgcn_sched_barrier(0);
  }
  const T rt = T(rtF), band = T(kTieBand * rtF), lam = T(a.lam);
#pragma unroll
  for (int p = 0; p < NQ; ++p) {
    const T vx = rt * node<Q1, T>(p % Q1) + T(uF), vy = rt * node<Q1, T>(p / Q1) + T(vF);
    const T vn = AXIS == 0 ? vx : vy, vt = AXIS == 0 ? vy : vx;
    const T dtv = T(-0.5) * lam * vt;
    const T recL = P[0][p] + (T(0.5) - T(0.5) * lam * vn) * limit<LIM, T>(P[0][p] - P[2][p], P[1][p] - P[0][p]) +
                   dtv * limit<LIM, T>(P[0][p] - P[5][p], P[4][p] - P[0][p]);
    const T recR = P[1][p] + (T(-0.5) - T(0.5) * lam * vn) * limit<LIM, T>(P[1][p] - P[0][p], P[3][p] - P[1][p]) +
                   dtv * limit<LIM, T>(P[1][p] - P[7][p], P[6][p] - P[1][p]);
    bar[P0 + p] = vn > band ? recL : (vn < -band ? recR : T(0.5) * (recL + recR));
  }
}

// One face along AXIS between cells L = (lx, ly) and R = L + e_AXIS.
template <typename T, int LIM, int AXIS>
__device__ __forceinline__ void q25_face(const StepArgs& a, const Q25Bufs& b, int lx, int ly,
                                         size_t fidx, size_t nface) {
  // stencil slots: 0 L, 1 R, 2 L-e_a, 3 R+e_a, 4 L+e_t, 5 L-e_t, 6 R+e_t, 7 R-e_t
  const int ex = AXIS == 0 ? 1 : 0, ey = 1 - ex;
  const int rx = lx + ex, ry = ly + ey;
  const int tx = ey, ty = ex;  // transverse unit vector
  const int cxs[8] = {lx, rx, lx - ex, rx + ex, lx + tx, lx - tx, rx + tx, rx - tx};
  const int cys[8] = {ly, ry, ly - ey, ry + ey, ly + ty, ly - ty, ry + ty, ry - ty};
  double frL[3], frR[3];
  {
    T tmp[9];
    q25_slot<T, kQ25, 9>(a, b, cxs[0], cys[0], tmp, frL);
    q25_slot<T, kQ25, 9>(a, b, cxs[1], cys[1], tmp, frR);
  }
  double uF = 0.5 * (frL[0] + frR[0]), vF = 0.5 * (frL[1] + frR[1]);
  double TF = 0.5 * (frL[2] + frR[2]);
  T bar[kNP25];
  double rho_b = 0.0, ub = 0.0, vb = 0.0, Tb = 0.0;
  for (int pass = 0; pass <= a.n_corr; ++pass) {
    const double rtF = sqrt(TF);
    q25_part<T, LIM, AXIS, 5, 0>(a, b, cxs, cys, uF, vF, TF, bar);
    q25_part<T, LIM, AXIS, 3, kQ25>(a, b, cxs, cys, uF, vF, TF, bar);
    // face moments in FP64 (eq. ConservationLaws in lambda_F)
    double m0 = 0.0, mx = 0.0, my = 0.0, e = 0.0;
#pragma unroll
    for (int p = 0; p < kQ25; ++p) {
      const double vx = rtF * node<5, double>(p % 5) + uF, vy = rtF * node<5, double>(p / 5) + vF;
      const double fb = double(bar[p]);
      m0 += fb;
      mx += vx * fb;
      my += vy * fb;
      e += 0.5 * (vx * vx + vy * vy) * fb;
    }
#pragma unroll
    for (int p = 0; p < 9; ++p) e += double(bar[kQ25 + p]);
    rho_b = m0;
    ub = mx / m0;
    vb = my / m0;
    Tb = (e - 0.5 * m0 * (ub * ub + vb * vb)) / (a.cv * m0);
    if (pass < a.n_corr) {
      uF = ub;
      vF = vb;
      TF = Tb;
    }
  }
  raise_flag(a.flag, !(rho_b > 0.0) || !(Tb > 0.0), 1);
  // face equilibrium rho_b G W (eq. NonComovingEq): the comoving equilibrium
  // of (u_b, T_b) projected into lambda_F
  T eqc[kNP25], eq[kNP25];
  const T rb = T(rho_b), rgb = T(a.geq * Tb * rho_b);
#pragma unroll
  for (int p = 0; p < kQ25; ++p) eqc[p] = rb * w25<T>(p);
#pragma unroll
  for (int p = 0; p < 9; ++p) eqc[kQ25 + p] = rgb * w9<T>(p);
  const double irtF = 1.0 / sqrt(TF);
  xform25<T>(sqrt(Tb), ub, vb, irtF, uF, vF, eqc, eq);
  // inversion of eq. FluxTransf and the conserved flux
  const T c1 = T(a.c_face1), c2 = T(a.c_face2);
  T* fp = static_cast<T*>(b.fp[AXIS]);
  const double rtF = sqrt(TF);
  double F0 = 0.0, Fx = 0.0, Fy = 0.0, FE = 0.0;
#pragma unroll
  for (int p = 0; p < kNP25; ++p) {
    const T phi = c1 * bar[p] + c2 * eq[p];
    fp[p * nface + fidx] = phi;
    const double ph = double(phi);
    if (p < kQ25) {
      const double vx = rtF * node<5, double>(p % 5) + uF, vy = rtF * node<5, double>(p / 5) + vF;
      const double vn = AXIS == 0 ? vx : vy;
      F0 += vn * ph;
      Fx += vn * vx * ph;
      Fy += vn * vy * ph;
      FE += vn * 0.5 * (vx * vx + vy * vy) * ph;
    } else {
      const int q = p - kQ25;
      const double vn = AXIS == 0 ? rtF * node<3, double>(q % 3) + uF : rtF * node<3, double>(q / 3) + vF;
      FE += vn * ph;
    }
  }
  b.ff[AXIS][fidx] = uF;
  b.ff[AXIS][nface + fidx] = vF;
  b.ff[AXIS][2 * nface + fidx] = TF;
  int bad = 0;
  long long* psi = b.psi[AXIS];
  psi[fidx] = to_fixed(a.lam * F0, a.scale, &bad);
  psi[nface + fidx] = to_fixed(a.lam * Fx, a.scale, &bad);
  psi[2 * nface + fidx] = to_fixed(a.lam * Fy, a.scale, &bad);
  psi[3 * nface + fidx] = to_fixed(a.lam * FE, a.scale, &bad);
  raise_flag(a.flag, bad != 0, 2);
}

template <typename T, int AXIS>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) q25_face_kernel(StepArgs a, Q25Bufs b) {
  // x-faces: (nx + 1) per row; y-faces: nx per row, ny + 1 rows
  const size_t nface = AXIS == 0 ? size_t(a.nx + 1) * a.ny : size_t(a.nx) * (a.ny + 1);
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nface) return;
  const int w = AXIS == 0 ? a.nx + 1 : a.nx;
  const int i = int(k % size_t(w)), j = int(k / size_t(w));
  // x-face i of row j lies between cells (i-1, j) and (i, j); y-face j of
  // column i between (i, j-1) and (i, j)
  const int lx = AXIS == 0 ? i - 1 : i, ly = AXIS == 0 ? j : j - 1;
  if (a.limiter == LIM_MINMOD) q25_face<T, LIM_MINMOD, AXIS>(a, b, lx, ly, k, nface);
  else q25_face<T, LIM_VANLEER, AXIS>(a, b, lx, ly, k, nface);
}

template <typename T>
__global__ void __launch_bounds__(256) q25_cell_kernel(StepArgs a, Q25Bufs b) {
  const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= a.cells) return;
  const int x = int(k % size_t(a.nx)), y = int(k / size_t(a.nx));
  long long U[4];
  T n[kNP25];
  const T* nin = static_cast<const T*>(a.n_in);
#pragma unroll
  for (int q = 0; q < 4; ++q) U[q] = a.U_in[q * a.cells + k];
#pragma unroll
  for (int i = 0; i < kNP25; ++i) n[i] = nin[i * a.cells + k];
  const Frame f0 = gauge(U, a);
  qe_half25<T>(n, n + kQ25, T(a.kappa));
  // faces: west, east (x-faces), south, north (y-faces), sign -1 / +1
  const size_t nfx = size_t(a.nx + 1) * a.ny, nfy = size_t(a.nx) * (a.ny + 1);
  const size_t fi[4] = {size_t(x) + size_t(a.nx + 1) * y, size_t(x + 1) + size_t(a.nx + 1) * y,
                        size_t(x) + size_t(a.nx) * y, size_t(x) + size_t(a.nx) * (y + 1)};
  T acc[kNP25];
#pragma unroll
  for (int p = 0; p < kNP25; ++p) acc[p] = T(0);
  long long dU[4] = {0, 0, 0, 0};
  const T rt0 = T(f0.rt);
#pragma unroll
  for (int fc = 0; fc < 4; ++fc) {
    const int ax = fc / 2;
    const size_t nf = ax == 0 ? nfx : nfy, id = fi[fc];
    const T* fp = static_cast<const T*>(b.fp[ax]);
    T in[kNP25], out[kNP25];
#pragma unroll
    for (int p = 0; p < kNP25; ++p) in[p] = fp[p * nf + id];
    const double uF = b.ff[ax][id], vF = b.ff[ax][nf + id], TF = b.ff[ax][2 * nf + id];
    xform25<T>(sqrt(TF), uF, vF, f0.irt, f0.ux, f0.uy, in, out);
    const T sg = fc % 2 == 0 ? T(-1) : T(1);
    const T u0 = T(ax == 0 ? f0.ux : f0.uy);
#pragma unroll
    for (int p = 0; p < kNP25; ++p) {
      const T c = p < kQ25 ? (ax == 0 ? node<5, T>(p % 5) : node<5, T>(p / 5))
                           : (ax == 0 ? node<3, T>((p - kQ25) % 3) : node<3, T>((p - kQ25) / 3));
      acc[p] += sg * (rt0 * c + u0) * out[p];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) dU[q] += fc % 2 == 0 ? -b.psi[ax][q * nf + id] : b.psi[ax][q * nf + id];
  }
  // DUGKS update (eq. FinalUpdateDUGKS) in the cell frame
  const T bu = T(a.b_upd), lam = T(a.lam);
  const T r = T(f0.rho), rg = T(a.geq * f0.T * f0.rho);
  T ft[kNP25];
#pragma unroll
  for (int p = 0; p < kQ25; ++p) ft[p] = r * w25<T>(p) + bu * n[p] - lam * acc[p];
#pragma unroll
  for (int p = 0; p < 9; ++p) ft[kQ25 + p] = rg * w9<T>(p) + bu * n[kQ25 + p] - lam * acc[kQ25 + p];
  long long U2[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) U2[q] = U[q] - dU[q];
  const Frame nf = gauge(U2, a);
  T n2[kNP25];
  xform25<T>(f0.rt, f0.ux, f0.uy, nf.irt, nf.ux, nf.uy, ft, n2);
  const T r2 = T(nf.rho), rg2 = T(a.geq * nf.T * nf.rho);
#pragma unroll
  for (int p = 0; p < kQ25; ++p) n2[p] -= r2 * w25<T>(p);
#pragma unroll
  for (int p = 0; p < 9; ++p) n2[kQ25 + p] -= rg2 * w9<T>(p);
  qe_half25<T>(n2, n2 + kQ25, T(a.kappa));
  raise_flag(a.flag, !(nf.rho > 0.0) || !(nf.T > 0.0) || !isfinite(double(n2[0])), 1);
  bool over = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) over |= (U2[q] > (1LL << 62)) || (U2[q] < -(1LL << 62));
  raise_flag(a.flag, over, 2);
  T* nout = static_cast<T*>(a.n_out);
#pragma unroll
  for (int p = 0; p < kNP25; ++p) nout[p * a.cells + k] = n2[p];
#pragma unroll
  for (int q = 0; q < 4; ++q) a.U_out[q * a.cells + k] = U2[q];
}

}  // namespace

hipError_t launch_q25_step(bool fp64, const StepArgs& a, void* P, double* fr, void* fpx, void* fpy,
                           double* ffx, double* ffy, long long* psx, long long* psy,
                           hipStream_t st) {
  Q25Bufs b{P, fr, {fpx, fpy}, {ffx, ffy}, {psx, psy}};
  const dim3 block(256);
  const dim3 gc(unsigned((a.cells + 255) / 256));
  const dim3 gx(unsigned((size_t(a.nx + 1) * a.ny + 255) / 256));
  const dim3 gy(unsigned((size_t(a.nx) * (a.ny + 1) + 255) / 256));
  if (fp64) {
    hipLaunchKernelGGL(q25_prep_kernel<double>, gc, block, 0, st, a, b);
    hipLaunchKernelGGL((q25_face_kernel<double, 0>), gx, block, 0, st, a, b);
    hipLaunchKernelGGL((q25_face_kernel<double, 1>), gy, block, 0, st, a, b);
    hipLaunchKernelGGL(q25_cell_kernel<double>, gc, block, 0, st, a, b);
  } else {
    hipLaunchKernelGGL(q25_prep_kernel<float>, gc, block, 0, st, a, b);
    hipLaunchKernelGGL((q25_face_kernel<float, 0>), gx, block, 0, st, a, b);
    hipLaunchKernelGGL((q25_face_kernel<float, 1>), gy, block, 0, st, a, b);
    hipLaunchKernelGGL(q25_cell_kernel<float>, gc, block, 0, st, a, b);
  }
  return hipGetLastError();
}

hipError_t launch_step_1d(bool fp64, const StepArgs& a, hipStream_t st) {
  const dim3 grid(a.tiles_x * a.tiles_y), block(kThreads);
  if (fp64) hipLaunchKernelGGL((step_kernel<1, double>), grid, block, 0, st, a);
  else hipLaunchKernelGGL((step_kernel<1, float>), grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_step_batch(bool fp64, unsigned kind_mask, const BatchEntry* tab, int n,
                             int total_tiles, int parity, hipStream_t st) {
  const dim3 grid(total_tiles), block(kThreads);
  if (kind_mask & (1u << kind_of(TF_LAGRANGE, 0))) {
    if (fp64) hipLaunchKernelGGL((step_batch_kernel<2, double, TF_LAGRANGE, 0>), grid, block, 0, st, tab, n, parity);
    else hipLaunchKernelGGL((step_batch_kernel<2, float, TF_LAGRANGE, 0>), grid, block, 0, st, tab, n, parity);
  }
  if (kind_mask & (1u << kind_of(TF_GRAD, 0))) {
    if (fp64) hipLaunchKernelGGL((step_batch_kernel<2, double, TF_GRAD, 0>), grid, block, 0, st, tab, n, parity);
    else hipLaunchKernelGGL((step_batch_kernel<2, float, TF_GRAD, 0>), grid, block, 0, st, tab, n, parity);
  }
  if (kind_mask & (1u << kind_of(TF_LAGRANGE, 2))) {
    if (fp64) hipLaunchKernelGGL((step_batch_kernel<2, double, TF_LAGRANGE, 2>), grid, block, 0, st, tab, n, parity);
    else hipLaunchKernelGGL((step_batch_kernel<2, float, TF_LAGRANGE, 2>), grid, block, 0, st, tab, n, parity);
  }
  if (kind_mask & (1u << kind_of(TF_GRAD, 2))) {
    if (fp64) hipLaunchKernelGGL((step_batch_kernel<2, double, TF_GRAD, 2>), grid, block, 0, st, tab, n, parity);
    else hipLaunchKernelGGL((step_batch_kernel<2, float, TF_GRAD, 2>), grid, block, 0, st, tab, n, parity);
  }
  if (kind_mask & (1u << kind_of(TF_GRAD, 3))) {
    if (fp64) hipLaunchKernelGGL((step_batch_kernel<2, double, TF_GRAD, 3>), grid, block, 0, st, tab, n, parity);
    else hipLaunchKernelGGL((step_batch_kernel<2, float, TF_GRAD, 3>), grid, block, 0, st, tab, n, parity);
  }
  if (kind_mask & (1u << kind_of(TF_GRAD, 1))) {
    if (fp64) hipLaunchKernelGGL((step_batch_kernel<2, double, TF_GRAD, 1>), grid, block, 0, st, tab, n, parity);
    else hipLaunchKernelGGL((step_batch_kernel<2, float, TF_GRAD, 1>), grid, block, 0, st, tab, n, parity);
  }
  return hipGetLastError();
}

hipError_t launch_wall_ghosts(bool fp64, const StepArgs& a, long long* wU, void* wN,
                              hipStream_t st) {
  const dim3 grid(unsigned((a.wall_n + 255) / 256)), block(256);
  if (fp64) hipLaunchKernelGGL(wall_ghost_kernel<double>, grid, block, 0, st, a, wU, static_cast<double*>(wN));
  else hipLaunchKernelGGL(wall_ghost_kernel<float>, grid, block, 0, st, a, wU, static_cast<float*>(wN));
  return hipGetLastError();
}

hipError_t launch_switch(const StepArgs& a, const long long* U, double threshold, double gamma,
                         int* q16_out,
                         double* theta, unsigned char* lat_out, hipStream_t st) {
  const dim3 grid(unsigned((a.cells + 255) / 256)), block(256);
  hipLaunchKernelGGL(switch_theta_kernel, grid, block, 0, st, a, U, gamma, theta, q16_out);
  hipLaunchKernelGGL(switch_lattice_kernel, grid, block, 0, st, a, theta, threshold, lat_out, q16_out);
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
