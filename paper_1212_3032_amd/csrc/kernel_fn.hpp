// Laplace-domain elastodynamic fundamental solutions and element integrals.
//
// Sec. 2.1 defines U_ij = (phi delta_ij - psi r_i r_j) / (4 pi mu) and
// T_ij = G_ikj n_k(y).  At the damped frequency s = sigma + i omega of the
// exponential window (Sec. 3.1) the exp(i k r) factors become exp(-s r / c).
// With z = s r / c_s, gamma = c_s / c_p and z_p = gamma z:
//   r phi  = e^{-z}(1 + 1/z + 1/z^2) - gamma^2 e^{-z_p}(1/z_p + 1/z_p^2)
//   r psi  = e^{-z}(1 + 3/z + 3/z^2) - gamma^2 e^{-z_p}(1 + 3/z_p + 3/z_p^2)
//   r^2 phi' = -r phi - [e^{-z}(z + 1 + 2/z + 2/z^2) - gamma^2 e^{-z_p}(1 + 2/z_p + 2/z_p^2)]
//   r^2 psi' = -r psi - [e^{-z}(z + 3 + 6/z + 6/z^2) - gamma^2 e^{-z_p}(z_p + 3 + 6/z_p + 6/z_p^2)]
// (the P-wave terms carry gamma^2, without which U has no static limit; r_i
// is the unit vector from the load point x to the field point y).  Below
// |z| = 1/2 these forms cancel catastrophically and the Taylor series in z
// (coefficients filled on the host into KParams) is evaluated instead.
// The traction kernel expands to
//   T_ij = [A (delta_ij dr/dn + n_i r_j) + B r_i r_j dr/dn + C r_i n_j] / (4 pi)
// with A = phi' - psi/r, B = 2 (2 psi/r - psi'),
//      C = (c_p/c_s)^2 (phi' - psi' - 2 psi/r) - 2 (phi' - psi' - psi/r).
#pragma once

#include "common.hpp"

namespace ewbem {

// r = |d| and ir = 1 / r from d2 = |d|^2 > 0: the hardware reciprocal square
// root (about single precision) refined by two Newton steps
// y <- y + y (1 - d2 y^2) / 2, each squaring the relative error, then r = d2 y;
// both to a few units in the last place, in fewer operations than a square
// root and a division.
__device__ __forceinline__ void dist_inv(double d2, double& r, double& ir) {
  double y = __builtin_amdgcn_rsq(d2);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d2, y * y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  ir = y;
  r = d2 * y;
}

struct Radial {
  cd rphi, rpsi, r2dphi, r2dpsi;
};

// r phi, r psi (and r^2 phi', r^2 psi' when DERIV) at distance r, with
// ir = 1 / r.  TAIL drops the static n = 2 terms, leaving the part that stays
// bounded as r -> 0.  1 / z = (c_s / s) / r takes a product, not a division.
template <bool TAIL, bool DERIV>
__device__ __forceinline__ Radial radial(double r, double ir, const KParams& P) {
  const cd z = P.s * (r * P.inv_cs);
  Radial o;
  if (norm2(z) < P.series_z2) {
    const double* __restrict__ c_phi = P.ser;
    const double* __restrict__ c_psi = P.ser + NSER;
    const double* __restrict__ c_dphi = P.ser + 2 * NSER;
    const double* __restrict__ c_dpsi = P.ser + 3 * NSER;
    cd a = mk(c_phi[NSER - 1]), b = mk(c_psi[NSER - 1]);
    cd c = mk(c_dphi[NSER - 1]), d = mk(c_dpsi[NSER - 1]);
    for (int m = NSER - 2; m >= 1; --m) {
      a = a * z + c_phi[m];
      b = b * z + c_psi[m];
      if (DERIV) {
        c = c * z + c_dphi[m];
        d = d * z + c_dpsi[m];
      }
    }
    a = a * z;
    b = b * z;
    if (DERIV) {
      c = c * z;
      d = d * z;
    }
    if (!TAIL) {
      a = a + c_phi[0];
      b = b + c_psi[0];
      if (DERIV) {
        c = c + c_dphi[0];
        d = d + c_dpsi[0];
      }
    }
    o.rphi = a;
    o.rpsi = b;
    o.r2dphi = c;
    o.r2dpsi = d;
    return o;
  }
  double sn, cs;
  const double e1 = exp(-z.x);
  sincos(z.y, &sn, &cs);
  const cd es = cd{e1 * cs, -e1 * sn};
  const double g = P.gamma, g2 = P.g2;
  const double e2 = exp(-g * z.x);
  sincos(g * z.y, &sn, &cs);
  const cd ep = cd{e2 * cs, -e2 * sn};
  const cd iz = P.cs_over_s * ir;
  const cd iz2 = iz * iz;
  const cd gi = iz * g;  // gamma^2 / z_p
  const cd rphi = es * (1.0 + iz + iz2) - ep * (gi + iz2);
  const cd rpsi = es * (1.0 + 3.0 * iz + 3.0 * iz2) - ep * (g2 + 3.0 * gi + 3.0 * iz2);
  o.rphi = rphi;
  o.rpsi = rpsi;
  if (DERIV) {
    o.r2dphi = -rphi - (es * (z + 1.0 + 2.0 * iz + 2.0 * iz2) - ep * (g2 + 2.0 * gi + 2.0 * iz2));
    o.r2dpsi = -rpsi - (es * (z + 3.0 + 6.0 * iz + 6.0 * iz2) -
                        ep * ((g2 * g) * z + 3.0 * g2 + 6.0 * gi + 6.0 * iz2));
  }
  if (TAIL) {
    o.rphi = o.rphi - P.stat_rphi;
    o.rpsi = o.rpsi - P.stat_rpsi;
    if (DERIV) {
      o.r2dphi = o.r2dphi + P.stat_rphi;
      o.r2dpsi = o.r2dpsi + P.stat_rpsi;
    }
  }
  return o;
}

// The coefficients of w T_ij(x, y; n) = A n_i h_j + B h_i h_j + C h_i n_j
// + Ad delta_ij, with h the unit vector from x to y.
struct TCoef {
  double h[3];
  cd A, B, C, Ad;
};

template <bool TAIL>
__device__ __forceinline__ TCoef t_coef(const double* x, const double* y, const double* n, double w,
                                        const KParams& P) {
  TCoef o;
  const double d0 = y[0] - x[0], d1 = y[1] - x[1], d2 = y[2] - x[2];
  double r, ir;
  dist_inv(d0 * d0 + d1 * d1 + d2 * d2, r, ir);
  o.h[0] = d0 * ir;
  o.h[1] = d1 * ir;
  o.h[2] = d2 * ir;
  const double drdn = o.h[0] * n[0] + o.h[1] * n[1] + o.h[2] * n[2];
  const Radial R = radial<TAIL, true>(r, ir, P);
  const double ir2 = ir * ir;
  const cd psir = R.rpsi * ir2;
  const cd dphi = R.r2dphi * ir2;
  const cd dpsi = R.r2dpsi * ir2;
  const double sc = w * P.inv4pi;
  o.A = (dphi - psir) * sc;
  o.B = (2.0 * (2.0 * psir - dpsi)) * (sc * drdn);
  o.C = (P.ratio * (dphi - dpsi - 2.0 * psir) - 2.0 * (dphi - dpsi - psir)) * sc;
  o.Ad = o.A * drdn;
  return o;
}

// T[3i+j] += w * T_ij(x, y; n)
template <bool TAIL>
__device__ __forceinline__ void acc_T(const double* x, const double* y, const double* n, double w,
                                      const KParams& P, cd* T) {
  const TCoef c = t_coef<TAIL>(x, y, n, w, P);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cd v = c.A * (n[i] * c.h[j]) + c.B * (c.h[i] * c.h[j]) + c.C * (c.h[i] * n[j]);
      if (i == j) v += c.Ad;
      T[3 * i + j] += v;
    }
  }
}

// T[3i+j] = sum_q w_q T_ij(x, y_q; n) over the seven points y_q (weights w_q)
// of one element, whose normal n is shared: T = n a^T + S + c n^T with
// a = sum A_q h_q, c = sum C_q h_q and the symmetric S = sum (B_q h_q h_q^T
// + Ad_q I), so that a point costs 12 complex updates instead of 9 full
// entries.  UNROLL: the points unrolled (more registers) or in a loop.
template <bool UNROLL>
__device__ __forceinline__ void elem_T(const double* x, const double* y, const double* w, const double* n,
                                       const KParams& P, cd* T) {
  cd a[3], c[3], S[6];
#pragma unroll
  for (int i = 0; i < 3; ++i) a[i] = c[i] = mk(0.0);
#pragma unroll
  for (int i = 0; i < 6; ++i) S[i] = mk(0.0);
  auto point = [&](int q) {
    const TCoef k = t_coef<false>(x, y + 3 * q, n, w[q], P);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      a[i] += k.A * k.h[i];
      c[i] += k.C * k.h[i];
    }
    S[0] += k.B * (k.h[0] * k.h[0]) + k.Ad;
    S[1] += k.B * (k.h[0] * k.h[1]);
    S[2] += k.B * (k.h[0] * k.h[2]);
    S[3] += k.B * (k.h[1] * k.h[1]) + k.Ad;
    S[4] += k.B * (k.h[1] * k.h[2]);
    S[5] += k.B * (k.h[2] * k.h[2]) + k.Ad;
  };
  if (UNROLL) {
#pragma unroll
    for (int q = 0; q < 7; ++q) point(q);
  } else {
#pragma unroll 1
    for (int q = 0; q < 7; ++q) point(q);
  }
  constexpr int si[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) T[3 * i + j] = a[j] * n[i] + S[si[i][j]] + c[i] * n[j];
}

// U[3i+j] += w * U_ij(x, y)   (only the 6 distinct entries are formed)
template <bool TAIL>
__device__ __forceinline__ void acc_U(const double* x, const double* y, double w,
                                      const KParams& P, cd* U) {
  const double d0 = y[0] - x[0], d1 = y[1] - x[1], d2 = y[2] - x[2];
  double r, ir;
  dist_inv(d0 * d0 + d1 * d1 + d2 * d2, r, ir);
  const double h[3] = {d0 * ir, d1 * ir, d2 * ir};
  const Radial R = radial<TAIL, false>(r, ir, P);
  const double sc = w * P.inv4pimu * ir;
  const cd phi = R.rphi * sc;
  const cd psi = R.rpsi * sc;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = i; j < 3; ++j) {
      cd v = psi * (-h[i] * h[j]);
      if (i == j) v += phi;
      U[3 * i + j] += v;
      if (j != i) U[3 * j + i] += v;
    }
  }
}

// u[i] += w * U_ij(x, y) t_j  = w/(4 pi mu) [phi t_i - psi rh_i (rh . t)]
__device__ __forceinline__ void acc_Ut(const double* x, const double* y, double w, const double* t,
                                       const KParams& P, cd* u) {
  const double d0 = y[0] - x[0], d1 = y[1] - x[1], d2 = y[2] - x[2];
  double r, ir;
  dist_inv(d0 * d0 + d1 * d1 + d2 * d2, r, ir);
  const double h0 = d0 * ir, h1 = d1 * ir, h2 = d2 * ir;
  const Radial R = radial<false, false>(r, ir, P);
  const double sc = w * P.inv4pimu * ir;
  const double ht = h0 * t[0] + h1 * t[1] + h2 * t[2];
  const cd phi = R.rphi * sc;
  const cd psi = R.rpsi * (sc * ht);
  u[0] += phi * t[0] - psi * h0;
  u[1] += phi * t[1] - psi * h1;
  u[2] += phi * t[2] - psi * h2;
}

}  // namespace ewbem
