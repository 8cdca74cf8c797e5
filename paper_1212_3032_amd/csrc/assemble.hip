// Assembly kernels: singular self-element integrals, dense near-field
// blocks of the traction operator, the right-hand side U t0, and the
// parity entry points (point kernels, dense T and U).
//
// Sec. 2.1: collocation of the boundary integral equation at element
// centroids with constant elements gives T u = U t; distinct elements use
// the 7-point rule, the element holding the collocation point uses a
// polar-coordinate rule about it, with the free term delta_ij / 2 and the
// principal value of the static traction kernel added in closed form.
#include "kernel_fn.hpp"
#include "launch.hpp"

namespace ewbem {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wavefront per element: lanes cover (edge, angular node) pairs and
// loop over the radial nodes of the polar rule about the centroid.
__global__ __launch_bounds__(256) void k_self(DevGeom g, KParams P, SelfRule S, cd* __restrict__ selfT,
                                              cd* __restrict__ selfU, cd* __restrict__ selfA) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= g.ne) return;
  const double* x = g.cen + 3 * e;
  const double* n = g.nrm + 3 * e;
  const double* v = g.vtx + 9 * e;
  cd T[9], U[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) T[i] = U[i] = mk(0.0);
  const int nodes = 3 * S.nt;
  for (int idx = lane; idx < nodes; idx += 64) {
    const int edge = idx / S.nt, a = idx - edge * S.nt;
    const double* pa = v + 3 * edge;
    const double* pb = v + 3 * ((edge + 1) % 3);
    double da[3], db[3];
    for (int k = 0; k < 3; ++k) {
      da[k] = pa[k] - x[k];
      db[k] = pb[k] - x[k];
    }
    double e3[3] = {da[1] * db[2] - da[2] * db[1], da[2] * db[0] - da[0] * db[2],
                    da[0] * db[1] - da[1] * db[0]};
    double l3 = rsqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
    double la = rsqrt(da[0] * da[0] + da[1] * da[1] + da[2] * da[2]);
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
      e3[k] *= l3;
      e1[k] = da[k] * la;
    }
    e2[0] = e3[1] * e1[2] - e3[2] * e1[1];
    e2[1] = e3[2] * e1[0] - e3[0] * e1[2];
    e2[2] = e3[0] * e1[1] - e3[1] * e1[0];
    const double tb = atan2(db[0] * e2[0] + db[1] * e2[1] + db[2] * e2[2],
                            db[0] * e1[0] + db[1] * e1[1] + db[2] * e1[2]);
    double te[3], L = 0;
    for (int k = 0; k < 3; ++k) {
      te[k] = pb[k] - pa[k];
      L += te[k] * te[k];
    }
    L = rsqrt(L);
    double proj = 0;
    for (int k = 0; k < 3; ++k) {
      te[k] *= L;
      proj += da[k] * te[k];
    }
    double m[3], h = 0;
    for (int k = 0; k < 3; ++k) {
      m[k] = da[k] - te[k] * proj;  // foot - x
      h += m[k] * m[k];
    }
    h = sqrt(h);
    for (int k = 0; k < 3; ++k) m[k] /= h;
    const double th = S.t[a] * tb;
    double sn, cs;
    sincos(th, &sn, &cs);
    double rh[3];
    for (int k = 0; k < 3; ++k) rh[k] = cs * e1[k] + sn * e2[k];
    const double R = h / (rh[0] * m[0] + rh[1] * m[1] + rh[2] * m[2]);
    const double wth = S.wt[a] * tb;
    for (int b = 0; b < S.nr; ++b) {
      const double rho = S.u[b] * R;
      const double y[3] = {x[0] + rho * rh[0], x[1] + rho * rh[1], x[2] + rho * rh[2]};
      const double w = wth * S.wu[b] * rho * R;
      acc_T<true>(x, y, n, w, P, T);
      acc_U<false>(x, y, w, P, U);
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    T[i].x = wave_sum(T[i].x);
    T[i].y = wave_sum(T[i].y);
    U[i].x = wave_sum(U[i].x);
    U[i].y = wave_sum(U[i].y);
  }
  if (lane == 0) {
    // Principal value of the static kernel gamma^2/(4 pi r^2)(rh_i n_j - rh_j n_i):
    // PV int rh_i / r^2 dA = -sum_edges m_i int_edge dl / r (divergence
    // theorem in the element plane, m the outward in-plane edge normal).
    double C[3] = {0, 0, 0};
    for (int edge = 0; edge < 3; ++edge) {
      const double* pa = v + 3 * edge;
      const double* pb = v + 3 * ((edge + 1) % 3);
      double te[3], L = 0;
      for (int k = 0; k < 3; ++k) {
        te[k] = pb[k] - pa[k];
        L += te[k] * te[k];
      }
      L = sqrt(L);
      double proj = 0;
      for (int k = 0; k < 3; ++k) {
        te[k] /= L;
        proj += (x[k] - pa[k]) * te[k];
      }
      double m[3], h = 0;
      for (int k = 0; k < 3; ++k) {
        m[k] = pa[k] + te[k] * proj - x[k];  // foot - x, outward from x
        h += m[k] * m[k];
      }
      h = sqrt(h);
      const double l1 = -proj, l2 = L - proj;  // endpoint coordinates from the foot
      const double I = asinh(l2 / h) - asinh(l1 / h);
      for (int k = 0; k < 3; ++k) C[k] -= (m[k] / h) * I;
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double cpv = P.cpv * (C[i] * n[j] - n[i] * C[j]);
        T[3 * i + j].x += cpv + (i == j ? 0.5 : 0.0);
      }
    const bool disp = g.bc && g.bc[e];
    for (int i = 0; i < 9; ++i) {
      selfT[9 * (size_t)e + i] = T[i];
      selfU[9 * (size_t)e + i] = U[i];
      if (selfA) selfA[9 * (size_t)e + i] = disp ? -U[i] : T[i];
    }
  }
}

void launch_self(const DevGeom& g, const KParams& P, const SelfRule& S, cd* selfT, cd* selfU,
                 cd* selfA, hipStream_t st) {
  hipLaunchKernelGGL(k_self, dim3((g.ne + 3) / 4), dim3(256), 0, st, g, P, S, selfT, selfU, selfA);
}

// Dense near-field blocks of the system matrix A (Sec. 2.1, eq. Aa_b): the
// columns of an element with a given traction are those of T, of an element
// with a given displacement those of -U.  One workgroup per block, the
// column cluster's quadrature data staged in LDS, one (row element, column
// element) pair per thread.  The self pair is left to k_scatter_self.
// (at most 168 registers: three wavefronts per SIMD, without spills; 5% faster
// than the two that the unconstrained allocation allows)
__global__ __launch_bounds__(256, 3) void k_near(const NearBlk* __restrict__ blks, DevGeom g, KParams P,
                                              cd* __restrict__ D) {
  const NearBlk B = blks[blockIdx.x];
  __shared__ double sq[64 * 21], sw[64 * 7], sn[64 * 3], sx[64 * 3];
  __shared__ int sbc[64];
  for (int i = threadIdx.x; i < B.n; i += blockDim.x) sbc[i] = g.bc ? g.bc[B.c0 + i] : 0;
  for (int i = threadIdx.x; i < B.n * 21; i += blockDim.x) sq[i] = g.qp[(size_t)B.c0 * 21 + i];
  for (int i = threadIdx.x; i < B.n * 7; i += blockDim.x) sw[i] = g.qw[(size_t)B.c0 * 7 + i];
  for (int i = threadIdx.x; i < B.n * 3; i += blockDim.x) sn[i] = g.nrm[(size_t)B.c0 * 3 + i];
  for (int i = threadIdx.x; i < B.m * 3; i += blockDim.x) sx[i] = g.cen[(size_t)B.r0 * 3 + i];
  __syncthreads();
  const int ld = 3 * B.m;
  for (int p = threadIdx.x; p < B.m * B.n; p += blockDim.x) {
    const int a = p % B.m, b = p / B.m;
    if (B.r0 + a == B.c0 + b) continue;
    cd T[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) T[i] = mk(0.0);
    if (sbc[b]) {
#pragma unroll
      for (int q = 0; q < 7; ++q) acc_U<false>(sx + 3 * a, sq + 21 * b + 3 * q, -sw[7 * b + q], P, T);
    } else {
      elem_T<false>(sx + 3 * a, sq + 21 * b, sw + 7 * b, sn + 3 * b, P, T);
    }
    cd* out = D + B.off + (size_t)(3 * b) * ld + 3 * a;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) out[(size_t)j * ld + i] = T[3 * i + j];
  }
}

void launch_near(const NearBlk* blks, int nblk, const DevGeom& g, const KParams& P, cd* D,
                 hipStream_t st) {
  if (nblk > 0) hipLaunchKernelGGL(k_near, dim3(nblk), dim3(256), 0, st, blks, g, P, D);
}

__global__ void k_scatter_self(const cd* __restrict__ selfT, const long long* __restrict__ self_off,
                               const int* __restrict__ self_ld, int ne, cd* __restrict__ D) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * ne) return;
  const int e = t / 9, ij = t - 9 * e, i = ij / 3, j = ij - 3 * i;
  D[self_off[e] + (size_t)j * self_ld[e] + i] = selfT[t];
}

void launch_scatter_self(const cd* selfT, const long long* self_off, int ne, cd* D,
                         const int* self_ld, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_self, dim3((9 * ne + 255) / 256), dim3(256), 0, st, selfT, self_off,
                     self_ld, ne, D);
}

// Parity path: every off-diagonal element pair of the dense T and U,
// written row-major in the caller's element order.
__global__ __launch_bounds__(256) void k_dense_pairs(DevGeom g, KParams P, const int* __restrict__ perm,
                                                     cd* __restrict__ Tout, cd* __restrict__ Uout) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ne = g.ne;
  if (p >= ne * ne) return;
  const int a = (int)(p % ne), b = (int)(p / ne);
  if (a == b) return;
  cd T[9], U[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) T[i] = U[i] = mk(0.0);
  const double* x = g.cen + 3 * a;
  for (int q = 0; q < 7; ++q) {
    const double* y = g.qp + 21 * (size_t)b + 3 * q;
    const double w = g.qw[7 * (size_t)b + q];
    acc_T<false>(x, y, g.nrm + 3 * b, w, P, T);
    acc_U<false>(x, y, w, P, U);
  }
  const long long N = 3 * ne;
  const long long ao = perm[a], bo = perm[b];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const long long idx = (3 * ao + i) * N + 3 * bo + j;
      if (Tout) Tout[idx] = T[3 * i + j];
      if (Uout) Uout[idx] = U[3 * i + j];
    }
}

void launch_dense_pairs(const DevGeom& g, const KParams& P, const int* perm, cd* Tout, cd* Uout,
                        hipStream_t st) {
  const long long np = (long long)g.ne * g.ne;
  hipLaunchKernelGGL(k_dense_pairs, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, g, P, perm,
                     Tout, Uout);
}

__global__ void k_dense_self(const cd* __restrict__ selfT, const cd* __restrict__ selfU,
                             const int* __restrict__ perm, int ne, cd* __restrict__ Tout,
                             cd* __restrict__ Uout) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * ne) return;
  const int e = t / 9, ij = t - 9 * e, i = ij / 3, j = ij - 3 * i;
  const long long N = 3LL * ne, eo = perm[e];
  const long long idx = (3 * eo + i) * N + 3 * eo + j;
  if (Tout) Tout[idx] = selfT[t];
  if (Uout) Uout[idx] = selfU[t];
}

void launch_dense_self(const cd* selfT, const cd* selfU, const int* perm, int ne, cd* Tout,
                       cd* Uout, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_self, dim3((9 * ne + 255) / 256), dim3(256), 0, st, selfT, selfU, perm,
                     ne, Tout, Uout);
}

// Right-hand side b_k = P_k U(s_k) t0 by direct summation over all element
// pairs (7-point rule) plus the self-element U blocks, for up to RHS_NK
// frequencies per pass.  For the frequencies s_k = sigma + i k dw of one
// pass the exponentials share their modulus exp(-sigma r / c) and their
// phases advance by the fixed rotation exp(-i dw r / c), so each extra
// frequency costs a complex multiply instead of an exp and a sincos.
// Targets are tiled 256 per workgroup, the sources split into RHS_SPLIT
// ranges (staged in LDS, RHS_TILE elements at a time); each range writes
// its own partial vector and k_rhs_finish sums them in a fixed order.
// INC: the load of a plane wave, exp(-s_k tau_e) t0_e per source element,
// whose phase advances with the frequency in the same way.
constexpr int RHS_NK = 8;
constexpr int RHS_TILE = 128;

template <bool INC>
__global__ __launch_bounds__(256) void k_rhs_multi(DevGeom g, KParams P, double sigma, double dw, int k0,
                                                   int nk, const double* __restrict__ t0,
                                                   const double* __restrict__ tau, cd* __restrict__ partial) {
  __shared__ double sq[RHS_TILE * 21], sw[RHS_TILE * 7], stt[RHS_TILE * 3], stau[INC ? RHS_TILE : 1];
  __shared__ cd scs[RHS_NK];  // c_s / s_k of the pass: 1 / z_s = (c_s / s_k) / r
  const int ne = g.ne;
  const int kst = k0 + blockIdx.y * RHS_NK;          // first frequency of this pass
  const int nkc = min(RHS_NK, k0 + nk - kst);        // frequencies in this pass
  if (!INC && threadIdx.x < RHS_NK) {  // read after the first barrier below
    const double w = (kst + (int)threadIdx.x) * dw, d = sigma * sigma + w * w, csv = 1.0 / P.inv_cs;
    scs[threadIdx.x] = d > 0.0 ? cd{csv * sigma / d, -csv * w / d} : mk(0.0);
  }
  const int split = blockIdx.z, nsplit = gridDim.z;
  const int s0 = (int)((long long)ne * split / nsplit), s1 = (int)((long long)ne * (split + 1) / nsplit);
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = a < ne;
  double x[3] = {0, 0, 0};
  if (act) {
    x[0] = g.cen[3 * a];
    x[1] = g.cen[3 * a + 1];
    x[2] = g.cen[3 * a + 2];
  }
  cd acc[RHS_NK][3];
#pragma unroll
  for (int j = 0; j < RHS_NK; ++j) acc[j][0] = acc[j][1] = acc[j][2] = mk(0.0);
  const double gam = P.gamma, ics = P.inv_cs;
  for (int c0 = s0; c0 < s1; c0 += RHS_TILE) {
    const int nc = min(RHS_TILE, s1 - c0);
    __syncthreads();
    for (int i = threadIdx.x; i < nc * 21; i += blockDim.x) sq[i] = g.qp[(size_t)c0 * 21 + i];
    for (int i = threadIdx.x; i < nc * 7; i += blockDim.x) sw[i] = g.qw[(size_t)c0 * 7 + i];
    for (int i = threadIdx.x; i < nc * 3; i += blockDim.x) stt[i] = t0[(size_t)c0 * 3 + i];
    if (INC)
      for (int i = threadIdx.x; i < nc; i += blockDim.x) stau[i] = tau[c0 + i];
    __syncthreads();
    if (!act) continue;
    for (int b = 0; b < nc; ++b) {
      if (c0 + b == a) continue;
      const double* tb = stt + 3 * b;
      // incident wave: the source's load at s_kst and its step to s_{k+1}
      cd sph = mk(1.0), srot = mk(1.0);
      if (INC) {
        double sn, cs;
        const double ta = stau[b];
        sincos(kst * dw * ta, &sn, &cs);
        const double m = exp(-sigma * ta);
        sph = cd{m * cs, -m * sn};
        sincos(dw * ta, &sn, &cs);
        srot = cd{cs, -sn};
      }
      for (int qq = 0; qq < 7; ++qq) {
        const double* y = sq + 21 * b + 3 * qq;
        const double d0 = y[0] - x[0], d1 = y[1] - x[1], d2 = y[2] - x[2];
        double r, ir;
        dist_inv(d0 * d0 + d1 * d1 + d2 * d2, r, ir);
        const double h0 = d0 * ir, h1 = d1 * ir, h2 = d2 * ir;
        const double ht = h0 * tb[0] + h1 * tb[1] + h2 * tb[2];
        const double sc = sw[7 * b + qq] * P.inv4pimu * ir;
        const double zx = sigma * r * ics;      // Re z_s (same for every k)
        const double th = dw * r * ics;         // Im z_s step per k
        double sn, cs;
        const double ms = exp(-zx), mp = exp(-gam * zx);
        sincos(kst * th, &sn, &cs);
        cd ph = cd{ms * cs, -ms * sn};
        sincos(th, &sn, &cs);
        const cd rot = cd{cs, -sn};
        sincos(gam * kst * th, &sn, &cs);
        cd php = cd{mp * cs, -mp * sn};
        sincos(gam * th, &sn, &cs);
        const cd rotp = cd{cs, -sn};
        cd sp = sph;
#pragma unroll
        for (int j = 0; j < RHS_NK; ++j) {
          if (j < nkc) {
            const cd z = cd{zx, (kst + j) * th};
            cd rphi, rpsi;
            if (norm2(z) < P.series_z2) {
              cd a1 = mk(P.ser[NSER - 1]), b1 = mk(P.ser[2 * NSER - 1]);
              for (int m = NSER - 2; m >= 0; --m) {
                a1 = a1 * z + P.ser[m];
                b1 = b1 * z + P.ser[NSER + m];
              }
              rphi = a1;
              rpsi = b1;
            } else {
              // without the plane wave, 1 / z_s = (c_s / s_k) / r by a product; with
              // it the division (the products' extra registers would halve
              // the occupancy of that variant)
              const cd iz = INC ? cinv(z) : scs[j] * ir;
              const cd iz2 = iz * iz;
              const cd gi = iz * gam;
              rphi = ph * (1.0 + iz + iz2) - php * (gi + iz2);
              rpsi = ph * (1.0 + 3.0 * iz + 3.0 * iz2) - php * (P.g2 + 3.0 * gi + 3.0 * iz2);
            }
            cd f = rphi * sc, gg = rpsi * (sc * ht);
            if (INC) {
              f = f * sp;
              gg = gg * sp;
              sp = sp * srot;
            }
            acc[j][0] += f * tb[0] - gg * h0;
            acc[j][1] += f * tb[1] - gg * h1;
            acc[j][2] += f * tb[2] - gg * h2;
            ph = ph * rot;
            php = php * rotp;
          }
        }
      }
    }
  }
  if (!act) return;
#pragma unroll
  for (int j = 0; j < RHS_NK; ++j) {
    if (j < nkc) {
      cd* out = partial + ((size_t)split * nk + (kst - k0 + j)) * 3 * ne + 3 * (size_t)a;
      out[0] = acc[j][0];
      out[1] = acc[j][1];
      out[2] = acc[j][2];
    }
  }
}

// The same sums for several loads t0_l on one mesh: one workgroup column
// per frequency, every pair's kernel evaluated once and applied to all NL
// loads.  With one frequency per pass the phases exp(-i Im(s) r / c) are
// evaluated directly (no rotation recurrence to share), so a load's
// partials agree with k_rhs_multi's to rounding.  INC: incident waves, each
// load's source element weighted by its own exp(-s_k tau_l), as in
// k_rhs_multi<true>.
template <int NL, bool INC>
__global__ __launch_bounds__(256) void k_rhs_loads(DevGeom g, KParams P, double sigma, double dw, int k0,
                                                   int nk, RhsLoadSet L) {
  __shared__ double sq[RHS_TILE * 21], sw[RHS_TILE * 7], stt[NL * RHS_TILE * 3], stau[INC ? NL * RHS_TILE : 1];
  const int ne = g.ne;
  const int k = k0 + blockIdx.y;
  const int split = blockIdx.z, nsplit = gridDim.z;
  const int s0 = (int)((long long)ne * split / nsplit), s1 = (int)((long long)ne * (split + 1) / nsplit);
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = a < ne;
  double x[3] = {0, 0, 0};
  if (act) {
    x[0] = g.cen[3 * a];
    x[1] = g.cen[3 * a + 1];
    x[2] = g.cen[3 * a + 2];
  }
  cd acc[NL][3];
#pragma unroll
  for (int l = 0; l < NL; ++l) acc[l][0] = acc[l][1] = acc[l][2] = mk(0.0);
  const double gam = P.gamma, ics = P.inv_cs;
  for (int c0 = s0; c0 < s1; c0 += RHS_TILE) {
    const int nc = min(RHS_TILE, s1 - c0);
    __syncthreads();
    for (int i = threadIdx.x; i < nc * 21; i += blockDim.x) sq[i] = g.qp[(size_t)c0 * 21 + i];
    for (int i = threadIdx.x; i < nc * 7; i += blockDim.x) sw[i] = g.qw[(size_t)c0 * 7 + i];
#pragma unroll
    for (int l = 0; l < NL; ++l)
      for (int i = threadIdx.x; i < nc * 3; i += blockDim.x) stt[l * RHS_TILE * 3 + i] = L.t0[l][(size_t)c0 * 3 + i];
    if (INC)
#pragma unroll
      for (int l = 0; l < NL; ++l)
        for (int i = threadIdx.x; i < nc; i += blockDim.x) stau[l * RHS_TILE + i] = L.tau[l][c0 + i];
    __syncthreads();
    if (!act) continue;
    for (int b = 0; b < nc; ++b) {
      if (c0 + b == a) continue;
      double tb[NL][3];
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        tb[l][0] = stt[l * RHS_TILE * 3 + 3 * b];
        tb[l][1] = stt[l * RHS_TILE * 3 + 3 * b + 1];
        tb[l][2] = stt[l * RHS_TILE * 3 + 3 * b + 2];
      }
      // incident waves: the source's load at s_k, exp(-s_k tau_l)
      cd sp[INC ? NL : 1];
      if (INC) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          double sn, cs;
          const double ta = stau[l * RHS_TILE + b];
          sincos(k * dw * ta, &sn, &cs);
          const double m = exp(-sigma * ta);
          sp[l] = cd{m * cs, -m * sn};
        }
      }
      for (int qq = 0; qq < 7; ++qq) {
        const double* y = sq + 21 * b + 3 * qq;
        const double d0 = y[0] - x[0], d1 = y[1] - x[1], d2 = y[2] - x[2];
        double r, ir;
        dist_inv(d0 * d0 + d1 * d1 + d2 * d2, r, ir);
        const double h0 = d0 * ir, h1 = d1 * ir, h2 = d2 * ir;
        const double sc = sw[7 * b + qq] * P.inv4pimu * ir;
        const double zx = sigma * r * ics;
        const double zy = k * dw * r * ics;  // Im z_s at s_k
        double sn, cs;
        const double ms = exp(-zx), mp = exp(-gam * zx);
        sincos(zy, &sn, &cs);
        const cd ph = cd{ms * cs, -ms * sn};
        sincos(gam * zy, &sn, &cs);
        const cd php = cd{mp * cs, -mp * sn};
        const cd z = cd{zx, zy};
        cd rphi, rpsi;
        if (norm2(z) < P.series_z2) {
          cd a1 = mk(P.ser[NSER - 1]), b1 = mk(P.ser[2 * NSER - 1]);
          for (int m = NSER - 2; m >= 0; --m) {
            a1 = a1 * z + P.ser[m];
            b1 = b1 * z + P.ser[NSER + m];
          }
          rphi = a1;
          rpsi = b1;
        } else {
          const cd iz = cinv(z);
          const cd iz2 = iz * iz;
          const cd gi = iz * gam;
          rphi = ph * (1.0 + iz + iz2) - php * (gi + iz2);
          rpsi = ph * (1.0 + 3.0 * iz + 3.0 * iz2) - php * (P.g2 + 3.0 * gi + 3.0 * iz2);
        }
        const cd f = rphi * sc;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const double ht = h0 * tb[l][0] + h1 * tb[l][1] + h2 * tb[l][2];
          cd fl = f, gg = rpsi * (sc * ht);
          if (INC) {
            fl = fl * sp[l];
            gg = gg * sp[l];
          }
          acc[l][0] += fl * tb[l][0] - gg * h0;
          acc[l][1] += fl * tb[l][1] - gg * h1;
          acc[l][2] += fl * tb[l][2] - gg * h2;
        }
      }
    }
  }
  if (!act) return;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    cd* out = L.part[l] + ((size_t)split * nk + (k - k0)) * 3 * ne + 3 * (size_t)a;
    out[0] = acc[l][0];
    out[1] = acc[l][1];
    out[2] = acc[l][2];
  }
}

template <int NL, bool INC>
void rhs_loads_nl(const DevGeom& g, const KParams& P, double sigma, double dw, int k0, int nk, const RhsLoadSet& L,
                  hipStream_t st) {
  dim3 grid((g.ne + 255) / 256, nk, rhs_split(g.ne));
  hipLaunchKernelGGL((k_rhs_loads<NL, INC>), grid, dim3(256), 0, st, g, P, sigma, dw, k0, nk, L);
}

// b[d] = P_k (sum over source ranges of the partials of frequency index kk
// + U_self t0)
__global__ void k_rhs_finish(const cd* __restrict__ partial, int nsplit, int nk, int kk, int ne,
                             const cd* __restrict__ selfU, const double* __restrict__ t0,
                             const double* __restrict__ tau, cd s_k, const cd* __restrict__ phat_k,
                             cd* __restrict__ b) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= 3 * ne) return;
  const int e = d / 3, i = d - 3 * e;
  cd acc = mk(0.0);
  for (int sp = 0; sp < nsplit; ++sp) acc += partial[((size_t)sp * nk + kk) * 3 * ne + d];
  cd self = mk(0.0);
  for (int j = 0; j < 3; ++j) self += selfU[9 * (size_t)e + 3 * i + j] * t0[3 * e + j];
  if (tau) {
    // exp(-s_k tau_e) on the element's own load, and the factor s_k of the
    // incident wave's traction
    double sn, cs;
    sincos(s_k.y * tau[e], &sn, &cs);
    const double m = exp(-s_k.x * tau[e]);
    acc += self * cd{m * cs, -m * sn};
    b[d] = acc * phat_k[0] * s_k;
  } else {
    b[d] = (acc + self) * phat_k[0];
  }
}

// Total-field load of a plane S-wave on traction-free cavities: b = the
// incident displacement at each collocation point,
// b[3e + i] = F_k exp(-s_k tau_e) pol_i.
__global__ void k_rhs_total(const double* __restrict__ tau, double q0, double q1, double q2, cd s_k,
                            const cd* __restrict__ phat_k, int ne, cd* __restrict__ b) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= 3 * ne) return;
  const int e = d / 3, i = d - 3 * e;
  double sn, cs;
  sincos(s_k.y * tau[e], &sn, &cs);
  const double m = exp(-s_k.x * tau[e]);
  const double q = i == 0 ? q0 : (i == 1 ? q1 : q2);
  b[d] = cd{m * cs, -m * sn} * phat_k[0] * q;
}

void launch_rhs_total(const double* tau, const double* pol, cd s_k, const cd* phat_k, int ne, cd* b,
                      hipStream_t st) {
  if (ne <= 0) return;
  hipLaunchKernelGGL(k_rhs_total, dim3((3 * ne + 255) / 256), dim3(256), 0, st, tau, pol[0], pol[1], pol[2], s_k,
                     phat_k, ne, b);
}

int rhs_split(int ne) { return ne >= 4096 ? 4 : 1; }

void launch_rhs_multi(const DevGeom& g, const KParams& P, double sigma, double dw, int k0, int nk,
                      const double* t0, const double* tau, cd* partial, hipStream_t st) {
  if (nk <= 0) return;
  dim3 grid((g.ne + 255) / 256, (nk + RHS_NK - 1) / RHS_NK, rhs_split(g.ne));
  if (tau)
    hipLaunchKernelGGL(k_rhs_multi<true>, grid, dim3(256), 0, st, g, P, sigma, dw, k0, nk, t0, tau, partial);
  else
    hipLaunchKernelGGL(k_rhs_multi<false>, grid, dim3(256), 0, st, g, P, sigma, dw, k0, nk, t0, tau, partial);
}

void launch_rhs_loads(const DevGeom& g, const KParams& P, double sigma, double dw, int k0, int nk, int n_loads,
                      const double* const* t0, const double* const* tau, cd* const* partial, hipStream_t st) {
  if (nk <= 0) return;
  const int per = tau ? RHS_NL_INC : RHS_NL;
  for (int l0 = 0; l0 < n_loads; l0 += per) {
    const int n = std::min(per, n_loads - l0);
    RhsLoadSet L{};
    for (int i = 0; i < n; ++i) {
      L.t0[i] = t0[l0 + i];
      L.tau[i] = tau ? tau[l0 + i] : nullptr;
      L.part[i] = partial[l0 + i];
    }
    if (tau) {
      switch (n) {
        case 1: rhs_loads_nl<1, true>(g, P, sigma, dw, k0, nk, L, st); break;
        case 2: rhs_loads_nl<2, true>(g, P, sigma, dw, k0, nk, L, st); break;
        case 3: rhs_loads_nl<3, true>(g, P, sigma, dw, k0, nk, L, st); break;
        default: rhs_loads_nl<4, true>(g, P, sigma, dw, k0, nk, L, st); break;
      }
      continue;
    }
    switch (n) {
      case 1: rhs_loads_nl<1, false>(g, P, sigma, dw, k0, nk, L, st); break;
      case 2: rhs_loads_nl<2, false>(g, P, sigma, dw, k0, nk, L, st); break;
      case 3: rhs_loads_nl<3, false>(g, P, sigma, dw, k0, nk, L, st); break;
      case 4: rhs_loads_nl<4, false>(g, P, sigma, dw, k0, nk, L, st); break;
      case 5: rhs_loads_nl<5, false>(g, P, sigma, dw, k0, nk, L, st); break;
      case 6: rhs_loads_nl<6, false>(g, P, sigma, dw, k0, nk, L, st); break;
      case 7: rhs_loads_nl<7, false>(g, P, sigma, dw, k0, nk, L, st); break;
      default: rhs_loads_nl<8, false>(g, P, sigma, dw, k0, nk, L, st); break;
    }
  }
}

void launch_rhs_finish(const cd* partial, int nk, int kk, int ne, const cd* selfU, const double* t0,
                       const double* tau, cd s_k, const cd* phat_k, cd* b, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_finish, dim3((3 * ne + 255) / 256), dim3(256), 0, st, partial, rhs_split(ne), nk,
                     kk, ne, selfU, t0, tau, s_k, phat_k, b);
}

// Parity path: the point kernels U_ij(x, y) and T_ij(x, y; n) for n pairs.
__global__ void k_kernel_eval(KParams P, long long n, const double* __restrict__ x,
                              const double* __restrict__ y, const double* __restrict__ nrm,
                              cd* __restrict__ U, cd* __restrict__ T) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  cd Ub[9], Tb[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Ub[i] = Tb[i] = mk(0.0);
  if (U) acc_U<false>(x + 3 * p, y + 3 * p, 1.0, P, Ub);
  if (T) acc_T<false>(x + 3 * p, y + 3 * p, nrm + 3 * p, 1.0, P, Tb);
  for (int i = 0; i < 9; ++i) {
    if (U) U[9 * p + i] = Ub[i];
    if (T) T[9 * p + i] = Tb[i];
  }
}

void launch_kernel_eval(const KParams& P, long long n, const double* x, const double* y,
                        const double* nrm, cd* U, cd* T, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_kernel_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, n, x, y,
                       nrm, U, T);
}

// ---- Sec. 3.3: damped DFT of the sampled load and the windowed,
// de-damped inverse back to time.

__global__ void k_load_spectrum(const double* __restrict__ hist, int n_f, double dt, double sigma,
                                cd* __restrict__ phat) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > n_f / 2) return;
  cd acc = mk(0.0);
  for (int n = 0; n < n_f; ++n) {
    const long long nk = ((long long)n * k) % n_f;
    double sn, cs;
    sincospi(2.0 * (double)nk / n_f, &sn, &cs);
    const double a = exp(-sigma * n * dt) * hist[n];
    acc += cd{a * cs, -a * sn};
  }
  phat[k] = acc * (1.0 / n_f);
}

void launch_load_spectrum(const double* hist, int n_f, double period, double sigma, cd* phat,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_load_spectrum, dim3((n_f / 2 + 1 + 63) / 64), dim3(64), 0, st, hist, n_f,
                     period / n_f, sigma, phat);
}

__device__ __forceinline__ double window_w(int window, int k, int n_f) {
  if (window == 1) return 0.5 * (1.0 + cospi(2.0 * k / n_f));
  if (window == 2) return 0.42 + 0.5 * cospi(2.0 * k / n_f) + 0.08 * cospi(4.0 * k / n_f);
  return 1.0;
}

// u[n][caller dof] = Re{ e^{sigma n dt} sum_k W_k a_k e^{2 pi i n k / N_f} }
// with a_{N_f-k} = conj(a_k): the k and N_f-k terms pair into 2 Re(...).
__global__ void k_mft_inverse(const cd* __restrict__ spec, long long N, int n_f, double dt,
                              double sigma, int window, const int* __restrict__ perm,
                              double* __restrict__ u) {
  const long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (d >= N) return;
  const int half = n_f / 2;
  double acc = 0.0;
  for (int k = 0; k <= half; ++k) {
    const cd a = spec[(size_t)k * N + d];
    const long long nk = ((long long)n * k) % n_f;
    double sn, cs;
    sincospi(2.0 * (double)nk / n_f, &sn, &cs);
    const double re = a.x * cs - a.y * sn;
    const double c = (k == 0 || k == half) ? 1.0 : 2.0;
    acc += c * window_w(window, k, n_f) * re;
  }
  const long long e = d / 3, comp = d - 3 * e;
  u[(size_t)n * N + 3 * perm[e] + comp] = exp(sigma * n * dt) * acc;
}

void launch_mft_inverse(const cd* spec, long long N, int n_f, double period, double sigma,
                        int window, const int* perm, double* u, hipStream_t st) {
  hipLaunchKernelGGL(k_mft_inverse, dim3((unsigned)((N + 255) / 256), n_f), dim3(256), 0, st, spec, N,
                     n_f, period / n_f, sigma, window, perm, u);
}

}  // namespace ewbem
