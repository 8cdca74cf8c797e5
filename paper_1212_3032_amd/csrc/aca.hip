// Adaptive cross approximation of the admissible (far-field) blocks of the
// system matrix (columns of T, or of -U for elements with a given
// displacement), A_b ~ U V^T, one workgroup per block.
//
// Each step takes the three rows of one row element (a 3 x 3n residual
// cross row computed from the kernel minus the current approximation), picks
// the column element whose 3 x 3 entry is largest, computes its three
// residual columns, and eliminates the 3 x 3 pivot block with complete
// pivoting.  Every accepted pivot adds one rank-one term, so a step adds up
// to three terms; pivots below 1e-10 of the block's largest are dropped.
// The approximation stops when the new terms satisfy
//   sqrt(sum_t |u_t|^2 |v_t|^2) <= tol * |S|_F,
// with |S|_F^2 estimated as sum_l |u_l|^2 |v_l|^2 (the cross terms between
// different terms are left out, which keeps each step linear in the block
// size), or when the capacity is exhausted (reported so the host can
// retry).  The
// next row element is the unused one with the largest entries in the new
// columns.
#include "kernel_fn.hpp"
#include "launch.hpp"
#include "aca.hpp"

namespace ewbem {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// 3 x 3 T block between collocation point x and element e (7-point rule).
__device__ __forceinline__ void T_elem(const double* x, int e, const DevGeom& g, const KParams& P,
                                       cd* T) {
#pragma unroll
  for (int i = 0; i < 9; ++i) T[i] = mk(0.0);
  const double* n = g.nrm + 3 * (size_t)e;
#pragma unroll
  for (int q = 0; q < 7; ++q)
    acc_T<false>(x, g.qp + 21 * (size_t)e + 3 * q, n, g.qw[7 * (size_t)e + q], P, T);
}

template <int WG>
__device__ __forceinline__ void block_argmax(double& v, int& idx, double* sv, int* si) {
  // wave level
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off, 64);
    int oi = __shfl_xor(idx, off, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  constexpr int W = WG / 64;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (W > 1) {
    __syncthreads();
    if (lane == 0) {
      sv[w] = v;
      si[w] = idx;
    }
    __syncthreads();
    v = sv[0];
    idx = si[0];
    for (int k = 1; k < W; ++k)
      if (sv[k] > v || (sv[k] == v && si[k] < idx)) {
        v = sv[k];
        idx = si[k];
      }
  }
}

template <int WG>
__device__ __forceinline__ double block_sum(double v, double* sv) {
  v = wsum(v);
  constexpr int W = WG / 64;
  if (W > 1) {
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sv[threadIdx.x >> 6] = v;
    __syncthreads();
    v = 0;
    for (int k = 0; k < W; ++k) v += sv[k];
  }
  return v;
}

// 3 x 3 block of T between collocation point x and element e, the 7
// quadrature points split over LPE consecutive lanes and summed by
// butterfly shuffles (every lane of the group ends with the full block).
template <int LPE>
__device__ __forceinline__ void T_elem_split(const double* x, int e, bool valid, int q, const DevGeom& g,
                                             const KParams& P, cd* T) {
#pragma unroll
  for (int i = 0; i < 9; ++i) T[i] = mk(0.0);
  if (valid) {
    if (g.bc && g.bc[e]) {
      // column of an element with a given displacement: -U (Sec. 2.1, eq. Aa_b)
      for (int pt = q; pt < 7; pt += LPE)
        acc_U<false>(x, g.qp + 21 * (size_t)e + 3 * pt, -g.qw[7 * (size_t)e + pt], P, T);
    } else {
      const double* n = g.nrm + 3 * (size_t)e;
      for (int pt = q; pt < 7; pt += LPE)
        acc_T<false>(x, g.qp + 21 * (size_t)e + 3 * pt, n, g.qw[7 * (size_t)e + pt], P, T);
    }
  }
#pragma unroll
  for (int off = 1; off < LPE; off <<= 1)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      T[i].x += __shfl_xor(T[i].x, off, 64);
      T[i].y += __shfl_xor(T[i].y, off, 64);
    }
}

template <int WG, int KMAX>
__global__ __launch_bounds__(WG) void k_aca(const FarBlk* __restrict__ blks, const int* __restrict__ order,
                                            DevGeom g, KParams P, double tol, int* __restrict__ rank_out,
                                            int* __restrict__ status_out) {
  constexpr int LPE = 4;           // lanes per element in the cross evaluations
  constexpr int EPP = WG / LPE;    // elements per pass
  constexpr int W = WG / 64;
  const int bid = order[blockIdx.x];
  const FarBlk B = blks[bid];
  const int R = 3 * B.m, C = 3 * B.n, kcap = B.kcap;
  cd* __restrict__ U = B.U;
  cd* __restrict__ V = B.V;
  __shared__ cd s_urow[3][KMAX];
  __shared__ cd s_vcol[3][KMAX];
  __shared__ unsigned s_used[ACA_MAXM / 32];
  __shared__ double s_rv[W + 1];
  __shared__ int s_ri[W + 1];
  __shared__ double s_red[W][6];
  __shared__ cd s_alpha[3][3], s_beta[3][3];
  __shared__ int s_nacc;

  const int tid = threadIdx.x;
  const int q = tid % LPE, eo = tid / LPE;
  for (int i = tid; i < ACA_MAXM / 32; i += WG) s_used[i] = 0u;
  int k = 0, astar = 0, fails = 0, status = 0;
  double normS2 = 0.0, first_max = -1.0;
  __syncthreads();

  for (;;) {
    // ---- residual row cross: rows 3a*+i, all 3n columns, into V[:, k+i]
    for (int l = tid; l < 3 * k; l += WG) {
      const int i = l / k, ll = l - i * k;
      s_urow[i][ll] = U[(size_t)ll * R + 3 * astar + i];
    }
    __syncthreads();
    double bestv = -1.0;
    int besti = 0x7fffffff;
    {
      const double* xa = g.cen + 3 * (size_t)(B.r0 + astar);
      const double x[3] = {xa[0], xa[1], xa[2]};
      for (int b0 = 0; b0 < B.n; b0 += EPP) {
        const int b = b0 + eo;
        cd T[9];
        T_elem_split<LPE>(x, B.c0 + b, b < B.n, q, g, P, T);
        if (b < B.n && q < 3) {
          const int c = 3 * b + q;
          cd r0 = T[q], r1 = T[3 + q], r2 = T[6 + q];
#pragma unroll 4
          for (int l = 0; l < k; ++l) {
            const cd vv = V[(size_t)l * C + c];
            r0 -= s_urow[0][l] * vv;
            r1 -= s_urow[1][l] * vv;
            r2 -= s_urow[2][l] * vv;
          }
          V[(size_t)(k + 0) * C + c] = r0;
          V[(size_t)(k + 1) * C + c] = r1;
          V[(size_t)(k + 2) * C + c] = r2;
          const double mx = fmax(norm2(r0), fmax(norm2(r1), norm2(r2)));
          if (mx > bestv) {
            bestv = mx;
            besti = b;
          }
        }
      }
    }
    block_argmax<WG>(bestv, besti, s_rv, s_ri);
    if (tid == 0) s_used[astar >> 5] |= 1u << (astar & 31);
    if (first_max < 0) first_max = bestv;
    __syncthreads();
    if (!(bestv > 1e-24 * first_max) || bestv == 0.0) {
      // the row is already represented: try the next unused row
      ++fails;
      int next = -1;
      for (int a = 0; a < B.m; ++a)
        if (!(s_used[a >> 5] & (1u << (a & 31)))) {
          next = a;
          break;
        }
      if (next < 0 || fails > 3) break;
      astar = next;
      continue;
    }
    const int bstar = besti;
    // ---- residual column cross: all 3m rows, columns 3b*+j, into U[:, k+j]
    for (int l = tid; l < 3 * k; l += WG) {
      const int j = l / k, ll = l - j * k;
      s_vcol[j][ll] = V[(size_t)ll * C + 3 * bstar + j];
    }
    __syncthreads();
    for (int a0 = 0; a0 < B.m; a0 += EPP) {
      const int a = a0 + eo;
      const int ac = a < B.m ? a : 0;
      const double* xa = g.cen + 3 * (size_t)(B.r0 + ac);
      const double x[3] = {xa[0], xa[1], xa[2]};
      cd T[9];
      T_elem_split<LPE>(x, B.c0 + bstar, a < B.m, q, g, P, T);
      if (a < B.m && q < 3) {
        const int r = 3 * a + q;
        cd c0 = T[3 * q], c1 = T[3 * q + 1], c2 = T[3 * q + 2];
#pragma unroll 4
        for (int l = 0; l < k; ++l) {
          const cd uu = U[(size_t)l * R + r];
          c0 -= uu * s_vcol[0][l];
          c1 -= uu * s_vcol[1][l];
          c2 -= uu * s_vcol[2][l];
        }
        U[(size_t)(k + 0) * R + r] = c0;
        U[(size_t)(k + 1) * R + r] = c1;
        U[(size_t)(k + 2) * R + r] = c2;
      }
    }
    __syncthreads();
    // ---- 3 x 3 pivot block: complete-pivoting elimination plan (one thread)
    if (tid == 0) {
      cd Pm[3][3], Br[3][3], Ac[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          Pm[i][j] = V[(size_t)(k + i) * C + 3 * bstar + j];
          Br[i][j] = Ac[i][j] = mk(i == j ? 1.0 : 0.0);
          s_alpha[i][j] = s_beta[i][j] = mk(0.0);
        }
      int rowl = 7, coll = 7, nacc = 0;
      double pmax0 = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) pmax0 = fmax(pmax0, norm2(Pm[i][j]));
      for (int stp = 0; stp < 3; ++stp) {
        int p = -1, qq = -1;
        double best = -1.0;
        for (int i = 0; i < 3; ++i) {
          if (!(rowl & (1 << i))) continue;
          for (int j = 0; j < 3; ++j) {
            if (!(coll & (1 << j))) continue;
            const double v = norm2(Pm[i][j]);
            if (v > best) {
              best = v;
              p = i;
              qq = j;
            }
          }
        }
        if (p < 0 || !(best > 1e-20 * pmax0) || best == 0.0) break;
        const cd ipiv = cinv(Pm[p][qq]);
        for (int j = 0; j < 3; ++j) {
          s_alpha[nacc][j] = Ac[qq][j];
          s_beta[nacc][j] = Br[p][j] * ipiv;
        }
        cd f[3], h[3];
        for (int i = 0; i < 3; ++i) f[i] = Pm[i][qq] * ipiv;
        for (int j = 0; j < 3; ++j) h[j] = Pm[p][j] * ipiv;
        for (int i = 0; i < 3; ++i) {
          if (!(rowl & (1 << i)) || i == p) continue;
          for (int j = 0; j < 3; ++j) Br[i][j] -= f[i] * Br[p][j];
        }
        for (int j = 0; j < 3; ++j) {
          if (!(coll & (1 << j)) || j == qq) continue;
          for (int i = 0; i < 3; ++i) Ac[j][i] -= h[j] * Ac[qq][i];
        }
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            if (i != p && j != qq) Pm[i][j] -= Pm[i][qq] * h[j];
        rowl &= ~(1 << p);
        coll &= ~(1 << qq);
        ++nacc;
      }
      s_nacc = nacc;
    }
    __syncthreads();
    const int nacc = s_nacc;
    // ---- form the accepted terms in place: U[:, k+t] = sum_j alpha[t][j] C_j,
    //      V[:, k+t] = sum_i beta[t][i] R_i; accumulate their squared norms
    double nu[3] = {0.0, 0.0, 0.0}, nvv[3] = {0.0, 0.0, 0.0};
    for (int r = tid; r < R; r += WG) {
      const cd c0 = U[(size_t)k * R + r], c1 = U[(size_t)(k + 1) * R + r], c2 = U[(size_t)(k + 2) * R + r];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (t < nacc) {
          const cd v = s_alpha[t][0] * c0 + s_alpha[t][1] * c1 + s_alpha[t][2] * c2;
          U[(size_t)(k + t) * R + r] = v;
          nu[t] += norm2(v);
        }
      }
    }
    for (int c = tid; c < C; c += WG) {
      const cd r0 = V[(size_t)k * C + c], r1 = V[(size_t)(k + 1) * C + c], r2 = V[(size_t)(k + 2) * C + c];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (t < nacc) {
          const cd v = s_beta[t][0] * r0 + s_beta[t][1] * r1 + s_beta[t][2] * r2;
          V[(size_t)(k + t) * C + c] = v;
          nvv[t] += norm2(v);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      nu[t] = wsum(nu[t]);
      nvv[t] = wsum(nvv[t]);
    }
    if ((tid & 63) == 0) {
      for (int t = 0; t < 3; ++t) {
        s_red[tid >> 6][t] = nu[t];
        s_red[tid >> 6][3 + t] = nvv[t];
      }
    }
    __syncthreads();
    if (nacc == 0) {
      ++fails;
      int next = -1;
      for (int a = 0; a < B.m; ++a)
        if (!(s_used[a >> 5] & (1u << (a & 31)))) {
          next = a;
          break;
        }
      if (next < 0 || fails > 3) break;
      astar = next;
      continue;
    }
    // ---- stopping test with |S|_F^2 estimated by sum_l |u_l|^2 |v_l|^2
    double termsq = 0.0;
    for (int t = 0; t < nacc; ++t) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < W; ++w) {
        a += s_red[w][t];
        b += s_red[w][3 + t];
      }
      termsq += a * b;
    }
    normS2 += termsq;
    k += nacc;
    fails = 0;
    if (termsq <= tol * tol * normS2) break;
    if (k + 3 > kcap) {
      status = 1;
      break;
    }
    // ---- next row element: largest entries of the new columns among unused rows
    double nv = -1.0;
    int ni = 0x7fffffff;
    for (int a = tid; a < B.m; a += WG) {
      if (s_used[a >> 5] & (1u << (a & 31))) continue;
      double sc = 0.0;
      for (int t = k - nacc; t < k; ++t)
        for (int i = 0; i < 3; ++i) sc += norm2(U[(size_t)t * R + 3 * a + i]);
      if (sc > nv) {
        nv = sc;
        ni = a;
      }
    }
    block_argmax<WG>(nv, ni, s_rv, s_ri);
    __syncthreads();
    if (nv < 0.0) break;  // every row used: the approximation is exact
    astar = ni;
  }
  if (tid == 0) {
    rank_out[bid] = k;
    status_out[bid] = status;
  }
}

void launch_aca(const FarBlk* blks, const int* order_small, int n_small, const int* order_big,
                int n_big, const DevGeom& g, const KParams& P, double tol, int* rank, int* status,
                hipStream_t st) {
  if (n_small > 0)
    hipLaunchKernelGGL((k_aca<64, ACA_KMAX_SMALL>), dim3(n_small), dim3(64), 0, st, blks, order_small, g, P, tol, rank,
                       status);
  if (n_big > 0)
    hipLaunchKernelGGL((k_aca<256, ACA_KMAX>), dim3(n_big), dim3(256), 0, st, blks, order_big, g, P, tol, rank,
                       status);
}

// complex128 -> complex64 copy of the first rank columns of every block,
// into a compact store laid out by the host.
__global__ void k_to_c64(const FarBlk* __restrict__ blks, const int* __restrict__ rank,
                         const long long* __restrict__ uo, const long long* __restrict__ vo,
                         cf* __restrict__ out) {
  const FarBlk B = blks[blockIdx.x];
  const int k = rank[blockIdx.x];
  const long long nu = 3LL * B.m * k, nvv = 3LL * B.n * k;
  cf* Uo = out + uo[blockIdx.x];
  cf* Vo = out + vo[blockIdx.x];
  for (long long i = threadIdx.x; i < nu; i += blockDim.x) Uo[i] = to_cf(B.U[i]);
  for (long long i = threadIdx.x; i < nvv; i += blockDim.x) Vo[i] = to_cf(B.V[i]);
}

void launch_to_c64(const FarBlk* blks, int nblk, const int* rank, const long long* uo,
                   const long long* vo, cf* out, hipStream_t st) {
  if (nblk > 0) hipLaunchKernelGGL(k_to_c64, dim3(nblk), dim3(256), 0, st, blks, rank, uo, vo, out);
}

}  // namespace ewbem
