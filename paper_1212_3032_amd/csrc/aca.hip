// Adaptive cross approximation of the admissible (far-field) blocks of the
// system matrix (columns of T, or of -U for elements with a given
// displacement), A_b ~ U V^T, for all far blocks at once.
//
// The blocks advance in lock step.  One step of every active block is:
//   k_aca_row_eval  one thread per (block, column element): the three rows
//                   of the current row element a* against all columns, into
//                   V[:, k..k+2];
//   k_aca_row_res   one wavefront per 64 columns of a block: subtract
//                   U(a*, :) V^T (the residual rows), and keep the largest
//                   entry's column element b* by a packed atomic maximum;
//   k_aca_pivot     one thread per block: marks the row used (a row that is
//                   already represented is skipped for the next unused one)
//                   and eliminates the 3 x 3 pivot block with complete
//                   pivoting: each accepted pivot is one rank-one term,
//                   pivots below 1e-10 of the largest are dropped;
//   k_aca_col_eval  one thread per (block, row element): the three columns of
//                   b* against all rows, into U[:, k..k+2];
//   k_aca_col_res   one wavefront per 21 row elements: subtract U V(b*, :)^T
//                   (the residual columns), form the accepted terms' U
//                   columns in place, their squared norms, and the next row
//                   element (largest entries of the new columns among the
//                   unused rows);
//   k_aca_form_v    one wavefront per 64 columns: the terms' V columns in
//                   place, and their squared norms;
//   k_aca_finalize  one wavefront per block: the stopping test
//                   sqrt(sum_t |u_t|^2 |v_t|^2) <= tol |S|_F, with |S|_F^2
//                   estimated by sum_l |u_l|^2 |v_l|^2;
//   k_aca_compact   the next step's list of active blocks.
// Evaluation (compute bound, many registers) and the residual updates
// (streaming the factors, few registers) are separate kernels so that each
// runs at its own occupancy.  Norm sums go through per-wavefront partials
// summed in a fixed order, so the result does not depend on scheduling.
// A block stops when converged, when every row has been used, or when its
// capacity is exhausted (reported for a retry with more capacity).
#include "kernel_fn.hpp"
#include "launch.hpp"
#include "aca.hpp"

namespace ewbem {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// 3 x 3 block of the system matrix between collocation point x and element e.
__device__ __forceinline__ void A_elem(const double* x, int e, const DevGeom& g, const KParams& P, cd* T) {
#pragma unroll
  for (int i = 0; i < 9; ++i) T[i] = mk(0.0);
  if (g.bc && g.bc[e]) {
#pragma unroll 1
    for (int q = 0; q < 7; ++q) acc_U<false>(x, g.qp + 21 * (size_t)e + 3 * q, -g.qw[7 * (size_t)e + q], P, T);
  } else {
    elem_T<false>(x, g.qp + 21 * (size_t)e, g.qw + 7 * (size_t)e, g.nrm + 3 * (size_t)e, P, T);
  }
}

// index i with offs[i] <= t < offs[i+1]
__device__ __forceinline__ int find_seg(const int* __restrict__ offs, int n, int t) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offs[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Packed (score, index) for an unsigned maximum: score >= 0 as float bits in
// the high word (they order like the value), ties go to the smaller index.
__device__ __forceinline__ unsigned long long pack_best(double score, int idx) {
  const float f = (float)score;
  return ((unsigned long long)__float_as_uint(f) << 32) | (unsigned)(0x7fffffff - idx);
}
__device__ __forceinline__ int unpack_idx(unsigned long long p) { return 0x7fffffff - (int)(p & 0xffffffffu); }
__device__ __forceinline__ double unpack_score(unsigned long long p) {
  return (double)__uint_as_float((unsigned)(p >> 32));
}

__device__ __forceinline__ int first_unused(const unsigned* __restrict__ used, int m) {
  for (int w = 0; w < (m + 31) / 32; ++w) {
    const unsigned free_bits = ~used[w];
    if (free_bits) {
      const int a = 32 * w + __ffs(free_bits) - 1;
      return a < m ? a : -1;
    }
  }
  return -1;
}

__global__ void k_aca_init(const int* __restrict__ ids, int n, const FarBlk* __restrict__ blks,
                           AcaState* __restrict__ st, unsigned* __restrict__ used, int* __restrict__ nlist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = ids[i];
  AcaState s{};
  s.status = ACA_ACTIVE;
  s.first_max = -1.0;
  st[b] = s;
  const FarBlk B = blks[b];
  for (int w = 0; w < (B.m + 31) / 32; ++w) used[B.bitoff + w] = 0u;
  nlist[2 * b] = 0;
  nlist[2 * b + 1] = 0;
}

// Exclusive scans over the active list (one workgroup) of the element
// counts n and m, of the 64-column wavefront tasks ceil(3n / 64) and of the
// 21-row-element wavefront tasks ceil(m / 21).
__global__ __launch_bounds__(1024) void k_aca_scan(const int* __restrict__ act, const int* __restrict__ nact_dev,
                                                   const FarBlk* __restrict__ blks, int* __restrict__ offs,
                                                   int stride, int* __restrict__ totals) {
  const int nact = *nact_dev;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ int wt[4][16];  // per-wavefront totals, then their exclusive prefixes
  __shared__ int ct[4];      // total of the chunk
  int carry[4] = {0, 0, 0, 0};
  for (int base = 0; base < nact; base += 1024) {
    const int i = base + threadIdx.x;
    int v[4] = {0, 0, 0, 0};
    if (i < nact) {
      const FarBlk B = blks[act[i]];
      v[0] = B.n;
      v[1] = B.m;
      v[2] = (3 * B.n + 63) / 64;
      v[3] = (B.m + ACA_ROWS_PER_WAVE - 1) / ACA_ROWS_PER_WAVE;
    }
    int inc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int x = v[q];
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
      }
      inc[q] = x;
    }
    __syncthreads();  // the previous chunk is done with wt / ct
    if (lane == 63)
#pragma unroll
      for (int q = 0; q < 4; ++q) wt[q][w] = inc[q];
    __syncthreads();
    if (w == 0 && lane < 16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int own = wt[q][lane];
        int x = own;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          const int y = __shfl_up(x, off, 64);
          if (lane >= off) x += y;
        }
        wt[q][lane] = x - own;
        if (lane == 15) ct[q] = x;
      }
    }
    __syncthreads();
    if (i < nact)
#pragma unroll
      for (int q = 0; q < 4; ++q) offs[q * stride + i] = carry[q] + wt[q][w] + inc[q] - v[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) carry[q] += ct[q];
  }
  if (threadIdx.x < 4) {
    offs[threadIdx.x * stride + nact] = carry[threadIdx.x];
    totals[threadIdx.x] = carry[threadIdx.x];
  }
  if (threadIdx.x == 0) totals[4] = nact;
}

// Row step, evaluation: one thread per (block, column element) writes the
// 3 x 3 entries A(3a* + j, 3b + jj) into V[3b + jj, k + j].
__global__ __launch_bounds__(256, 4) void k_aca_row_eval(const int* __restrict__ act, int nact,
                                                      const int* __restrict__ offs_n,
                                                      const FarBlk* __restrict__ blks,
                                                      const AcaState* __restrict__ st, DevGeom g, KParams P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= offs_n[nact]) return;
  const int i = find_seg(offs_n, nact, t);
  const int blk = act[i];
  const int b = t - offs_n[i];
  const FarBlk B = blks[blk];
  const int k = st[blk].k, astar = st[blk].astar;
  const size_t C = 3 * (size_t)B.n;
  const double* xa = g.cen + 3 * (size_t)(B.r0 + astar);
  const double x[3] = {xa[0], xa[1], xa[2]};
  cd T[9];
  A_elem(x, B.c0 + b, g, P, T);
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) B.V[(k + j) * C + 3 * b + jj] = T[3 * j + jj];
}

// Row step, residual: one wavefront per 64 columns of one block,
// V[c, k + j] -= sum_l U[3a* + j, l] V[c, l]; the wavefront's largest
// residual entry (with its column element) goes to the block's pivot search.
// The U entries of row element a* are staged 64 terms at a time in LDS.
__global__ __launch_bounds__(64) void k_aca_row_res(const int* __restrict__ act, int nact,
                                                    const int* __restrict__ offs_w,
                                                    const FarBlk* __restrict__ blks, AcaState* __restrict__ st) {
  __shared__ cd su[64][3];
  const int t = blockIdx.x;
  const int i = find_seg(offs_w, nact, t);
  const int blk = act[i];
  const FarBlk B = blks[blk];
  const int k = st[blk].k, astar = st[blk].astar;
  const size_t R = 3 * (size_t)B.m, C = 3 * (size_t)B.n;
  const int c = (t - offs_w[i]) * 64 + threadIdx.x;
  const bool valid = c < (int)C;
  cd r0 = mk(0.0), r1 = mk(0.0), r2 = mk(0.0);
  if (valid) {
    r0 = B.V[(size_t)k * C + c];
    r1 = B.V[(size_t)(k + 1) * C + c];
    r2 = B.V[(size_t)(k + 2) * C + c];
  }
  for (int l0 = 0; l0 < k; l0 += 64) {
    const int nl = min(64, k - l0);
    __syncthreads();
    if ((int)threadIdx.x < nl) {
      const cd* u = B.U + (size_t)(l0 + threadIdx.x) * R + 3 * astar;
      su[threadIdx.x][0] = u[0];
      su[threadIdx.x][1] = u[1];
      su[threadIdx.x][2] = u[2];
    }
    __syncthreads();
    if (valid) {
      const cd* v = B.V + (size_t)l0 * C + c;
      int l = 0;
      for (; l + 4 <= nl; l += 4) {
        const cd v0 = v[(size_t)l * C], v1 = v[(size_t)(l + 1) * C], v2 = v[(size_t)(l + 2) * C],
                 v3 = v[(size_t)(l + 3) * C];
        r0 -= su[l][0] * v0 + su[l + 1][0] * v1 + su[l + 2][0] * v2 + su[l + 3][0] * v3;
        r1 -= su[l][1] * v0 + su[l + 1][1] * v1 + su[l + 2][1] * v2 + su[l + 3][1] * v3;
        r2 -= su[l][2] * v0 + su[l + 1][2] * v1 + su[l + 2][2] * v2 + su[l + 3][2] * v3;
      }
      for (; l < nl; ++l) {
        const cd vv = v[(size_t)l * C];
        r0 -= su[l][0] * vv;
        r1 -= su[l][1] * vv;
        r2 -= su[l][2] * vv;
      }
    }
  }
  unsigned long long best = 0ull;
  if (valid) {
    if (k > 0) {
      B.V[(size_t)k * C + c] = r0;
      B.V[(size_t)(k + 1) * C + c] = r1;
      B.V[(size_t)(k + 2) * C + c] = r2;
    }
    best = pack_best(sqrt(fmax(norm2(r0), fmax(norm2(r1), norm2(r2)))), c / 3);
  }
  best = wave_max_u64(best);
  if (threadIdx.x == 0) atomicMax(&st[blk].best, best);
}

__device__ __forceinline__ cd sel3(int i, cd a, cd b, cd c) {
  const bool i0 = i == 0, i1 = i == 1;
  return cd{i0 ? a.x : (i1 ? b.x : c.x), i0 ? a.y : (i1 ? b.y : c.y)};
}

// One step of complete-pivoting elimination on the 3 x 3 pivot block Pm:
// the largest remaining entry (p, q) becomes term STP with column weights
// alpha[STP] (residual column q in terms of the cross columns) and row
// weights beta[STP] (residual row p over the pivot, in terms of the cross
// rows); Br / Ac track the residual rows / columns in those terms.
template <int STP>
__device__ __forceinline__ void plan_step(cd (&Pm)[3][3], cd (&Br)[3][3], cd (&Ac)[3][3], cd (&alpha)[3][3],
                                          cd (&beta)[3][3], bool (&rowl)[3], bool (&coll)[3], double pmax0,
                                          int& nacc) {
  if (nacc != STP) return;
  double best = -1.0;
  int p = 0, q = 0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = norm2(Pm[r][c]);
      if (rowl[r] && coll[c] && v > best) {
        best = v;
        p = r;
        q = c;
      }
    }
  if (!(best > 1e-20 * pmax0 && best > 0.0)) return;
  cd prow[3], qcol[3], brp[3], acq[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    prow[c] = sel3(p, Pm[0][c], Pm[1][c], Pm[2][c]);
    brp[c] = sel3(p, Br[0][c], Br[1][c], Br[2][c]);
    acq[c] = sel3(q, Ac[0][c], Ac[1][c], Ac[2][c]);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) qcol[r] = sel3(q, Pm[r][0], Pm[r][1], Pm[r][2]);
  const cd piv = sel3(q, prow[0], prow[1], prow[2]);
  const cd ipiv = cinv(piv);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    alpha[STP][c] = acq[c];
    beta[STP][c] = brp[c] * ipiv;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const cd f = qcol[r] * ipiv;
    if (rowl[r] && r != p)
#pragma unroll
      for (int c = 0; c < 3; ++c) Br[r][c] -= f * brp[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cd h = prow[c] * ipiv;
    if (coll[c] && c != q)
#pragma unroll
      for (int r = 0; r < 3; ++r) Ac[c][r] -= h * acq[r];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (r != p && c != q) Pm[r][c] -= qcol[r] * (prow[c] * ipiv);
#pragma unroll
  for (int r = 0; r < 3; ++r)
    if (r == p) rowl[r] = false;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (c == q) coll[c] = false;
  ++nacc;
}

// A row that adds nothing: try the next unused one, or stop.
__device__ __forceinline__ void row_failed(AcaState& s, const unsigned* u, int m) {
  s.skip = 1;
  s.fails += 1;
  const int next = first_unused(u, m);
  if (next < 0 || s.fails > 3)
    s.status = ACA_DONE;
  else
    s.astar = next;
}

__global__ __launch_bounds__(64) void k_aca_pivot(const int* __restrict__ act, int nact, const FarBlk* __restrict__ blks,
                            AcaState* __restrict__ st, AcaPlan* __restrict__ plan, unsigned* __restrict__ used) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nact) return;
  const int blk = act[i];
  const FarBlk B = blks[blk];
  AcaState s = st[blk];
  const unsigned long long best = s.best;
  s.best = 0ull;
  s.best_row = 0ull;
  const double score = unpack_score(best);
  s.bstar = unpack_idx(best);
  unsigned* u = used + B.bitoff;
  u[s.astar >> 5] |= 1u << (s.astar & 31);
  if (s.first_max < 0.0) s.first_max = score;
  s.skip = 0;
  s.nacc = 0;
  if (!(score > 1e-12 * s.first_max) || score == 0.0 || s.bstar < 0 || s.bstar >= B.n) {
    row_failed(s, u, B.m);  // the row is already represented
    st[blk] = s;
    return;
  }
  // complete-pivoting plan on the 3 x 3 pivot block (registers only)
  const size_t C = 3 * (size_t)B.n;
  cd Pm[3][3], Br[3][3], Ac[3][3], alpha[3][3], beta[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Pm[r][c] = B.V[(size_t)(s.k + r) * C + 3 * s.bstar + c];
      Br[r][c] = Ac[r][c] = mk(r == c ? 1.0 : 0.0);
      alpha[r][c] = beta[r][c] = mk(0.0);
    }
  double pmax0 = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) pmax0 = fmax(pmax0, norm2(Pm[r][c]));
  bool rowl[3] = {true, true, true}, coll[3] = {true, true, true};
  int nacc = 0;
  plan_step<0>(Pm, Br, Ac, alpha, beta, rowl, coll, pmax0, nacc);
  plan_step<1>(Pm, Br, Ac, alpha, beta, rowl, coll, pmax0, nacc);
  plan_step<2>(Pm, Br, Ac, alpha, beta, rowl, coll, pmax0, nacc);
  if (nacc == 0) {
    row_failed(s, u, B.m);
    st[blk] = s;
    return;
  }
  s.nacc = nacc;
  AcaPlan pl;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pl.alpha[r][c] = alpha[r][c];
      pl.beta[r][c] = beta[r][c];
    }
  plan[blk] = pl;
  st[blk] = s;
}

// Column step, evaluation: one thread per (block, row element) writes
// A(3a + ii, 3b* + jj) into U[3a + ii, k + jj].
__global__ __launch_bounds__(256, 4) void k_aca_col_eval(const int* __restrict__ act, int nact,
                                                      const int* __restrict__ offs_m,
                                                      const FarBlk* __restrict__ blks,
                                                      const AcaState* __restrict__ st, DevGeom g, KParams P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= offs_m[nact]) return;
  const int i = find_seg(offs_m, nact, t);
  const int blk = act[i];
  if (st[blk].skip) return;
  const int a = t - offs_m[i];
  const FarBlk B = blks[blk];
  const int k = st[blk].k, bstar = st[blk].bstar;
  const size_t R = 3 * (size_t)B.m;
  const double* xa = g.cen + 3 * (size_t)(B.r0 + a);
  const double x[3] = {xa[0], xa[1], xa[2]};
  cd T[9];
  A_elem(x, B.c0 + bstar, g, P, T);
#pragma unroll
  for (int jj = 0; jj < 3; ++jj)
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) B.U[(k + jj) * R + 3 * a + ii] = T[3 * ii + jj];
}

// Column step, residual and U terms: one wavefront per 21 row elements (63
// rows) of one block.  U[r, k + jj] -= sum_l U[r, l] V[3b* + jj, l] with the
// V entries of b* staged in LDS; then the accepted terms
// U[r, k + t] = sum_jj alpha[t][jj] U[r, k + jj], their squared norms per
// wavefront into part (3 per task), and the largest new-column energy of an
// unused row element into the block's next-row search.
__global__ __launch_bounds__(64) void k_aca_col_res(const int* __restrict__ act, int nact,
                                                    const int* __restrict__ offs_w,
                                                    const FarBlk* __restrict__ blks, AcaState* __restrict__ st,
                                                    const AcaPlan* __restrict__ plan,
                                                    const unsigned* __restrict__ used, double* __restrict__ part) {
  __shared__ cd sv[64][3];
  const int t = blockIdx.x;
  const int i = find_seg(offs_w, nact, t);
  const int blk = act[i];
  if (st[blk].skip) return;
  const FarBlk B = blks[blk];
  const int k = st[blk].k, bstar = st[blk].bstar, nacc = st[blk].nacc;
  const size_t R = 3 * (size_t)B.m, C = 3 * (size_t)B.n;
  const int lane = threadIdx.x;
  const int r = (t - offs_w[i]) * (3 * ACA_ROWS_PER_WAVE) + lane;
  const bool valid = lane < 3 * ACA_ROWS_PER_WAVE && r < (int)R;
  cd c0 = mk(0.0), c1 = mk(0.0), c2 = mk(0.0);
  if (valid) {
    c0 = B.U[(size_t)k * R + r];
    c1 = B.U[(size_t)(k + 1) * R + r];
    c2 = B.U[(size_t)(k + 2) * R + r];
  }
  for (int l0 = 0; l0 < k; l0 += 64) {
    const int nl = min(64, k - l0);
    __syncthreads();
    if (lane < nl) {
      const cd* v = B.V + (size_t)(l0 + lane) * C + 3 * bstar;
      sv[lane][0] = v[0];
      sv[lane][1] = v[1];
      sv[lane][2] = v[2];
    }
    __syncthreads();
    if (valid) {
      const cd* u = B.U + (size_t)l0 * R + r;
      int l = 0;
      for (; l + 4 <= nl; l += 4) {
        const cd u0 = u[(size_t)l * R], u1 = u[(size_t)(l + 1) * R], u2 = u[(size_t)(l + 2) * R],
                 u3 = u[(size_t)(l + 3) * R];
        c0 -= u0 * sv[l][0] + u1 * sv[l + 1][0] + u2 * sv[l + 2][0] + u3 * sv[l + 3][0];
        c1 -= u0 * sv[l][1] + u1 * sv[l + 1][1] + u2 * sv[l + 2][1] + u3 * sv[l + 3][1];
        c2 -= u0 * sv[l][2] + u1 * sv[l + 1][2] + u2 * sv[l + 2][2] + u3 * sv[l + 3][2];
      }
      for (; l < nl; ++l) {
        const cd uu = u[(size_t)l * R];
        c0 -= uu * sv[l][0];
        c1 -= uu * sv[l][1];
        c2 -= uu * sv[l][2];
      }
    }
  }
  const AcaPlan& pl = plan[blk];
  double nu[3] = {0.0, 0.0, 0.0}, e = 0.0;
#pragma unroll
  for (int tt = 0; tt < 3; ++tt)
    if (tt < nacc) {
      const cd v = pl.alpha[tt][0] * c0 + pl.alpha[tt][1] * c1 + pl.alpha[tt][2] * c2;
      if (valid) B.U[(size_t)(k + tt) * R + r] = v;
      const double q = valid ? norm2(v) : 0.0;
      nu[tt] = q;
      e += q;
    }
  // energy of the row element 3a..3a+2 (lanes 3j..3j+2 of the wavefront)
  const double e1 = __shfl_down(e, 1, 64), e2 = __shfl_down(e, 2, 64);
  unsigned long long cand = 0ull;
  if (valid && lane % 3 == 0) {
    const int a = r / 3;
    if (!(used[B.bitoff + (a >> 5)] & (1u << (a & 31)))) cand = pack_best(sqrt(e + e1 + e2), a);
  }
  cand = wave_max_u64(cand);
#pragma unroll
  for (int tt = 0; tt < 3; ++tt) nu[tt] = wsum(nu[tt]);
  if (lane == 0) {
    if (cand) atomicMax(&st[blk].best_row, cand);
    double* p = part + 3 * (size_t)t;
    p[0] = nu[0];
    p[1] = nu[1];
    p[2] = nu[2];
  }
}

// V terms: one wavefront per 64 columns, V[c, k + t] = sum_j beta[t][j]
// V[c, k + j], squared norms per wavefront into part (3 per task).
__global__ __launch_bounds__(64) void k_aca_form_v(const int* __restrict__ act, int nact,
                                                   const int* __restrict__ offs_w,
                                                   const FarBlk* __restrict__ blks,
                                                   const AcaState* __restrict__ st,
                                                   const AcaPlan* __restrict__ plan, double* __restrict__ part) {
  const int t = blockIdx.x;
  const int i = find_seg(offs_w, nact, t);
  const int blk = act[i];
  if (st[blk].skip) return;
  const FarBlk B = blks[blk];
  const int k = st[blk].k, nacc = st[blk].nacc;
  const size_t C = 3 * (size_t)B.n;
  const int c = (t - offs_w[i]) * 64 + threadIdx.x;
  const bool valid = c < (int)C;
  cd r0 = mk(0.0), r1 = mk(0.0), r2 = mk(0.0);
  if (valid) {
    r0 = B.V[(size_t)k * C + c];
    r1 = B.V[(size_t)(k + 1) * C + c];
    r2 = B.V[(size_t)(k + 2) * C + c];
  }
  const AcaPlan& pl = plan[blk];
  double nv[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int tt = 0; tt < 3; ++tt)
    if (tt < nacc) {
      const cd v = pl.beta[tt][0] * r0 + pl.beta[tt][1] * r1 + pl.beta[tt][2] * r2;
      if (valid) {
        B.V[(size_t)(k + tt) * C + c] = v;
        nv[tt] = norm2(v);
      }
    }
#pragma unroll
  for (int tt = 0; tt < 3; ++tt) nv[tt] = wsum(nv[tt]);
  if (threadIdx.x == 0) {
    double* p = part + 3 * (size_t)t;
    p[0] = nv[0];
    p[1] = nv[1];
    p[2] = nv[2];
  }
}

// One wavefront per active block: sums the norm partials in task order, the
// stopping test and the next row.
__global__ __launch_bounds__(256) void k_aca_finalize(const int* __restrict__ act, int nact,
                                                      const int* __restrict__ offs_wu,
                                                      const int* __restrict__ offs_wv,
                                                      const FarBlk* __restrict__ blks, AcaState* __restrict__ st,
                                                      const double* __restrict__ part_u,
                                                      const double* __restrict__ part_v, double tol,
                                                      int* __restrict__ plist, int* __restrict__ nlist) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nact) return;
  const int blk = act[i];
  AcaState s = st[blk];
  if (!s.skip) {
    double nu[3] = {0.0, 0.0, 0.0}, nv[3] = {0.0, 0.0, 0.0};
    for (int q = offs_wu[i] + lane; q < offs_wu[i + 1]; q += 64)
#pragma unroll
      for (int tt = 0; tt < 3; ++tt) nu[tt] += part_u[3 * (size_t)q + tt];
    for (int q = offs_wv[i] + lane; q < offs_wv[i + 1]; q += 64)
#pragma unroll
      for (int tt = 0; tt < 3; ++tt) nv[tt] += part_v[3 * (size_t)q + tt];
    double termsq = 0.0;
#pragma unroll
    for (int tt = 0; tt < 3; ++tt) termsq += wsum(nu[tt]) * wsum(nv[tt]);
    const FarBlk B = blks[blk];
    s.normS2 += termsq;
    s.k += s.nacc;
    s.fails = 0;
    // this step's pivot elements, for a warm start at the next frequency
    if (lane == 0) {
      const int nr = nlist[2 * blk], nc = nlist[2 * blk + 1];
      if (nr >= 0 && nr < B.m && nc < B.m) {
        plist[B.poff + nr] = s.astar;
        plist[B.poff + B.m + nc] = s.bstar;
        nlist[2 * blk] = nr + 1;
        nlist[2 * blk + 1] = nc + 1;
      } else {
        nlist[2 * blk] = -1;
      }
    }
    if (termsq <= tol * tol * s.normS2 || s.k >= 3 * min(B.m, B.n) || s.best_row == 0ull)
      s.status = ACA_DONE;  // converged, full rank, or every row used (exact)
    else if (s.k + 3 > B.kcap)
      s.status = ACA_OVERFLOW;
    else
      s.astar = unpack_idx(s.best_row);
  }
  if (lane == 0) st[blk] = s;
}

// The next step's active list (one thread per block, so the appends to the
// shared counter combine per wavefront).
__global__ void k_aca_compact(const int* __restrict__ act, int nact, const AcaState* __restrict__ st,
                              int* __restrict__ act_out, int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nact) return;
  const int blk = act[i];
  if (st[blk].status == ACA_ACTIVE) act_out[atomicAdd(count, 1)] = blk;
}

__global__ void k_aca_finish(const int* __restrict__ ids, int n, const AcaState* __restrict__ st,
                             int* __restrict__ rank, int* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = ids[i];
  rank[b] = st[b].k;
  status[b] = st[b].status == ACA_OVERFLOW ? 1 : 0;
}

void launch_aca_init(const int* ids, int n, const FarBlk* blks, AcaState* st, unsigned* used, int* nlist,
                     hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_aca_init, dim3((n + 255) / 256), dim3(256), 0, s, ids, n, blks, st, used, nlist);
}

void launch_aca_compact(const int* ids, int n, const AcaState* st, int* act_out, int* count, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_aca_compact, dim3((n + 255) / 256), dim3(256), 0, s, ids, n, st, act_out, count);
}

void launch_aca_scan(const int* act, const int* nact_dev, const FarBlk* blks, int* offs, int stride,
                     int* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_aca_scan, dim3(1), dim3(1024), 0, s, act, nact_dev, blks, offs, stride, totals);
}

void launch_aca_step(const AcaLists& L, const AcaWork& W, const DevGeom& g, const KParams& P, double tol,
                     int* act_out, int* count, hipStream_t s) {
  const int nact = L.nact;
  if (nact <= 0) return;
  hipLaunchKernelGGL(k_aca_row_eval, dim3((L.tot_n + 255) / 256), dim3(256), 0, s, L.act, nact, L.offs_n, W.blks,
                     W.st, g, P);
  hipLaunchKernelGGL(k_aca_row_res, dim3(L.tot_wn), dim3(64), 0, s, L.act, nact, L.offs_wn, W.blks, W.st);
  hipLaunchKernelGGL(k_aca_pivot, dim3((nact + 63) / 64), dim3(64), 0, s, L.act, nact, W.blks, W.st, W.plan,
                     W.used);
  hipLaunchKernelGGL(k_aca_col_eval, dim3((L.tot_m + 255) / 256), dim3(256), 0, s, L.act, nact, L.offs_m, W.blks,
                     W.st, g, P);
  hipLaunchKernelGGL(k_aca_col_res, dim3(L.tot_wm), dim3(64), 0, s, L.act, nact, L.offs_wm, W.blks, W.st, W.plan,
                     W.used, W.part_u);
  hipLaunchKernelGGL(k_aca_form_v, dim3(L.tot_wn), dim3(64), 0, s, L.act, nact, L.offs_wn, W.blks, W.st, W.plan,
                     W.part_v);
  hipLaunchKernelGGL(k_aca_finalize, dim3((nact + 3) / 4), dim3(256), 0, s, L.act, nact, L.offs_wm, L.offs_wn,
                     W.blks, W.st, W.part_u, W.part_v, tol, W.plist, W.nlist);
  hipLaunchKernelGGL(k_aca_compact, dim3((nact + 255) / 256), dim3(256), 0, s, L.act, nact, W.st, act_out, count);
}

void launch_aca_finish(const int* ids, int n, const AcaState* st, int* rank, int* status, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_aca_finish, dim3((n + 255) / 256), dim3(256), 0, s, ids, n, st, rank, status);
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

// The same conversion for the blocks ids[0..n) into per-block destinations.
__global__ void k_to_c64_ptr(const FarBlk* __restrict__ blks, const int* __restrict__ ids,
                             const int* __restrict__ rank, cf* const* __restrict__ up, cf* const* __restrict__ vp) {
  const int b = ids[blockIdx.x];
  const FarBlk B = blks[b];
  const int k = rank[b];
  const long long nu = 3LL * B.m * k, nvv = 3LL * B.n * k;
  cf* Uo = up[blockIdx.x];
  cf* Vo = vp[blockIdx.x];
  for (long long i = threadIdx.x; i < nu; i += blockDim.x) Uo[i] = to_cf(B.U[i]);
  for (long long i = threadIdx.x; i < nvv; i += blockDim.x) Vo[i] = to_cf(B.V[i]);
}

void launch_to_c64_ptr(const FarBlk* blks, const int* ids, int n, const int* rank, cf* const* up, cf* const* vp,
                       hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_to_c64_ptr, dim3(n), dim3(256), 0, st, blks, ids, rank, up, vp);
}

void launch_to_c64(const FarBlk* blks, int nblk, const int* rank, const long long* uo,
                   const long long* vo, cf* out, hipStream_t st) {
  if (nblk > 0) hipLaunchKernelGGL(k_to_c64, dim3(nblk), dim3(256), 0, st, blks, rank, uo, vo, out);
}

}  // namespace ewbem
