// Warm start of the cross approximation from the previous frequency's pivots.
//
// At consecutive frequencies the kernel of a far block changes smoothly, so
// the rows and columns that made a good cross at s_{k-1} make a good cross
// at s_k.  For a block whose previous approximation accepted pivots in row
// elements I_e and column elements J_e (rows I = 3 I_e + {0,1,2}, columns
// J likewise):
//   k_ws_init       state, used-row bits (every listed row is used);
//   k_ws_eval_rows  A(I, :) into Rr, one thread per (listed row element,
//                   column element);
//   k_ws_eval_cols  A(:, J) into Cc, one thread per (listed column element,
//                   row element);
//   k_ws_lu_reg,    one workgroup per block: W = A(I, J), Gaussian
//   k_ws_lu         elimination with complete pivoting (cores of at most
//                   128 x 128 in registers, larger ones in LDS or global
//                   memory), stopping at the first pivot below a set
//                   fraction of the first one's modulus
//                   (ewbem_op_opts.ws_pivot_rel, by default the ACA
//                   tolerance: a term's norm is at least its pivot's
//                   modulus, so later terms rarely pass the stopping test);
//                   the pivot order (p_t, q_t) and the eliminated W;
//   k_ws_panels     per chunk of 16 terms, the panels of the substitutions
//                   U = C_Q M^{-1} (M unit upper triangular,
//                   M[l][t] = W[p_l][q_t] / W[p_l][q_l]) and
//                   V = R_P^T N^{-T} (N^T[l][t] = W[p_t][q_l], l <= t);
//   k_ws_form_mfma  the terms u_t (residual of column q_t) and v_t (residual
//                   of row p_t over its pivot) as chunked products on the
//                   matrix cores; column norms, and the next row element
//                   (largest entry of the last term among unused rows);
//   k_ws_finish     the terms up to the first that meets the stopping test,
//                   the norm estimate sum_t |u_t|^2 |v_t|^2, the lists cut to
//                   the kept pivots' elements, and the next row, so the
//                   ordinary steps continue from there.
// The terms are those the cold steps would form with the same pivots in the
// same order; the approximation equals A(:, Jp) A(Ip, Jp)^{-1} A(Ip, :) on
// the accepted pivots.  The ordinary steps that follow keep the usual
// stopping test, so the warm start changes the cost, not the tolerance.
#include "kernel_fn.hpp"
#include "launch.hpp"
#include "aca.hpp"

namespace ewbem {

namespace {

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

__device__ __forceinline__ unsigned long long pack_best(double score, int idx) {
  const float f = (float)score;
  return ((unsigned long long)__float_as_uint(f) << 32) | (unsigned)(0x7fffffff - idx);
}

// acc -= x * m as four fused multiply-adds
__device__ __forceinline__ void cms(cd& acc, cd x, cd m) {
  acc.x = fma(-x.x, m.x, acc.x);
  acc.x = fma(x.y, m.y, acc.x);
  acc.y = fma(-x.x, m.y, acc.y);
  acc.y = fma(-x.y, m.x, acc.y);
}

// LDS written by some lanes of a wavefront, then read by others: the
// wavefront's LDS operations complete in order; this keeps the compiler
// from moving them across the point.
typedef double wfv4d __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace

__global__ void k_ws_init(const WsBlk* __restrict__ wb, int nwarm, const FarBlk* __restrict__ blks,
                          AcaState* __restrict__ st, unsigned* __restrict__ used, const int* __restrict__ plist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nwarm) return;
  const WsBlk w = wb[i];
  const FarBlk B = blks[w.blk];
  AcaState s{};
  s.status = ACA_ACTIVE;
  s.first_max = -1.0;
  st[w.blk] = s;
  unsigned* u = used + B.bitoff;
  for (int q = 0; q < (B.m + 31) / 32; ++q) u[q] = 0u;
  for (int q = 0; q < w.nr; ++q) {
    const int a = plist[B.poff + q];
    u[a >> 5] |= 1u << (a & 31);
  }
}

// Rr[(3s + j), 3b + jj] = A(3 a_s + j, 3b + jj): thread per (block, s, b).
// At most 128 registers, four wavefronts per SIMD (a few bytes of the
// quadrature loop's state spill; measured faster than three wavefronts).
__global__ __launch_bounds__(256, 4) void k_ws_eval_rows(const WsBlk* __restrict__ wb, int nwarm,
                                                      const int* __restrict__ off, const FarBlk* __restrict__ blks,
                                                      const int* __restrict__ plist, cd* __restrict__ cross, DevGeom g,
                                                      KParams P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= off[nwarm]) return;
  const int i = find_seg(off, nwarm, t);
  const WsBlk w = wb[i];
  const FarBlk B = blks[w.blk];
  const int loc = t - off[i];
  const int sidx = loc / B.n, b = loc - sidx * B.n;
  const int a = plist[B.poff + sidx];
  const size_t N3 = 3 * (size_t)B.n;
  const double* xa = g.cen + 3 * (size_t)(B.r0 + a);
  const double x[3] = {xa[0], xa[1], xa[2]};
  cd T[9];
  A_elem(x, B.c0 + b, g, P, T);
  cd* Rr = cross + w.rr;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) Rr[(3 * (size_t)sidx + j) * N3 + 3 * b + jj] = T[3 * j + jj];
}

// Cc[3a + ii, (3s + jj)] = A(3a + ii, 3 b_s + jj): thread per (block, s, a).
__global__ __launch_bounds__(256, 4) void k_ws_eval_cols(const WsBlk* __restrict__ wb, int nwarm,
                                                      const int* __restrict__ off, const FarBlk* __restrict__ blks,
                                                      const int* __restrict__ plist, cd* __restrict__ cross, DevGeom g,
                                                      KParams P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= off[nwarm]) return;
  const int i = find_seg(off, nwarm, t);
  const WsBlk w = wb[i];
  const FarBlk B = blks[w.blk];
  const int loc = t - off[i];
  const int sidx = loc / B.m, a = loc - sidx * B.m;
  const int b = plist[B.poff + B.m + sidx];
  const size_t M3 = 3 * (size_t)B.m;
  const double* xa = g.cen + 3 * (size_t)(B.r0 + a);
  const double x[3] = {xa[0], xa[1], xa[2]};
  cd T[9];
  A_elem(x, B.c0 + b, g, P, T);
  cd* Cc = cross + w.cc;
#pragma unroll
  for (int jj = 0; jj < 3; ++jj)
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) Cc[(3 * (size_t)sidx + jj) * M3 + 3 * a + ii] = T[3 * ii + jj];
}


// Wavefront argmax of (value, linear index), ties to the smaller index.
__device__ __forceinline__ void wave_argmax(double& v, int& e) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oe = __shfl_xor(e, off, 64);
    if (ov > v || (ov == v && oe < e)) {
      v = ov;
      e = oe;
    }
  }
}

// Elimination of W with complete pivoting: one workgroup of WS_LU_NW
// wavefronts per block.  Lanes own rows (row i = lane + 64 r; the alive rows
// and the pivot column's entries of a lane's rows are in registers); the
// wavefronts split the list of alive columns, which is double-buffered so
// that each pivot costs one barrier.  W is in LDS when it has at most MAXE
// entries; MAXE = 0 works on the copy of W in global memory (large cores).
// NR: row chunks of 64 a lane covers (R3 <= 64 NR).
constexpr int WS_LU_NW = 8;      // wavefronts per elimination workgroup, cores in global memory
constexpr int WS_LU_NW_LDS = 8;  // the same for the LDS classes (tiny cores: 2)
template <int MAXE, int NR, int NW>
__global__ __launch_bounds__(64 * NW) void k_ws_lu(const WsBlk* __restrict__ wb, const int* __restrict__ list,
                                               const FarBlk* __restrict__ blks, const int* __restrict__ plist,
                                               cd* __restrict__ cross, int* __restrict__ pq,
                                               int* __restrict__ rho_out, double stop2) {
  __shared__ cd Wl[MAXE > 0 ? MAXE : 1];
  __shared__ short cl[2][3 * WS_MAXLIST];
  __shared__ short sP[3 * WS_MAXLIST], sQ[3 * WS_MAXLIST];
  __shared__ double sv[2][NW];
  __shared__ int se[2][NW];
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = list[blockIdx.x];
  const WsBlk w = wb[wi];
  const FarBlk B = blks[w.blk];
  const int R3 = 3 * w.nr, C3 = 3 * w.nc, tot = R3 * C3;
  const size_t M3 = 3 * (size_t)B.m;
  const cd* Cc = cross + w.cc;
  cd* W = MAXE > 0 ? Wl : cross + w.w;
  const int* rows = plist + B.poff;
  double best = -1.0;
  int be = 0x7fffffff;
  for (int e = tid; e < tot; e += NT) {
    const int i = e % R3, j = e / R3;
    const cd v = Cc[(size_t)j * M3 + 3 * rows[i / 3] + i % 3];
    W[e] = v;
    const double a = norm2(v);
    if (a > best) {
      best = a;
      be = e;
    }
  }
  for (int j = tid; j < C3; j += NT) cl[0][j] = (short)j;
  unsigned alive = 0u;
  for (int r = 0; r * 64 + lane < R3; ++r) alive |= 1u << r;
  wave_argmax(best, be);
  if (lane == 0) {
    sv[0][wv] = best;
    se[0][wv] = be;
  }
  __syncthreads();
  auto pick = [&](int slot) {
    best = sv[slot][0];
    be = se[slot][0];
#pragma unroll
    for (int q = 1; q < NW; ++q)
      if (sv[slot][q] > best || (sv[slot][q] == best && se[slot][q] < be)) {
        best = sv[slot][q];
        be = se[slot][q];
      }
  };
  pick(0);
  const double max0 = best;
  int t = 0, nac = C3;
  while (t < w.rcap && best > stop2 * max0 && best > 0.0) {
    const int p = be % R3, q = be / R3;
    const short* L = cl[t & 1];
    short* Ln = cl[(t + 1) & 1];
    if (tid == 0) {
      sP[t] = (short)p;
      sQ[t] = (short)q;
    }
    if ((p & 63) == lane) alive &= ~(1u << (p >> 6));
    // next step's column list: this one without q (the last entry takes its place)
    const short last = L[nac - 1];
    for (int jj = tid; jj < nac - 1; jj += NT) Ln[jj] = L[jj] == q ? last : L[jj];
    const cd ipiv = cinv(W[q * R3 + p]);
    cd pc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) pc[r] = (alive & (1u << r)) ? W[q * R3 + r * 64 + lane] : mk(0.0);
    best = -1.0;
    be = 0x7fffffff;
    // eight columns per wavefront pass (jb, jb + NW, ..., jb + 7 NW), all
    // loads of a row chunk issued before its stores
    for (int jb = wv; jb < nac; jb += 8 * NW) {
      int jc[8];
      cd pr[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int jj = jb + NW * u;
        jc[u] = jj < nac ? L[jj] : q;
        pr[u] = jc[u] != q ? W[jc[u] * R3 + p] * ipiv : mk(0.0);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r * 64 >= R3) break;
        if (!(alive & (1u << r))) continue;
        const int i = r * 64 + lane;
        cd v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = jc[u] != q ? W[jc[u] * R3 + i] : mk(0.0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (jc[u] != q) {
            const int e = jc[u] * R3 + i;
            cms(v[u], pc[r], pr[u]);
            W[e] = v[u];
            const double a = norm2(v[u]);
            if (a > best || (a == best && e < be)) {
              best = a;
              be = e;
            }
          }
        }
      }
    }
    wave_argmax(best, be);
    ++t;
    --nac;
    if (lane == 0) {
      sv[t & 1][wv] = best;
      se[t & 1][wv] = be;
    }
    __syncthreads();
    pick(t & 1);
  }
  const int rho = t;
  if (tid == 0) rho_out[wi] = rho;
  int* Pp = pq + w.pq;
  int* Qp = Pp + w.rcap;
  for (int tt = tid; tt < rho; tt += NT) {
    Pp[tt] = sP[tt];
    Qp[tt] = sQ[tt];
  }
  // the eliminated core to its global copy (the LDS classes), for the
  // substitution panels
  if (MAXE > 0) {
    cd* Wg = cross + w.w;
    for (int e = tid; e < tot; e += NT) Wg[e] = W[e];
  }
}

// The same elimination with the core in registers, for cores of at most
// 64 NRC rows and NW CPW columns.  Column j belongs to wavefront j % NW (its
// slot j / NW); lane l holds rows l + 64 r of its wavefront's columns, so the
// rank-one update of a pivot touches registers only.  After the update each
// wavefront puts the column of its own largest entry into LDS beside the
// entry's key; one barrier later every wavefront knows the pivot (p, q),
// reads column q from the winner's slot and broadcasts row p of its own
// columns from the lane that holds it.  The candidate columns are
// double-buffered by pivot parity: a slot is rewritten two pivots later,
// after a barrier every wavefront has passed with its reads done.
// Each lane keeps its largest live entry exactly; across lanes and
// wavefronts the entries compare by a key that packs the squared modulus
// rounded to float (monotone bits) above the complement of the column-major
// index, so one unsigned maximum picks the largest entry and, among entries
// equal in float, the first: complete pivoting up to float rounding of the
// comparison.  The update scales the pivot column (zero on eliminated rows,
// which then keep their values) instead of the pivot row; the stopping rule
// is that of k_ws_lu.  At the end the eliminated core goes to the global copy
// of W for the substitution panels.
__device__ __forceinline__ double bcast_lane(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ unsigned long long lu_key(double v, int e) {
  return ((unsigned long long)__float_as_uint((float)v) << 32) | (unsigned)(0x7fffffff - e);
}
__device__ __forceinline__ double key_val(unsigned long long k) { return (double)__uint_as_float((unsigned)(k >> 32)); }
__device__ __forceinline__ int key_idx(unsigned long long k) { return 0x7fffffff - (int)(unsigned)(k & 0xffffffffu); }

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_max(unsigned long long k) {
  const unsigned lo = (unsigned)k, hi = (unsigned)(k >> 32);
  const unsigned olo = (unsigned)__builtin_amdgcn_update_dpp((int)lo, (int)lo, CTRL, 0xf, 0xf, false);
  const unsigned ohi = (unsigned)__builtin_amdgcn_update_dpp((int)hi, (int)hi, CTRL, 0xf, 0xf, false);
  const unsigned long long o = ((unsigned long long)ohi << 32) | olo;
  return o > k ? o : k;
}

// Largest key of the wavefront (every lane active), wavefront-uniform:
// within rows of 16 lanes by DPP (quad swaps, half-row and row mirrors),
// then across the four rows by lane reads.
__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long k) {
  k = dpp_max<0xB1>(k);   // quad_perm [1, 0, 3, 2]
  k = dpp_max<0x4E>(k);   // quad_perm [2, 3, 0, 1]
  k = dpp_max<0x141>(k);  // row_half_mirror
  k = dpp_max<0x140>(k);  // row_mirror
  const unsigned lo = (unsigned)k, hi = (unsigned)(k >> 32);
  unsigned long long m = 0ull;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned long long o =
        ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)hi, 16 * r) << 32) |
        (unsigned)__builtin_amdgcn_readlane((int)lo, 16 * r);
    m = o > m ? o : m;
  }
  return m;
}

template <int NW, int CPW, int NRC>
__global__ __launch_bounds__(64 * NW) void k_ws_lu_reg(const WsBlk* __restrict__ wb, const int* __restrict__ list,
                                                   const FarBlk* __restrict__ blks, const int* __restrict__ plist,
                                                   cd* __restrict__ cross, int* __restrict__ pq,
                                                   int* __restrict__ rho_out, double stop2) {
  __shared__ cd pcand[2][NW][64 * NRC];
  __shared__ unsigned long long skey[2][NW];
  __shared__ short sP[64 * NRC], sQ[64 * NRC];
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi = list[blockIdx.x];
  const WsBlk w = wb[wi];
  const FarBlk B = blks[w.blk];
  const int R3 = 3 * w.nr, C3 = 3 * w.nc;
  const size_t M3 = 3 * (size_t)B.m;
  const cd* Cc = cross + w.cc;
  cd* Wg = cross + w.w;
  const int* rows = plist + B.poff;
  cd a[CPW][NRC];
  unsigned ralive = 0u, calive = 0u;
  // this lane's largest live entry: squared modulus and column-major index
  // (entries are scanned in increasing index, so a strict comparison keeps
  // the first of equals)
  double best = -1.0;
  int be = 0x7fffffff;
#pragma unroll
  for (int s = 0; s < CPW; ++s)
#pragma unroll
    for (int r = 0; r < NRC; ++r) {
      const int i = r * 64 + lane;
      const int j = wv + NW * s;
      const bool ok = i < R3 && j < C3;
      const size_t ro = i < R3 ? 3 * (size_t)rows[i / 3] + i % 3 : 0;
      const cd v = Cc[ok ? (size_t)j * M3 + ro : 0];
      a[s][r] = ok ? v : mk(0.0);
      const double m = norm2(v);
      const bool take = ok && m > best;
      best = take ? m : best;
      be = take ? j * R3 + i : be;
    }
#pragma unroll
  for (int r = 0; r < NRC; ++r)
    if (r * 64 + lane < R3) ralive |= 1u << r;
#pragma unroll
  for (int s = 0; s < CPW; ++s)
    if (wv + NW * s < C3) calive |= 1u << s;
  // a wavefront's candidate: its largest entry's key and that entry's column
  auto offer = [&](int slot) {
    const unsigned long long key = wave_max_key(best >= 0.0 ? lu_key(best, be) : 0ull);
    if (key != 0ull) {
      const int sc = (key_idx(key) / R3 - wv) / NW;  // wavefront-uniform
#pragma unroll
      for (int s = 0; s < CPW; ++s)
        if (s == sc) {
#pragma unroll
          for (int r = 0; r < NRC; ++r) pcand[slot][wv][r * 64 + lane] = a[s][r];
        }
    }
    if (lane == 0) skey[slot][wv] = key;
  };
  auto pick = [&](int slot) {
    unsigned long long kk[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) kk[q] = skey[slot][q];
    unsigned long long m = kk[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) m = kk[q] > m ? kk[q] : m;
    return m;
  };
  offer(0);
  __syncthreads();
  unsigned long long key = pick(0);
  const double max0 = key_val(key);
  int t = 0;
  while (t < w.rcap && key != 0ull && key_val(key) > stop2 * max0 && key_val(key) > 0.0) {
    const int slot = t & 1;
    const int kb = key_idx(key);
    const int p = kb % R3, q = kb / R3;
    const int qw = q % NW, pl = p & 63, pr = p >> 6;
    if (tid == 0) {
      sP[t] = (short)p;
      sQ[t] = (short)q;
    }
    if (pl == lane) ralive &= ~(1u << pr);
    if (wv == qw) calive &= ~(1u << (q / NW));
    const cd* col = pcand[slot][qw];
    const cd ipiv = cinv(col[p]);
    // the pivot column over the pivot, zero on eliminated rows: their
    // entries then stay as they are (a - 0 x = a)
    cd pcs[NRC];
#pragma unroll
    for (int r = 0; r < NRC; ++r) {
      const cd v = col[r * 64 + lane] * ipiv;
      pcs[r] = ((ralive >> r) & 1u) ? v : mk(0.0);
    }
    best = -1.0;
    be = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < CPW; ++s) {
      if (!(calive & (1u << s))) continue;  // wavefront-uniform
      cd rv = a[s][0];
#pragma unroll
      for (int r = 1; r < NRC; ++r)
        if (pr == r) rv = a[s][r];
      const cd prow = cd{bcast_lane(rv.x, pl), bcast_lane(rv.y, pl)};
      const int j = wv + NW * s;
#pragma unroll
      for (int r = 0; r < NRC; ++r) {
        cms(a[s][r], pcs[r], prow);
        const double m = norm2(a[s][r]);
        const bool take = ((ralive >> r) & 1u) && m > best;
        best = take ? m : best;
        be = take ? j * R3 + r * 64 + lane : be;
      }
    }
    ++t;
    offer(t & 1);
    __syncthreads();
    key = pick(t & 1);
  }
  const int rho = t;
  // the eliminated core to its global copy, for the substitution panels
#pragma unroll
  for (int s = 0; s < CPW; ++s) {
    const int j = wv + NW * s;
    if (j < C3) {
#pragma unroll
      for (int r = 0; r < NRC; ++r) {
        const int i = r * 64 + lane;
        if (i < R3) Wg[(size_t)j * R3 + i] = a[s][r];
      }
    }
  }
  if (tid == 0) rho_out[wi] = rho;
  int* Pp = pq + w.pq;
  int* Qp = Pp + w.rcap;
  for (int tt = tid; tt < rho; tt += NT) {
    Pp[tt] = sP[tt];
    Qp[tt] = sQ[tt];
  }
}

// The substitutions as products on the FP64 matrix cores.
//
// With the pivot order (p_t, q_t) of the eliminated core W, the terms are
//   U = C_Q M^{-1},  M[l][t] = W[p_l][q_t] / W[p_l][q_l] (unit upper),
//   V = R_P^T N^{-T}, N^T[l][t] = W[p_t][q_l] (upper, diagonal W[p_t][q_t]),
// C_Q the cross columns q_t and R_P the cross rows p_t.  Taken in chunks
// T_k of 16 terms, with D_k the inverse of S[T_k, T_k] (S = M or N^T),
//   X[:, T_k] = (Src[:, T_k] - X[:, T_<k] S[T_<k, T_k]) D_k
//             = [Src[:, T_k] | X[:, T_<k]] P_k,  P_k = [D_k ; -S[T_<k, T_k] D_k],
// so each chunk is one product whose first 16 inner rows read the source
// columns and the rest the terms already formed.  k_ws_panels forms the
// panels P_k ((16 + 16 k) x 16, row-major; columns of terms past rho are
// zero), one workgroup per warm block.  The algebra is that of the forward
// substitutions; only the summation order differs.
__global__ __launch_bounds__(256) void k_ws_panels(WsArgs A) {
  __shared__ cd Sd[2][16][16];  // S[T_k, T_k] of each side
  __shared__ cd Dk[2][16][16];  // its inverse
  __shared__ cd sInv[16];       // 1 / W[p_t][q_t] of the chunk's terms
  __shared__ int sP[3 * WS_MAXLIST], sQ[3 * WS_MAXLIST];
  const int i = blockIdx.x;
  const WsBlk w = A.wb[i];
  const int rho = A.rho[i];
  if (rho == 0) return;  // the whole workgroup
  const int tid = threadIdx.x, nt = blockDim.x;
  const int R3 = 3 * w.nr;
  const cd* __restrict__ W = A.cross + w.w;
  cd* PU = A.coef + w.co;
  cd* PV = PU + ws_panel_elems(w.rcap);
  for (int t = tid; t < rho; t += nt) {
    sP[t] = A.pq[w.pq + t];
    sQ[t] = A.pq[w.pq + w.rcap + t];
  }
  __syncthreads();
  // W[p_l][q_t]
  auto Wlt = [&](int l, int t) { return W[(size_t)sQ[t] * R3 + sP[l]]; };
  const int nk = (rho + 15) / 16;
  for (int k = 0; k < nk; ++k) {
    const int t0 = 16 * k;
    // the chunk's pivot inverses, once each (the diagonal of S_1, and the row
    // scales of S_0), so that no division sits in the serial substitution below
    if (tid < 16) sInv[tid] = t0 + tid < rho ? cinv(Wlt(t0 + tid, t0 + tid)) : mk(1.0);
    __syncthreads();
    // the diagonal blocks: S_0[j][l] = M = W[p_j][q_l] / W[p_j][q_j],
    // S_1[j][l] = N^T = W[p_l][q_j] (j <= l; zero elsewhere and past rho)
    for (int e = tid; e < 512; e += nt) {
      const int side = e >> 8, j = (e >> 4) & 15, l = e & 15;
      cd v = mk(0.0);
      if (j <= l && t0 + l < rho) {
        if (side == 0)
          v = j == l ? mk(1.0) : Wlt(t0 + j, t0 + l) * sInv[j];
        else
          v = Wlt(t0 + l, t0 + j);
      }
      Sd[side][j][l] = v;
      Dk[side][j][l] = mk(0.0);
    }
    __syncthreads();
    // column c of D_k: back substitution S[T_k, T_k] x = e_c, one thread each
    // (the diagonal of S_0 is one, that of S_1 the pivots)
    if (tid < 32) {
      const int side = tid >> 4, c = tid & 15;
      if (t0 + c < rho) {
        Dk[side][c][c] = side == 0 ? mk(1.0) : sInv[c];
        for (int j = c - 1; j >= 0; --j) {
          cd acc = mk(0.0);
          for (int l = j + 1; l <= c; ++l) acc += Sd[side][j][l] * Dk[side][l][c];
          Dk[side][j][c] = -(side == 0 ? acc : acc * sInv[j]);
        }
      }
    }
    __syncthreads();
    const size_t pof = 256 * (size_t)(k * (k + 1) / 2);
    // rows 0..15: D_k
    for (int e = tid; e < 512; e += nt) {
      const int side = e >> 8, r = (e >> 4) & 15, c = e & 15;
      (side == 0 ? PU : PV)[pof + (size_t)r * 16 + c] = Dk[side][r][c];
    }
    // rows 16 + l, l < t0: -S[l, T_k] D_k, one thread per (side, l)
    for (int e = tid; e < 2 * t0; e += nt) {
      const int side = e / t0, l = e - side * t0;
      cd srow[16];
      const cd il = side == 0 ? cinv(Wlt(l, l)) : mk(0.0);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int t = t0 + j < rho ? t0 + j : rho - 1;
        srow[j] = side == 0 ? Wlt(l, t) * il : Wlt(t, l);
      }
      cd* dst = (side == 0 ? PU : PV) + pof + (size_t)(16 + l) * 16;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        cd acc = mk(0.0);
#pragma unroll
        for (int j = 0; j <= c; ++j) acc += srow[j] * Dk[side][j][c];
        dst[c] = -acc;
      }
    }
    __syncthreads();  // Sd and Dk are rewritten by the next chunk
  }
}

// X = [Src | X] P_k chunk by chunk: one wavefront per 48 rows of a block
// (16 row elements of the U side; three 16-row tiles of the product), four
// independent wavefronts per workgroup.  Per step of four inner rows,
// v_mfma_f64_16x16x4f64 twice per tile and half-chunk of eight terms, with
// A the 16 x 4 source entries (lane l: row l % 16, inner row l / 16) and B
// the panel entries in the layout [Re P | Im P] and [-Im P | Re P]
// (lane l: inner row l / 16, term (l % 16) % 8); lane l ends with rows
// l / 16 + 4 v of column l % 16: the real (l % 16 < 8) or imaginary part of
// a term.  The chunk's terms are stored, and their squared norms summed per
// wavefront; the U side also offers the next row element (largest entry of
// the last term among unused rows).  A chunk reads the terms that earlier
// chunks of the same wavefront stored (other lanes' stores): the wavefront
// waits for its stores before the next chunk's loads.
template <bool USIDE>
__global__ __launch_bounds__(256) void k_ws_form_mfma(WsArgs A, const FarBlk* __restrict__ blks,
                                                      AcaState* __restrict__ st, const unsigned* __restrict__ used) {
  __shared__ double rowsq[4][WS_TILE_ROWS];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int task = blockIdx.x * 4 + wv;
  const int ntask = USIDE ? A.tot_tu : A.tot_tv;
  if (task >= ntask) return;  // wavefront-uniform; no barrier below
  const int* off = USIDE ? A.tu_off : A.tv_off;
  const int i = find_seg(off, A.nwarm, task);
  const WsBlk w = A.wb[i];
  const FarBlk B = blks[w.blk];
  const int rho = A.rho[i];
  if (rho == 0) return;
  const int tile = task - off[i];
  const int nrow = USIDE ? 3 * B.m : 3 * B.n;
  const int r0 = tile * WS_TILE_ROWS;
  const int* __restrict__ perm = A.pq + w.pq + (USIDE ? w.rcap : 0);  // q_t (U) or p_t (V)
  const cd* src = A.cross + (USIDE ? w.cc : w.rr);                   // column t: src + perm[t] nrow
  cd* out = USIDE ? B.U : B.V;
  const cd* pan = A.coef + w.co + (USIDE ? 0 : ws_panel_elems(w.rcap));
  double* part = A.part + (USIDE ? w.pu : w.pv) + (size_t)tile * w.rcap;
  const int kr = lane >> 4, n = lane & 15;
  const int nk = (rho + 15) / 16;
  // sources, formed terms and panels through buffer resources (vector
  // memory counter only; every span is far below 4 GiB)
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)src, 0, (unsigned)((size_t)nrow * (USIDE ? 3 * w.nc : 3 * w.nr) * sizeof(cd)), 0x00020000);
  const __amdgpu_buffer_rsrc_t rout =
      __builtin_amdgcn_make_buffer_rsrc((void*)out, 0, (unsigned)((size_t)nrow * rho * sizeof(cd)), 0x00020000);
  const __amdgpu_buffer_rsrc_t rpan = __builtin_amdgcn_make_buffer_rsrc(
      (void*)pan, 0, (unsigned)(ws_panel_elems(w.rcap) * sizeof(cd)), 0x00020000);
  auto bload = [](__amdgpu_buffer_rsrc_t rs, unsigned i) -> cd {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, i * (unsigned)sizeof(cd), 0, 0);
    const double2 d = __builtin_bit_cast(double2, v);
    return cd{d.x, d.y};
  };
  for (int k = 0; k < nk; ++k) {
    const int t0 = 16 * k;
    const unsigned pofs = 256u * (unsigned)(k * (k + 1) / 2);
    wfv4d acc[3][2];
#pragma unroll
    for (int tt = 0; tt < 3; ++tt)
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[tt][h] = wfv4d{0.0, 0.0, 0.0, 0.0};
    const int K = 16 + t0;
    // one step's operands; the next step's are loaded before this step's
    // products
    auto load = [&](int kk, cd (&a)[3], cd& p0, cd& p1) {
      const int kap = kk + kr;
      // inner rows below 16 read the source columns of this chunk's terms
      // (terms past rho read the last one; their panel rows are zero), the
      // rest the terms already formed
      const bool fromsrc = kk < 16;
      const int t = t0 + kap < rho ? t0 + kap : rho - 1;
      const unsigned col = fromsrc ? (unsigned)perm[t] * (unsigned)nrow : (unsigned)(kap - 16) * (unsigned)nrow;
#pragma unroll
      for (int tt = 0; tt < 3; ++tt) {
        const int r = r0 + 16 * tt + n;
        const unsigned i = col + (unsigned)(r < nrow ? r : nrow - 1);
        const cd v = fromsrc ? bload(rsrc, i) : bload(rout, i);
        a[tt] = r < nrow ? v : mk(0.0);
      }
      p0 = bload(rpan, pofs + (unsigned)kap * 16u + (unsigned)(n & 7));
      p1 = bload(rpan, pofs + (unsigned)kap * 16u + 8u + (unsigned)(n & 7));
    };
    // the six accumulators in turn, so that no product waits on the one
    // just issued
    auto mma = [&](const cd (&a)[3], const cd& p0, const cd& p1) {
      double b1[2], b2[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const cd pb = h ? p1 : p0;
        b1[h] = n < 8 ? pb.x : pb.y;
        b2[h] = n < 8 ? -pb.y : pb.x;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int tt = 0; tt < 3; ++tt)
          acc[tt][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[tt].x, b1[h], acc[tt][h], 0, 0, 0);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int tt = 0; tt < 3; ++tt)
          acc[tt][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[tt].y, b2[h], acc[tt][h], 0, 0, 0);
    };
    cd a0[3], a1[3], p00, p01, p10, p11;
    load(0, a0, p00, p01);
    for (int kk = 0; kk < K; kk += 8) {
      if (kk + 4 < K) load(kk + 4, a1, p10, p11);
      mma(a0, p00, p01);
      if (kk + 4 < K) {
        if (kk + 8 < K) load(kk + 8, a0, p00, p01);
        mma(a1, p10, p11);
      }
    }
    // store the chunk's terms; squared norms per term over this tile's rows
    double sq[2] = {0.0, 0.0};
    const int comp = n >> 3;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = t0 + 8 * h + (n & 7);
#pragma unroll
      for (int tt = 0; tt < 3; ++tt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = r0 + 16 * tt + kr + 4 * v;
          if (r < nrow && t < rho) {
            const double x = acc[tt][h][v];
            const unsigned off = ((unsigned)t * (unsigned)nrow + (unsigned)r) * (unsigned)sizeof(cd) + 8u * comp;
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), rout, off, 0, 0);
            sq[h] += x * x;
          }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double q = sq[h];
      q += __shfl_xor(q, 8, 64);
      q += __shfl_xor(q, 16, 64);
      q += __shfl_xor(q, 32, 64);
      if (lane < 8 && t0 + 8 * h + lane < rho) part[t0 + 8 * h + lane] = q;
    }
    if (USIDE && k == nk - 1) {
      // the last term's squared entries per row, then per row element
      const int tl = rho - 1 - t0, hl = tl >> 3, nl = tl & 7;
#pragma unroll
      for (int tt = 0; tt < 3; ++tt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double x = hl ? acc[tt][1][v] : acc[tt][0][v];
          double q = x * x;
          q += __shfl_xor(q, 8, 64);
          if (n == nl) rowsq[wv][16 * tt + kr + 4 * v] = q;
        }
      wave_sync();
      unsigned long long cand = 0ull;
      if (lane < WS_TILE_ROWS / 3) {
        const int a = r0 / 3 + lane;
        if (3 * a < nrow && !(used[B.bitoff + (a >> 5)] & (1u << (a & 31)))) {
          const double e = rowsq[wv][3 * lane] + rowsq[wv][3 * lane + 1] + rowsq[wv][3 * lane + 2];
          cand = pack_best(sqrt(e), a);
        }
      }
      cand = wave_max_u64(cand);
      if (lane == 0 && cand) atomicMax(&st[w.blk].best_row, cand);
    }
    // the next chunk reads these stores (other lanes'): wait for them
    __builtin_amdgcn_s_waitcnt(0);
    wave_sync();
  }
}

// One wavefront per warm block.  The terms are taken in pivot order until
// the stopping test of a cold step holds for one of them,
// |u_t|^2 |v_t|^2 <= tol^2 sum_{l<=t} |u_l|^2 |v_l|^2 (that term is kept, as
// a cold step keeps its last terms), or all of them with keep_all; the
// pivot lists shrink to the elements of the kept pivots.  At least one ordinary step follows, on a row outside
// the cross, so growth of the rank at the new frequency is still detected.
__global__ __launch_bounds__(256) void k_ws_finish(WsArgs A, const FarBlk* __restrict__ blks,
                                                   AcaState* __restrict__ st, const unsigned* __restrict__ used,
                                                   int* __restrict__ plist, int* __restrict__ nlist, double tol) {
  __shared__ unsigned char keep[4][2 * WS_MAXLIST];
  const int wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + wv;
  const int lane = threadIdx.x & 63;
  if (i >= A.nwarm) return;
  const WsBlk w = A.wb[i];
  const FarBlk B = blks[w.blk];
  const int rho = A.rho[i];
  const int ntu = A.tu_off[i + 1] - A.tu_off[i], ntv = A.tv_off[i + 1] - A.tv_off[i];
  const int* Pp = A.pq + w.pq;
  const int* Qp = Pp + w.rcap;
  // running norm estimate over the terms, 64 at a time
  double normS2 = 0.0;
  int kept = rho;
  for (int t0 = 0; t0 < rho && kept == rho; t0 += 64) {
    const int t = t0 + lane;
    double term = 0.0;
    if (t < rho) {
      double nu = 0.0, nv = 0.0;
      for (int q = 0; q < ntu; ++q) nu += A.part[w.pu + (size_t)q * w.rcap + t];
      for (int q = 0; q < ntv; ++q) nv += A.part[w.pv + (size_t)q * w.rcap + t];
      term = nu * nv;
    }
    // inclusive prefix sum of the terms over the lanes
    double inc = term;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    const bool stop = !A.keep_all && t < rho && term <= tol * tol * (normS2 + inc);
    const unsigned long long bal = __ballot(stop);
    if (bal) {
      const int first = __ffsll((long long)bal) - 1;
      kept = t0 + first + 1;
      normS2 += __shfl(inc, first, 64);
    } else {
      normS2 += __shfl(inc, 63, 64);
    }
  }
  // pivot lists of the next frequency: elements of the kept pivots
  unsigned char* kr = keep[wv];
  unsigned char* kc = keep[wv] + WS_MAXLIST;
  for (int q = lane; q < WS_MAXLIST; q += 64) kr[q] = kc[q] = 0;
  wave_sync();
  for (int t = lane; t < kept; t += 64) {
    kr[Pp[t] / 3] = 1;
    kc[Qp[t] / 3] = 1;
  }
  wave_sync();
  // the lists compacted by the whole wavefront: every entry read first (and
  // waited for), then each kept one stored at its rank among the kept
  int* rl = plist + B.poff;
  int* cl = plist + B.poff + B.m;
  constexpr int NQ = (WS_MAXLIST + 63) / 64;
  int rv[NQ], cv[NQ];
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int q = lane + 64 * u;
    rv[u] = q < w.nr ? rl[q] : 0;
    cv[u] = q < w.nc ? cl[q] : 0;
  }
  __builtin_amdgcn_s_waitcnt(0);
  wave_sync();
  int nr = 0, nc = 0;
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int q = lane + 64 * u;
    const bool kr_ = q < w.nr && kr[q], kc_ = q < w.nc && kc[q];
    const unsigned long long br = __ballot(kr_), bc = __ballot(kc_);
    const unsigned long long below = (1ull << lane) - 1ull;
    if (kr_) rl[nr + __popcll(br & below)] = rv[u];
    if (kc_) cl[nc + __popcll(bc & below)] = cv[u];
    nr += __popcll(br);
    nc += __popcll(bc);
  }
  if (lane != 0) return;
  nlist[2 * w.blk] = nr;
  nlist[2 * w.blk + 1] = nc;
  atomicAdd(&A.cnt[0], (unsigned long long)rho);
  atomicAdd(&A.cnt[1], (unsigned long long)kept);
  AcaState s = st[w.blk];
  s.k = kept;
  s.normS2 = normS2;
  if (kept >= 3 * min(B.m, B.n)) {
    s.status = ACA_DONE;  // full rank
  } else if (kept + 3 > B.kcap) {
    s.status = ACA_OVERFLOW;
  } else if (kept == 0 || s.best_row == 0ull) {
    // no candidate from the last term: the first row outside the cross
    int a = -1;
    const unsigned* u = used + B.bitoff;
    for (int q = 0; q < (B.m + 31) / 32 && a < 0; ++q) {
      const unsigned f = ~u[q];
      if (f) a = 32 * q + __ffs(f) - 1;
    }
    if (a < 0 || a >= B.m)
      s.status = ACA_DONE;  // every row is in the cross
    else
      s.astar = a;
  } else {
    s.astar = 0x7fffffff - (int)(s.best_row & 0xffffffffu);
  }
  s.best_row = 0ull;
  st[w.blk] = s;
}

void launch_ws(const WsArgs& A, const AcaWork& W, const DevGeom& g, const KParams& P, double tol, hipStream_t s,
               const WsSide& side) {
  if (A.nwarm <= 0) return;
  hipLaunchKernelGGL(k_ws_init, dim3((A.nwarm + 255) / 256), dim3(256), 0, s, A.wb, A.nwarm, W.blks, W.st, W.used,
                     W.plist);
  if (A.tot_er > 0)
    hipLaunchKernelGGL(k_ws_eval_rows, dim3((A.tot_er + 255) / 256), dim3(256), 0, s, A.wb, A.nwarm, A.er_off, W.blks,
                       W.plist, A.cross, g, P);
  if (A.tot_ec > 0)
    hipLaunchKernelGGL(k_ws_eval_cols, dim3((A.tot_ec + 255) / 256), dim3(256), 0, s, A.wb, A.nwarm, A.ec_off, W.blks,
                       W.plist, A.cross, g, P);
  // the elimination in seven size classes: cores of at most 64 x 64 and
  // 128 x 128 in registers; the rest with W of up to 1024 entries and 64
  // rows with two wavefronts, of up to 2304, 4480 and 8960 entries with
  // eight, all in LDS, larger in global memory
  const int nt = 64 * WS_LU_NW, ntl = 64 * WS_LU_NW_LDS;
  const int* lst = A.lu_list;
  // classes 0..4 on the side stream when there is one: it starts after the
  // cross evaluation and the caller's stream waits for it before the panels
  const bool fork = side.stream && A.n_lu[0] + A.n_lu[1] + A.n_lu[2] + A.n_lu[3] + A.n_lu[4] > 0;
  const hipStream_t s0 = s;
  if (fork) {
    EWBEM_HIP_CHECK(hipEventRecord(side.fork, s0));
    EWBEM_HIP_CHECK(hipStreamWaitEvent(side.stream, side.fork, 0));
    s = side.stream;
  }
  if (A.n_lu[0] > 0)
    hipLaunchKernelGGL((k_ws_lu<WS_LDS_SMALL, WS_LU_NR_LDS, WS_LU_NW_LDS>), dim3(A.n_lu[0]), dim3(ntl), 0, s, A.wb,
                       lst, W.blks, W.plist, A.cross, A.pq, A.rho, A.stop2);
  lst += A.n_lu[0];
  if (A.n_lu[1] > 0)
    hipLaunchKernelGGL((k_ws_lu<WS_LDS_MID, WS_LU_NR_LDS, WS_LU_NW_LDS>), dim3(A.n_lu[1]), dim3(ntl), 0, s, A.wb,
                       lst, W.blks, W.plist, A.cross, A.pq, A.rho, A.stop2);
  lst += A.n_lu[1];
  if (A.n_lu[2] > 0)
    hipLaunchKernelGGL((k_ws_lu<WS_LDS_LARGE, WS_LU_NR_LDS, WS_LU_NW_LDS>), dim3(A.n_lu[2]), dim3(ntl), 0, s, A.wb,
                       lst, W.blks, W.plist, A.cross, A.pq, A.rho, A.stop2);
  lst += A.n_lu[2];
  if (A.n_lu[3] > 0)
    hipLaunchKernelGGL((k_ws_lu<0, (3 * WS_MAXLIST + 63) / 64, WS_LU_NW>), dim3(A.n_lu[3]), dim3(nt), 0, s, A.wb, lst,
                       W.blks, W.plist, A.cross, A.pq, A.rho, A.stop2);
  lst += A.n_lu[3];
  if (A.n_lu[4] > 0)
    hipLaunchKernelGGL((k_ws_lu<WS_LDS_TINY, 1, 2>), dim3(A.n_lu[4]), dim3(128), 0, s, A.wb, lst, W.blks, W.plist,
                       A.cross, A.pq, A.rho, A.stop2);
  lst += A.n_lu[4];
  if (fork) {
    EWBEM_HIP_CHECK(hipEventRecord(side.join, s));
    s = s0;
  }
  // cores in registers: 4 x 16 columns of 64 rows, 8 x 16 columns of 128 rows
  if (A.n_lu[5] > 0)
    hipLaunchKernelGGL((k_ws_lu_reg<WS_REG_SMALL / 16, 16, 1>), dim3(A.n_lu[5]), dim3(WS_REG_SMALL / 16 * 64), 0,
                       s, A.wb, lst, W.blks, W.plist, A.cross, A.pq, A.rho, A.stop2);
  lst += A.n_lu[5];
  if (A.n_lu[6] > 0)
    hipLaunchKernelGGL((k_ws_lu_reg<WS_REG_LARGE / 16, 16, 2>), dim3(A.n_lu[6]), dim3(WS_REG_LARGE / 16 * 64), 0,
                       s, A.wb, lst, W.blks, W.plist, A.cross, A.pq, A.rho, A.stop2);
  if (fork) EWBEM_HIP_CHECK(hipStreamWaitEvent(s, side.join, 0));
  hipLaunchKernelGGL(k_ws_panels, dim3(A.nwarm), dim3(256), 0, s, A);
  hipLaunchKernelGGL((k_ws_form_mfma<true>), dim3((A.tot_tu + 3) / 4), dim3(256), 0, s, A, W.blks, W.st, W.used);
  hipLaunchKernelGGL((k_ws_form_mfma<false>), dim3((A.tot_tv + 3) / 4), dim3(256), 0, s, A, W.blks, W.st, W.used);
  hipLaunchKernelGGL(k_ws_finish, dim3((A.nwarm + 3) / 4), dim3(256), 0, s, A, W.blks, W.st, W.used, W.plist,
                     W.nlist, tol);
}

}  // namespace ewbem
