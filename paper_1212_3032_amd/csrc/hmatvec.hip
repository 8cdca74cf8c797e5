// Hierarchical-matrix matvec y = A x, A = sum_near D + sum_far U V^T.
//
// Phase 1 (k_far_vt): z_b = V_b^T x_sigma for every far block, one
// wavefront per group of up to four factor columns; each column is read
// once, coalesced, and reduced across the wavefront.
// Phase 2 (k_hmv): row ownership by leaf cluster.  Every leaf's rows see a
// panel made of its dense near blocks (times x) and the matching row slices
// of the U factors of the far blocks above it (times z).  The panel is cut
// into tasks of similar column counts; one workgroup streams one task
// (column-major, coalesced along rows) and writes a partial result.
// k_hmv_reduce sums the partials of each leaf in a fixed order, so the
// result is deterministic (no atomics).
#include "aca.hpp"

namespace ewbem {

__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename TS>
__global__ __launch_bounds__(256) void k_far_vt(const VtTask* __restrict__ tasks, int ntask,
                                                const cd* __restrict__ x, cd* __restrict__ z) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= ntask) return;
  const VtTask T = tasks[t];
  const TS* __restrict__ V = (const TS*)T.V;
  const cd* __restrict__ xs = x + T.x0;
  cd a0 = mk(0.0), a1 = mk(0.0), a2 = mk(0.0), a3 = mk(0.0);
  const int C = T.C;
  const int nc = T.ncol;
  // columns past ncol read column 0 again (in bounds) and are discarded
  const TS* __restrict__ V1 = V + (size_t)(nc > 1 ? 1 : 0) * C;
  const TS* __restrict__ V2 = V + (size_t)(nc > 2 ? 2 : 0) * C;
  const TS* __restrict__ V3 = V + (size_t)(nc > 3 ? 3 : 0) * C;
  for (int c = lane; c < C; c += 64) {
    const cd xv = xs[c];
    a0 += to_cd(V[c]) * xv;
    a1 += to_cd(V1[c]) * xv;
    a2 += to_cd(V2[c]) * xv;
    a3 += to_cd(V3[c]) * xv;
  }
  a0.x = wsum64(a0.x);
  a0.y = wsum64(a0.y);
  a1.x = wsum64(a1.x);
  a1.y = wsum64(a1.y);
  a2.x = wsum64(a2.x);
  a2.y = wsum64(a2.y);
  a3.x = wsum64(a3.x);
  a3.y = wsum64(a3.y);
  // every lane holds the sums; lane 0 stores them (no lane-indexed select,
  // which the compiler would place in scratch memory)
  if (lane == 0) {
    cd* zz = z + T.zidx;
    zz[0] = a0;
    if (nc > 1) zz[1] = a1;
    if (nc > 2) zz[2] = a2;
    if (nc > 3) zz[3] = a3;
  }
}

void launch_far_vt(const VtTask* tasks, int ntask, int store_c64, const cd* x, cd* z,
                   hipStream_t st) {
  if (ntask <= 0) return;
  dim3 grid((ntask + 3) / 4);
  if (store_c64)
    hipLaunchKernelGGL(k_far_vt<cf>, grid, dim3(256), 0, st, tasks, ntask, x, z);
  else
    hipLaunchKernelGGL(k_far_vt<cd>, grid, dim3(256), 0, st, tasks, ntask, x, z);
}

template <typename TS>
__device__ __forceinline__ cd panel_dot(const TS* __restrict__ A, const cd* __restrict__ src, int ld,
                                        int ncols, int r, int g, int G) {
  cd acc = mk(0.0);
  int c = g;
  for (; c + 3 * G < ncols; c += 4 * G) {
    const cd a0 = to_cd(A[(size_t)c * ld + r]);
    const cd a1 = to_cd(A[(size_t)(c + G) * ld + r]);
    const cd a2 = to_cd(A[(size_t)(c + 2 * G) * ld + r]);
    const cd a3 = to_cd(A[(size_t)(c + 3 * G) * ld + r]);
    acc += a0 * src[c];
    acc += a1 * src[c + G];
    acc += a2 * src[c + 2 * G];
    acc += a3 * src[c + 3 * G];
  }
  for (; c < ncols; c += G) acc += to_cd(A[(size_t)c * ld + r]) * src[c];
  return acc;
}

__global__ __launch_bounds__(256) void k_hmv(const RowTask* __restrict__ tasks, const Seg* __restrict__ segs,
                                             const cd* __restrict__ x, const cd* __restrict__ z,
                                             cd* __restrict__ partial) {
  const RowTask T = tasks[blockIdx.x];
  const int rows_pad = (T.rows + 63) & ~63;
  const int G = 256 / rows_pad;
  const int r = threadIdx.x % rows_pad, g = threadIdx.x / rows_pad;
  __shared__ cd red[256];
  cd acc = mk(0.0);
  if (g < G && r < T.rows) {
    for (int s = T.s0; s < T.s1; ++s) {
      const Seg S = segs[s];
      const cd* src = ((S.flags & SEG_FROM_Z) ? z : x) + S.src;
      if (S.flags & SEG_C64)
        acc += panel_dot((const cf*)S.A, src, S.ld, S.ncols, r, g, G);
      else
        acc += panel_dot((const cd*)S.A, src, S.ld, S.ncols, r, g, G);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < T.rows) {
    cd s = red[threadIdx.x];
    for (int q = 1; q < G; ++q) s += red[q * rows_pad + threadIdx.x];
    partial[(size_t)blockIdx.x * HMV_MAXROWS + threadIdx.x] = s;
  }
}

void launch_hmv(const RowTask* tasks, int ntask, const Seg* segs, const cd* x, const cd* z,
                cd* partial, hipStream_t st) {
  if (ntask > 0) hipLaunchKernelGGL(k_hmv, dim3(ntask), dim3(256), 0, st, tasks, segs, x, z, partial);
}

__global__ void k_hmv_reduce(const LeafRange* __restrict__ leaves, const cd* __restrict__ partial,
                             cd* __restrict__ y) {
  const LeafRange L = leaves[blockIdx.x];
  const int r = threadIdx.x;
  if (r >= L.rows) return;
  cd s = mk(0.0);
  for (int t = L.t0; t < L.t1; ++t) s += partial[(size_t)t * HMV_MAXROWS + r];
  y[L.row0 + r] = s;
}

void launch_hmv_reduce(const LeafRange* leaves, int nleaf, const cd* partial, cd* y,
                       hipStream_t st) {
  if (nleaf > 0)
    hipLaunchKernelGGL(k_hmv_reduce, dim3(nleaf), dim3(HMV_MAXROWS), 0, st, leaves, partial, y);
}

}  // namespace ewbem
