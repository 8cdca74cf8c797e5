// Hierarchical-matrix matvec y = A x, A = sum_near D + sum_far U V^T.
//
// Phase 1 (k_far_vt): z_b = V_b^T x_sigma for every far block, one
// wavefront per group of up to 2, 4 or 8 factor columns (tuned); each column
// is read once, coalesced, and reduced across the wavefront.
// Phase 2 (k_hmv): row ownership by leaf cluster.  Every leaf's rows see a
// panel made of its dense near blocks (times x) and the matching row slices
// of the U factors of the far blocks above it (times z).  The panel is cut
// into tasks of similar column counts; one workgroup streams one task
// (column-major, coalesced along rows) and writes a partial result.
// k_hmv_reduce sums the partials of each leaf in a fixed order, so the
// result is deterministic (no atomics).  All three take one to four
// right-hand sides (the extrapolated guess applies the operator to several
// earlier solutions at once).
#include "aca.hpp"

namespace ewbem {

__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One entry of a panel through a buffer resource: counted by the vector
// memory counter only (a flat load would also hold every wait on the scalar
// x loads), and bounded by the resource's size.  POL is the load's cache
// policy: 0, or CPOL_NT (the non-temporal hint for data read once: the
// matvec's complex128 panels and phase-1 factor columns on the vector units,
// measured 9% faster with it; complex64 panels measured 1% slower, and the
// matrix-core products, which touch each line twice, 6% slower).
constexpr int CPOL_NT = 2;
template <typename TS, int POL = 0>
__device__ __forceinline__ cd panel_load(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  if constexpr (sizeof(TS) == 16) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, POL);
    const double2 d = __builtin_bit_cast(double2, v);
    return cd{d.x, d.y};
  } else {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, POL);
    const float2 f = __builtin_bit_cast(float2, v);
    return cd{(double)f.x, (double)f.y};
  }
}

// NR right-hand sides at once (columns of x, z, partial and y, strides ldx,
// ldz, ldp, ldy): every factor and near-block entry is loaded once and
// multiplied against the NR vectors.  Phase 1 takes NC factor columns per
// wavefront (a tuning choice).
// Columns per pass: with several right-hand sides the NC x NR accumulators
// would crowd the registers (and the occupancy), so a task's columns are
// taken in passes of NCS, the x slice being re-read from cache each pass.
template <int NR, int NC>
constexpr int far_vt_pass_cols() {
  return NR == 1 ? NC : (NR == 2 ? (NC < 4 ? NC : 4) : 2);
}

template <typename TS, int NR, int NC>
__global__ __launch_bounds__(256) void k_far_vt(const VtTask* __restrict__ tasks, int ntask,
                                                const cd* __restrict__ x, long long ldx, cd* __restrict__ z,
                                                long long ldz) {
  constexpr int NCS = far_vt_pass_cols<NR, NC>();
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= ntask) return;
  const VtTask T = tasks[t];
  const TS* __restrict__ V = (const TS*)T.V;
  const cd* __restrict__ xs = x + T.x0;
  const int C = T.C;
  const int nc = T.ncol;
  for (int k0 = 0; k0 < NC && k0 < nc; k0 += NCS) {
    cd a[NCS][NR];
#pragma unroll
    for (int k = 0; k < NCS; ++k)
#pragma unroll
      for (int q = 0; q < NR; ++q) a[k][q] = mk(0.0);
    // columns past ncol read column 0 again (in bounds) and are discarded
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)V, 0, (unsigned)((size_t)nc * C * sizeof(TS)), 0x00020000);
    unsigned Vc[NCS];
#pragma unroll
    for (int k = 0; k < NCS; ++k) Vc[k] = (unsigned)(nc > k0 + k ? k0 + k : 0) * (unsigned)C;
    for (int c = lane; c < C; c += 64) {
      cd v[NCS];
#pragma unroll
      for (int k = 0; k < NCS; ++k) v[k] = panel_load<TS, sizeof(TS) == 16 ? CPOL_NT : 0>(rs, (Vc[k] + (unsigned)c) * (unsigned)sizeof(TS));
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const cd xv = xs[c + q * ldx];
#pragma unroll
        for (int k = 0; k < NCS; ++k) a[k][q] += v[k] * xv;
      }
    }
#pragma unroll
    for (int k = 0; k < NCS; ++k)
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        a[k][q].x = wsum64(a[k][q].x);
        a[k][q].y = wsum64(a[k][q].y);
      }
    // every lane holds the sums; lane 0 stores them (no lane-indexed select,
    // which the compiler would place in scratch memory)
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        cd* zz = z + T.zidx + q * ldz + k0;
#pragma unroll
        for (int k = 0; k < NCS; ++k)
          if (nc > k0 + k) zz[k] = a[k][q];
      }
    }
  }
}

// Phase 1 for eight right-hand sides on the matrix cores: one wavefront per
// task of up to 16 factor columns j (a task list of its own).  Per four rows
// c of the factor, v_mfma_f64_16x16x4f64 twice with A the 16 x 4 block
// V(c, j)^T (lane l: column j = l % 16, row index l / 16) and B the x
// entries (lane l: the same row, output column n = l % 16):
//   Z += Re(V^T) [Re X | Im X] + Im(V^T) [-Im X | Re X] = [Re V^T X | Im V^T X].
// Lane l ends with Z rows (factor columns) l / 16 + 4 v of output column
// l % 16 (real parts of the eight products, then imaginary parts).
typedef double fvt_v4d __attribute__((ext_vector_type(4)));

template <typename TS>
__global__ __launch_bounds__(256) void k_far_vt_mfma8(const VtTask* __restrict__ tasks, int ntask,
                                                      const cd* __restrict__ x, long long ldx, cd* __restrict__ z,
                                                      long long ldz) {
  const int t = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform task
  const int lane = threadIdx.x & 63;
  if (t >= ntask) return;
  const VtTask T = tasks[t];
  const TS* __restrict__ V = (const TS*)T.V;
  const cd* __restrict__ xs = x + T.x0;
  const int C = T.C, nc = T.ncol;
  const int j = lane & 15, kr = lane >> 4, q = j & 7;
  const bool jv = j < nc;
  // the task's factor columns through a buffer resource (vector memory
  // counter only); columns past ncol read column 0 and multiply zero
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)V, 0, (unsigned)((size_t)nc * C * sizeof(TS)), 0x00020000);
  const unsigned vcol = (unsigned)(jv ? j : 0) * (unsigned)C;
  const cd* __restrict__ xq = xs + q * ldx;
  // four accumulators (row half h, real or imaginary factor part), summed
  // at the end, so that no product waits on the one just issued
  fvt_v4d acc4[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc4[u] = fvt_v4d{0.0, 0.0, 0.0, 0.0};
  // a step is eight rows, two products: product h pairs lane row kr with
  // factor row c0 + 2 kr + h, so a lane's two rows are adjacent in memory
  // (rows past C read row C - 1 and are zeroed)
  auto load = [&](int c0, cd (&a)[2], cd (&xv)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = c0 + 2 * kr + h;
      const bool cv = c < C;
      const int cc = cv ? c : C - 1;
      const cd av = panel_load<TS>(rs, (vcol + (unsigned)cc) * (unsigned)sizeof(TS));
      const cd xx = xq[cc];
      a[h] = (jv && cv) ? av : mk(0.0);
      xv[h] = cv ? xx : mk(0.0);
    }
  };
  auto mma = [&](const cd (&a)[2], const cd (&xv)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double b1 = j < 8 ? xv[h].x : xv[h].y;
      const double b2 = j < 8 ? -xv[h].y : xv[h].x;
      acc4[2 * h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h].x, b1, acc4[2 * h], 0, 0, 0);
      acc4[2 * h + 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h].y, b2, acc4[2 * h + 1], 0, 0, 0);
    }
  };
  // three steps in flight: the loads of steps s + 1 and s + 2 are issued
  // before the products of step s
  cd a0[2], x0[2], a1[2], x1[2], a2[2], x2[2];
  load(0, a0, x0);
  if (8 < C) load(8, a1, x1);
  for (int c0 = 0; c0 < C; c0 += 24) {
    if (c0 + 16 < C) load(c0 + 16, a2, x2);
    mma(a0, x0);
    if (c0 + 8 < C) {
      if (c0 + 24 < C) load(c0 + 24, a0, x0);
      mma(a1, x1);
    }
    if (c0 + 16 < C) {
      if (c0 + 32 < C) load(c0 + 32, a1, x1);
      mma(a2, x2);
    }
  }
  const fvt_v4d acc = (acc4[0] + acc4[2]) + (acc4[1] + acc4[3]);
  const int comp = j >> 3;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = kr + 4 * v;
    if (i < nc) ((double*)(z + T.zidx + i + q * ldz))[comp] = acc[v];
  }
}

template <int NR, int NC>
void far_vt_nr(const VtTask* tasks, int ntask, int store_c64, const cd* x, long long ldx, cd* z, long long ldz,
               hipStream_t st) {
  dim3 grid((ntask + 3) / 4);
  if (store_c64)
    hipLaunchKernelGGL((k_far_vt<cf, NR, NC>), grid, dim3(256), 0, st, tasks, ntask, x, ldx, z, ldz);
  else
    hipLaunchKernelGGL((k_far_vt<cd, NR, NC>), grid, dim3(256), 0, st, tasks, ntask, x, ldx, z, ldz);
}

template <int NC>
void far_vt_nc(const VtTask* tasks, int ntask, int store_c64, const cd* x, long long ldx, int nrhs, cd* z,
               long long ldz, hipStream_t st) {
  switch (nrhs) {
    case 1: far_vt_nr<1, NC>(tasks, ntask, store_c64, x, ldx, z, ldz, st); break;
    case 2: far_vt_nr<2, NC>(tasks, ntask, store_c64, x, ldx, z, ldz, st); break;
    case 3: far_vt_nr<3, NC>(tasks, ntask, store_c64, x, ldx, z, ldz, st); break;
    case 4: far_vt_nr<4, NC>(tasks, ntask, store_c64, x, ldx, z, ldz, st); break;
    case 5: far_vt_nr<5, NC>(tasks, ntask, store_c64, x, ldx, z, ldz, st); break;
    case 6: far_vt_nr<6, NC>(tasks, ntask, store_c64, x, ldx, z, ldz, st); break;
    case 7: far_vt_nr<7, NC>(tasks, ntask, store_c64, x, ldx, z, ldz, st); break;
    case 8: far_vt_nr<8, NC>(tasks, ntask, store_c64, x, ldx, z, ldz, st); break;
    default: throw ApiError(-1, "matvec: 1 to 8 right-hand sides");
  }
}

void launch_far_vt(const VtTask* tasks, int ntask, int cols_per_wave, int store_c64, const cd* x, long long ldx,
                   int nrhs, cd* z, long long ldz, hipStream_t st, int mfma) {
  if (ntask <= 0) return;
  if (nrhs == 8 && mfma) {
    dim3 grid((ntask + 3) / 4);
    if (store_c64)
      hipLaunchKernelGGL((k_far_vt_mfma8<cf>), grid, dim3(256), 0, st, tasks, ntask, x, ldx, z, ldz);
    else
      hipLaunchKernelGGL((k_far_vt_mfma8<cd>), grid, dim3(256), 0, st, tasks, ntask, x, ldx, z, ldz);
    return;
  }
  switch (cols_per_wave) {
    case 2: far_vt_nc<2>(tasks, ntask, store_c64, x, ldx, nrhs, z, ldz, st); break;
    case 4: far_vt_nc<4>(tasks, ntask, store_c64, x, ldx, nrhs, z, ldz, st); break;
    case 8: far_vt_nc<8>(tasks, ntask, store_c64, x, ldx, nrhs, z, ldz, st); break;
    default: throw ApiError(-1, "matvec: 2, 4 or 8 factor columns per wavefront");
  }
}

// acc[q] += sum_c A[c, r] x(c, q) over the columns c = g, g + G, ... of a
// column-major panel (ld rows; its span below 4 GiB, checked on the host),
// with x(c, q) = src[c + q lds], or, with XL, src[c NR + q] (a slice staged
// in LDS).  Four columns per step; the next step's four entries are loaded
// before this step's products, so their latency overlaps the arithmetic
// (the products are summed in column order either way).
template <typename TS, int NR, bool XL = false>
__device__ __forceinline__ void panel_dot(const TS* __restrict__ A, const cd* __restrict__ src, long long lds,
                                          int ld, int ncols, int r, int g, int G, cd (&acc)[NR]) {
  auto xv = [&](int c, int q) -> cd { return XL ? src[c * NR + q] : src[c + q * lds]; };
  const unsigned span = (unsigned)(((size_t)(ncols - 1) * ld + ld) * sizeof(TS));
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)A, 0, span, 0x00020000);
  const unsigned es = sizeof(TS);
  const unsigned stride = (unsigned)G * (unsigned)ld * es;
  int c = g;
  unsigned off = ((unsigned)c * (unsigned)ld + (unsigned)r) * es;
  // one step: load the next four entries into nxt, then the products of the
  // current four in cur; the two register sets alternate, so no copy has to
  // wait for a load.  The loads are unconditional (no branch for the wait
  // counts to merge): past the panel's span a buffer load returns zero, and
  // those values are not used.
  auto step = [&](cd (&cur)[4], cd (&nxt)[4]) -> bool {
    const int cn = c + 4 * G;
    const unsigned offn = off + 4 * stride;
    const bool more = cn + 3 * G < ncols;
#pragma unroll
    for (int i = 0; i < 4; ++i) nxt[i] = panel_load<TS, sizeof(TS) == 16 ? CPOL_NT : 0>(rs, offn + i * stride);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      acc[q] += cur[0] * xv(c, q);
      acc[q] += cur[1] * xv(c + G, q);
      acc[q] += cur[2] * xv(c + 2 * G, q);
      acc[q] += cur[3] * xv(c + 3 * G, q);
    }
    c = cn;
    off = offn;
    return more;
  };
  if (c + 3 * G < ncols) {
    cd a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = panel_load<TS, sizeof(TS) == 16 ? CPOL_NT : 0>(rs, off + i * stride);
    while (step(a, b) && step(b, a)) {
    }
  }
  for (; c < ncols; c += G, off += stride) {
    const cd a0 = panel_load<TS, sizeof(TS) == 16 ? CPOL_NT : 0>(rs, off);
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] += a0 * xv(c, q);
  }
}

// Columns of x staged in LDS per pass, for four or more right-hand sides
// (their x loads would otherwise be NR scalar loads per column, which miss
// the small scalar cache when many waves read different segments).
constexpr int HMV_XCH = 64;

template <int NR>
__global__ __launch_bounds__(256) void k_hmv(const RowTask* __restrict__ tasks, const Seg* __restrict__ segs,
                                             const cd* __restrict__ x, long long ldx, const cd* __restrict__ z,
                                             long long ldz, cd* __restrict__ partial, long long ldp) {
  const RowTask T = tasks[blockIdx.x];
  const int rows_pad = (T.rows + 63) & ~63;
  const int G = 256 / rows_pad;
  // rows_pad is a multiple of 64, so a wavefront's threads share g: made
  // explicit, it lets every x load of the panel loop be one uniform load
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x / rows_pad);
  const int r = threadIdx.x - g * rows_pad;
  __shared__ cd red[NR][256];
  cd acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = mk(0.0);
  const bool active = g < G && r < T.rows;
  if constexpr (NR >= 4) {
    // x in chunks of HMV_XCH columns through LDS; every thread takes part in
    // the staging and reaches every barrier (segments and chunks are the
    // same for the whole workgroup)
    __shared__ cd xs[HMV_XCH * NR];
    for (int s = T.s0; s < T.s1; ++s) {
      const Seg S = segs[s];
      const bool fz = (S.flags & SEG_FROM_Z) != 0;
      const cd* src = (fz ? z : x) + S.src;
      const long long lds = fz ? ldz : ldx;
      for (int c0 = 0; c0 < S.ncols; c0 += HMV_XCH) {
        const int nch = min(HMV_XCH, S.ncols - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < nch * NR; i += blockDim.x) {
          const int q = i / nch, cc = i - q * nch;
          xs[cc * NR + q] = src[c0 + cc + q * lds];
        }
        __syncthreads();
        if (active) {
          if (S.flags & SEG_C64)
            panel_dot<cf, NR, true>((const cf*)S.A + (size_t)c0 * S.ld, xs, 0, S.ld, nch, r, g, G, acc);
          else
            panel_dot<cd, NR, true>((const cd*)S.A + (size_t)c0 * S.ld, xs, 0, S.ld, nch, r, g, G, acc);
        }
      }
    }
  } else if (active) {
    for (int s = T.s0; s < T.s1; ++s) {
      const Seg S = segs[s];
      const bool fz = (S.flags & SEG_FROM_Z) != 0;
      const cd* src = (fz ? z : x) + S.src;
      const long long lds = fz ? ldz : ldx;
      if (S.flags & SEG_C64)
        panel_dot<cf, NR>((const cf*)S.A, src, lds, S.ld, S.ncols, r, g, G, acc);
      else
        panel_dot<cd, NR>((const cd*)S.A, src, lds, S.ld, S.ncols, r, g, G, acc);
    }
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  if (threadIdx.x < T.rows) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      cd s = red[q][threadIdx.x];
      for (int k = 1; k < G; ++k) s += red[q][k * rows_pad + threadIdx.x];
      partial[q * ldp + (size_t)blockIdx.x * HMV_MAXROWS + threadIdx.x] = s;
    }
  }
}

// Phase 2 for eight right-hand sides on the matrix cores.  A task's rows
// form up to twelve tiles of 16; wave w of the four takes tiles w, w + 4,
// w + 8.  Per step of four panel columns and tile, v_mfma_f64_16x16x4f64
// twice: with A the tile's 16 x 4 entries (lane l: row l % 16, column
// l / 16) and B the x entries (lane l: column l / 16, output column
// n = l % 16, read directly: no staging, no barrier),
//   C += Re(A) [Re X | Im X] + Im(A) [-Im X | Re X] = [Re AX | Im AX],
// the 16 output columns holding the real parts of the eight products, then
// their imaginary parts.  Lane l holds C rows l / 16 + 4 v, v < 4, of
// output column l % 16 (the layout of this instruction's result, checked on
// the device).
typedef double hmv_v4d __attribute__((ext_vector_type(4)));

// acc[tile] += panel(tile rows, columns of one segment) X(columns, 8) with
// the x entries read directly (lane l: column l / 16, vector (l % 16) % 8);
// the next step's four columns are loaded before this step's products.
template <typename TS>
__device__ __forceinline__ void seg_mfma(const void* A, int ld, int rows, int ncols, const cd* src, long long lds,
                                         int lane, int w, hmv_v4d (&acc)[3]) {
  const int kr = lane >> 4, n = lane & 15;
  const cd* __restrict__ xq = src + (n & 7) * lds;
  // the panel through a buffer resource (vector memory counter only; its
  // span is below 4 GiB, checked on the host); columns past the segment and
  // rows past the task read an in-bounds entry and are zeroed
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)A, 0, (unsigned)(((size_t)(ncols - 1) * ld + rows) * sizeof(TS)), 0x00020000);
  auto load = [&](int c0, cd (&a)[3], cd& xv) {
    const int col = c0 + kr;
    const bool cv = col < ncols;
    const int cc = cv ? col : ncols - 1;
    const unsigned cb = (unsigned)cc * (unsigned)ld;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int row = 16 * (w + 4 * q) + n;
      const cd v = panel_load<TS>(rs, (cb + (unsigned)(row < rows ? row : rows - 1)) * (unsigned)sizeof(TS));
      a[q] = (cv && row < rows) ? v : mk(0.0);
    }
    const cd xx = xq[cc];
    xv = cv ? xx : mk(0.0);
  };
  // the three accumulators in turn, so that no product waits on the one
  // just issued
  auto mma = [&](const cd (&a)[3], const cd& xv) {
    const double b1 = n < 8 ? xv.x : xv.y;
    const double b2 = n < 8 ? -xv.y : xv.x;
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].x, b1, acc[q], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].y, b2, acc[q], 0, 0, 0);
  };
  cd a0[3], a1[3], x0, x1;
  load(0, a0, x0);
  for (int c0 = 0; c0 < ncols; c0 += 8) {
    if (c0 + 4 < ncols) load(c0 + 4, a1, x1);
    mma(a0, x0);
    if (c0 + 4 < ncols) {
      if (c0 + 8 < ncols) load(c0 + 8, a0, x0);
      mma(a1, x1);
    }
  }
}

__global__ __launch_bounds__(256) void k_hmv_mfma8(const RowTask* __restrict__ tasks, const Seg* __restrict__ segs,
                                                   const cd* __restrict__ x, long long ldx,
                                                   const cd* __restrict__ z, long long ldz,
                                                   cd* __restrict__ partial, long long ldp) {
  const RowTask T = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  hmv_v4d acc[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) acc[q] = hmv_v4d{0.0, 0.0, 0.0, 0.0};
  // a wavefront whose tiles all lie past the task's rows has nothing to do
  if (16 * w < T.rows) {
    for (int s = T.s0; s < T.s1; ++s) {
      const Seg S = segs[s];
      const bool fz = (S.flags & SEG_FROM_Z) != 0;
      const cd* src = (fz ? z : x) + S.src;
      const long long lds = fz ? ldz : ldx;
      if (S.flags & SEG_C64)
        seg_mfma<cf>(S.A, S.ld, T.rows, S.ncols, src, lds, lane, w, acc);
      else
        seg_mfma<cd>(S.A, S.ld, T.rows, S.ncols, src, lds, lane, w, acc);
    }
  }
  const int j = lane & 15, q = j & 7, comp = j >> 3;
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * (w + 4 * t) + (lane >> 4) + 4 * v;
      if (row < T.rows) {
        double* p = (double*)(partial + q * ldp + (size_t)blockIdx.x * HMV_MAXROWS + row);
        p[comp] = acc[t][v];
      }
    }
}

void launch_hmv(const RowTask* tasks, int ntask, const Seg* segs, const cd* x, long long ldx, int nrhs,
                const cd* z, long long ldz, cd* partial, long long ldp, hipStream_t st, int mfma) {
  if (ntask > 0 && nrhs == 8 && mfma) {
    hipLaunchKernelGGL(k_hmv_mfma8, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp);
    return;
  }
  if (ntask <= 0) return;
  switch (nrhs) {
    case 1: hipLaunchKernelGGL(k_hmv<1>, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp); break;
    case 2: hipLaunchKernelGGL(k_hmv<2>, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp); break;
    case 3: hipLaunchKernelGGL(k_hmv<3>, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp); break;
    case 4: hipLaunchKernelGGL(k_hmv<4>, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp); break;
    case 5: hipLaunchKernelGGL(k_hmv<5>, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp); break;
    case 6: hipLaunchKernelGGL(k_hmv<6>, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp); break;
    case 7: hipLaunchKernelGGL(k_hmv<7>, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp); break;
    case 8: hipLaunchKernelGGL(k_hmv<8>, dim3(ntask), dim3(256), 0, st, tasks, segs, x, ldx, z, ldz, partial, ldp); break;
    default: throw ApiError(-1, "matvec: 1 to 8 right-hand sides");
  }
}

__global__ void k_hmv_reduce(const LeafRange* __restrict__ leaves, const cd* __restrict__ partial, long long ldp,
                             cd* __restrict__ y, long long ldy) {
  const LeafRange L = leaves[blockIdx.x];
  const int r = threadIdx.x;
  if (r >= L.rows) return;
  const int q = blockIdx.y;
  const cd* pq = partial + q * ldp;
  cd s = mk(0.0);
  for (int t = L.t0; t < L.t1; ++t) s += pq[(size_t)t * HMV_MAXROWS + r];
  y[q * ldy + L.row0 + r] = s;
}

void launch_hmv_reduce(const LeafRange* leaves, int nleaf, const cd* partial, long long ldp, int nrhs, cd* y,
                       long long ldy, hipStream_t st) {
  if (nleaf > 0)
    hipLaunchKernelGGL(k_hmv_reduce, dim3(nleaf, nrhs), dim3(HMV_MAXROWS), 0, st, leaves, partial, ldp, y, ldy);
}

}  // namespace ewbem
