// Vector kernels of the Krylov solver (complex128) and the block-diagonal
// preconditioner.  Inner products are formed as per-chunk partial sums
// reduced in a fixed order, so results do not depend on scheduling.
#include "solver.hpp"

namespace ewbem {

__device__ __forceinline__ double wsumv(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// partial[c * nchunk + chunk] = sum_{r in chunk} conj(V[r + c ld]) w[r]
__global__ __launch_bounds__(256) void k_dots(const cd* __restrict__ V, long long ld, const cd* __restrict__ w,
                                              long long n, int nchunk, cd* __restrict__ partial) {
  const int c = blockIdx.y;
  const long long per = (n + nchunk - 1) / nchunk;
  const long long r0 = (long long)blockIdx.x * per;
  const long long r1 = min(n, r0 + per);
  const cd* __restrict__ v = V + (size_t)c * ld;
  cd acc = mk(0.0);
  for (long long r = r0 + threadIdx.x; r < r1; r += 256) acc += cmulc(v[r], w[r]);
  __shared__ double sx[4], sy[4];
  acc.x = wsumv(acc.x);
  acc.y = wsumv(acc.y);
  if ((threadIdx.x & 63) == 0) {
    sx[threadIdx.x >> 6] = acc.x;
    sy[threadIdx.x >> 6] = acc.y;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    partial[(size_t)c * nchunk + blockIdx.x] = cd{sx[0] + sx[1] + sx[2] + sx[3], sy[0] + sy[1] + sy[2] + sy[3]};
}

__global__ void k_reduce_cols(const cd* __restrict__ partial, int nchunk, int ncols, cd* __restrict__ out) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  cd acc = mk(0.0);
  for (int i = lane; i < nchunk; i += 64) acc += partial[(size_t)c * nchunk + i];
  acc.x = wsumv(acc.x);
  acc.y = wsumv(acc.y);
  if (lane == 0 && c < ncols) out[c] = acc;
}

int dots_chunks(long long n) {
  long long c = (n + 4095) / 4096;
  if (c < 1) c = 1;
  if (c > 512) c = 512;
  return (int)c;
}

// nrm[c] = |V(:, c)|_2 for c < ncols: one 256-thread workgroup per column,
// fixed summation order
__global__ __launch_bounds__(256) void k_col_norms(const cd* __restrict__ V, long long ld, long long n,
                                                   double* __restrict__ nrm) {
  const cd* __restrict__ v = V + (size_t)blockIdx.x * ld;
  double acc = 0.0;
  for (long long r = threadIdx.x; r < n; r += 256) acc += v[r].x * v[r].x + v[r].y * v[r].y;
  __shared__ double sp[4];
  acc = wsumv(acc);
  if ((threadIdx.x & 63) == 0) sp[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) nrm[blockIdx.x] = sqrt(sp[0] + sp[1] + sp[2] + sp[3]);
}

// V(:, c) *= f[c] (inv = 0) or / f[c] (inv = 1; a zero f leaves the column)
__global__ void k_col_scale(cd* __restrict__ V, long long ld, long long n, const double* __restrict__ f,
                            int inv) {
  const double g = f[blockIdx.y];
  const double a = inv ? (g > 0.0 ? 1.0 / g : 1.0) : g;
  cd* __restrict__ v = V + (size_t)blockIdx.y * ld;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (long long)gridDim.x * blockDim.x)
    v[r] = cd{a * v[r].x, a * v[r].y};
}

void launch_col_norms(const cd* V, long long ld, int ncols, long long n, double* nrm, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_col_norms, dim3(ncols), dim3(256), 0, st, V, ld, n, nrm);
}

void launch_col_scale(cd* V, long long ld, int ncols, long long n, const double* f, int inv, hipStream_t st) {
  if (ncols <= 0 || n <= 0) return;
  const long long bx = std::min<long long>((n + 255) / 256, 64);
  hipLaunchKernelGGL(k_col_scale, dim3((unsigned)bx, ncols), dim3(256), 0, st, V, ld, n, f, inv);
}

void launch_dots(const cd* V, long long ld, int ncols, const cd* w, long long n, cd* partial,
                 cd* out, hipStream_t st) {
  if (ncols <= 0) return;
  const int nchunk = dots_chunks(n);
  hipLaunchKernelGGL(k_dots, dim3(nchunk, ncols), dim3(256), 0, st, V, ld, w, n, nchunk, partial);
  hipLaunchKernelGGL(k_reduce_cols, dim3(ncols), dim3(64), 0, st, partial, nchunk, ncols, out);
}

// w[r] -= sum_c V[r + c ld] h[c]
__global__ void k_gemv_sub(const cd* __restrict__ V, long long ld, int ncols, const cd* __restrict__ h,
                           cd* __restrict__ w, long long n) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  cd acc = w[r];
  for (int c = 0; c < ncols; ++c) acc -= V[(size_t)c * ld + r] * h[c];
  w[r] = acc;
}

void launch_gemv_sub(const cd* V, long long ld, int ncols, const cd* h, cd* w, long long n,
                     hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_gemv_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, V, ld, ncols, h, w,
                     n);
}

// out[r] = beta * out[r] + sum_c V[r + c ld] h[c]   (h on the device)
__global__ void k_gemv_acc(const cd* __restrict__ V, long long ld, int ncols, const cd* __restrict__ h,
                           cd beta, cd* __restrict__ out, long long n) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  cd acc = (beta.x == 0.0 && beta.y == 0.0) ? mk(0.0) : out[r] * beta;
  for (int c = 0; c < ncols; ++c) acc += V[(size_t)c * ld + r] * h[c];
  out[r] = acc;
}

void launch_gemv_acc(const cd* V, long long ld, int ncols, const cd* h, cd beta, cd* out, long long n,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_acc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, V, ld, ncols, h,
                     beta, out, n);
}

// y = a x + b y
__global__ void k_axpby(cd a, const cd* x, cd b, cd* y, long long n) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  // y is not read when b = 0 (it may be uninitialised)
  y[r] = (b.x == 0.0 && b.y == 0.0) ? a * x[r] : a * x[r] + b * y[r];
}

void launch_axpby(cd a, const cd* x, cd b, cd* y, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, x, b, y, n);
}

// Gather/scatter between the caller's dof order and tree order.
// to_tree: out[3t+i] = in[3 perm[t] + i];  from_tree: out[3 perm[t] + i] = in[3t+i]
__global__ void k_permute(const cd* __restrict__ in, const int* __restrict__ perm, int ne, int to_tree,
                          cd* __restrict__ out) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= 3 * ne) return;
  const int t = d / 3, i = d - 3 * t;
  const size_t o = 3 * (size_t)perm[t] + i;
  if (to_tree)
    out[d] = in[o];
  else
    out[o] = in[d];
}

void launch_permute(const cd* in, const int* perm, int ne, int to_tree, cd* out, hipStream_t st) {
  hipLaunchKernelGGL(k_permute, dim3((3 * ne + 255) / 256), dim3(256), 0, st, in, perm, ne, to_tree,
                     out);
}

// ---- element (3 x 3) block-diagonal preconditioner: the diagonal 3 x 3
// blocks of T are the self-element blocks.
__global__ void k_inv3(const cd* __restrict__ A, int ne, cd* __restrict__ Ainv) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  cd a[3][3], inv[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a[i][j] = A[9 * (size_t)e + 3 * i + j];
  // adjugate / determinant
  inv[0][0] = a[1][1] * a[2][2] - a[1][2] * a[2][1];
  inv[0][1] = a[0][2] * a[2][1] - a[0][1] * a[2][2];
  inv[0][2] = a[0][1] * a[1][2] - a[0][2] * a[1][1];
  inv[1][0] = a[1][2] * a[2][0] - a[1][0] * a[2][2];
  inv[1][1] = a[0][0] * a[2][2] - a[0][2] * a[2][0];
  inv[1][2] = a[0][2] * a[1][0] - a[0][0] * a[1][2];
  inv[2][0] = a[1][0] * a[2][1] - a[1][1] * a[2][0];
  inv[2][1] = a[0][1] * a[2][0] - a[0][0] * a[2][1];
  inv[2][2] = a[0][0] * a[1][1] - a[0][1] * a[1][0];
  const cd det = a[0][0] * inv[0][0] + a[0][1] * inv[1][0] + a[0][2] * inv[2][0];
  const cd id = cinv(det);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ainv[9 * (size_t)e + 3 * i + j] = inv[i][j] * id;
}

void launch_inv3(const cd* A, int ne, cd* Ainv, hipStream_t st) {
  hipLaunchKernelGGL(k_inv3, dim3((ne + 255) / 256), dim3(256), 0, st, A, ne, Ainv);
}

__global__ void k_apply3(const cd* __restrict__ M, int ne, const cd* __restrict__ v, cd* __restrict__ z) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= 3 * ne) return;
  const int e = d / 3, i = d - 3 * e;
  const cd* m = M + 9 * (size_t)e + 3 * i;
  const cd* x = v + 3 * (size_t)e;
  z[d] = m[0] * x[0] + m[1] * x[1] + m[2] * x[2];
}

void launch_apply3(const cd* M, int ne, const cd* v, cd* z, hipStream_t st) {
  hipLaunchKernelGGL(k_apply3, dim3((3 * ne + 255) / 256), dim3(256), 0, st, M, ne, v, z);
}

// ---- leaf block-diagonal preconditioner: Gauss-Jordan inversion with
// partial pivoting of each diagonal near block (n x n, column-major).
//
// Blocks of up to BI_NP = 128 rows: the whole block lives in the registers
// of one 1024-thread workgroup (thread = row r, columns g, g + 8, ...), and
// rows are never swapped: at step k the pivot is the unused row p with the
// largest |A[p][k]|, row p is scaled and column k eliminated from every
// other row in place.  The result B then holds the inverse with rows and
// columns permuted: inv[i][c] = B[piv[i]][q[c]], q the inverse of piv, which
// the final store undoes.  Three barriers per pivot, no global traffic
// between the load and the store.
constexpr int BI_NP = 128;                 // rows per block, padded
constexpr int BI_G = 1024 / BI_NP;         // column groups
constexpr int BI_CPT = BI_NP / BI_G;       // columns per thread

__global__ __launch_bounds__(1024) void k_block_inv_reg(const long long* __restrict__ offs,
                                                        const int* __restrict__ dims, cd* __restrict__ W,
                                                        int* __restrict__ piv_fail) {
  const int b = blockIdx.x;
  const int n = dims[b];
  if (n > BI_NP) return;  // larger blocks: k_block_inv
  cd* A = W + offs[b];
  const int t = threadIdx.x;
  const int r = t % BI_NP, g = t / BI_NP;
  const int lane = t & 63, wv = r >> 6;  // wave index within the column group
  // s_col alternates with the step: rows still updating from step k read
  // it while column k + 1 is written
  __shared__ cd s_row[BI_NP], s_col[2][BI_NP];
  __shared__ double s_bv[2];
  __shared__ int s_bi[2], s_piv[BI_NP], s_q[BI_NP];
  __shared__ cd s_inv;
  cd a[BI_CPT];
#pragma unroll
  for (int j = 0; j < BI_CPT; ++j) {
    const int c = g + BI_G * j;
    a[j] = (r < n && c < n) ? A[(size_t)c * n + r] : mk(0.0);
  }
  bool used = r >= n;
  for (int k = 0; k < n; ++k) {
    const int gk = k % BI_G, jk = k / BI_G;
    // this thread's entry of column k (meaningful in group gk)
    cd ck = mk(0.0);
#pragma unroll
    for (int j = 0; j < BI_CPT; ++j)
      if (j == jk) ck = a[j];
    if (g == gk) {
      // arg max over the unused rows; used rows score -1, ties to the lower row
      double v = used ? -1.0 : norm2(ck);
      int vi = r;
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(vi, off, 64);
        if (ov > v || (ov == v && oi < vi)) {
          v = ov;
          vi = oi;
        }
      }
      if (lane == 0) {
        s_bv[wv] = v;
        s_bi[wv] = vi;
      }
      if (r < n) s_col[k & 1][r] = ck;
    }
    __syncthreads();
    const int p = (s_bv[1] > s_bv[0] || (s_bv[1] == s_bv[0] && s_bi[1] < s_bi[0])) ? s_bi[1] : s_bi[0];
    if (r == p) {
      // the pivot's row, scaled; column k of the result holds 1 / pivot
      if (g == gk) {
        const bool ok = norm2(ck) > 0.0;
        if (!ok) piv_fail[b] = 1;
        s_inv = ok ? cinv(ck) : mk(0.0);
        s_piv[k] = p;
        s_q[p] = k;
      }
    }
    __syncthreads();
    const cd ip = s_inv;
    if (r == p) {
#pragma unroll
      for (int j = 0; j < BI_CPT; ++j) {
        const int c = g + BI_G * j;
        if (c < n) {
          a[j] = (c == k) ? ip : a[j] * ip;
          s_row[c] = a[j];
        }
      }
      used = true;
    }
    __syncthreads();
    if (r != p && r < n) {
      const cd f = s_col[k & 1][r];
#pragma unroll
      for (int j = 0; j < BI_CPT; ++j) {
        const int c = g + BI_G * j;
        if (c < n) a[j] = (c == k) ? -(f * ip) : a[j] - f * s_row[c];
      }
    }
  }
  __syncthreads();
  if (r < n) {
    const int i = s_q[r];
#pragma unroll
    for (int j = 0; j < BI_CPT; ++j) {
      const int c = g + BI_G * j;
      if (c < n) A[(size_t)s_piv[c] * n + i] = a[j];
    }
  }
}

// Larger blocks (up to HMV_MAXROWS_S rows): one 256-thread workgroup per
// block, in place in global memory, explicit row swaps.
__global__ __launch_bounds__(256) void k_block_inv(const long long* __restrict__ offs, const int* __restrict__ dims,
                                                   cd* __restrict__ W, int* __restrict__ piv_fail) {
  const int b = blockIdx.x;
  const int n = dims[b];
  if (n <= BI_NP) return;  // k_block_inv_reg
  cd* A = W + offs[b];
  __shared__ int s_piv[HMV_MAXROWS_S];
  __shared__ double s_v[256];
  __shared__ int s_i[256];
  __shared__ cd s_col[HMV_MAXROWS_S];
  __shared__ cd s_row[HMV_MAXROWS_S];
  for (int k = 0; k < n; ++k) {
    // pivot search in column k, rows k..n-1
    double best = -1.0;
    int bi = k;
    for (int r = k + threadIdx.x; r < n; r += 256) {
      const double v = norm2(A[(size_t)k * n + r]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
    s_v[threadIdx.x] = best;
    s_i[threadIdx.x] = bi;
    __syncthreads();
    if (threadIdx.x == 0) {
      double bv = s_v[0];
      int bb = s_i[0];
      for (int t = 1; t < 256; ++t)
        if (s_v[t] > bv) {
          bv = s_v[t];
          bb = s_i[t];
        }
      s_piv[k] = bb;
      if (!(bv > 0.0)) piv_fail[b] = 1;
    }
    __syncthreads();
    const int p = s_piv[k];
    // swap rows k and p
    if (p != k)
      for (int c = threadIdx.x; c < n; c += 256) {
        const cd t = A[(size_t)c * n + k];
        A[(size_t)c * n + k] = A[(size_t)c * n + p];
        A[(size_t)c * n + p] = t;
      }
    __syncthreads();
    const cd ip = cinv(A[(size_t)k * n + k]);
    // save column k (multipliers) and scaled row k
    for (int r = threadIdx.x; r < n; r += 256) s_col[r] = A[(size_t)k * n + r];
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += 256) {
      const cd v = (c == k) ? ip : A[(size_t)c * n + k] * ip;
      s_row[c] = v;
      A[(size_t)c * n + k] = v;
    }
    __syncthreads();
    // eliminate: A[r][c] -= col[r] * row[c] for r != k; column k becomes -col[r]*ip
    for (int idx = threadIdx.x; idx < n * n; idx += 256) {
      const int c = idx / n, r = idx - c * n;
      if (r == k) continue;
      if (c == k)
        A[(size_t)c * n + r] = -(s_col[r] * ip);
      else
        A[(size_t)c * n + r] -= s_col[r] * s_row[c];
    }
    __syncthreads();
  }
  // undo the row swaps as column swaps, last to first
  for (int k = n - 1; k >= 0; --k) {
    const int p = s_piv[k];
    if (p != k)
      for (int r = threadIdx.x; r < n; r += 256) {
        const cd t = A[(size_t)k * n + r];
        A[(size_t)k * n + r] = A[(size_t)p * n + r];
        A[(size_t)p * n + r] = t;
      }
    __syncthreads();
  }
}

void launch_block_inv(const long long* offs, const int* dims, int nblk, cd* W, int* piv_fail,
                      hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(k_block_inv_reg, dim3(nblk), dim3(1024), 0, st, offs, dims, W, piv_fail);
  hipLaunchKernelGGL(k_block_inv, dim3(nblk), dim3(256), 0, st, offs, dims, W, piv_fail);
}

// z[row0 + r] = sum_c Minv_b[r, c] v[row0 + c], one workgroup per leaf
__global__ __launch_bounds__(256) void k_block_apply(const long long* __restrict__ offs, const int* __restrict__ dims,
                                                     const int* __restrict__ row0s, const cd* __restrict__ W,
                                                     const cd* __restrict__ v, cd* __restrict__ z) {
  const int b = blockIdx.x;
  const int n = dims[b], row0 = row0s[b];
  const cd* A = W + offs[b];
  __shared__ cd sv[HMV_MAXROWS_S];
  for (int c = threadIdx.x; c < n; c += 256) sv[c] = v[row0 + c];
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += 256) {
    cd acc = mk(0.0);
    for (int c = 0; c < n; ++c) acc += A[(size_t)c * n + r] * sv[c];
    z[row0 + r] = acc;
  }
}

void launch_block_apply(const long long* offs, const int* dims, const int* row0s, int nblk,
                        const cd* W, const cd* v, cd* z, hipStream_t st) {
  if (nblk > 0) hipLaunchKernelGGL(k_block_apply, dim3(nblk), dim3(256), 0, st, offs, dims, row0s, W, v, z);
}

__global__ void k_copy_blocks(const long long* __restrict__ src_offs, const int* __restrict__ src_ld,
                              const long long* __restrict__ dst_offs, const int* __restrict__ dims,
                              const cd* __restrict__ D, cd* __restrict__ W) {
  const int b = blockIdx.x;
  const int n = dims[b];
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int c = idx / n, r = idx - c * n;
    W[dst_offs[b] + idx] = D[src_offs[b] + (size_t)c * src_ld[b] + r];
  }
}

void launch_copy_blocks(const long long* src_offs, const int* src_ld, const long long* dst_offs,
                        const int* dims, int nblk, const cd* D, cd* W, hipStream_t st) {
  if (nblk > 0)
    hipLaunchKernelGGL(k_copy_blocks, dim3(nblk), dim3(256), 0, st, src_offs, src_ld, dst_offs, dims, D, W);
}

}  // namespace ewbem
