// Learned initial guess: the network's forward, backward and Adam kernels,
// and the kernels that turn reduced coordinates into training samples and a
// network output back into a guess.
//
// Every matrix product of the network runs on the bf16 matrix cores
// (v_mfma_f32_16x16x16 bf16): both operands are rounded to bf16 (nearest,
// ties to even) from their fp32 values when a tile is staged into LDS, and
// the products accumulate in fp32.  Biases, GELU, the loss, the bias
// gradients and Adam stay in fp32 (the loss sum in fp64).
#include "learn.hpp"

#include <algorithm>
#include <stdexcept>

namespace ewbem {
namespace {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) {  // inf stays inf, NaN stays a quiet NaN
    return (unsigned short)((u >> 16) | ((u & 0x007fffffu) ? 0x0040u : 0u));
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

constexpr int GT = 64;        // output tile (rows and columns) of one workgroup
constexpr int GK = 32;        // k extent of one LDS stage
constexpr int GKP = GK + 8;   // padded LDS row (bf16 elements), 8-byte aligned fragments

// C(i, j) = sum_k A(i, k) B(k, j) over a 64 x 64 tile; four waves, each a
// 32 x 32 quarter as 2 x 2 MFMA 16 x 16 blocks.  A(i, k) = A[i a_i + k a_k],
// B(k, j) = B[k b_k + j b_j]; out-of-range elements read as zero.
template <int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm(GemmArgs g) {
  __shared__ unsigned short As[GT][GKP];  // [row][k]
  __shared__ unsigned short Bs[GT][GKP];  // [column][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int row0 = blockIdx.y * GT, col0 = blockIdx.x * GT;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  f32x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  // consecutive threads walk the operand's contiguous index
  const bool a_kfast = g.a_k == 1, b_kfast = g.b_k == 1;
  for (int k0 = 0; k0 < g.K; k0 += GK) {
#pragma unroll
    for (int q = 0; q < GT * GK / 256; ++q) {
      const int e = tid + 256 * q;
      const int r = a_kfast ? e / GK : e % GT;
      const int kk = a_kfast ? e % GK : e / GT;
      const long long gi = row0 + r, gk = k0 + kk;
      const float v = (gi < g.M && gk < g.K) ? g.A[gi * g.a_i + gk * g.a_k] : 0.f;
      As[r][kk] = to_bf16(v);
    }
#pragma unroll
    for (int q = 0; q < GT * GK / 256; ++q) {
      const int e = tid + 256 * q;
      const int c = b_kfast ? e / GK : e % GT;
      const int kk = b_kfast ? e % GK : e / GT;
      const long long gj = col0 + c, gk = k0 + kk;
      const float v = (gj < g.N && gk < g.K) ? g.B[gk * g.b_k + gj * g.b_j] : 0.f;
      Bs[c][kk] = to_bf16(v);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      // lane l supplies rows (columns) l % 16 at k = ks + 4 (l / 16) .. +3
      const int kq = ks + 4 * (lane >> 4);
      s16x4 fa[2], fb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        fa[t] = *reinterpret_cast<const s16x4*>(&As[wr + 16 * t + (lane & 15)][kq]);
        fb[t] = *reinterpret_cast<const s16x4*>(&Bs[wc + 16 * t + (lane & 15)][kq]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane l holds rows 4 (l / 16) .. +3 of column l % 16 of each 16 x 16 block
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const long long i = row0 + wr + 16 * a + 4 * (lane >> 4) + t;
        const long long j = col0 + wc + 16 * b + (lane & 15);
        if (i >= g.M || j >= g.N) continue;
        float v = acc[a][b][t];
        if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) v += g.bias[j];
        if (EPI == EPI_BIAS_GELU) {
          g.Z[i * g.ldz + j] = v;
          v = gelu(v);
        }
        if (EPI == EPI_GELU_BWD) v *= gelu_grad(g.aux[i * g.ld_aux + j]);
        g.C[i * g.ldc + j] = v;
      }
}

// out[j] = sum_i D[i ld + j] (bias gradients): 64 columns per block, four
// waves over interleaved rows, fixed summation order.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ D, long long ld, long long M, int N,
                                               float* __restrict__ out) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (j < N)
    for (long long i = w; i < M; i += 4) s += D[i * ld + j];
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < N) out[j] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// dY = scale (Y - T); partial[b] = sum over block b's elements of (Y - T)^2.
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ T,
                                                 long long n, float scale, float* __restrict__ dY,
                                                 double* __restrict__ partial) {
  __shared__ double red[4];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const float e = Y[i] - T[i];
    if (dY) dY[i] = scale * e;
    s += (double)e * (double)e;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, AdamStep a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = a.beta1 * m[i] + (1.f - a.beta1) * gi;
  const float vi = a.beta2 * v[i] + (1.f - a.beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= a.lr * (mi / a.corr1) / (sqrtf(vi / a.corr2) + a.eps);
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One wave per sample.
__global__ __launch_bounds__(64) void k_learn_samples(const cd* __restrict__ coef, const cd* __restrict__ base, int r,
                                                     const int* __restrict__ idx, const float* __restrict__ kf, int n,
                                                     float* __restrict__ X, float* __restrict__ T,
                                                     double* __restrict__ nu) {
  const int s = blockIdx.x, lane = threadIdx.x;
  if (s >= n) return;
  const cd* c1 = coef + (size_t)idx[4 * s] * r;
  const cd* c2 = coef + (size_t)idx[4 * s + 1] * r;
  const cd* c3 = coef + (size_t)idx[4 * s + 2] * r;
  const int i0 = idx[4 * s + 3];
  double q = 0.0;
  for (int j = lane; j < r; j += 64) q += norm2(c1[j]);
  q = wave_sum(q);
  const double v = q > 0.0 ? sqrt(q) : 1.0;
  const double iv = 1.0 / v;
  const int d0 = 6 * r + 2;
  float* x = X + (size_t)s * d0;
  for (int j = lane; j < r; j += 64) {
    const cd a = c1[j], b = c2[j], c = c3[j];
    x[j] = (float)(a.x * iv);
    x[r + j] = (float)(a.y * iv);
    x[2 * r + j] = (float)(b.x * iv);
    x[3 * r + j] = (float)(b.y * iv);
    x[4 * r + j] = (float)(c.x * iv);
    x[5 * r + j] = (float)(c.y * iv);
    if (T && i0 >= 0) {
      const cd t0 = coef[(size_t)i0 * r + j];
      // residual of the base prediction: the table's row for the target's
      // snapshot, else the extrapolation 3 c_{k-1} - 3 c_{k-2} + c_{k-3}
      const cd e = t0 - (base ? base[(size_t)i0 * r + j] : 3.0 * a - 3.0 * b + c);
      T[(size_t)s * 2 * r + j] = (float)(e.x * iv);
      T[(size_t)s * 2 * r + r + j] = (float)(e.y * iv);
    }
  }
  if (lane == 0) {
    x[6 * r] = kf[s];
    x[6 * r + 1] = kf[s] * kf[s];
    if (nu) nu[s] = v;
  }
}

// p = (bp ? bp : 3 c1 - 3 c2 + c3) + nu (y_re + i y_im), the predicted
// coordinates; out = p (rel = 0) or p - (3 c1 - 3 c2 + c3) (rel = 1).
__global__ void k_learn_compose(const cd* __restrict__ coef, int r, const int* __restrict__ idx,
                                const double* __restrict__ nu, const float* __restrict__ y,
                                const cd* __restrict__ bp, int rel, cd* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  const double v = nu[0];
  const cd corr{v * (double)y[j], v * (double)y[r + j]};
  const cd a = coef[(size_t)idx[0] * r + j], b = coef[(size_t)idx[1] * r + j], c = coef[(size_t)idx[2] * r + j];
  const cd q = 3.0 * a - 3.0 * b + c;
  const cd p = (bp ? bp[j] : q) + corr;
  out[j] = rel ? p - q : p;
}

}  // namespace

size_t MlpShape::n_params() const {
  size_t n = 0;
  for (int l = 0; l + 1 < (int)dims.size(); ++l) n += (size_t)dims[l + 1] * dims[l] + dims[l + 1];
  return n;
}
size_t MlpShape::woff(int l) const {
  size_t n = 0;
  for (int i = 0; i < l; ++i) n += (size_t)dims[i + 1] * dims[i] + dims[i + 1];
  return n;
}
size_t MlpShape::boff(int l) const { return woff(l) + (size_t)dims[l + 1] * dims[l]; }
int MlpShape::max_width() const { return *std::max_element(dims.begin(), dims.end()); }
size_t MlpShape::hidden_sum() const {
  size_t n = 0;
  for (int l = 1; l + 1 < (int)dims.size(); ++l) n += dims[l];
  return n;
}

void launch_mlp_gemm(int epi, const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  const dim3 grid((unsigned)((g.N + GT - 1) / GT), (unsigned)((g.M + GT - 1) / GT));
  switch (epi) {
    case EPI_STORE: hipLaunchKernelGGL(k_mlp_gemm<EPI_STORE>, grid, dim3(256), 0, st, g); break;
    case EPI_BIAS: hipLaunchKernelGGL(k_mlp_gemm<EPI_BIAS>, grid, dim3(256), 0, st, g); break;
    case EPI_BIAS_GELU: hipLaunchKernelGGL(k_mlp_gemm<EPI_BIAS_GELU>, grid, dim3(256), 0, st, g); break;
    case EPI_GELU_BWD: hipLaunchKernelGGL(k_mlp_gemm<EPI_GELU_BWD>, grid, dim3(256), 0, st, g); break;
    default: throw std::runtime_error("mlp gemm: unknown epilogue");
  }
}

void mlp_forward(const MlpShape& s, const float* P, long long M, const float* X, float* act, float* pre, float* Y,
                 hipStream_t st) {
  const int L = s.n_layers();
  const float* in = X;
  size_t off = 0;
  for (int l = 0; l < L; ++l) {
    const int din = s.dims[l], dout = s.dims[l + 1];
    GemmArgs g{};
    g.M = (int)M;
    g.N = dout;
    g.K = din;
    g.A = in;       // A(i, k) = in[i din + k]
    g.a_i = din;
    g.a_k = 1;
    g.B = P + s.woff(l);  // B(k, j) = W[j din + k]
    g.b_k = 1;
    g.b_j = din;
    g.bias = P + s.boff(l);
    if (l + 1 < L) {
      g.C = act + off * M;
      g.ldc = dout;
      g.Z = pre + off * M;
      g.ldz = dout;
      launch_mlp_gemm(EPI_BIAS_GELU, g, st);
      in = g.C;
      off += dout;
    } else {
      g.C = Y;
      g.ldc = dout;
      launch_mlp_gemm(EPI_BIAS, g, st);
    }
  }
}

void mlp_backward(const MlpShape& s, const float* P, long long M, const float* X, const float* act, const float* pre,
                  const float* dY, float* work, float* G, hipStream_t st) {
  const int L = s.n_layers();
  // offsets of each hidden layer's activations in act / pre
  std::vector<size_t> hoff(L, 0);
  for (int l = 1; l < L; ++l) hoff[l] = hoff[l - 1] + (l > 1 ? s.dims[l - 1] : 0);
  // hoff[l] = start (in units of M floats) of the output of layer l - 1, l >= 1
  const size_t mw = (size_t)s.max_width();
  float* bufs[2] = {work, work + mw * M};
  const float* dz = dY;  // gradient at the output of layer l (pre-activation for hidden ones)
  for (int l = L - 1; l >= 0; --l) {
    const int din = s.dims[l], dout = s.dims[l + 1];
    const float* in = l == 0 ? X : act + hoff[l] * M;
    // weight gradient: G_W(j, k) = sum_i dz[i dout + j] in[i din + k]
    GemmArgs gw{};
    gw.M = dout;
    gw.N = din;
    gw.K = (int)M;
    gw.A = dz;  // A(j, i) = dz[i dout + j]
    gw.a_i = 1;
    gw.a_k = dout;
    gw.B = in;  // B(i, k) = in[i din + k]
    gw.b_k = din;
    gw.b_j = 1;
    gw.C = G + s.woff(l);
    gw.ldc = din;
    launch_mlp_gemm(EPI_STORE, gw, st);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((dout + 63) / 64)), dim3(256), 0, st, dz, (long long)dout, M, dout,
                       G + s.boff(l));
    if (l == 0) break;
    // input gradient through GELU: dz'(i, k) = gelu'(pre(i, k)) sum_j dz[i dout + j] W[j din + k]
    GemmArgs gd{};
    gd.M = (int)M;
    gd.N = din;
    gd.K = dout;
    gd.A = dz;  // A(i, j) = dz[i dout + j]
    gd.a_i = dout;
    gd.a_k = 1;
    gd.B = P + s.woff(l);  // B(j, k) = W[j din + k]
    gd.b_k = din;
    gd.b_j = 1;
    gd.aux = pre + hoff[l] * M;
    gd.ld_aux = din;
    float* out = bufs[l & 1];
    gd.C = out;
    gd.ldc = din;
    launch_mlp_gemm(EPI_GELU_BWD, gd, st);
    dz = out;
  }
}

int loss_blocks(long long n) { return (int)std::max(1LL, std::min(256LL, (n + 4095) / 4096)); }

void launch_mlp_loss(const float* Y, const float* T, long long n, float scale, float* dY, double* partial,
                     hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mlp_loss, dim3(loss_blocks(n)), dim3(256), 0, st, Y, T, n, scale, dY, partial);
}

void launch_adam(float* p, const float* g, float* m, float* v, long long n, const AdamStep& a, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, a);
}

void launch_learn_samples(const cd* coef, const cd* base, int r, const int* idx, const float* kf, int n, float* X,
                          float* T, double* nu, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_learn_samples, dim3(n), dim3(64), 0, st, coef, base, r, idx, kf, n, X, T, nu);
}

void launch_learn_compose(const cd* coef, int r, const int* idx, const double* nu, const float* y, const cd* bp,
                          int rel, cd* out, hipStream_t st) {
  hipLaunchKernelGGL(k_learn_compose, dim3((unsigned)((r + 63) / 64)), dim3(64), 0, st, coef, r, idx, nu, y, bp,
                     rel, out);
}

}  // namespace ewbem
