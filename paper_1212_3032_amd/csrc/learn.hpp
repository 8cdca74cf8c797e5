// Learned initial guess: a network maps the reduced coordinates of the three
// previous frequencies' solutions to a correction of their quadratic
// extrapolation at the next frequency.  The reduced coordinates are the
// components on an orthonormal basis of the dominant subspace of training
// solutions (proper orthogonal decomposition); the network's prediction is
// one more column of the least-squares extrapolation of Sec. 4.2, so it can
// only lower the initial residual that extrapolation alone would give.
//
// Network: dims[0] -> dims[1] -> ... -> dims[L], GELU after every layer but
// the last; parameters flat in fp32, layer by layer: W_l (dims[l+1] x
// dims[l], row-major) then b_l (dims[l+1]).  Products run on bf16 matrix
// cores with fp32 accumulation.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace ewbem {

struct MlpShape {
  std::vector<int> dims;
  int n_layers() const { return (int)dims.size() - 1; }
  size_t n_params() const;
  size_t woff(int l) const;  // offset of W_l in the flat parameters
  size_t boff(int l) const;  // offset of b_l
  int max_width() const;
  size_t hidden_sum() const;  // sum of the hidden widths (activation floats per sample)
};

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };

// C(i, j) = sum_k A(i, k) B(k, j), i < M, j < N, k < K, with
// A(i, k) = A[i a_i + k a_k], B(k, j) = B[k b_k + j b_j] (fp32 storage,
// bf16 operands), and the epilogue
//   EPI_STORE:     C = acc
//   EPI_BIAS:      C = acc + bias[j]
//   EPI_BIAS_GELU: Z = acc + bias[j], C = gelu(Z)
//   EPI_GELU_BWD:  C = acc * gelu'(aux[i ld_aux + j])
struct GemmArgs {
  int M, N, K;
  const float* A;
  long long a_i, a_k;
  const float* B;
  long long b_k, b_j;
  const float* bias;
  const float* aux;
  long long ld_aux;
  float* C;
  long long ldc;
  float* Z;
  long long ldz;
};
void launch_mlp_gemm(int epi, const GemmArgs& g, hipStream_t st);

// Forward pass of M samples X (M x dims[0]): hidden outputs into act and
// their pre-activations into pre (each M x hidden_sum, layer after layer,
// each layer M x width row-major), the output into Y (M x dims[L]).
void mlp_forward(const MlpShape& s, const float* P, long long M, const float* X, float* act, float* pre, float* Y,
                 hipStream_t st);
// Backward pass from dY = dLoss/dY (M x dims[L]); work: 2 M max_width
// floats; G: gradient, laid out like the parameters.
void mlp_backward(const MlpShape& s, const float* P, long long M, const float* X, const float* act, const float* pre,
                  const float* dY, float* work, float* G, hipStream_t st);

// Squared-error loss: dY = scale (Y - T) (dY may be null) and per-block
// partial sums of (Y - T)^2 in fp64 (loss_blocks(n) of them).
int loss_blocks(long long n);
void launch_mlp_loss(const float* Y, const float* T, long long n, float scale, float* dY, double* partial,
                     hipStream_t st);

struct AdamStep {
  float lr, beta1, beta2, eps, corr1, corr2;  // corr = 1 - beta^t
};
void launch_adam(float* p, const float* g, float* m, float* v, long long n, const AdamStep& a, hipStream_t st);

// Samples from a table of reduced coordinates (rows of r complex values).
// Sample s uses rows idx[4s .. 4s+2] as the solutions at k-1, k-2, k-3 and
// row idx[4s+3] (or -1) as the target at k.  With nu = |c_{k-1}| (1 if 0):
//   X row (6 r + 2): [Re c1, Im c1, Re c2, Im c2, Re c3, Im c3] / nu, f, f^2
//   T row (2 r):     [Re e, Im e] / nu,  e = c_k - base_k
// with f = kf[s] and base_k row idx[4s+3] of ``base`` (same layout as coef),
// or 3 c1 - 3 c2 + c3 when base is null.  T and nu may be null.
void launch_learn_samples(const cd* coef, const cd* base, int r, const int* idx, const float* kf, int n, float* X,
                          float* T, double* nu, hipStream_t st);
// p (r) = (bp ? bp : 3 c1 - 3 c2 + c3) + nu (y[0..r) + i y[r..2r)) for the
// rows idx[0..2] of coef; out = p (rel = 0) or p - (3 c1 - 3 c2 + c3) (rel = 1).
void launch_learn_compose(const cd* coef, int r, const int* idx, const double* nu, const float* y, const cd* bp,
                          int rel, cd* out, hipStream_t st);

// ---- host helpers (small dense matrices, row-major)

// Cholesky factorisation A = L L^H of a Hermitian positive definite n x n
// matrix (lower triangle used), in place; false if not positive definite.
bool cholesky(std::vector<std::complex<double>>& A, int n);
// Inverse of the upper-triangular L^H of a Cholesky factor (upper triangular).
std::vector<std::complex<double>> inverse_lh(const std::vector<std::complex<double>>& L, int n);
// The least-squares map of one frequency in its dual form: X (d x n) and Y
// (r x n), both column-major; A = (X^H X + lam I)^{-1} with
// lam = eps tr(X^H X) / n (returned in lam); W = Y A (r x n, column-major)
// and adiag = diag(A).  False if the Gram matrix is zero or does not factor.
bool ridge_dual(const std::vector<std::complex<double>>& X, const std::vector<std::complex<double>>& Y, int d,
                int r, int n, double eps, std::vector<std::complex<double>>& W, std::vector<double>& adiag,
                double& lam);
// Eigen-decomposition of a Hermitian n x n matrix by cyclic Jacobi
// rotations: eigenvalues in descending order, eigenvectors as the columns of
// V (row-major n x n).
void herm_eig(std::vector<std::complex<double>> A, int n, std::vector<double>& w,
              std::vector<std::complex<double>>& V);

}  // namespace ewbem
