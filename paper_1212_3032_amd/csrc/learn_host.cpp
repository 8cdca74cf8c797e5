// Host helpers of the learned initial guess: the small dense factorisations
// of the randomized range finder (Cholesky-QR and the final Hermitian
// eigenproblem of the sketch) and of the per-frequency least-squares map
// (an n x n Gram matrix per frequency, n the training loads).
#include "learn.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace ewbem {

using zc = std::complex<double>;

bool cholesky(std::vector<zc>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(A[(size_t)j * n + k]);
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      zc s = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * std::conj(A[(size_t)j * n + k]);
      A[(size_t)i * n + j] = s / d;
    }
    for (int i = 0; i < j; ++i) A[(size_t)i * n + j] = 0.0;
  }
  return true;
}

std::vector<zc> inverse_lh(const std::vector<zc>& L, int n) {
  // R = L^H is upper triangular; solve R X = I column by column
  std::vector<zc> X((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    for (int i = n - 1; i >= 0; --i) {
      zc s = (i == c) ? 1.0 : 0.0;
      for (int k = i + 1; k < n; ++k) s -= std::conj(L[(size_t)k * n + i]) * X[(size_t)k * n + c];
      X[(size_t)i * n + c] = s / std::conj(L[(size_t)i * n + i]);
    }
  }
  return X;
}

void herm_eig(std::vector<zc> A, int n, std::vector<double>& w, std::vector<zc>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto at = [&](int i, int j) -> zc& { return A[(size_t)i * n + j]; };
  double fro = 0.0;
  for (const zc& a : A) fro += std::norm(a);
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        if (i != j) off += std::norm(at(i, j));
    if (std::sqrt(off) <= 1e-15 * fro || fro == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const zc b = at(p, q);
        const double ab = std::abs(b);
        if (ab <= 1e-300) continue;
        // G = diag(1, e^{-i phi}) R(theta) makes the (p, q) entry zero:
        // the phase turns b real, then a real Jacobi rotation
        const zc ph = b / ab;  // e^{i phi}
        const double a = at(p, p).real(), d = at(q, q).real();
        const double th = (d - a) / (2.0 * ab);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::abs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        const zc gpp = c, gpq = s, gqp = -s * std::conj(ph), gqq = c * std::conj(ph);
        for (int i = 0; i < n; ++i) {  // A <- A G
          const zc x = at(i, p), y = at(i, q);
          at(i, p) = x * gpp + y * gqp;
          at(i, q) = x * gpq + y * gqq;
        }
        for (int j = 0; j < n; ++j) {  // A <- G^H A
          const zc x = at(p, j), y = at(q, j);
          at(p, j) = std::conj(gpp) * x + std::conj(gqp) * y;
          at(q, j) = std::conj(gpq) * x + std::conj(gqq) * y;
        }
        at(p, q) = 0.0;
        at(q, p) = 0.0;
        at(p, p) = at(p, p).real();
        at(q, q) = at(q, q).real();
        for (int i = 0; i < n; ++i) {  // V <- V G
          const zc x = V[(size_t)i * n + p], y = V[(size_t)i * n + q];
          V[(size_t)i * n + p] = x * gpp + y * gqp;
          V[(size_t)i * n + q] = x * gpq + y * gqq;
        }
      }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return at(x, x).real() > at(y, y).real(); });
  w.resize(n);
  std::vector<zc> Vs((size_t)n * n);
  for (int c = 0; c < n; ++c) {
    w[c] = at(ord[c], ord[c]).real();
    for (int i = 0; i < n; ++i) Vs[(size_t)i * n + c] = V[(size_t)i * n + ord[c]];
  }
  V.swap(Vs);
}

bool ridge_dual(const std::vector<zc>& X, const std::vector<zc>& Y, int d, int r, int n, double eps,
                std::vector<zc>& W, std::vector<double>& adiag, double& lam_out) {
  // G = X^H X (row-major n x n), columns of X contiguous
  std::vector<zc> G((size_t)n * n);
  double tr = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      zc acc = 0.0;
      for (int q = 0; q < d; ++q) acc += std::conj(X[(size_t)i * d + q]) * X[(size_t)j * d + q];
      G[(size_t)i * n + j] = acc;
      G[(size_t)j * n + i] = std::conj(acc);
    }
  for (int i = 0; i < n; ++i) tr += G[(size_t)i * n + i].real();
  if (!(tr > 0)) return false;
  const double lam = eps * tr / n;
  lam_out = lam;
  for (int i = 0; i < n; ++i) G[(size_t)i * n + i] += lam;
  if (!cholesky(G, n)) return false;
  // A = (L L^H)^{-1} = R R^H with R = (L^H)^{-1} upper triangular
  const std::vector<zc> R = inverse_lh(G, n);
  std::vector<zc> A((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      zc acc = 0.0;
      for (int q = std::max(i, j); q < n; ++q) acc += R[(size_t)i * n + q] * std::conj(R[(size_t)j * n + q]);
      A[(size_t)i * n + j] = acc;
    }
  W.assign((size_t)r * n, 0.0);
  adiag.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    adiag[j] = A[(size_t)j * n + j].real();
    for (int q = 0; q < n; ++q) {
      const zc a = A[(size_t)q * n + j];
      for (int i = 0; i < r; ++i) W[(size_t)j * r + i] += Y[(size_t)q * r + i] * a;
    }
  }
  return true;
}

}  // namespace ewbem
