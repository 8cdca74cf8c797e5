// Shared types and helpers of the ewbem HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace ewbem {

// Interleaved complex128 (same layout as ewbem_z / torch.complex128).
struct cd {
  double x, y;
};
// Interleaved complex64, used for reduced-precision storage of low-rank factors.
struct cf {
  float x, y;
};

__host__ __device__ inline cd mk(double a, double b = 0.0) { return cd{a, b}; }
__host__ __device__ inline cd operator+(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cd operator-(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cd operator-(cd a) { return cd{-a.x, -a.y}; }
__host__ __device__ inline cd operator*(cd a, cd b) {
  return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline cd operator*(double s, cd a) { return cd{s * a.x, s * a.y}; }
__host__ __device__ inline cd operator*(cd a, double s) { return cd{s * a.x, s * a.y}; }
__host__ __device__ inline cd operator+(cd a, double s) { return cd{a.x + s, a.y}; }
__host__ __device__ inline cd operator+(double s, cd a) { return cd{a.x + s, a.y}; }
__host__ __device__ inline cd operator-(cd a, double s) { return cd{a.x - s, a.y}; }
__host__ __device__ inline cd& operator+=(cd& a, cd b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline cd& operator-=(cd& a, cd b) { a.x -= b.x; a.y -= b.y; return a; }
__host__ __device__ inline cd conj(cd a) { return cd{a.x, -a.y}; }
__host__ __device__ inline double norm2(cd a) { return a.x * a.x + a.y * a.y; }
// conj(a) * b
__host__ __device__ inline cd cmulc(cd a, cd b) {
  return cd{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline cd cinv(cd a) {
  double d = 1.0 / (a.x * a.x + a.y * a.y);
  return cd{a.x * d, -a.y * d};
}
__host__ __device__ inline cd to_cd(cf a) { return cd{(double)a.x, (double)a.y}; }
__host__ __device__ inline cd to_cd(cd a) { return a; }
__host__ __device__ inline cf to_cf(cd a) { return cf{(float)a.x, (float)a.y}; }

// Number of Taylor terms (n = 2 .. NSER+1) kept for small |z_s|.
constexpr int NSER = 18;
// Maximum self-element polar rule order (per direction).
constexpr int MAX_SELF_ORDER = 32;

// Everything a kernel evaluation needs at one Laplace parameter s.
struct KParams {
  cd s;              // Laplace parameter sigma + i omega_k
  cd cs_over_s;      // c_s / s, so that 1 / z_s = (c_s / s) / r (zero at s = 0,
                     // where every |z| takes the series branch)
  double inv_cs;     // 1 / c_s
  double gamma;      // c_s / c_p
  double g2;         // gamma^2
  double ratio;      // (c_p / c_s)^2
  double inv4pi;     // 1 / (4 pi)
  double inv4pimu;   // 1 / (4 pi mu)
  double cpv;        // gamma^2 / (4 pi)
  double series_z2;  // |z_s|^2 below which the series is used
  double stat_rphi, stat_rpsi;  // static (n = 2) terms of r phi, r psi
  // device, 4 x NSER: Taylor coefficients of r phi, r psi, r^2 phi', r^2 psi'
  // in z (material constants; read only on the rare small-|z| branch, so they
  // are not kernel arguments held in scalar registers)
  const double* ser;
};

// Geometry of the mesh on the device, elements in cluster-tree order.
struct DevGeom {
  int ne;
  const double* cen;   // [ne][3] collocation points (centroids)
  const double* nrm;   // [ne][3] unit normals pointing out of the solid
  const double* qp;    // [ne][7][3] quadrature points of the 7-point rule
  const double* qw;    // [ne][7] quadrature weights times area
  const double* vtx;   // [ne][3][3] vertices
  // per element: 0 = traction given (unknown displacement, columns of T),
  // 1 = displacement given (unknown traction, columns of -U); null = all 0
  const int* bc;
};

}  // namespace ewbem

#define EWBEM_HIP_CHECK(expr)                                  \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) {                                    \
      throw ::ewbem::HipError(_e, #expr, __FILE__, __LINE__);  \
    }                                                          \
  } while (0)

#include <stdexcept>
#include <string>
namespace ewbem {
struct HipError : std::runtime_error {
  hipError_t code;
  HipError(hipError_t e, const char* what, const char* file, int line)
      : std::runtime_error(std::string("HIP error '") + hipGetErrorString(e) + "' in " + what +
                           " at " + file + ":" + std::to_string(line)),
        code(e) {}
};
struct ApiError : std::runtime_error {
  int status;
  ApiError(int st, const std::string& m) : std::runtime_error(m), status(st) {}
};
}  // namespace ewbem
