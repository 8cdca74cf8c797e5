// Host launchers of the HIP kernels (all enqueue on the given stream).
#pragma once

#include "common.hpp"

namespace ewbem {

struct SelfRule {
  int nt, nr;                         // angular and radial orders
  double t[MAX_SELF_ORDER], wt[MAX_SELF_ORDER];
  double u[MAX_SELF_ORDER], wu[MAX_SELF_ORDER];
};

// Dense near-field block: rows = leaf elements [r0, r0+m), columns = leaf
// elements [c0, c0+n) in tree order, stored column-major with ld = 3m at
// D + off (complex128).
struct NearBlk {
  int r0, m, c0, n;
  long long off;
};

// ---- assembly
// selfT, selfU: the self blocks of T (free term and principal value
// included) and U; selfA (optional): those of the system matrix A (T, or -U
// for an element with a given displacement).
void launch_self(const DevGeom& g, const KParams& P, const SelfRule& S, cd* selfT, cd* selfU,
                 cd* selfA, hipStream_t st);
void launch_near(const NearBlk* blks, int nblk, const DevGeom& g, const KParams& P, cd* D,
                 hipStream_t st);
void launch_scatter_self(const cd* selfT, const long long* self_off, int ne, cd* D,
                         const int* self_ld, hipStream_t st);
void launch_dense_pairs(const DevGeom& g, const KParams& P, const int* perm, cd* Tout, cd* Uout,
                        hipStream_t st);
void launch_dense_self(const cd* selfT, const cd* selfU, const int* perm, int ne, cd* Tout,
                       cd* Uout, hipStream_t st);
// Off-diagonal part of U(s_k) t0 for k = k0 .. k0+nk-1 (s_k = sigma + i k dw)
// into partial[rhs_split(ne)][nk][3 ne]; then b_k = P_k (sum + U_self t0).
// With tau (per element, tree order) the load of element e at s_k is
// exp(-s_k tau_e) t0_e (a plane wave arriving at tau_e), and
// b_k = P_k s_k (sum + U_self exp(-s_k tau) t0).
int rhs_split(int ne);
void launch_rhs_multi(const DevGeom& g, const KParams& P, double sigma, double dw, int k0, int nk,
                      const double* t0, const double* tau, cd* partial, hipStream_t st);
// The same partials for n_loads loads (t0[l] and partial[l] per load; with
// tau, tau[l] per load: incident waves, as for launch_rhs_multi), each
// pair's kernel evaluated once for up to RHS_NL loads (RHS_NL_INC with
// tau); every load's partials agree with launch_rhs_multi's for it to
// rounding.
constexpr int RHS_NL = 8;
constexpr int RHS_NL_INC = 4;
struct RhsLoadSet {
  const double* t0[RHS_NL];
  const double* tau[RHS_NL];
  cd* part[RHS_NL];
};
void launch_rhs_loads(const DevGeom& g, const KParams& P, double sigma, double dw, int k0, int nk, int n_loads,
                      const double* const* t0, const double* const* tau, cd* const* partial, hipStream_t st);
void launch_rhs_finish(const cd* partial, int nk, int kk, int ne, const cd* selfU, const double* t0,
                       const double* tau, cd s_k, const cd* phat_k, cd* b, hipStream_t st);
// b = F_k exp(-s_k tau_e) pol at every collocation point (the incident
// displacement: total-field load of a plane wave; pol on the host)
void launch_rhs_total(const double* tau, const double* pol, cd s_k, const cd* phat_k, int ne, cd* b,
                      hipStream_t st);
void launch_kernel_eval(const KParams& P, long long n, const double* x, const double* y,
                        const double* nrm, cd* U, cd* T, hipStream_t st);

// ---- transforms (Sec. 2.2 / 3.3)
void launch_load_spectrum(const double* hist, int n_f, double period, double sigma, cd* phat,
                          hipStream_t st);
void launch_mft_inverse(const cd* spec, long long N, int n_f, double period, double sigma,
                        int window, const int* perm, double* u, hipStream_t st);

}  // namespace ewbem
