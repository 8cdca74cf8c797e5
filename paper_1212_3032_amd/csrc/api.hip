// C-ABI of the ewbem library: context, setup, per-frequency assembly,
// hierarchical matvec, GMRES with solution extrapolation, and the modified
// Fourier transform back to time.  See include/ewbem.h for the contract.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <exception>
#include <functional>
#include <thread>
#include <tuple>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "ewbem.h"
#include "aca.hpp"
#include "host.hpp"
#include "launch.hpp"
#include "learn.hpp"
#include "solver.hpp"

using namespace ewbem;

namespace {

// device bytes held by the library's buffers, all contexts of the process
std::atomic<long long> g_dev_bytes{0};

// Debugging aid: with EWBEM_POISON_ALLOC set in the environment, every new
// floating-point buffer starts as all-ones bytes (NaN), so a kernel that
// reads device memory no kernel wrote shows NaN in its results instead of
// whatever the allocation held.  Integer buffers are left alone (an index
// read unwritten could point anywhere).
bool poison_alloc() {
  static const bool on = std::getenv("EWBEM_POISON_ALLOC") != nullptr;
  return on;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      (void)hipFree(p);
      g_dev_bytes -= (long long)(n * sizeof(T));
    }
    p = nullptr;
    n = 0;
  }
  void reserve(size_t cnt) {
    if (cnt <= n) return;
    // nothing in flight may still use the old allocation
    if (p) EWBEM_HIP_CHECK(hipDeviceSynchronize());
    release();
    if (cnt) {
      EWBEM_HIP_CHECK(hipMalloc((void**)&p, cnt * sizeof(T)));
      n = cnt;
      g_dev_bytes += (long long)(n * sizeof(T));
      if (std::is_floating_point<T>::value || std::is_same<T, cd>::value || std::is_same<T, cf>::value)
        if (poison_alloc()) {
          EWBEM_HIP_CHECK(hipMemset(p, 0xff, cnt * sizeof(T)));
          EWBEM_HIP_CHECK(hipDeviceSynchronize());
        }
    }
  }
  // for buffers that grow with the frequency (ranks, task lists): a quarter
  // of headroom, so they are not reallocated at every frequency
  void reserve_grow(size_t cnt) {
    if (cnt <= n) return;
    reserve(std::max(cnt, n + n / 4));
  }
  void upload(const std::vector<T>& v, hipStream_t st) {
    reserve_grow(v.size());
    if (!v.empty())
      EWBEM_HIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  }
};

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    EWBEM_HIP_CHECK(hipEventCreate(&a));
    EWBEM_HIP_CHECK(hipEventCreate(&b));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  float elapsed() {
    float ms = 0.f;
    EWBEM_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
};

void fail(int st, const std::string& m) { throw ApiError(st, m); }

}  // namespace

namespace {
// A trained network with its reduced basis (what ewbem_guess_save stores).
struct LearnedModel {
  bool ok = false;
  int r = 0;                               // reduced coordinates
  MlpShape shape;                          // dims: 6 r + 2, hidden..., 2 r
  std::vector<float> params;               // flat fp32 parameters
  std::vector<std::complex<double>> phi;   // basis, N x r column-major, caller dof order
  double energy = 0, loss0 = 0, loss1 = 0;  // training snapshots' energy in the basis; fit losses
  // the least-squares map of each frequency k = 3 .. rk - 1 over rn training
  // loads (rn = 0: none): X_k (3 r x rn) and W_k (r x rn), column-major,
  // frequency after frequency; the prediction is W_k X_k^H [c1; c2; c3]
  int rn = 0, rk = 0;
  std::vector<std::complex<double>> rx, rw;
};
}  // namespace

struct ewbem_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  std::string err;

  // ---- inputs
  bool have_mesh = false, have_mat = false, have_time = false, have_load = false;
  std::vector<double> xyz;
  std::vector<int32_t> tri;
  int nv = 0, nt = 0;
  bool exterior = true;
  double rho = 1, mu = 1, nu = 0.25;
  double period = 1;
  int n_f = 2;
  double sigma = 0;
  int window = EWBEM_WINDOW_HANN;
  bool load_is_pressure = false;
  // plane S-wave incident load: u_inc = pol f(t - dir . x / c_s), f Ricker
  bool load_incident = false;
  bool inc_total = false;  // total-field formulation: b = u_inc, the unknown is u_sc + u_inc
  double inc_dir[3] = {1, 0, 0}, inc_pol[3] = {0, 0, 1}, inc_fc = 0, inc_t0 = 0;
  std::vector<int> bc_caller;       // empty: every element has a given traction
  std::vector<double> load_caller;  // t0 (nt*3) or p (nt), caller order
  std::vector<double> history;
  ewbem_op_opts op{};
  ewbem_solver_opts so{};

  // ---- derived structure (host)
  bool structure_ok = false;  // tree + geometry + partition match the inputs
  bool device_ok = false;     // device copies of the structure are current
  HostGeom hg;
  Partition part;
  std::vector<NearBlk> near_h;
  std::vector<long long> self_off_h;
  std::vector<int> self_ld_h;
  long long near_entries = 0;
  std::vector<FarBlk> far_h;
  std::vector<int> rank_h, status_h, kcap_prev;

  // ---- device state
  DevBuf<double> d_cen, d_nrm, d_qp, d_qw, d_vtx, d_t0, d_hist, d_tau;
  DevBuf<int> d_perm, d_bc;
  DevBuf<cd> d_phat, d_selfT, d_selfU, d_selfA;
  DevBuf<NearBlk> d_near;
  DevBuf<long long> d_self_off;
  DevBuf<int> d_self_ld;
  DevBuf<cd> d_D;
  DevBuf<FarBlk> d_far;
  // far factors in two slots: the next frequency's ACA fills one while the
  // current frequency's GMRES reads the other (fslot: the matvec's slot)
  DevBuf<cd> d_wsf[2];
  int fslot = 0;
  hipStream_t astream = nullptr;  // the overlapped ACA's stream (library-owned)
  WsSide ws_side;                 // the warm start's second stream (library-owned)
  // one buffer per capacity-retry round of the current frequency; all stay
  // alive until the next frequency is assembled (blocks retried in an
  // earlier round keep pointing into their round's buffer)
  std::vector<std::unique_ptr<DevBuf<cd>>> d_retry[2];
  DevBuf<cf> d_f32;
  DevBuf<long long> d_uo, d_vo;
  // streamed complex64 store (op.aca_batch_mb > 0): chunks filled in block
  // order as the batches finish; block b's factors at u32_h[b], v32_h[b]
  std::vector<std::unique_ptr<DevBuf<cf>>> d_f32s;
  std::vector<cf*> u32_h, v32_h;
  bool streamed = false;  // the factors in use came from a streamed run
  DevBuf<int> d_batch_ids;
  DevBuf<cf*> d_u32p, d_v32p;
  DevBuf<int> d_rank, d_status;
  // lock-step ACA: per-block state, used-row bits, active lists and scans
  DevBuf<AcaState> d_acast;
  DevBuf<AcaPlan> d_acaplan;
  DevBuf<double> d_aca_part;
  DevBuf<int> d_aca_cold;
  // warm starts: pivot lists (kept across frequencies) and their work areas
  bool plist_ok = false;
  DevBuf<int> d_plist, d_nlist;
  std::vector<int> nlist_h;
  DevBuf<WsBlk> d_wsb;
  DevBuf<int> d_wsoff, d_wspq, d_wsrho, d_wslu;
  DevBuf<unsigned long long> d_wscnt;  // warm-start pivot and kept-term counts of one call
  DevBuf<double> d_ser;  // series coefficients of the kernels (KParams::ser)
  double ser_g = -1.0;   // the c_s / c_p they were formed for
  DevBuf<cd> d_cross, d_wscoef;
  DevBuf<double> d_wspart;
  DevBuf<unsigned> d_used;
  DevBuf<int> d_aca_ids, d_act, d_act2, d_offs, d_tot;
  DevBuf<VtTask> d_vt;
  DevBuf<Seg> d_seg;
  DevBuf<RowTask> d_rt;
  DevBuf<LeafRange> d_lr;
  // host copies of the matvec tables, for the batch's concatenated launch
  std::vector<VtTask> vt_h;
  DevBuf<VtTask> d_vt16;  // phase-1 tasks of 16 factor columns (eight vectors on the matrix cores)
  int n_vt16 = 0;
  std::vector<Seg> seg_h;
  std::vector<RowTask> rt_h;
  std::vector<LeafRange> lr_h;
  int n_vt = 0, n_rt = 0, n_lr = 0;
  // matvec task shapes: factor columns per phase-1 wavefront and the phase-2
  // task size (total panel columns / mv_div per task); chosen by timing on
  // the first assembled operator when op.autotune is set
  int mv_cols = 4, mv_div = 4096, vt_cols = 4;
  bool mv_tuned = false;
  bool mv_tune_cached = false;  // shapes from an earlier context's tuning
  double mv_best_ms = 0, mv_default_ms = 0;  // tuning: fastest and default shapes' matvec time
  DevBuf<cd> d_z, d_hpart, d_mvpart;
  long long z_len = 0, mvpart_len = 0;  // one right-hand side's share of d_z, d_mvpart
  DevBuf<cd> d_rhs_part;
  int boff_k0 = 0, boff_nk = 0;   // frequencies whose off-diagonal U t0 is in d_rhs_part
  // preconditioner
  DevBuf<cd> d_M3, d_Minv;
  DevBuf<long long> d_minv_off, d_minv_src;
  DevBuf<int> d_minv_dim, d_minv_row0, d_minv_ld, d_pivfail;
  int n_minv = 0;
  // vectors (tree order)
  DevBuf<cd> d_b, d_x, d_r, d_w, d_u, d_zt, d_V, d_small, d_tmp_in, d_tmp_out;
  DevBuf<cd> d_amx;  // ewbem_apply_multi: the columns in tree order, in and out
  DevBuf<cd> d_Y, d_hist_sol, d_spec;
  int hist_n = 0, hist_head = 0;  // ring buffer of the last sem_k solutions
  std::vector<int> hist_slot;  // newest first
  std::vector<int> hist_kidx;  // frequency index of each of those slots

  // learned initial guess: the model (host, caller dof order) and its device
  // copies; reduced coordinates of the last three solutions in a ring
  LearnedModel lm;
  bool lm_dev = false;  // device copies of lm current
  DevBuf<cd> d_phi, d_lcoef, d_lpred, d_lx;
  DevBuf<cd> d_rx, d_rw, d_lh, d_lz, d_lbase;  // least-squares map and its inference buffers
  DevBuf<float> d_lp, d_lfeat, d_lact, d_lpre, d_ly, d_lkf;
  DevBuf<int> d_lidx;
  DevBuf<double> d_lnu;
  std::vector<int> lc_slot, lc_kidx;  // newest first

  int assembled_k = -1;
  KParams P{};
  SelfRule S{};
  int store_c64_active = 0;
  double matvec_bytes = 0, stored_bytes = 0;
  double matvec_rhs_bytes = 0;  // the part of matvec_bytes each right-hand side adds
  int64_t rank_sum = 0, rank_max = 0;

  // per-call accumulators
  ewbem_stats acc{};
};

namespace {

// Kernel parameters at s; the series coefficients (material constants) live
// in a small device buffer of the context, uploaded when the material changes.
KParams make_params(ewbem_ctx* c, cd s) {
  const double rho = c->rho, mu = c->mu, nu = c->nu;
  KParams P{};
  const double lam = 2.0 * mu * nu / (1.0 - 2.0 * nu);
  const double cs = std::sqrt(mu / rho), cp = std::sqrt((lam + 2.0 * mu) / rho);
  const double g = cs / cp;
  P.s = s;
  const double s2 = s.x * s.x + s.y * s.y;
  P.cs_over_s = s2 > 0.0 ? cd{cs * s.x / s2, -cs * s.y / s2} : mk(0.0);
  P.inv_cs = 1.0 / cs;
  P.gamma = g;
  P.g2 = g * g;
  P.ratio = (cp / cs) * (cp / cs);
  P.inv4pi = 1.0 / (4.0 * M_PI);
  P.inv4pimu = 1.0 / (4.0 * M_PI * mu);
  P.cpv = g * g / (4.0 * M_PI);
  P.series_z2 = 0.25;
  // Taylor coefficients of r phi, r psi in z = s r / c_s (index m = n - 2):
  //   r phi: (-1)^n (n-1)(n-1+g^n)/n!,  r psi: (-1)^n (n-1)(n-3)(1-g^n)/n!,
  //   r^2 phi', r^2 psi': the same times (n-3).
  double ser[4 * NSER];  // c_phi, c_psi, c_dphi, c_dpsi
  double fact = 1.0;     // n!
  for (int n = 2; n < NSER + 2; ++n) {
    fact *= n;
    const double sgn = (n % 2 == 0) ? 1.0 : -1.0;
    const double gn = std::pow(g, n);
    const double cphi = sgn * (n - 1) * (n - 1 + gn) / fact;
    const double cpsi = sgn * (n - 1) * (n - 3) * (1.0 - gn) / fact;
    ser[n - 2] = cphi;
    ser[NSER + n - 2] = cpsi;
    ser[2 * NSER + n - 2] = (n - 3) * cphi;
    ser[3 * NSER + n - 2] = (n - 3) * cpsi;
  }
  P.stat_rphi = ser[0];
  P.stat_rpsi = ser[NSER];
  if (c->device >= 0 && (!c->d_ser.p || c->ser_g != g)) {
    c->d_ser.reserve(4 * NSER);
    EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_ser.p, ser, sizeof(ser), hipMemcpyHostToDevice, c->stream));
    EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
    c->ser_g = g;
  }
  P.ser = c->d_ser.p;
  return P;
}

void require_gpu(ewbem_ctx* c) {
  if (c->device < 0) fail(EWBEM_ESTATE, "host-only context: no GPU work possible");
}

void ensure_structure(ewbem_ctx* c) {
  if (!c->have_mesh) fail(EWBEM_ESTATE, "mesh not set");
  if (c->structure_ok) return;
  c->part = Partition();
  std::vector<int> perm = build_tree(c->nv, c->xyz.data(), c->nt, c->tri.data(), c->op.leaf_size,
                                     c->part.clusters);
  build_geometry(c->nv, c->xyz.data(), c->nt, c->tri.data(), c->exterior, perm, c->hg);
  build_partition(c->op.kind == EWBEM_OP_DENSE ? 0.0 : c->op.eta_adm, c->part, ACA_MAXM);
  // near-block layout (each block column-major, ld = 3 m) and the position
  // of every element's self block inside its diagonal near block
  c->near_h.clear();
  c->self_off_h.assign(c->nt, -1);
  c->self_ld_h.assign(c->nt, 0);
  long long off = 0;
  for (const BlockPair& bp : c->part.near) {
    const Cluster& r = c->part.clusters[bp.row];
    const Cluster& s = c->part.clusters[bp.col];
    NearBlk nb{r.begin, r.size(), s.begin, s.size(), off};
    c->near_h.push_back(nb);
    if (bp.row == bp.col)
      for (int a = 0; a < r.size(); ++a) {
        c->self_off_h[r.begin + a] = off + (long long)(3 * a) * (3 * r.size()) + 3 * a;
        c->self_ld_h[r.begin + a] = 3 * r.size();
      }
    off += 9LL * r.size() * s.size();
  }
  c->near_entries = off;
  for (int e = 0; e < c->nt; ++e)
    if (c->self_off_h[e] < 0) fail(EWBEM_EINVAL, "internal: element without a diagonal near block");
  c->far_h.clear();
  for (const BlockPair& bp : c->part.far) {
    const Cluster& r = c->part.clusters[bp.row];
    const Cluster& s = c->part.clusters[bp.col];
    if (r.size() > ACA_MAXM || s.size() > ACA_MAXM)
      fail(EWBEM_EINVAL, "internal: far block with more than 16384 elements on a side");
    FarBlk fb{};
    fb.r0 = r.begin;
    fb.m = r.size();
    fb.c0 = s.begin;
    fb.n = s.size();
    c->far_h.push_back(fb);
  }
  c->kcap_prev.assign(c->far_h.size(), 0);
  c->plist_ok = false;
  c->mv_tuned = false;
  c->mv_tune_cached = false;
  c->mv_cols = 4;
  c->mv_div = 4096;
  c->rank_h.assign(c->far_h.size(), 0);
  c->status_h.assign(c->far_h.size(), 0);
  c->structure_ok = true;
  c->device_ok = false;
  c->assembled_k = -1;
}

// The plane S-wave along unit d polarised along unit q, per element in tree
// order: the frequency-independent factor g of the scattered-field load
//   t_sc(s) = s F(s) exp(-s tau) g,  g = (mu / c_s)(q (d.n) + d (q.n))
// (the negated traction of the plane wave on a surface of normal n), and the
// arrival delay tau = d.x / c_s at each collocation point.
void incident_factors(const ewbem_ctx* c, const double* d, const double* q, std::vector<double>& g0,
                      std::vector<double>& tau) {
  const HostGeom& g = c->hg;
  const double cs = std::sqrt(c->mu / c->rho), f = c->mu / cs;
  g0.assign(3 * (size_t)c->nt, 0.0);
  tau.assign(c->nt, 0.0);
  for (int t = 0; t < c->nt; ++t) {
    const double* n = &g.nrm[3 * (size_t)t];
    const double dn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    const double qn = q[0] * n[0] + q[1] * n[1] + q[2] * n[2];
    for (int k = 0; k < 3; ++k) g0[3 * (size_t)t + k] = f * (q[k] * dn + d[k] * qn);
    tau[t] = (d[0] * g.cen[3 * (size_t)t] + d[1] * g.cen[3 * (size_t)t + 1] + d[2] * g.cen[3 * (size_t)t + 2]) / cs;
  }
}

std::vector<double> tree_load(ewbem_ctx* c) {
  // traction per element in tree order; for the incident S-wave, the factor
  // g of incident_factors
  const HostGeom& g = c->hg;
  std::vector<double> t0(3 * (size_t)c->nt);
  if (c->load_incident) {
    std::vector<double> tau;
    incident_factors(c, c->inc_dir, c->inc_pol, t0, tau);
    return t0;
  }
  for (int t = 0; t < c->nt; ++t) {
    const int e = g.perm[t];
    for (int k = 0; k < 3; ++k)
      t0[3 * t + k] = c->load_is_pressure ? -c->load_caller[e] * g.nrm[3 * t + k]
                                          : c->load_caller[3 * (size_t)e + k];
  }
  return t0;
}

// Device copies of the learned model: the basis in tree order, the
// parameters, and the inference buffers (one sample).
void learned_upload(ewbem_ctx* c) {
  const LearnedModel& m = c->lm;
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  const int r = m.r;
  std::vector<cd> ph((size_t)N * r);
  for (int j = 0; j < r; ++j)
    for (int t = 0; t < c->nt; ++t) {
      const size_t e = (size_t)c->hg.perm[t];
      for (int i = 0; i < 3; ++i) {
        const std::complex<double> v = m.phi[(size_t)j * N + 3 * e + i];
        ph[(size_t)j * N + 3 * (size_t)t + i] = cd{v.real(), v.imag()};
      }
    }
  c->d_phi.upload(ph, st);
  c->d_lp.upload(m.params, st);
  if (m.rn > 0) {
    std::vector<cd> rx(m.rx.size()), rw(m.rw.size());
    for (size_t i = 0; i < rx.size(); ++i) rx[i] = cd{m.rx[i].real(), m.rx[i].imag()};
    for (size_t i = 0; i < rw.size(); ++i) rw[i] = cd{m.rw[i].real(), m.rw[i].imag()};
    c->d_rx.upload(rx, st);
    c->d_rw.upload(rw, st);
    c->d_lh.reserve(3 * (size_t)r);
    c->d_lz.reserve(m.rn);
    c->d_lbase.reserve(r);
  }
  const int L = m.shape.n_layers();
  c->d_lcoef.reserve(4 * (size_t)r);  // the ring of three, then scratch for Phi^H x
  c->d_lpred.reserve(r);
  c->d_lx.reserve(N);
  c->d_lfeat.reserve(m.shape.dims[0]);
  c->d_lact.reserve(std::max<size_t>(1, m.shape.hidden_sum()));
  c->d_lpre.reserve(std::max<size_t>(1, m.shape.hidden_sum()));
  c->d_ly.reserve(m.shape.dims[L]);
  c->d_lkf.reserve(1);
  c->d_lidx.reserve(4);
  c->d_lnu.reserve(1);
  c->d_hpart.reserve((size_t)dots_chunks(N) * std::max(r, m.rn));
  c->lc_slot.clear();
  c->lc_kidx.clear();
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  c->lm_dev = true;
}

void ensure_device(ewbem_ctx* c) {
  require_gpu(c);
  ensure_structure(c);
  if (!c->have_mat) fail(EWBEM_ESTATE, "material not set");
  if (!c->have_time) fail(EWBEM_ESTATE, "time grid not set");
  if (!c->have_load) fail(EWBEM_ESTATE, "load not set");
  if (c->device_ok) {
    if (c->lm.ok && !c->lm_dev) learned_upload(c);
    return;
  }
  EWBEM_HIP_CHECK(hipSetDevice(c->device));
  if (!c->astream) EWBEM_HIP_CHECK(hipStreamCreateWithFlags(&c->astream, hipStreamNonBlocking));
  if (!c->ws_side.stream) {
    EWBEM_HIP_CHECK(hipStreamCreateWithFlags(&c->ws_side.stream, hipStreamNonBlocking));
    EWBEM_HIP_CHECK(hipEventCreateWithFlags(&c->ws_side.fork, hipEventDisableTiming));
    EWBEM_HIP_CHECK(hipEventCreateWithFlags(&c->ws_side.join, hipEventDisableTiming));
  }
  hipStream_t st = c->stream;
  const HostGeom& g = c->hg;
  c->d_cen.upload(g.cen, st);
  c->d_nrm.upload(g.nrm, st);
  c->d_qp.upload(g.qp, st);
  c->d_qw.upload(g.qw, st);
  c->d_vtx.upload(g.vtx, st);
  c->d_perm.upload(g.perm, st);
  std::vector<double> t0 = tree_load(c);
  c->d_t0.upload(t0, st);
  if (c->load_incident) {
    // arrival delay of the plane wave at each collocation point
    std::vector<double> g0, tau;
    incident_factors(c, c->inc_dir, c->inc_pol, g0, tau);
    c->d_tau.upload(tau, st);
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));  // tau is a temporary
  }
  if (!c->bc_caller.empty()) {
    std::vector<int> bct(c->nt);
    for (int t = 0; t < c->nt; ++t) bct[t] = c->bc_caller[g.perm[t]];
    c->d_bc.upload(bct, st);
  }
  c->d_hist.upload(c->history, st);
  c->d_phat.reserve(c->n_f / 2 + 1);
  launch_load_spectrum(c->d_hist.p, c->n_f, c->period, c->sigma, c->d_phat.p, st);
  c->d_near.upload(c->near_h, st);
  c->d_self_off.upload(c->self_off_h, st);
  c->d_self_ld.upload(c->self_ld_h, st);
  c->d_D.reserve(std::max<long long>(c->near_entries, 1));
  const long long N = 3LL * c->nt;
  c->d_selfT.reserve(9 * (size_t)c->nt);
  c->d_selfU.reserve(9 * (size_t)c->nt);
  c->d_selfA.reserve(9 * (size_t)c->nt);
  c->boff_nk = 0;
  for (DevBuf<cd>* v : {&c->d_b, &c->d_x, &c->d_r, &c->d_w, &c->d_u, &c->d_zt, &c->d_tmp_in, &c->d_tmp_out})
    v->reserve(N);
  const int m = c->so.restart;
  c->d_V.reserve((size_t)std::max(m + 1, c->so.sem_k + 1) * N);
  c->d_small.reserve(4 * (size_t)(m + 2) + 16);
  c->d_hpart.reserve((size_t)dots_chunks(N) * std::max(m + 2, c->so.sem_k + 1));
  c->d_Y.reserve((size_t)(c->so.sem_k + 1) * N);
  c->d_hist_sol.reserve((size_t)std::max(1, c->so.sem_k) * N);
  c->d_spec.reserve((size_t)(c->n_f / 2 + 1) * N);
  c->d_M3.reserve(9 * (size_t)c->nt);
  // self rule
  c->S.nt = c->S.nr = c->op.self_order;
  gauss_legendre01(c->op.self_order, c->S.t, c->S.wt);
  gauss_legendre01(c->op.self_order, c->S.u, c->S.wu);
  c->P = make_params(c, mk(0.0));
  c->hist_n = 0;
  c->hist_head = 0;
  c->hist_slot.clear();
  c->hist_kidx.clear();
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  c->lm_dev = false;
  if (c->lm.ok) learned_upload(c);
  c->device_ok = true;
  c->assembled_k = -1;
}

DevGeom dev_geom(ewbem_ctx* c) {
  DevGeom g;
  g.ne = c->nt;
  g.cen = c->d_cen.p;
  g.nrm = c->d_nrm.p;
  g.qp = c->d_qp.p;
  g.qw = c->d_qw.p;
  g.vtx = c->d_vtx.p;
  g.bc = c->bc_caller.empty() ? nullptr : c->d_bc.p;
  return g;
}

cd s_of_k(ewbem_ctx* c, int k) { return cd{c->sigma, 2.0 * M_PI * k / c->period}; }

// ---- ACA with capacity retries, then matvec task lists

// Cores of at most 128 x 128 are eliminated in registers (k_ws_lu_reg).
constexpr bool kWsLuReg = true;

// Lock-step cross approximation of the far blocks ids (their FarBlk
// entries already on the device).  Blocks with pivot lists from the previous
// frequency (and warm set) start from the cross on those pivots, the others
// from scratch; then all run the ordinary steps, one host round trip per
// step (the scan of the active list gives the grid sizes).
void aca_lockstep(ewbem_ctx* c, const DevGeom& g, const std::vector<int>& ids, bool warm, bool count_starts,
                  hipStream_t st) {
  const int n = (int)ids.size();
  if (n == 0) return;
  std::vector<int> cold;
  std::vector<WsBlk> wb;
  std::vector<int> woff;  // er, ec, tu, tv offsets, 4 x (nwarm + 1)
  long long cross = 0, er = 0, ec = 0, tu = 0, tv = 0, pqn = 0, part = 0, coefn = 0;
  for (int b : ids) {
    const FarBlk& f = c->far_h[b];
    const int nr = c->nlist_h[2 * b], nc = c->nlist_h[2 * b + 1];
    if (!warm || nr <= 0 || nc <= 0 || nr > WS_MAXLIST || nc > WS_MAXLIST) {
      cold.push_back(b);
      continue;
    }
    WsBlk w{};
    w.blk = b;
    w.nr = nr;
    w.nc = nc;
    w.rcap = std::min(3 * std::min(nr, nc), f.kcap);
    w.rr = cross;
    cross += 9LL * nr * f.n;
    w.cc = cross;
    cross += 9LL * nc * f.m;
    w.w = cross;
    cross += 9LL * nr * nc;
    w.pq = (int)pqn;
    pqn += 2LL * w.rcap;
    const int ntu = (3 * f.m + WS_TILE_ROWS - 1) / WS_TILE_ROWS, ntv = (3 * f.n + WS_TILE_ROWS - 1) / WS_TILE_ROWS;
    w.tu = (int)tu;
    w.tv = (int)tv;
    w.pu = part;
    part += (long long)ntu * w.rcap;
    w.pv = part;
    part += (long long)ntv * w.rcap;
    w.co = coefn;
    coefn += 2 * ws_panel_elems(w.rcap);  // substitution panels, U and V sides
    wb.push_back(w);
    er += (long long)nr * f.n;
    ec += (long long)nc * f.m;
    tu += ntu;
    tv += ntv;
  }
  const int nw = (int)wb.size();
  int n_lu_count[WS_NCLASS] = {0, 0, 0, 0, 0, 0, 0};
  unsigned long long ws_cnt[2] = {0ull, 0ull};
  if (er > INT32_MAX / 2 || ec > INT32_MAX / 2 || tu > INT32_MAX / 2 || tv > INT32_MAX / 2 || pqn > INT32_MAX / 2)
    fail(EWBEM_EINVAL, "warm start larger than its index range");
  AcaWork W0{c->d_far.p, c->d_acast.p, c->d_acaplan.p, c->d_used.p, nullptr, nullptr, c->d_plist.p, c->d_nlist.p};
  c->d_aca_ids.upload(ids, st);
  c->d_act.reserve(n);
  c->d_act2.reserve(n);
  c->d_tot.reserve(6);
  int* count = c->d_tot.p + 5;
  if (!cold.empty()) {
    c->d_aca_cold.upload(cold, st);
    launch_aca_init(c->d_aca_cold.p, (int)cold.size(), c->d_far.p, c->d_acast.p, c->d_used.p, c->d_nlist.p, st);
  }
  if (nw > 0) {
    woff.assign(4 * (size_t)(nw + 1), 0);
    for (int i = 0; i < nw; ++i) {
      const FarBlk& f = c->far_h[wb[i].blk];
      woff[i + 1] = woff[i] + wb[i].nr * f.n;
      woff[(nw + 1) + i + 1] = woff[(nw + 1) + i] + wb[i].nc * f.m;
      woff[2 * (nw + 1) + i + 1] = woff[2 * (nw + 1) + i] + (3 * f.m + WS_TILE_ROWS - 1) / WS_TILE_ROWS;
      woff[3 * (nw + 1) + i + 1] = woff[3 * (nw + 1) + i] + (3 * f.n + WS_TILE_ROWS - 1) / WS_TILE_ROWS;
    }
    c->d_wsb.upload(wb, st);
    c->d_wsoff.upload(woff, st);
    c->d_cross.reserve_grow(std::max<long long>(cross, 1));
    c->d_wspq.reserve_grow(std::max<long long>(pqn, 1));
    c->d_wsrho.reserve(nw);
    c->d_wspart.reserve_grow(std::max<long long>(part, 1));
    c->d_wscoef.reserve_grow(std::max<long long>(coefn, 1));
    // size classes of the core elimination
    std::vector<int> lu_list;
    int n_lu[WS_NCLASS] = {0, 0, 0, 0, 0, 0, 0};
    std::vector<int> cls_of(nw);
    for (int i = 0; i < nw; ++i) {
      const int R3 = 3 * wb[i].nr, C3 = 3 * wb[i].nc;
      const long long e = (long long)R3 * C3;
      cls_of[i] = (kWsLuReg && R3 <= WS_REG_SMALL && C3 <= WS_REG_SMALL)   ? 5
                  : (kWsLuReg && R3 <= WS_REG_LARGE && C3 <= WS_REG_LARGE) ? 6
                  : R3 > 64 * WS_LU_NR_LDS                                  ? 3
                  : (R3 <= 64 && e <= WS_LDS_TINY)                          ? 4
                  : e <= WS_LDS_SMALL                                       ? 0
                  : e <= WS_LDS_MID                                         ? 1
                  : e <= WS_LDS_LARGE                                       ? 2
                                                                            : 3;
    }
    for (int cls = 0; cls < WS_NCLASS; ++cls)
      for (int i = 0; i < nw; ++i)
        if (cls_of[i] == cls) {
          lu_list.push_back(i);
          ++n_lu[cls];
        }
    c->d_wslu.upload(lu_list, st);
    for (int cls = 0; cls < WS_NCLASS; ++cls) n_lu_count[cls] = n_lu[cls];
    WsArgs A{c->d_wsb.p, nw, c->d_wsoff.p, c->d_wsoff.p + (nw + 1), c->d_wsoff.p + 2 * (nw + 1),
             c->d_wsoff.p + 3 * (nw + 1), (int)er, (int)ec, (int)tu, (int)tv, c->d_cross.p, c->d_wspq.p,
             c->d_wsrho.p, c->d_wspart.p, c->d_wscoef.p, c->d_wslu.p,
             {n_lu[0], n_lu[1], n_lu[2], n_lu[3], n_lu[4], n_lu[5], n_lu[6]}, 0.0, 0, nullptr};
    const double prel = c->op.ws_pivot_rel > 0 ? c->op.ws_pivot_rel : c->op.aca_tol;
    A.stop2 = prel * prel;
    A.keep_all = c->op.ws_keep;
    c->d_wscnt.reserve(2);
    A.cnt = c->d_wscnt.p;
    EWBEM_HIP_CHECK(hipMemsetAsync(A.cnt, 0, 2 * sizeof(unsigned long long), st));
    launch_ws(A, W0, g, c->P, c->op.aca_tol, st, c->ws_side);
    // read with the first step's synchronisation below
    EWBEM_HIP_CHECK(hipMemcpyAsync(ws_cnt, A.cnt, sizeof(ws_cnt), hipMemcpyDeviceToHost, st));
  }
  if (count_starts) {
    c->acc.aca_warm_blocks += nw;
    c->acc.aca_cold_blocks += (long long)cold.size();
    for (int cls = 0; cls < WS_NCLASS; ++cls) c->acc.aca_core_blocks[cls] += n_lu_count[cls];
  }
  bool counted = !count_starts || nw == 0;
  // the active list: every block still ACA_ACTIVE after its start
  EWBEM_HIP_CHECK(hipMemsetD32Async((hipDeviceptr_t)count, 0, 1, st));
  launch_aca_compact(c->d_aca_ids.p, n, c->d_acast.p, c->d_act.p, count, st);
  const int stride = n + 1;
  c->d_offs.reserve(4 * (size_t)stride);
  int* act = c->d_act.p;
  int* nxt = c->d_act2.p;
  // every step either adds at least one term or counts a failed row (at
  // most four in a row), so the number of steps is bounded
  const int max_steps = 5 * ACA_KMAX + 16;
  int tot[5] = {0, 0, 0, 0, 0};
  bool sized = false;
  for (int it = 0;; ++it) {
    launch_aca_scan(act, count, c->d_far.p, c->d_offs.p, stride, c->d_tot.p, st);
    EWBEM_HIP_CHECK(hipMemcpyAsync(tot, c->d_tot.p, 5 * sizeof(int), hipMemcpyDeviceToHost, st));
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    if (!counted) {
      c->acc.aca_warm_pivots += (long long)ws_cnt[0];
      c->acc.aca_warm_kept += (long long)ws_cnt[1];
      counted = true;
    }
    const int nact = tot[4];
    if (it == 0) c->acc.aca_step_first += nact;
    if (nact == 0) break;
    c->acc.aca_steps += 1;
    c->acc.aca_step_blocks += nact;
    if (nact < 0 || nact > n || it > max_steps) fail(EWBEM_EINVAL, "internal: ACA active list out of range");
    EWBEM_HIP_CHECK(hipMemsetD32Async((hipDeviceptr_t)count, 0, 1, st));
    // the first step has the most active blocks, so the largest task counts
    if (!sized) {
      c->d_aca_part.reserve_grow(3 * ((size_t)tot[2] + (size_t)tot[3]));
      sized = true;
    }
    if ((size_t)3 * ((size_t)tot[2] + (size_t)tot[3]) > c->d_aca_part.n)
      fail(EWBEM_EINVAL, "internal: ACA task count grew");
    AcaLists L{act, nact, tot[0], tot[1], tot[2], tot[3], c->d_offs.p, c->d_offs.p + stride,
               c->d_offs.p + 2 * stride, c->d_offs.p + 3 * stride};
    AcaWork W = W0;
    W.part_u = c->d_aca_part.p;
    W.part_v = c->d_aca_part.p + 3 * (size_t)tot[3];
    launch_aca_step(L, W, g, c->P, c->op.aca_tol, nxt, count, st);
    std::swap(act, nxt);
  }
  launch_aca_finish(c->d_aca_ids.p, n, c->d_acast.p, c->d_rank.p, c->d_status.p, st);
}

// Far factors of every block into factor slot ``slot`` on stream st.  With
// op.aca_batch_mb > 0 the blocks go in batches through one complex128 work
// area, each batch converted into the streamed complex64 store as it
// finishes.
void run_aca(ewbem_ctx* c, const DevGeom& g, EventPair& ev, double& aca_ms, hipStream_t st, int slot) {
  const int nf = (int)c->far_h.size();
  if (nf == 0) return;
  // Capacity: 50% (at least 24 terms) above the previous frequency's rank
  // (ranks grow with frequency), else a size-based first guess; retries
  // are the exception.
  // 3 min(m, n) + 2 columns always suffice: a block stops at full rank, and
  // a step adds at most three terms.
  // pivot lists for warm starts: allocated with the partition, empty until a
  // first approximation has run
  if (!c->plist_ok) {
    long long poff = 0;
    for (int b = 0; b < nf; ++b) {
      c->far_h[b].poff = (int)poff;
      poff += 2LL * c->far_h[b].m;
    }
    if (poff > INT32_MAX) fail(EWBEM_EINVAL, "too many far-block rows");
    c->d_plist.reserve(std::max<long long>(poff, 1));
    c->d_nlist.reserve(2 * (size_t)nf);
    EWBEM_HIP_CHECK(hipMemsetAsync(c->d_nlist.p, 0, 2 * (size_t)nf * sizeof(int), st));
    c->nlist_h.assign(2 * (size_t)nf, 0);
    c->plist_ok = true;
  }
  const bool warm = c->op.aca_reuse != 0;
  std::vector<int> kcap(nf);
  for (int b = 0; b < nf; ++b) {
    const FarBlk& f = c->far_h[b];
    const int full = 3 * std::min(f.m, f.n) + 2;
    int want = c->kcap_prev[b] > 0 ? c->rank_h[b] + std::max(24, c->rank_h[b] / 2)
                                   : 24 + (f.m + f.n) / 8;
    const int nr = c->nlist_h[2 * b], nc = c->nlist_h[2 * b + 1];
    if (warm && nr > 0 && nc > 0) want = std::max(want, 3 * std::min(nr, nc) + 6);
    want = ((want + 2) / 3) * 3;
    kcap[b] = std::max(3, std::min({want, full, ACA_KMAX}));
  }
  // batches of blocks (one batch of all unless streamed)
  const bool streamed = c->op.aca_batch_mb > 0 && c->op.far_store == EWBEM_STORE_C64;
  std::vector<std::vector<int>> batches(1);
  if (streamed) {
    const double budget = (double)c->op.aca_batch_mb * 1048576.0;
    double acc = 0;
    for (int b = 0; b < nf; ++b) {
      const FarBlk& f = c->far_h[b];
      const double nr = c->nlist_h[2 * b], nc = c->nlist_h[2 * b + 1];
      const double rc = 3.0 * std::min(nr, nc);
      const double need = 16.0 * (3.0 * (f.m + f.n) * kcap[b] + 9.0 * (nr * f.n + nc * f.m + nr * nc) +
                                  2.0 * (rc + 8) * rc);
      if (!batches.back().empty() && acc + need > budget) {
        batches.emplace_back();
        acc = 0;
      }
      batches.back().push_back(b);
      acc += need;
    }
  } else {
    batches[0].resize(nf);
    for (int b = 0; b < nf; ++b) batches[0][b] = b;
  }
  c->streamed = streamed;
  if (streamed) {
    c->u32_h.assign(nf, nullptr);
    c->v32_h.assign(nf, nullptr);
  }
  size_t chunk_i = 0, chunk_used = 0;  // fill position in the streamed store
  auto store_alloc = [&](size_t n) -> cf* {
    constexpr size_t kChunk = size_t(1) << 29;  // 4 GiB of complex64 entries
    while (true) {
      if (chunk_i < c->d_f32s.size() && chunk_used + n <= c->d_f32s[chunk_i]->n) {
        cf* p = c->d_f32s[chunk_i]->p + chunk_used;
        chunk_used += n;
        return p;
      }
      if (chunk_i < c->d_f32s.size() && chunk_used > 0) {  // next chunk
        ++chunk_i;
        chunk_used = 0;
        continue;
      }
      if (chunk_i >= c->d_f32s.size()) {
        c->d_f32s.emplace_back(new DevBuf<cf>());
        c->d_f32s.back()->reserve(std::max(n, kChunk));
      } else {
        // an existing, empty chunk too small for this block: a larger one in its place
        c->d_f32s[chunk_i]->reserve(n);
      }
    }
  };
  DevBuf<cd>& ws = c->d_wsf[slot];
  c->d_retry[slot].clear();
  long long words = 0;
  for (int b = 0; b < nf; ++b) {
    FarBlk& f = c->far_h[b];
    if (words > INT32_MAX - 1024) fail(EWBEM_EINVAL, "too many far blocks");
    f.bitoff = (int)words;
    words += (f.m + 31) / 32;
  }
  c->d_used.reserve(words);
  c->d_acast.reserve(nf);
  c->d_acaplan.reserve(nf);
  c->d_rank.reserve(nf);
  c->d_status.reserve(nf);
  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const std::vector<int>& ids = batches[bi];
    // main layout (the previous batch's or frequency's retry buffers are no
    // longer used)
    c->d_retry[slot].clear();
    long long total = 0;
    for (int b : ids) total += (long long)(3 * c->far_h[b].m + 3 * c->far_h[b].n) * kcap[b];
    if (streamed)
      ws.reserve(std::max<long long>(total, 1));
    else
      ws.reserve_grow(total);
    long long off = 0;
    for (int b : ids) {
      FarBlk& f = c->far_h[b];
      f.kcap = kcap[b];
      f.U = ws.p + off;
      off += 3LL * f.m * kcap[b];
      f.V = ws.p + off;
      off += 3LL * f.n * kcap[b];
    }
    c->d_far.upload(c->far_h, st);
    EWBEM_HIP_CHECK(hipEventRecord(ev.a, st));
    aca_lockstep(c, g, ids, warm, true, st);
    EWBEM_HIP_CHECK(hipEventRecord(ev.b, st));
    EWBEM_HIP_CHECK(hipMemcpyAsync(c->rank_h.data(), c->d_rank.p, nf * sizeof(int), hipMemcpyDeviceToHost, st));
    EWBEM_HIP_CHECK(hipMemcpyAsync(c->status_h.data(), c->d_status.p, nf * sizeof(int), hipMemcpyDeviceToHost, st));
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    aca_ms += ev.elapsed();
    // retries for blocks that ran out of capacity, in a separate buffer
    for (int round = 0; round < 8; ++round) {
      std::vector<int> over;
      for (int b : ids)
        if (c->status_h[b] != 0) over.push_back(b);
      if (over.empty()) break;
      c->acc.aca_retries += (long long)over.size();
      long long tot2 = 0;
      for (int b : over) {
        FarBlk& f = c->far_h[b];
        const int full = 3 * std::min(f.m, f.n) + 2;
        if (f.kcap >= std::min(full, ACA_KMAX))
          fail(EWBEM_EINVAL, "ACA rank exceeds the per-block limit of 1024");
        f.kcap = std::min({full, ACA_KMAX, 2 * f.kcap + 6});
        tot2 += (long long)(3 * f.m + 3 * f.n) * f.kcap;
      }
      c->d_retry[slot].emplace_back(new DevBuf<cd>());
      DevBuf<cd>& buf = *c->d_retry[slot].back();
      buf.reserve(tot2);
      long long o2 = 0;
      for (int b : over) {
        FarBlk& f = c->far_h[b];
        f.U = buf.p + o2;
        o2 += 3LL * f.m * f.kcap;
        f.V = buf.p + o2;
        o2 += 3LL * f.n * f.kcap;
      }
      c->d_far.upload(c->far_h, st);
      // the retry starts warm from the elements of every pivot accepted so
      // far (the lists the overflowing run left), not from scratch
      if (warm) {
        EWBEM_HIP_CHECK(hipMemcpyAsync(c->nlist_h.data(), c->d_nlist.p, 2 * (size_t)nf * sizeof(int),
                                       hipMemcpyDeviceToHost, st));
        EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      }
      EWBEM_HIP_CHECK(hipEventRecord(ev.a, st));
      aca_lockstep(c, g, over, warm, false, st);
      EWBEM_HIP_CHECK(hipEventRecord(ev.b, st));
      EWBEM_HIP_CHECK(hipMemcpyAsync(c->rank_h.data(), c->d_rank.p, nf * sizeof(int), hipMemcpyDeviceToHost, st));
      EWBEM_HIP_CHECK(hipMemcpyAsync(c->status_h.data(), c->d_status.p, nf * sizeof(int), hipMemcpyDeviceToHost, st));
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      aca_ms += ev.elapsed();
    }
    for (int b : ids) {
      if (c->status_h[b] != 0) fail(EWBEM_EINVAL, "ACA did not converge within its capacity");
      if (c->rank_h[b] < 0 || c->rank_h[b] > c->far_h[b].kcap) fail(EWBEM_EINVAL, "internal: rank outside capacity");
      c->kcap_prev[b] = c->far_h[b].kcap;
    }
    if (streamed) {
      // this batch into the complex64 store, before its work area is reused
      std::vector<cf*> up(ids.size()), vp(ids.size());
      for (size_t i = 0; i < ids.size(); ++i) {
        const FarBlk& f = c->far_h[ids[i]];
        const int k = c->rank_h[ids[i]];
        up[i] = c->u32_h[ids[i]] = store_alloc(std::max<size_t>(1, 3 * (size_t)f.m * k));
        vp[i] = c->v32_h[ids[i]] = store_alloc(std::max<size_t>(1, 3 * (size_t)f.n * k));
      }
      c->d_batch_ids.upload(ids, st);
      c->d_u32p.upload(up, st);
      c->d_v32p.upload(vp, st);
      launch_to_c64_ptr(c->d_far.p, c->d_batch_ids.p, (int)ids.size(), c->d_rank.p, c->d_u32p.p, c->d_v32p.p, st);
      EWBEM_HIP_CHECK(hipGetLastError());
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));  // up, vp and the work area
    }
  }
  EWBEM_HIP_CHECK(hipMemcpyAsync(c->nlist_h.data(), c->d_nlist.p, 2 * (size_t)nf * sizeof(int),
                                 hipMemcpyDeviceToHost, st));
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
}

// Host-side check that a device range [p, p + n) lies inside one of the
// live factor allocations; a failure is a library bug, reported as an error
// instead of being launched.
bool in_alloc(const void* p, long long n_bytes, const void* base, size_t base_bytes) {
  const char* a = (const char*)p;
  const char* b = (const char*)base;
  return base && a >= b && n_bytes >= 0 && a + n_bytes <= b + base_bytes;
}

// The streamed store's chunk holding [p, p + n).
bool in_f32_chunks(const ewbem_ctx* c, const void* p, long long n_bytes) {
  for (const auto& ch : c->d_f32s)
    if (in_alloc(p, n_bytes, ch->p, ch->n * sizeof(cf))) return true;
  return false;
}

void check_far_ranges(ewbem_ctx* c) {
  if (c->streamed) {  // the complex128 pointers are stale: check the complex64 store
    for (size_t b = 0; b < c->far_h.size(); ++b) {
      const FarBlk& f = c->far_h[b];
      const long long k = c->rank_h[b];
      if (k < 0 || k > f.kcap) fail(EWBEM_EINVAL, "internal: rank outside capacity");
      if (!in_f32_chunks(c, c->u32_h[b], 3LL * f.m * std::max(1LL, k) * (long long)sizeof(cf)) ||
          !in_f32_chunks(c, c->v32_h[b], 3LL * f.n * std::max(1LL, k) * (long long)sizeof(cf)))
        fail(EWBEM_EINVAL, "internal: streamed factor range outside its chunk");
    }
    return;
  }
  for (size_t b = 0; b < c->far_h.size(); ++b) {
    const FarBlk& f = c->far_h[b];
    const long long nu = 3LL * f.m * f.kcap * (long long)sizeof(cd), nv = 3LL * f.n * f.kcap * (long long)sizeof(cd);
    const DevBuf<cd>& ws = c->d_wsf[c->fslot];
    bool ok = in_alloc(f.U, nu, ws.p, ws.n * sizeof(cd)) && in_alloc(f.V, nv, ws.p, ws.n * sizeof(cd));
    for (const auto& r : c->d_retry[c->fslot])
      ok = ok || (in_alloc(f.U, nu, r->p, r->n * sizeof(cd)) && in_alloc(f.V, nv, r->p, r->n * sizeof(cd)));
    if (!ok) fail(EWBEM_EINVAL, "internal: far-block factor range outside its allocation");
    if (c->rank_h[b] < 0 || c->rank_h[b] > f.kcap) fail(EWBEM_EINVAL, "internal: rank outside capacity");
  }
}

void build_matvec(ewbem_ctx* c) {
  check_far_ranges(c);
  hipStream_t st = c->stream;
  const int nf = (int)c->far_h.size();
  const bool c64 = c->op.far_store == EWBEM_STORE_C64 && nf > 0;
  c->store_c64_active = c64;
  // z offsets and (for complex64) the compact factor store
  std::vector<long long> zoff(nf + 1, 0), uo(nf), vo(nf);
  long long f32tot = 0;
  c->rank_sum = 0;
  c->rank_max = 0;
  for (int b = 0; b < nf; ++b) {
    const int k = c->rank_h[b];
    zoff[b + 1] = zoff[b] + k;
    uo[b] = f32tot;
    f32tot += 3LL * c->far_h[b].m * k;
    vo[b] = f32tot;
    f32tot += 3LL * c->far_h[b].n * k;
    c->rank_sum += k;
    c->rank_max = std::max<int64_t>(c->rank_max, k);
  }
  c->z_len = std::max<long long>(1, zoff[nf]);
  c->d_z.reserve_grow((size_t)HMV_MAXRHS * c->z_len);
  const bool streamed = c64 && c->streamed;  // factors already in the streamed store
  auto u32 = [&](int b) -> const cf* { return streamed ? c->u32_h[b] : c->d_f32.p + uo[b]; };
  auto v32 = [&](int b) -> const cf* { return streamed ? c->v32_h[b] : c->d_f32.p + vo[b]; };
  if (c64 && !streamed) {
    c->d_f32.reserve_grow(std::max<long long>(1, f32tot));
    c->d_uo.upload(uo, st);
    c->d_vo.upload(vo, st);
    launch_to_c64(c->d_far.p, nf, c->d_rank.p, c->d_uo.p, c->d_vo.p, c->d_f32.p, st);
  }
  // phase 1 tasks
  const int vc = c->mv_cols;
  // phase-1 tasks of vc factor columns, and of 16 for the eight-vector
  // product on the matrix cores
  std::vector<VtTask> vt, vt16;
  const bool want16 = c->op.mv_mfma != 0;
  for (int b = 0; b < nf; ++b) {
    const FarBlk& f = c->far_h[b];
    const int k = c->rank_h[b], C = 3 * f.n;
    for (int w = 0; w < (want16 ? 2 : 1); ++w) {
      const int cols = w == 0 ? vc : HMV_MFMA_COLS;
      for (int l0 = 0; l0 < k; l0 += cols) {
        VtTask t{};
        t.V = c64 ? (const void*)(v32(b) + (size_t)l0 * C) : (const void*)(f.V + (size_t)l0 * C);
        t.zidx = zoff[b] + l0;
        t.C = C;
        t.x0 = 3 * f.c0;
        t.ncol = std::min(cols, k - l0);
        (w == 0 ? vt : vt16).push_back(t);
      }
    }
  }
  // phase 2 segments per leaf
  const std::vector<int>& leaves = c->part.leaves;
  const int nl = (int)leaves.size();
  std::vector<int> leaf_begin(nl);
  for (int i = 0; i < nl; ++i) leaf_begin[i] = c->part.clusters[leaves[i]].begin;
  auto leaf_of = [&](int begin) {
    return (int)(std::lower_bound(leaf_begin.begin(), leaf_begin.end(), begin) - leaf_begin.begin());
  };
  std::vector<std::vector<Seg>> segs(nl);
  double bytes = 0, rhs_bytes = 0;
  const double be_far = c64 ? 8.0 : 16.0;
  for (const NearBlk& nb : c->near_h) {
    const int li = leaf_of(nb.r0);
    Seg s{};
    s.A = c->d_D.p + nb.off;
    s.src = 3LL * nb.c0;
    s.ld = 3 * nb.m;
    s.ncols = 3 * nb.n;
    s.flags = 0;
    segs[li].push_back(s);
    bytes += 9.0 * nb.m * nb.n * 16.0;
  }
  for (int b = 0; b < nf; ++b) {
    const FarBlk& f = c->far_h[b];
    const int k = c->rank_h[b];
    if (k == 0) continue;
    bytes += 3.0 * k * (f.m + f.n) * be_far + 2.0 * k * 16.0;
    rhs_bytes += 2.0 * k * 16.0;
    for (int li = leaf_of(f.r0); li < nl && leaf_begin[li] < f.r0 + f.m; ++li) {
      const Cluster& L = c->part.clusters[leaves[li]];
      Seg s{};
      const size_t roff = 3 * (size_t)(L.begin - f.r0);
      s.A = c64 ? (const void*)(u32(b) + roff) : (const void*)(f.U + roff);
      s.src = zoff[b];
      s.ld = 3 * f.m;
      s.ncols = k;
      s.flags = SEG_FROM_Z | (c64 ? SEG_C64 : 0);
      segs[li].push_back(s);
    }
  }
  const long long N = 3LL * c->nt;
  bytes += 2.0 * N * 16.0;  // read x, write y
  rhs_bytes += 2.0 * N * 16.0;
  c->matvec_bytes = bytes;
  c->matvec_rhs_bytes = rhs_bytes;
  c->stored_bytes = 0;
  for (const NearBlk& nb : c->near_h) c->stored_bytes += 9.0 * nb.m * nb.n * 16.0;
  for (int b = 0; b < nf; ++b)
    c->stored_bytes += 3.0 * c->rank_h[b] * (c->far_h[b].m + c->far_h[b].n) * be_far;
  long long total_cols = 0;
  for (auto& v : segs)
    for (auto& s : v) total_cols += s.ncols;
  const long long target = std::max<long long>(96, total_cols / c->mv_div);
  std::vector<Seg> flat;
  std::vector<RowTask> rt;
  std::vector<LeafRange> lr;
  for (int li = 0; li < nl; ++li) {
    const Cluster& L = c->part.clusters[leaves[li]];
    LeafRange range{3 * L.begin, 3 * L.size(), (int)rt.size(), 0};
    long long acc = 0;
    int s0 = (int)flat.size();
    for (const Seg& s : segs[li]) {
      flat.push_back(s);
      acc += s.ncols;
      if (acc >= target) {
        rt.push_back(RowTask{3 * L.begin, 3 * L.size(), s0, (int)flat.size()});
        s0 = (int)flat.size();
        acc = 0;
      }
    }
    if ((int)flat.size() > s0 || range.t0 == (int)rt.size())
      rt.push_back(RowTask{3 * L.begin, 3 * L.size(), s0, (int)flat.size()});
    range.t1 = (int)rt.size();
    lr.push_back(range);
  }
  // every range a kernel will touch must lie inside its allocation
  {
    const long long ztot = zoff[nf];
    auto store_ok = [&](const void* p, long long bytes) {
      if (streamed) return in_f32_chunks(c, p, bytes);
      if (c64) return in_alloc(p, bytes, c->d_f32.p, c->d_f32.n * sizeof(cf));
      bool ok = in_alloc(p, bytes, c->d_wsf[c->fslot].p, c->d_wsf[c->fslot].n * sizeof(cd));
      for (const auto& r : c->d_retry[c->fslot]) ok = ok || in_alloc(p, bytes, r->p, r->n * sizeof(cd));
      return ok;
    };
    const long long es = c64 ? (long long)sizeof(cf) : (long long)sizeof(cd);
    for (int w = 0; w < 2; ++w)
      for (const VtTask& t : w == 0 ? vt : vt16) {
        if (t.ncol < 1 || t.ncol > (w == 0 ? vc : HMV_MFMA_COLS) || t.C < 1 || t.x0 < 0 ||
            t.x0 + (long long)t.C > N || t.zidx < 0 || t.zidx + t.ncol > ztot ||
            !store_ok(t.V, (long long)t.ncol * t.C * es))
          fail(EWBEM_EINVAL, "internal: phase-1 task out of range");
      }
    for (size_t i = 0; i < rt.size(); ++i) {
      const RowTask& T = rt[i];
      if (T.rows < 1 || T.rows > HMV_MAXROWS || T.row0 < 0 || T.row0 + T.rows > N || T.s0 < 0 ||
          T.s1 > (int)flat.size() || T.s0 > T.s1)
        fail(EWBEM_EINVAL, "internal: row task out of range");
      for (int q = T.s0; q < T.s1; ++q) {
        const Seg& S = flat[q];
        const long long span = ((long long)(S.ncols - 1) * S.ld + T.rows);
        if (S.ncols < 1 || S.ld < T.rows) fail(EWBEM_EINVAL, "internal: segment shape");
        // the matvec addresses a panel with 32-bit byte offsets
        if ((long long)S.ncols * S.ld * ((S.flags & SEG_C64) ? 8 : 16) >= (1LL << 32))
          fail(EWBEM_EINVAL, "internal: panel of 4 GiB or more");
        if (S.flags & SEG_FROM_Z) {
          if (S.src < 0 || S.src + S.ncols > ztot || !store_ok(S.A, span * es))
            fail(EWBEM_EINVAL, "internal: far segment out of range");
        } else {
          if (S.src < 0 || S.src + S.ncols > N ||
              !in_alloc(S.A, span * (long long)sizeof(cd), c->d_D.p, c->d_D.n * sizeof(cd)))
            fail(EWBEM_EINVAL, "internal: near segment out of range");
        }
      }
    }
    for (const LeafRange& L : lr)
      if (L.t0 < 0 || L.t1 > (int)rt.size() || L.t0 >= L.t1 || L.rows > HMV_MAXROWS || L.row0 + L.rows > N)
        fail(EWBEM_EINVAL, "internal: leaf range out of range");
  }
  c->d_vt.upload(vt, st);
  c->vt_cols = vc;
  if (want16) c->d_vt16.upload(vt16, st);
  c->n_vt16 = (int)vt16.size();
  c->d_seg.upload(flat, st);
  c->d_rt.upload(rt, st);
  c->d_lr.upload(lr, st);
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));  // the uploads read the host tables kept below
  c->vt_h = std::move(vt);
  c->seg_h = std::move(flat);
  c->rt_h = std::move(rt);
  c->lr_h = std::move(lr);
  c->n_vt = (int)c->vt_h.size();
  c->n_rt = (int)c->rt_h.size();
  c->n_lr = (int)c->lr_h.size();
  c->mvpart_len = (long long)std::max(1, c->n_rt) * HMV_MAXROWS;
  c->d_mvpart.reserve_grow((size_t)HMV_MAXRHS * c->mvpart_len);
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
}

// y = A x in tree order (both device, length N); times the kernels with
// events when ``ev`` is given.
void apply_tree(ewbem_ctx* c, const cd* x, cd* y, EventPair* ev) {
  hipStream_t st = c->stream;
  if (ev) EWBEM_HIP_CHECK(hipEventRecord(ev->a, st));
  launch_far_vt(c->d_vt.p, c->n_vt, c->vt_cols, c->store_c64_active, x, 0, 1, c->d_z.p, 0, st);
  launch_hmv(c->d_rt.p, c->n_rt, c->d_seg.p, x, 0, 1, c->d_z.p, 0, c->d_mvpart.p, 0, st);
  launch_hmv_reduce(c->d_lr.p, c->n_lr, c->d_mvpart.p, 0, 1, y, 0, st);
  if (ev) EWBEM_HIP_CHECK(hipEventRecord(ev->b, st));
  c->acc.matvecs += 1;
}

// Y(:, j) = A X(:, j) for j < nrhs <= HMV_MAXRHS (8), columns N apart (tree order): the
// operator is read once for all of them.
void apply_tree_multi(ewbem_ctx* c, const cd* X, cd* Y, int nrhs) {
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  if (nrhs < 1 || nrhs > HMV_MAXRHS) fail(EWBEM_EINVAL, "internal: matvec right-hand sides out of range");
  if (c->op.mv_mfma && nrhs == HMV_MAXRHS)
    launch_far_vt(c->d_vt16.p, c->n_vt16, HMV_MFMA_COLS, c->store_c64_active, X, N, nrhs, c->d_z.p, c->z_len, st, 1);
  else
    launch_far_vt(c->d_vt.p, c->n_vt, c->vt_cols, c->store_c64_active, X, N, nrhs, c->d_z.p, c->z_len, st, 0);
  launch_hmv(c->d_rt.p, c->n_rt, c->d_seg.p, X, N, nrhs, c->d_z.p, c->z_len, c->d_mvpart.p, c->mvpart_len, st,
             c->op.mv_mfma);
  launch_hmv_reduce(c->d_lr.p, c->n_lr, c->d_mvpart.p, c->mvpart_len, nrhs, Y, N, st);
  c->acc.matvecs += nrhs;
}

// add one event-timed matvec (its kernels' time and algorithmic bytes)
void account_matvec(ewbem_ctx* c, EventPair& ev) {
  c->acc.t_matvec_ms += ev.elapsed();
  c->acc.matvec_bytes_total += c->matvec_bytes;
  c->acc.matvecs_timed += 1;
}

void precond_setup(ewbem_ctx* c) {
  hipStream_t st = c->stream;
  if (c->so.precond == EWBEM_PREC_ELEMENT) {
    launch_inv3(c->d_selfA.p, c->nt, c->d_M3.p, st);
  } else if (c->so.precond == EWBEM_PREC_LEAF) {
    // copy each leaf's diagonal near block into a compact work array, invert
    std::vector<long long> src, dst;
    std::vector<int> dims, row0, ld;
    long long off = 0;
    for (const NearBlk& nb : c->near_h) {
      if (nb.r0 != nb.c0) continue;
      src.push_back(nb.off);
      dst.push_back(off);
      dims.push_back(3 * nb.m);
      row0.push_back(3 * nb.r0);
      ld.push_back(3 * nb.m);
      off += 9LL * nb.m * nb.m;
    }
    c->d_Minv.reserve(off);
    c->d_minv_src.upload(src, st);
    c->d_minv_off.upload(dst, st);
    c->d_minv_dim.upload(dims, st);
    c->d_minv_row0.upload(row0, st);
    c->d_minv_ld.upload(ld, st);
    c->d_pivfail.reserve(dims.size());
    c->n_minv = (int)dims.size();
    EWBEM_HIP_CHECK(hipMemsetAsync(c->d_pivfail.p, 0, dims.size() * sizeof(int), st));
    launch_copy_blocks(c->d_minv_src.p, c->d_minv_ld.p, c->d_minv_off.p, c->d_minv_dim.p, (int)dims.size(),
                       c->d_D.p, c->d_Minv.p, st);
    launch_block_inv(c->d_minv_off.p, c->d_minv_dim.p, (int)dims.size(), c->d_Minv.p, c->d_pivfail.p, st);
    std::vector<int> pf(dims.size());
    EWBEM_HIP_CHECK(hipMemcpyAsync(pf.data(), c->d_pivfail.p, pf.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    for (int v : pf)
      if (v) fail(EWBEM_EINVAL, "singular diagonal block in the preconditioner");
  }
}

void precond_apply(ewbem_ctx* c, const cd* v, cd* z) {
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  if (c->so.precond == EWBEM_PREC_ELEMENT) {
    launch_apply3(c->d_M3.p, c->nt, v, z, st);
  } else if (c->so.precond == EWBEM_PREC_LEAF) {
    launch_block_apply(c->d_minv_off.p, c->d_minv_dim.p, c->d_minv_row0.p, c->n_minv,
                       c->d_Minv.p, v, z, st);
  } else {
    EWBEM_HIP_CHECK(hipMemcpyAsync(z, v, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
  }
}

// Off-diagonal U(s_k) t0 for frequencies k0 .. k0+nk-1 in one batched pass.
void rhs_precompute(ewbem_ctx* c, const DevGeom& g, int k0, int nk) {
  if (c->inc_total) {  // b is the incident displacement itself: no sums
    c->boff_k0 = k0;
    c->boff_nk = nk;
    return;
  }
  const size_t need = (size_t)rhs_split(c->nt) * nk * 3 * (size_t)c->nt;
  c->d_rhs_part.reserve(need);
  launch_rhs_multi(g, c->P, c->sigma, 2.0 * M_PI / c->period, k0, nk, c->d_t0.p,
                   c->load_incident ? c->d_tau.p : nullptr, c->d_rhs_part.p, c->stream);
  c->boff_k0 = k0;
  c->boff_nk = nk;
}

double dev_norm(ewbem_ctx* c, const cd* v);

// b_k of the current load from its off-diagonal sums (d_rhs_part) and the
// self elements' U of the assembled frequency.
void rhs_finish_k(ewbem_ctx* c, int k) {
  if (c->inc_total) {
    launch_rhs_total(c->d_tau.p, c->inc_pol, s_of_k(c, k), c->d_phat.p + k, c->nt, c->d_b.p, c->stream);
    return;
  }
  launch_rhs_finish(c->d_rhs_part.p, c->boff_nk, k - c->boff_k0, c->nt, c->d_selfU.p, c->d_t0.p,
                    c->load_incident ? c->d_tau.p : nullptr, s_of_k(c, k), c->d_phat.p + k, c->d_b.p, c->stream);
}

// Matvec task shapes by measurement: every pair of candidate phase-1 column
// counts and phase-2 task sizes is built and timed (one warm apply, then
// three timed) on the operator just assembled; the fastest is kept for the
// rest of the context's life (until the partition changes).
// Shapes tuned in this process, by device and partition: the candidates cut
// the same bytes in different ways, so contexts of one problem (a batch, the
// loads of a training set, a repeated bench) share the first one's timing.
struct TunedShapes {
  int cols, div;
  double best_ms, default_ms;
};
using TuneKey = std::tuple<int, long long, long long, long long, long long, long long, int>;
std::mutex g_tune_mu;
std::map<TuneKey, TunedShapes> g_tuned;

TuneKey tune_key(const ewbem_ctx* c) {
  long long far_rows = 0;
  for (const FarBlk& f : c->far_h) far_rows += (long long)f.m + f.n;
  return TuneKey{c->device, (long long)c->nt, (long long)c->near_h.size(), (long long)c->far_h.size(),
                 c->near_entries, far_rows, c->op.far_store};
}

void tune_matvec(ewbem_ctx* c) {
  static const int kCols[] = {2, 4, 8};
  static const int kDivs[] = {2048, 4096, 8192};
  const TuneKey key = tune_key(c);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      c->mv_cols = it->second.cols;
      c->mv_div = it->second.div;
      c->mv_best_ms = it->second.best_ms;
      c->mv_default_ms = it->second.default_ms;
      c->mv_tuned = true;
      c->mv_tune_cached = true;
      build_matvec(c);
      return;
    }
  }
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  {
    std::vector<cd> xh(N);
    for (long long i = 0; i < N; ++i) xh[i] = cd{std::cos(0.37 * i), std::sin(0.11 * i)};
    EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_tmp_in.p, xh.data(), N * sizeof(cd), hipMemcpyHostToDevice, st));
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  }
  EventPair ev;
  double best = 1e300, yref = 0.0;
  int bc = c->mv_cols, bd = c->mv_div;
  bool first = true;
  for (int nc : kCols)
    for (int dv : kDivs) {
      c->mv_cols = nc;
      c->mv_div = dv;
      build_matvec(c);
      apply_tree(c, c->d_tmp_in.p, c->d_tmp_out.p, nullptr);
      EWBEM_HIP_CHECK(hipEventRecord(ev.a, st));
      for (int i = 0; i < 3; ++i) apply_tree(c, c->d_tmp_in.p, c->d_tmp_out.p, nullptr);
      EWBEM_HIP_CHECK(hipEventRecord(ev.b, st));
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      const double ms = ev.elapsed() / 3.0;
      // every shape computes the same product up to summation order
      if (first) {
        EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_w.p, c->d_tmp_out.p, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
        yref = dev_norm(c, c->d_w.p);
        first = false;
      } else {
        EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_zt.p, c->d_tmp_out.p, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
        launch_axpby(cd{-1.0, 0.0}, c->d_w.p, cd{1.0, 0.0}, c->d_zt.p, N, st);
        if (dev_norm(c, c->d_zt.p) > 1e-12 * yref) fail(EWBEM_EINVAL, "internal: matvec task shapes disagree");
      }
      if (nc == 4 && dv == 4096) c->mv_default_ms = ms;
      if (ms < best) {
        best = ms;
        bc = nc;
        bd = dv;
      }
    }
  c->mv_cols = bc;
  c->mv_div = bd;
  c->mv_tuned = true;
  c->mv_tune_cached = false;
  c->mv_best_ms = best;
  build_matvec(c);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = TunedShapes{bc, bd, best, c->mv_default_ms};
}

// Operator, right-hand side and preconditioner of frequency k.  aca_done:
// the far factors of k are already in slot fslot (the overlapped ACA).
void assemble_k(ewbem_ctx* c, int k, bool aca_done = false) {
  ensure_device(c);
  if (k < 0 || k > c->n_f / 2) fail(EWBEM_EINVAL, "frequency index out of range 0..N_f/2");
  hipStream_t st = c->stream;
  const auto t0 = Clock::now();
  c->P = make_params(c, s_of_k(c, k));
  const DevGeom g = dev_geom(c);
  EventPair ev;
  EWBEM_HIP_CHECK(hipEventRecord(ev.a, st));
  launch_self(g, c->P, c->S, c->d_selfT.p, c->d_selfU.p, c->d_selfA.p, st);
  launch_near(c->d_near.p, (int)c->near_h.size(), g, c->P, c->d_D.p, st);
  launch_scatter_self(c->d_selfA.p, c->d_self_off.p, c->nt, c->d_D.p, c->d_self_ld.p, st);
  EWBEM_HIP_CHECK(hipEventRecord(ev.b, st));
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  c->acc.t_near_ms += ev.elapsed();
  if (!aca_done) {
    double aca_ms = 0;
    // with the pipeline the slot the matvec reads is left alone
    const int slot = c->so.pipeline ? 1 - c->fslot : c->fslot;
    run_aca(c, g, ev, aca_ms, st, slot);
    c->fslot = slot;
    c->acc.t_aca_ms += aca_ms;
  }
  build_matvec(c);
  if (c->op.autotune && !c->mv_tuned && !c->far_h.empty()) tune_matvec(c);
  EWBEM_HIP_CHECK(hipEventRecord(ev.a, st));
  if (k < c->boff_k0 || k >= c->boff_k0 + c->boff_nk) rhs_precompute(c, g, k, 1);
  rhs_finish_k(c, k);
  EWBEM_HIP_CHECK(hipEventRecord(ev.b, st));
  precond_setup(c);
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  c->acc.t_rhs_ms += ev.elapsed();
  c->assembled_k = k;
  c->acc.t_assemble_ms += ms_since(t0);
  c->acc.n_near = (int64_t)c->near_h.size();
  c->acc.n_far = (int64_t)c->far_h.size();
  c->acc.rank_sum = c->rank_sum;
  c->acc.rank_max = c->rank_max;
  c->acc.matvec_bytes = c->matvec_bytes;
  c->acc.stored_bytes = c->stored_bytes;
}

// |v|^2 etc.: host copies of small device results
double dev_norm(ewbem_ctx* c, const cd* v) {
  const long long N = 3LL * c->nt;
  cd h;
  launch_dots(v, N, 1, v, N, c->d_hpart.p, c->d_small.p, c->stream);
  EWBEM_HIP_CHECK(hipMemcpyAsync(&h, c->d_small.p, sizeof(cd), hipMemcpyDeviceToHost, c->stream));
  EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
  return std::sqrt(std::max(0.0, h.x));
}

// Right-preconditioned restarted GMRES with classical Gram-Schmidt applied
// twice; the least-squares problem is updated by Givens rotations on the
// host.  x holds x0 on entry, r = b - A x0.  Returns the final true
// relative residual; iterations are added to the stats.
double gmres(ewbem_ctx* c, cd* x, cd* r, int& iters_out, bool& converged) {
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  const int m = c->so.restart;
  const double tol = c->so.tol;
  const double bnorm = dev_norm(c, c->d_b.p);
  iters_out = 0;
  converged = true;
  if (bnorm == 0.0) {
    EWBEM_HIP_CHECK(hipMemsetAsync(x, 0, N * sizeof(cd), st));
    return 0.0;
  }
  double rnorm = dev_norm(c, r);
  double relres = rnorm / bnorm;
  EventPair ev;
  std::vector<std::complex<double>> H((size_t)(m + 1) * m), cs(m), sn(m), gvec(m + 1);
  std::vector<cd> hbuf(2 * (m + 2) + 2);
  cd* V = c->d_V.p;
  cd* hd = c->d_small.p;            // h (m+1)
  cd* hd2 = c->d_small.p + (m + 2); // second pass
  cd* nd = c->d_small.p + 2 * (m + 2);
  while (relres > tol && iters_out < c->so.maxit) {
    const double beta = rnorm;
    launch_axpby(cd{1.0 / beta, 0.0}, r, cd{0.0, 0.0}, V, N, st);
    std::fill(gvec.begin(), gvec.end(), 0.0);
    gvec[0] = beta;
    int j = 0;
    double est = relres;
    for (; j < m && iters_out < c->so.maxit; ++j) {
      cd* vj = V + (size_t)j * N;
      cd* w = V + (size_t)(j + 1) * N;
      precond_apply(c, vj, c->d_zt.p);
      apply_tree(c, c->d_zt.p, w, &ev);
      launch_dots(V, N, j + 1, w, N, c->d_hpart.p, hd, st);
      launch_gemv_sub(V, N, j + 1, hd, w, N, st);
      launch_dots(V, N, j + 1, w, N, c->d_hpart.p, hd2, st);
      launch_gemv_sub(V, N, j + 1, hd2, w, N, st);
      launch_dots(w, N, 1, w, N, c->d_hpart.p, nd, st);
      EWBEM_HIP_CHECK(hipMemcpyAsync(hbuf.data(), c->d_small.p, (2 * (m + 2) + 1) * sizeof(cd),
                                     hipMemcpyDeviceToHost, st));
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      account_matvec(c, ev);
      ++iters_out;
      const double hn = std::sqrt(std::max(0.0, hbuf[2 * (m + 2)].x));
      for (int i = 0; i <= j; ++i)
        H[(size_t)j * (m + 1) + i] = std::complex<double>(hbuf[i].x + hbuf[m + 2 + i].x,
                                                          hbuf[i].y + hbuf[m + 2 + i].y);
      H[(size_t)j * (m + 1) + j + 1] = hn;
      // apply previous rotations to column j
      for (int i = 0; i < j; ++i) {
        std::complex<double>& a = H[(size_t)j * (m + 1) + i];
        std::complex<double>& b = H[(size_t)j * (m + 1) + i + 1];
        const std::complex<double> t = std::conj(cs[i]) * a + std::conj(sn[i]) * b;
        b = -sn[i] * a + cs[i] * b;
        a = t;
      }
      // new rotation annihilating H[j+1, j]
      const std::complex<double> a = H[(size_t)j * (m + 1) + j];
      const double bb = hn;
      const double den = std::sqrt(std::norm(a) + bb * bb);
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / den;
        sn[j] = bb / den;
      }
      H[(size_t)j * (m + 1) + j] = den;
      H[(size_t)j * (m + 1) + j + 1] = 0.0;
      gvec[j + 1] = -sn[j] * gvec[j];
      gvec[j] = std::conj(cs[j]) * gvec[j];
      est = std::abs(gvec[j + 1]) / bnorm;
      if (hn > 0.0) launch_axpby(cd{1.0 / hn, 0.0}, w, cd{0.0, 0.0}, w, N, st);
      if (est <= tol || hn == 0.0) {
        ++j;
        break;
      }
    }
    // y = H^{-1} g (upper triangular j x j)
    std::vector<std::complex<double>> y(j);
    for (int i = j - 1; i >= 0; --i) {
      std::complex<double> sacc = gvec[i];
      for (int l = i + 1; l < j; ++l) sacc -= H[(size_t)l * (m + 1) + i] * y[l];
      y[i] = sacc / H[(size_t)i * (m + 1) + i];
    }
    std::vector<cd> yd(j);
    for (int i = 0; i < j; ++i) yd[i] = cd{y[i].real(), y[i].imag()};
    EWBEM_HIP_CHECK(hipMemcpyAsync(hd, yd.data(), j * sizeof(cd), hipMemcpyHostToDevice, st));
    launch_gemv_acc(V, N, j, hd, cd{0.0, 0.0}, c->d_u.p, N, st);
    precond_apply(c, c->d_u.p, c->d_zt.p);
    launch_axpby(cd{1.0, 0.0}, c->d_zt.p, cd{1.0, 0.0}, x, N, st);
    // true residual
    apply_tree(c, x, r, &ev);
    launch_axpby(cd{1.0, 0.0}, c->d_b.p, cd{-1.0, 0.0}, r, N, st);
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    account_matvec(c, ev);
    rnorm = dev_norm(c, r);
    relres = rnorm / bnorm;
    if (j == 0) break;
  }
  converged = relres <= tol;
  return relres;
}

// The same GMRES for up to eight systems A x_l = b_l on one operator, in
// lock-step: each step's preconditioned vectors of the systems still
// iterating go through one multi-right-hand-side matvec (the operator read
// once for all), and one host synchronisation serves all their Arnoldi
// coefficients.  Per system the arithmetic is that of gmres() in the same
// order, so each result equals a lone solve's.  Vm: nb x (m+1) x N Krylov
// bases; Z, W: nb x N staging; small: nb x (2 (m+2) + 2) coefficients.
struct GmresLane {
  cd* b = nullptr;
  cd* x = nullptr;
  cd* r = nullptr;
  cd* V = nullptr;
  cd* hd = nullptr;  // h (m+2), second pass (m+2), |w|^2
  double bnorm = 0, rnorm = 0, relres = 0;
  int j = 0, its = 0;
  bool done = false, arnoldi = false;
  std::vector<std::complex<double>> H, cs, sn, g;
};

void gmres_multi(ewbem_ctx* c, std::vector<GmresLane>& L, cd* Z, cd* W) {
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  const int m = c->so.restart;
  const double tol = c->so.tol;
  const int nb = (int)L.size();
  if (nb < 1 || nb > HMV_MAXRHS) fail(EWBEM_EINVAL, "internal: 1 to 8 systems per lock-step GMRES");
  const int hs = 2 * (m + 2) + 2;
  std::vector<cd> hb((size_t)nb * hs);
  EventPair ev;
  // |b|, |r0| of every system, one synchronisation
  auto norms = [&](bool of_b, const std::vector<int>& who) {
    for (int l : who) launch_dots(of_b ? L[l].b : L[l].r, N, 1, of_b ? L[l].b : L[l].r, N, c->d_hpart.p, L[l].hd, st);
    for (int l : who)
      EWBEM_HIP_CHECK(hipMemcpyAsync(&hb[(size_t)l * hs], L[l].hd, sizeof(cd), hipMemcpyDeviceToHost, st));
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    for (int l : who) (of_b ? L[l].bnorm : L[l].rnorm) = std::sqrt(std::max(0.0, hb[(size_t)l * hs].x));
  };
  std::vector<int> all(nb);
  for (int l = 0; l < nb; ++l) {
    all[l] = l;
    L[l].H.assign((size_t)(m + 1) * m, 0.0);
    L[l].cs.assign(m, 0.0);
    L[l].sn.assign(m, 0.0);
    L[l].g.assign(m + 1, 0.0);
    L[l].its = 0;
    L[l].done = L[l].arnoldi = false;
  }
  norms(true, all);
  norms(false, all);
  for (GmresLane& G : L) {
    if (G.bnorm == 0.0) {
      EWBEM_HIP_CHECK(hipMemsetAsync(G.x, 0, N * sizeof(cd), st));
      G.relres = 0.0;
      G.done = true;
      continue;
    }
    G.relres = G.rnorm / G.bnorm;
    if (!(G.relres > tol)) G.done = true;
  }
  std::vector<int> act, ends;
  for (;;) {
    // systems starting a cycle
    for (GmresLane& G : L) {
      if (G.done || G.arnoldi) continue;
      if (G.its >= c->so.maxit) {
        G.done = true;
        continue;
      }
      launch_axpby(cd{1.0 / G.rnorm, 0.0}, G.r, cd{0.0, 0.0}, G.V, N, st);
      std::fill(G.g.begin(), G.g.end(), 0.0);
      G.g[0] = G.rnorm;
      G.j = 0;
      G.arnoldi = true;
    }
    act.clear();
    for (int l = 0; l < nb; ++l)
      if (L[l].arnoldi) act.push_back(l);
    if (act.empty()) break;
    // one Arnoldi step of each: w = A M^{-1} v_j, Gram-Schmidt twice, |w|
    const int na = (int)act.size();
    for (int i = 0; i < na; ++i) precond_apply(c, L[act[i]].V + (size_t)L[act[i]].j * N, Z + (size_t)i * N);
    EWBEM_HIP_CHECK(hipEventRecord(ev.a, st));
    apply_tree_multi(c, Z, W, na);
    EWBEM_HIP_CHECK(hipEventRecord(ev.b, st));
    for (int i = 0; i < na; ++i) {
      GmresLane& G = L[act[i]];
      cd* w = W + (size_t)i * N;
      cd* hd2 = G.hd + (m + 2);
      cd* nd = G.hd + 2 * (m + 2);
      launch_dots(G.V, N, G.j + 1, w, N, c->d_hpart.p, G.hd, st);
      launch_gemv_sub(G.V, N, G.j + 1, G.hd, w, N, st);
      launch_dots(G.V, N, G.j + 1, w, N, c->d_hpart.p, hd2, st);
      launch_gemv_sub(G.V, N, G.j + 1, hd2, w, N, st);
      launch_dots(w, N, 1, w, N, c->d_hpart.p, nd, st);
      EWBEM_HIP_CHECK(hipMemcpyAsync(&hb[(size_t)act[i] * hs], G.hd, (2 * (m + 2) + 1) * sizeof(cd),
                                     hipMemcpyDeviceToHost, st));
    }
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    c->acc.t_matvec_ms += ev.elapsed();
    c->acc.matvec_bytes_total += c->matvec_bytes + (na - 1) * c->matvec_rhs_bytes;
    c->acc.matvecs_timed += 1;
    ends.clear();
    for (int i = 0; i < na; ++i) {
      GmresLane& G = L[act[i]];
      const cd* h = &hb[(size_t)act[i] * hs];
      const int j = G.j;
      auto Hc = [&](int row) -> std::complex<double>& { return G.H[(size_t)j * (m + 1) + row]; };
      ++G.its;
      const double hn = std::sqrt(std::max(0.0, h[2 * (m + 2)].x));
      for (int q = 0; q <= j; ++q) Hc(q) = std::complex<double>(h[q].x + h[m + 2 + q].x, h[q].y + h[m + 2 + q].y);
      Hc(j + 1) = hn;
      for (int q = 0; q < j; ++q) {
        std::complex<double>& a = Hc(q);
        std::complex<double>& b = Hc(q + 1);
        const std::complex<double> t = std::conj(G.cs[q]) * a + std::conj(G.sn[q]) * b;
        b = -G.sn[q] * a + G.cs[q] * b;
        a = t;
      }
      const std::complex<double> a = Hc(j);
      const double den = std::sqrt(std::norm(a) + hn * hn);
      if (den == 0.0) {
        G.cs[j] = 1.0;
        G.sn[j] = 0.0;
      } else {
        G.cs[j] = a / den;
        G.sn[j] = hn / den;
      }
      Hc(j) = den;
      Hc(j + 1) = 0.0;
      G.g[j + 1] = -G.sn[j] * G.g[j];
      G.g[j] = std::conj(G.cs[j]) * G.g[j];
      const double est = std::abs(G.g[j + 1]) / G.bnorm;
      // the normalised vector goes into the basis (w itself when hn = 0)
      if (hn > 0.0 && j + 1 <= m)
        launch_axpby(cd{1.0 / hn, 0.0}, W + (size_t)i * N, cd{0.0, 0.0}, G.V + (size_t)(j + 1) * N, N, st);
      G.j = j + 1;
      if (est <= tol || hn == 0.0 || G.j >= m || G.its >= c->so.maxit) ends.push_back(act[i]);
    }
    if (ends.empty()) continue;
    // cycle ends: x += M^{-1} V y, then the true residuals in one matvec
    const int ne = (int)ends.size();
    std::vector<std::vector<cd>> yd(ne);
    for (int e = 0; e < ne; ++e) {
      GmresLane& G = L[ends[e]];
      const int j = G.j;
      std::vector<std::complex<double>> y(j);
      for (int i = j - 1; i >= 0; --i) {
        std::complex<double> sacc = G.g[i];
        for (int q = i + 1; q < j; ++q) sacc -= G.H[(size_t)q * (m + 1) + i] * y[q];
        y[i] = sacc / G.H[(size_t)i * (m + 1) + i];
      }
      yd[e].resize(j);
      for (int i = 0; i < j; ++i) yd[e][i] = cd{y[i].real(), y[i].imag()};
      cd* u = W + (size_t)e * N;
      cd* z = Z + (size_t)e * N;
      EWBEM_HIP_CHECK(hipMemcpyAsync(G.hd, yd[e].data(), j * sizeof(cd), hipMemcpyHostToDevice, st));
      launch_gemv_acc(G.V, N, j, G.hd, cd{0.0, 0.0}, u, N, st);
      precond_apply(c, u, z);
      launch_axpby(cd{1.0, 0.0}, z, cd{1.0, 0.0}, G.x, N, st);
      EWBEM_HIP_CHECK(hipMemcpyAsync(z, G.x, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
    }
    EWBEM_HIP_CHECK(hipEventRecord(ev.a, st));
    apply_tree_multi(c, Z, W, ne);
    EWBEM_HIP_CHECK(hipEventRecord(ev.b, st));
    for (int e = 0; e < ne; ++e) {
      GmresLane& G = L[ends[e]];
      EWBEM_HIP_CHECK(hipMemcpyAsync(G.r, W + (size_t)e * N, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
      launch_axpby(cd{1.0, 0.0}, G.b, cd{-1.0, 0.0}, G.r, N, st);
    }
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    c->acc.t_matvec_ms += ev.elapsed();
    c->acc.matvec_bytes_total += c->matvec_bytes + (ne - 1) * c->matvec_rhs_bytes;
    c->acc.matvecs_timed += 1;
    norms(false, ends);
    for (int l : ends) {
      GmresLane& G = L[l];
      G.relres = G.rnorm / G.bnorm;
      G.arnoldi = false;
      if (!(G.relres > tol) || G.j == 0) G.done = true;
    }
  }
}

// Sec. 4.2: x0 = X R^{-1} Q^H b with Y = A X = Q R (X: the last K solutions,
// newest first); columns with |R_jj| < 1e-12 |R_00| are dropped.  Also
// returns r0 = b - Y s without another matvec.
// Least-squares extrapolation (Sec. 4.2, eqs. a0, lsem, a0-solution): x0 = X s
// with s minimising |b - A X s|, X the last K solutions and, when extra is
// given, one more column (the learned guess).  r receives b - A x0.
void sem_guess(ewbem_ctx* c, cd* x, cd* r, const cd* extra = nullptr) {
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  const int K = std::min(c->so.sem_k, c->hist_n);
  const int Kt = K + (extra ? 1 : 0);
  EWBEM_HIP_CHECK(hipMemsetAsync(x, 0, N * sizeof(cd), st));
  EWBEM_HIP_CHECK(hipMemcpyAsync(r, c->d_b.p, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
  if (Kt == 0) return;
  cd* Y = c->d_Y.p;
  cd* Q = c->d_V.p;  // GMRES basis as scratch
  // Y(:, j) = A X(:, j): the columns are copied into the order of Y, then the
  // operator is applied to up to eight at once
  for (int j = 0; j < K; ++j)
    EWBEM_HIP_CHECK(hipMemcpyAsync(Q + (size_t)j * N, c->d_hist_sol.p + (size_t)c->hist_slot[j] * N,
                                   N * sizeof(cd), hipMemcpyDeviceToDevice, st));
  if (extra)
    EWBEM_HIP_CHECK(hipMemcpyAsync(Q + (size_t)K * N, extra, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
  for (int j0 = 0; j0 < Kt; j0 += HMV_MAXRHS)
    apply_tree_multi(c, Q + (size_t)j0 * N, Y + (size_t)j0 * N, std::min(HMV_MAXRHS, Kt - j0));
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  // classical Gram-Schmidt twice on the columns of Y
  std::vector<std::complex<double>> R((size_t)Kt * Kt, 0.0);
  std::vector<int> kept;
  double r00 = 0;
  std::vector<cd> hb(2 * (Kt + 1));
  for (int j = 0; j < Kt; ++j) {
    const int q = (int)kept.size();
    cd* qj = Q + (size_t)q * N;
    EWBEM_HIP_CHECK(hipMemcpyAsync(qj, Y + (size_t)j * N, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
    std::vector<std::complex<double>> rcol(q, 0.0);
    for (int pass = 0; pass < 2 && q > 0; ++pass) {
      launch_dots(Q, N, q, qj, N, c->d_hpart.p, c->d_small.p, st);
      launch_gemv_sub(Q, N, q, c->d_small.p, qj, N, st);
      EWBEM_HIP_CHECK(hipMemcpyAsync(hb.data(), c->d_small.p, q * sizeof(cd), hipMemcpyDeviceToHost, st));
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      for (int i = 0; i < q; ++i) rcol[i] += std::complex<double>(hb[i].x, hb[i].y);
    }
    const double nrm = dev_norm(c, qj);
    if (j == 0) r00 = nrm;
    if (!(nrm > 1e-12 * r00) || nrm == 0.0) continue;  // dependent column
    launch_axpby(cd{1.0 / nrm, 0.0}, qj, cd{0.0, 0.0}, qj, N, st);
    for (int i = 0; i < q; ++i) R[(size_t)i * Kt + q] = rcol[i];
    R[(size_t)q * Kt + q] = nrm;
    kept.push_back(j);
  }
  const int q = (int)kept.size();
  if (q == 0) return;
  // s = R^{-1} Q^H b
  launch_dots(Q, N, q, c->d_b.p, N, c->d_hpart.p, c->d_small.p, st);
  EWBEM_HIP_CHECK(hipMemcpyAsync(hb.data(), c->d_small.p, q * sizeof(cd), hipMemcpyDeviceToHost, st));
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  std::vector<std::complex<double>> sv(q);
  for (int i = q - 1; i >= 0; --i) {
    std::complex<double> a(hb[i].x, hb[i].y);
    for (int l = i + 1; l < q; ++l) a -= R[(size_t)i * Kt + l] * sv[l];
    sv[i] = a / R[(size_t)i * Kt + i];
  }
  // coefficients over the history slots and the extra column (x0), and over
  // Y's columns (r0)
  const int ncap = std::max(1, c->so.sem_k);
  std::vector<cd> cx(ncap, cd{0, 0}), cy(Kt, cd{0, 0});
  cd cext{0, 0};
  for (int i = 0; i < q; ++i) {
    const cd v{sv[i].real(), sv[i].imag()};
    if (kept[i] < K)
      cx[c->hist_slot[kept[i]]] = v;
    else
      cext = v;
    cy[kept[i]] = v;
  }
  EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_small.p, cx.data(), ncap * sizeof(cd), hipMemcpyHostToDevice, st));
  // only the slots written so far (0..hist_n): the others hold whatever the
  // allocation held, and a zero coefficient times a NaN there is NaN
  launch_gemv_acc(c->d_hist_sol.p, N, c->hist_n, c->d_small.p, cd{0.0, 0.0}, x, N, st);
  if (extra) launch_axpby(cext, extra, cd{1.0, 0.0}, x, N, st);
  EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_small.p + ncap, cy.data(), Kt * sizeof(cd), hipMemcpyHostToDevice, st));
  launch_gemv_sub(Y, N, Kt, c->d_small.p + ncap, r, N, st);
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
}

void push_history(ewbem_ctx* c, const cd* a, int k) {
  const long long N = 3LL * c->nt;
  const int cap = std::max(1, c->so.sem_k);
  int slot;
  if (c->hist_n < cap) {
    slot = c->hist_n++;
  } else {
    slot = c->hist_slot.back();
    c->hist_slot.pop_back();
    c->hist_kidx.pop_back();
  }
  EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_hist_sol.p + (size_t)slot * N, a, N * sizeof(cd),
                                 hipMemcpyDeviceToDevice, c->stream));
  c->hist_slot.insert(c->hist_slot.begin(), slot);
  c->hist_kidx.insert(c->hist_kidx.begin(), k);
}

// ---- learned initial guess

// Reduced coordinates Phi^H a of the solution at frequency k into the ring
// of the last three.
void push_coords(ewbem_ctx* c, const cd* a, int k) {
  const long long N = 3LL * c->nt;
  const int r = c->lm.r;
  int slot;
  if ((int)c->lc_slot.size() < 3) {
    slot = (int)c->lc_slot.size();
  } else {
    slot = c->lc_slot.back();
    c->lc_slot.pop_back();
    c->lc_kidx.pop_back();
  }
  launch_dots(c->d_phi.p, N, r, a, N, c->d_hpart.p, c->d_lcoef.p + (size_t)slot * r, c->stream);
  c->lc_slot.insert(c->lc_slot.begin(), slot);
  c->lc_kidx.insert(c->lc_kidx.begin(), k);
}

// The learned prediction of frequency k's coordinates into d_lpred: the
// least-squares map's W_k X_k^H [c1; c2; c3] (when the model has one for
// this frequency grid; else the quadratic extrapolation 3 c1 - 3 c2 + c3)
// plus the network's correction nu y.  False when the coordinates of k-1,
// k-2 and k-3 are not all in the ring.
bool learned_coords(ewbem_ctx* c, int k) {
  if (k < 3 || c->lc_kidx.size() < 3 || c->lc_kidx[0] != k - 1 || c->lc_kidx[1] != k - 2 ||
      c->lc_kidx[2] != k - 3)
    return false;
  hipStream_t st = c->stream;
  const int r = c->lm.r;
  const int idx[4] = {c->lc_slot[0], c->lc_slot[1], c->lc_slot[2], -1};
  const float kf = (float)k / (float)(c->n_f / 2);
  EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_lidx.p, idx, sizeof(idx), hipMemcpyHostToDevice, st));
  EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_lkf.p, &kf, sizeof(float), hipMemcpyHostToDevice, st));
  launch_learn_samples(c->d_lcoef.p, nullptr, r, c->d_lidx.p, c->d_lkf.p, 1, c->d_lfeat.p, nullptr, c->d_lnu.p, st);
  mlp_forward(c->lm.shape, c->d_lp.p, 1, c->d_lfeat.p, c->d_lact.p, c->d_lpre.p, c->d_ly.p, st);
  const cd* bp = nullptr;
  const LearnedModel& m = c->lm;
  if (m.rn > 0 && m.rk == c->n_f / 2 + 1 && k < m.rk) {
    const size_t xs = 3 * (size_t)r * m.rn, wsz = (size_t)r * m.rn;
    for (int j = 0; j < 3; ++j)
      EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_lh.p + (size_t)j * r, c->d_lcoef.p + (size_t)idx[j] * r, r * sizeof(cd),
                                     hipMemcpyDeviceToDevice, st));
    launch_dots(c->d_rx.p + (size_t)(k - 3) * xs, 3 * r, m.rn, c->d_lh.p, 3 * r, c->d_hpart.p, c->d_lz.p, st);
    launch_gemv_acc(c->d_rw.p + (size_t)(k - 3) * wsz, r, m.rn, c->d_lz.p, cd{0.0, 0.0}, c->d_lbase.p, r, st);
    bp = c->d_lbase.p;
  }
  launch_learn_compose(c->d_lcoef.p, r, c->d_lidx.p, c->d_lnu.p, c->d_ly.p, bp, 0, c->d_lpred.p, st);
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));  // idx and kf live on this frame
  return true;
}

// The learned guess: the least-squares extrapolation x (residual r) with
// its part in the basis moved towards the prediction p, by the step that
// minimises the residual along v = Phi (p - Phi^H x):
//   y = A v,  gamma = (y^H r) / (y^H y),  x += gamma v,  r -= gamma y.
// One operator application; the residual never grows.
void learned_refine(ewbem_ctx* c, int k, cd* x, cd* r) {
  if (!learned_coords(c, k)) return;
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  const int rr = c->lm.r;
  cd* cx = c->d_lcoef.p + 3 * (size_t)rr;  // scratch after the ring's three slots
  launch_dots(c->d_phi.p, N, rr, x, N, c->d_hpart.p, cx, st);
  launch_axpby(cd{-1.0, 0.0}, cx, cd{1.0, 0.0}, c->d_lpred.p, rr, st);  // p - Phi^H x
  launch_gemv_acc(c->d_phi.p, N, rr, c->d_lpred.p, cd{0.0, 0.0}, c->d_lx.p, N, st);
  EventPair ev;
  apply_tree(c, c->d_lx.p, c->d_w.p, &ev);
  launch_dots(c->d_w.p, N, 1, r, N, c->d_hpart.p, c->d_small.p, st);
  launch_dots(c->d_w.p, N, 1, c->d_w.p, N, c->d_hpart.p, c->d_small.p + 1, st);
  cd h[2];
  EWBEM_HIP_CHECK(hipMemcpyAsync(h, c->d_small.p, sizeof(h), hipMemcpyDeviceToHost, st));
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  account_matvec(c, ev);
  if (!(h[1].x > 0.0)) return;
  const cd g{h[0].x / h[1].x, h[0].y / h[1].x};
  launch_axpby(g, c->d_lx.p, cd{1.0, 0.0}, x, N, st);
  launch_axpby(cd{-g.x, -g.y}, c->d_w.p, cd{1.0, 0.0}, r, N, st);
  c->acc.guess_learned += 1;
}

// The initial guess of frequency k into d_x and its residual into d_r (b in
// d_b, the operator assembled); x0 (caller order, device) optional.
void guess_k(ewbem_ctx* c, int k, const ewbem_z* x0) {
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  const auto tg = Clock::now();
  EventPair ev;
  if (x0) {
    launch_permute((const cd*)x0, c->d_perm.p, c->nt, 1, c->d_x.p, st);
    apply_tree(c, c->d_x.p, c->d_r.p, &ev);
    launch_axpby(cd{1, 0}, c->d_b.p, cd{-1, 0}, c->d_r.p, N, st);
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    account_matvec(c, ev);
  } else if (c->so.guess == EWBEM_GUESS_SEM || c->so.guess == EWBEM_GUESS_LEARNED) {
    if (c->so.guess == EWBEM_GUESS_LEARNED && !c->lm.ok) fail(EWBEM_ESTATE, "learned guess: no trained or loaded model");
    sem_guess(c, c->d_x.p, c->d_r.p, nullptr);
    if (c->so.guess == EWBEM_GUESS_LEARNED) learned_refine(c, k, c->d_x.p, c->d_r.p);
  } else if (c->so.guess == EWBEM_GUESS_QUAD && c->hist_n > 0) {
    const int K = std::min(3, c->hist_n);
    static const double coef[4][3] = {{0, 0, 0}, {1, 0, 0}, {2, -1, 0}, {3, -3, 1}};
    const int ncap = std::max(1, c->so.sem_k);
    std::vector<cd> cx(ncap, cd{0, 0});
    for (int j = 0; j < K; ++j) cx[c->hist_slot[j]] = cd{coef[K][j], 0};
    EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_small.p, cx.data(), ncap * sizeof(cd), hipMemcpyHostToDevice, st));
    launch_gemv_acc(c->d_hist_sol.p, N, c->hist_n, c->d_small.p, cd{0, 0}, c->d_x.p, N, st);  // written slots only
    apply_tree(c, c->d_x.p, c->d_r.p, &ev);
    launch_axpby(cd{1, 0}, c->d_b.p, cd{-1, 0}, c->d_r.p, N, st);
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    account_matvec(c, ev);
  } else {
    EWBEM_HIP_CHECK(hipMemsetAsync(c->d_x.p, 0, N * sizeof(cd), st));
    EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_r.p, c->d_b.p, N * sizeof(cd), hipMemcpyDeviceToDevice, st));
  }
  const double bn = dev_norm(c, c->d_b.p);
  c->acc.guess_resid_sum += bn > 0 ? dev_norm(c, c->d_r.p) / bn : 0.0;
  c->acc.t_guess_ms += ms_since(tg);
}

// After GMRES on frequency k (solution in d_x): statistics, extrapolation
// history and the spectrum.
void finish_k(ewbem_ctx* c, int k, int its, double rel) {
  hipStream_t st = c->stream;
  const long long N = 3LL * c->nt;
  c->acc.n_solves += 1;
  c->acc.iters_total += its;
  c->acc.iters_max = std::max(c->acc.iters_max, its);
  c->acc.resid_max = std::max(c->acc.resid_max, rel);
  push_history(c, c->d_x.p, k);
  if (c->so.guess == EWBEM_GUESS_LEARNED && c->lm.ok) push_coords(c, c->d_x.p, k);
  EWBEM_HIP_CHECK(hipMemcpyAsync(c->d_spec.p + (size_t)k * N, c->d_x.p, N * sizeof(cd),
                                 hipMemcpyDeviceToDevice, st));
}

// Solve frequency k into d_x (tree order); x0 (caller order, device) optional.
int solve_k(ewbem_ctx* c, int k, const ewbem_z* x0) {
  if (c->assembled_k != k) assemble_k(c, k);
  guess_k(c, k, x0);
  const auto ts = Clock::now();
  int its = 0;
  bool conv = true;
  const double rel = gmres(c, c->d_x.p, c->d_r.p, its, conv);
  c->acc.t_gmres_ms += ms_since(ts);
  finish_k(c, k, its, rel);
  return conv ? EWBEM_OK : EWBEM_ENOCONV;
}

// Every frequency of the current load in order, the solutions into d_spec.
int frequency_loop(ewbem_ctx* c) {
  c->hist_n = 0;
  c->hist_slot.clear();
  c->hist_kidx.clear();
  c->lc_slot.clear();
  c->lc_kidx.clear();
  {
    // every frequency's off-diagonal U t0 in one batched pass
    EventPair ev;
    const auto t0 = Clock::now();
    EWBEM_HIP_CHECK(hipEventRecord(ev.a, c->stream));
    rhs_precompute(c, dev_geom(c), 0, c->n_f / 2 + 1);
    EWBEM_HIP_CHECK(hipEventRecord(ev.b, c->stream));
    EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
    c->acc.t_rhs_ms += ev.elapsed();
    c->acc.t_assemble_ms += ms_since(t0);
  }
  int rc = EWBEM_OK;
  const int nk = c->n_f / 2 + 1;
  // the pipeline: while GMRES solves frequency k on the caller's stream,
  // the far factors of k + 1 are approximated on the library's second
  // stream by a second host thread, into the factor slot the matvec of k
  // does not read; the rest of k + 1's assembly follows the solve
  if (c->so.pipeline && c->op.aca_batch_mb > 0)
    fail(EWBEM_EINVAL, "the pipeline needs the whole complex128 far field (aca_batch_mb = 0)");
  const bool pipe = c->so.pipeline && !c->far_h.empty();
  for (int k = 0; k < nk; ++k) {
    if (!pipe || k + 1 == nk) {
      const int r = solve_k(c, k, nullptr);
      if (r != EWBEM_OK) rc = r;
      continue;
    }
    if (c->assembled_k != k) assemble_k(c, k);
    const int slot = 1 - c->fslot;
    c->P = make_params(c, s_of_k(c, k + 1));
    const DevGeom g = dev_geom(c);
    double aca_ms = 0.0, aca_wall = 0.0;
    std::exception_ptr err;
    std::thread th([&, g, slot] {
      try {
        EWBEM_HIP_CHECK(hipSetDevice(c->device));
        EventPair ev;
        const auto t0 = Clock::now();
        run_aca(c, g, ev, aca_ms, c->astream, slot);
        aca_wall = ms_since(t0);
      } catch (...) {
        err = std::current_exception();
      }
    });
    int r = EWBEM_OK;
    try {
      r = solve_k(c, k, nullptr);
    } catch (...) {
      th.join();
      throw;
    }
    th.join();
    if (err) std::rethrow_exception(err);
    c->fslot = slot;
    c->acc.t_aca_ms += aca_ms;
    c->acc.t_assemble_ms += aca_wall;
    assemble_k(c, k + 1, true);
    if (r != EWBEM_OK) rc = r;
  }
  return rc;
}

// ---- several loads (same history) through one frequency loop

// What differs between the loads of a multi-load run: the traction, its
// off-diagonal sums for every frequency, the extrapolation history, the
// current right-hand side, iterate and residual, and where the spectrum goes
// (tree order, N_f/2 + 1 rows of N).
struct LoadRun {
  DevBuf<double> t0;
  DevBuf<double> tau;  // incident waves: arrival delay per element
  DevBuf<cd> rhs_part;
  DevBuf<cd> hist_sol;
  DevBuf<cd> b, x, r;
  std::vector<int> hist_slot, hist_kidx;
  int hist_n = 0;
  cd* spec = nullptr;
};

template <typename T>
void swap_buf(DevBuf<T>& a, DevBuf<T>& b) {
  std::swap(a.p, b.p);
  std::swap(a.n, b.n);
}

// Exchange a load's state with the context's (twice restores it).
void swap_load(ewbem_ctx* c, LoadRun& L) {
  swap_buf(c->d_t0, L.t0);
  if (c->load_incident) swap_buf(c->d_tau, L.tau);
  swap_buf(c->d_rhs_part, L.rhs_part);
  swap_buf(c->d_hist_sol, L.hist_sol);
  swap_buf(c->d_b, L.b);
  swap_buf(c->d_x, L.x);
  swap_buf(c->d_r, L.r);
  std::swap(c->hist_slot, L.hist_slot);
  std::swap(c->hist_kidx, L.hist_kidx);
  std::swap(c->hist_n, L.hist_n);
}

// A load's state in the context for one scope.
struct LoadIn {
  ewbem_ctx* c;
  LoadRun& L;
  LoadIn(ewbem_ctx* c_, LoadRun& L_) : c(c_), L(L_) { swap_load(c, L); }
  ~LoadIn() { swap_load(c, L); }
  LoadIn(const LoadIn&) = delete;
  LoadIn& operator=(const LoadIn&) = delete;
};

// Every frequency once for all loads: the operator, preconditioner and self
// terms are assembled once per frequency; each load's right-hand side and
// extrapolated guess follow, and the loads' GMRES run in lock-step groups of
// up to eight, their matvecs as one multi-right-hand-side product.  A load's
// solutions equal those of frequency_loop for that load alone on the same
// operators.
int multi_load_loop(ewbem_ctx* c, std::vector<LoadRun>& loads) {
  const long long N = 3LL * c->nt;
  const int nk = c->n_f / 2 + 1;
  const int n = (int)loads.size();
  hipStream_t st = c->stream;
  const DevGeom g = dev_geom(c);
  const int ncap = std::max(1, c->so.sem_k);
  const int m = c->so.restart;
  const int hs = 2 * (m + 2) + 2;
  const int gmax = std::min(n, HMV_MAXRHS);
  DevBuf<cd> Vm, Zm, Wm, hm;
  Vm.reserve((size_t)gmax * (m + 1) * N);
  Zm.reserve((size_t)HMV_MAXRHS * N);
  Wm.reserve((size_t)HMV_MAXRHS * N);
  hm.reserve((size_t)gmax * hs);
  {
    EventPair ev;
    const auto t0 = Clock::now();
    EWBEM_HIP_CHECK(hipEventRecord(ev.a, st));
    // every load's off-diagonal U t0 for all frequencies, the kernel
    // evaluated once per pair for up to eight loads
    std::vector<const double*> t0s, taus;
    std::vector<cd*> parts;
    for (LoadRun& L : loads) {
      L.hist_sol.reserve((size_t)ncap * N);
      L.b.reserve(N);
      L.x.reserve(N);
      L.r.reserve(N);
      L.rhs_part.reserve((size_t)rhs_split(c->nt) * nk * N);
      t0s.push_back(L.t0.p);
      taus.push_back(L.tau.p);
      parts.push_back(L.rhs_part.p);
    }
    launch_rhs_loads(g, c->P, c->sigma, 2.0 * M_PI / c->period, 0, nk, n, t0s.data(),
                     c->load_incident ? taus.data() : nullptr, parts.data(), st);
    EWBEM_HIP_CHECK(hipGetLastError());
    c->boff_k0 = 0;
    c->boff_nk = nk;
    EWBEM_HIP_CHECK(hipEventRecord(ev.b, st));
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    c->acc.t_rhs_ms += ev.elapsed();
    c->acc.t_assemble_ms += ms_since(t0);
  }
  const int saved_guess = c->so.guess;
  if (c->so.guess == EWBEM_GUESS_LEARNED) c->so.guess = EWBEM_GUESS_SEM;  // no per-load coordinate rings
  int rc = EWBEM_OK;
  std::vector<GmresLane> lanes;
  try {
    for (int k = 0; k < nk; ++k)
      for (int g0 = 0; g0 < n; g0 += HMV_MAXRHS) {
        const int g1 = std::min(n, g0 + HMV_MAXRHS);
        for (int l = g0; l < g1; ++l) {
          LoadIn in(c, loads[l]);
          if (c->assembled_k != k)
            assemble_k(c, k);  // b of this load too
          else
            rhs_finish_k(c, k);
          guess_k(c, k, nullptr);
        }
        lanes.assign(g1 - g0, GmresLane{});
        for (int l = g0; l < g1; ++l) {
          GmresLane& G = lanes[l - g0];
          G.b = loads[l].b.p;
          G.x = loads[l].x.p;
          G.r = loads[l].r.p;
          G.V = Vm.p + (size_t)(l - g0) * (m + 1) * N;
          G.hd = hm.p + (size_t)(l - g0) * hs;
        }
        const auto ts = Clock::now();
        gmres_multi(c, lanes, Zm.p, Wm.p);
        c->acc.t_gmres_ms += ms_since(ts);
        for (int l = g0; l < g1; ++l) {
          const GmresLane& G = lanes[l - g0];
          LoadIn in(c, loads[l]);
          finish_k(c, k, G.its, G.relres);
          if (!(G.relres <= c->so.tol)) rc = EWBEM_ENOCONV;
          EWBEM_HIP_CHECK(hipMemcpyAsync(loads[l].spec + (size_t)k * N, c->d_x.p, N * sizeof(cd),
                                         hipMemcpyDeviceToDevice, st));
        }
      }
  } catch (...) {
    c->so.guess = saved_guess;
    c->assembled_k = -1;
    c->boff_nk = 0;
    throw;
  }
  c->so.guess = saved_guess;
  // the right-hand side and off-diagonal sums now in the context are the
  // last load's: the context's own load is rebuilt on its next solve
  c->assembled_k = -1;
  c->boff_nk = 0;
  EWBEM_HIP_CHECK(hipStreamSynchronize(st));
  return rc;
}

// One LoadRun per case: tree-order tractions from caller-order values
// (nt x 3 tractions, or nt pressures when pressure), spectra at spec_base.
std::vector<LoadRun> make_load_runs(ewbem_ctx* c, int n, const double* loads, bool pressure, cd* spec_base) {
  const long long N = 3LL * c->nt;
  const int nk = c->n_f / 2 + 1;
  const size_t per = pressure ? (size_t)c->nt : 3 * (size_t)c->nt;
  const std::vector<double> saved = c->load_caller;
  const bool saved_p = c->load_is_pressure;
  std::vector<LoadRun> runs(n);
  try {
    for (int i = 0; i < n; ++i) {
      c->load_caller.assign(loads + per * i, loads + per * (i + 1));
      c->load_is_pressure = pressure;
      runs[i].t0.upload(tree_load(c), c->stream);
      EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));  // the host vector is a temporary
      runs[i].spec = spec_base + (size_t)i * nk * N;
    }
  } catch (...) {
    c->load_caller = saved;
    c->load_is_pressure = saved_p;
    throw;
  }
  c->load_caller = saved;
  c->load_is_pressure = saved_p;
  return runs;
}

// One LoadRun per incident plane S-wave (unit direction dirs[3i], unit
// polarisation pols[3i], normal to each other): its factor g and arrival
// delays, spectra at spec_base.
std::vector<LoadRun> make_incident_runs(ewbem_ctx* c, int n, const double* dirs, const double* pols,
                                        cd* spec_base) {
  const long long N = 3LL * c->nt;
  const int nk = c->n_f / 2 + 1;
  std::vector<LoadRun> runs(n);
  std::vector<double> g0, tau;
  for (int i = 0; i < n; ++i) {
    incident_factors(c, dirs + 3 * i, pols + 3 * i, g0, tau);
    runs[i].t0.upload(g0, c->stream);
    runs[i].tau.upload(tau, c->stream);
    EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));  // the host vectors are reused
    runs[i].spec = spec_base + (size_t)i * nk * N;
  }
  return runs;
}

void begin_stats(ewbem_ctx* c);
void end_stats(ewbem_ctx* c, ewbem_stats* out);

// The loads' frequency loop, then each load's inverse transform into u (and
// its spectrum in caller order into spec, if given); sp holds the spectra.
int run_loads(ewbem_ctx* ctx, std::vector<LoadRun>& runs, const cd* sp, double* u, ewbem_z* spec,
              ewbem_stats* stats) {
  const long long N = 3LL * ctx->nt;
  const int nk = ctx->n_f / 2 + 1;
  const int rc = multi_load_loop(ctx, runs);
  const auto tp = Clock::now();
  for (size_t l = 0; l < runs.size(); ++l) {
    const cd* sl = sp + l * nk * N;
    launch_mft_inverse(sl, N, ctx->n_f, ctx->period, ctx->sigma, ctx->window, ctx->d_perm.p,
                       u + l * ctx->n_f * N, ctx->stream);
    if (spec)
      for (int k = 0; k < nk; ++k)
        launch_permute(sl + (size_t)k * N, ctx->d_perm.p, ctx->nt, 0, (cd*)spec + (l * nk + k) * N, ctx->stream);
  }
  EWBEM_HIP_CHECK(hipGetLastError());
  EWBEM_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  ctx->acc.t_post_ms += ms_since(tp);
  end_stats(ctx, stats);
  if (rc != EWBEM_OK) ctx->err = "GMRES did not reach the tolerance within maxit at some frequency";
  return rc;
}

int guard(ewbem_ctx* ctx, const std::function<int()>& f) {
  if (!ctx) return EWBEM_EINVAL;
  try {
    ctx->err.clear();
    return f();
  } catch (const ApiError& e) {
    ctx->err = e.what();
    return e.status;
  } catch (const HipError& e) {
    ctx->err = e.what();
    return e.code == hipErrorOutOfMemory ? EWBEM_ENOMEM : EWBEM_EHIP;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return EWBEM_ENOMEM;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return EWBEM_EINVAL;
  }
}

void begin_stats(ewbem_ctx* c) { c->acc = ewbem_stats{}; }
void end_stats(ewbem_ctx* c, ewbem_stats* out) {
  c->acc.matvec_bytes = c->matvec_bytes;
  c->acc.stored_bytes = c->stored_bytes;
  c->acc.rank_sum = c->rank_sum;
  c->acc.rank_max = c->rank_max;
  c->acc.n_near = (int64_t)c->near_h.size();
  c->acc.n_far = (int64_t)c->far_h.size();
  if (out) *out = c->acc;
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// ---- training of the learned guess

using zc = std::complex<double>;

std::vector<zc> to_host(ewbem_ctx* c, const cd* d, size_t n) {
  std::vector<cd> h(n);
  if (n) EWBEM_HIP_CHECK(hipMemcpyAsync(h.data(), d, n * sizeof(cd), hipMemcpyDeviceToHost, c->stream));
  EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
  std::vector<zc> z(n);
  for (size_t i = 0; i < n; ++i) z[i] = zc(h[i].x, h[i].y);
  return z;
}

void to_device(ewbem_ctx* c, const std::vector<zc>& z, cd* d) {
  std::vector<cd> h(z.size());
  for (size_t i = 0; i < z.size(); ++i) h[i] = cd{z[i].real(), z[i].imag()};
  if (!h.empty())
    EWBEM_HIP_CHECK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(cd), hipMemcpyHostToDevice, c->stream));
  EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
}

// Gram matrix G = Y^H Y (l x l, row-major, host) of the columns of Y (n x l, ld n).
std::vector<zc> gram(ewbem_ctx* c, const cd* Y, long long n, int l, cd* part, cd* g) {
  for (int j = 0; j < l; ++j) launch_dots(Y, n, l, Y + (size_t)j * n, n, part, g + (size_t)j * l, c->stream);
  const std::vector<zc> gc = to_host(c, g, (size_t)l * l);  // column j = Y^H y_j
  std::vector<zc> G((size_t)l * l);
  for (int i = 0; i < l; ++i)
    for (int j = 0; j < l; ++j) G[(size_t)i * l + j] = gc[(size_t)j * l + i];
  return G;
}

// Orthonormalise the columns of Y (n x l) in place by Cholesky-QR,
// Y <- Y R^{-1} with Y^H Y = R^H R, three times; a Gram matrix too
// ill-conditioned to factor gets a small diagonal shift first (shifted
// Cholesky-QR: the later passes restore orthogonality).  tmp: n x l.
void cholqr3(ewbem_ctx* c, cd* Y, long long n, int l, cd* tmp, cd* part, cd* g) {
  for (int pass = 0; pass < 3; ++pass) {
    std::vector<zc> G = gram(c, Y, n, l, part, g);
    double tr = 0.0;
    for (int i = 0; i < l; ++i) tr += G[(size_t)i * l + i].real();
    std::vector<zc> Lf = G;
    // a (numerically) rank-deficient sketch gets a tiny diagonal shift
    for (double shift = 0.0; !cholesky(Lf, l);) {
      shift = shift == 0.0 ? 1e-14 * tr : shift * 100.0;
      if (!(shift < tr)) fail(EWBEM_EINVAL, "guess training: the snapshots span too few directions");
      Lf = G;
      for (int i = 0; i < l; ++i) Lf[(size_t)i * l + i] += shift;
    }
    const std::vector<zc> Ri = inverse_lh(Lf, l);
    std::vector<zc> cols((size_t)l * l);  // column j of R^{-1}, contiguous
    for (int i = 0; i < l; ++i)
      for (int j = 0; j < l; ++j) cols[(size_t)j * l + i] = Ri[(size_t)i * l + j];
    to_device(c, cols, g);
    for (int j = 0; j < l; ++j)
      launch_gemv_acc(Y, n, l, g + (size_t)j * l, cd{0.0, 0.0}, tmp + (size_t)j * n, n, c->stream);
    EWBEM_HIP_CHECK(hipMemcpyAsync(Y, tmp, (size_t)n * l * sizeof(cd), hipMemcpyDeviceToDevice, c->stream));
  }
}

// Proper orthogonal decomposition of the snapshots S (N x M, ld N) by a
// randomized range finder with q subspace iterations and l columns, then
// the eigen-decomposition of the sketch: Phi (N x r) spans the r dominant
// left singular directions.  Returns the fraction of |S|_F^2 they hold.
double pod_basis(ewbem_ctx* c, const cd* S, long long N, int M, int r, int l, int q, uint64_t seed, cd* Phi) {
  hipStream_t st = c->stream;
  DevBuf<cd> om, Q, tq, Z, tz, g, part;
  om.reserve((size_t)M * l);
  Q.reserve((size_t)N * l);
  tq.reserve((size_t)N * l);
  Z.reserve((size_t)M * l);
  tz.reserve((size_t)M * l);
  g.reserve((size_t)l * l + 1);
  part.reserve((size_t)std::max({dots_chunks(N) * (long long)M, dots_chunks(N) * (long long)l,
                                 dots_chunks(M) * (long long)l, 512LL}));
  {
    std::mt19937_64 rng(seed ^ 0x9e3779b97f4a7c15ULL);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<zc> o((size_t)M * l);
    for (auto& v : o) v = zc(nd(rng), nd(rng));
    to_device(c, o, om.p);
  }
  auto range = [&](const cd* X, cd* Yo) {  // Yo = S X (X: M x l)
    for (int j = 0; j < l; ++j) launch_gemv_acc(S, N, M, X + (size_t)j * M, cd{0.0, 0.0}, Yo + (size_t)j * N, N, st);
  };
  auto corange = [&](const cd* Y, cd* Xo) {  // Xo = S^H Y (Y: N x l)
    for (int j = 0; j < l; ++j) launch_dots(S, N, M, Y + (size_t)j * N, N, part.p, Xo + (size_t)j * M, st);
  };
  range(om.p, Q.p);
  cholqr3(c, Q.p, N, l, tq.p, part.p, g.p);
  for (int it = 0; it < q; ++it) {
    corange(Q.p, Z.p);
    cholqr3(c, Z.p, M, l, tz.p, part.p, g.p);
    range(Z.p, Q.p);
    cholqr3(c, Q.p, N, l, tq.p, part.p, g.p);
  }
  // B = Q^H S; B B^H = Z^H Z with Z = S^H Q
  corange(Q.p, Z.p);
  const std::vector<zc> G = gram(c, Z.p, M, l, part.p, g.p);
  std::vector<double> w;
  std::vector<zc> V;
  herm_eig(G, l, w, V);
  std::vector<zc> cols((size_t)l * r);
  for (int j = 0; j < r; ++j)
    for (int i = 0; i < l; ++i) cols[(size_t)j * l + i] = V[(size_t)i * l + j];
  to_device(c, cols, g.p);
  for (int j = 0; j < r; ++j)
    launch_gemv_acc(Q.p, N, l, g.p + (size_t)j * l, cd{0.0, 0.0}, Phi + (size_t)j * N, N, st);
  launch_dots(S, N * (long long)M, 1, S, N * (long long)M, part.p, g.p, st);
  const double tot = to_host(c, g.p, 1)[0].real();
  double top = 0.0;
  for (int j = 0; j < r; ++j) top += std::max(0.0, w[j]);
  return tot > 0.0 ? top / tot : 1.0;
}

double loss_sum(ewbem_ctx* c, const double* part, int nb) {
  std::vector<double> h(nb);
  EWBEM_HIP_CHECK(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (double v : h) s += v;
  return s;
}

// Full-batch Adam on M samples (X: M x dims[0], T: M x dims[L]) minimising
// the mean squared error; P (device) in place.  cosine: the step size decays
// from lr to lr / 10 over the epochs, else stays lr.  loss0 / loss1: the
// mean squared error before the first and after the last step.
void train_mlp(ewbem_ctx* c, const MlpShape& s, float* P, long long M, const float* X, const float* T, int epochs,
               double lr, bool cosine, double& loss0, double& loss1) {
  hipStream_t st = c->stream;
  const size_t np = s.n_params();
  const int dL = s.dims[s.n_layers()];
  const long long nout = M * dL;
  DevBuf<float> G, m1, m2, act, pre, Y, dY, work;
  DevBuf<double> part;
  G.reserve(np);
  m1.reserve(np);
  m2.reserve(np);
  act.reserve(std::max<size_t>(1, s.hidden_sum() * M));
  pre.reserve(std::max<size_t>(1, s.hidden_sum() * M));
  Y.reserve(nout);
  dY.reserve(nout);
  work.reserve(2 * (size_t)s.max_width() * M);
  const int nb = loss_blocks(nout);
  part.reserve(nb);
  EWBEM_HIP_CHECK(hipMemsetAsync(m1.p, 0, np * sizeof(float), st));
  EWBEM_HIP_CHECK(hipMemsetAsync(m2.p, 0, np * sizeof(float), st));
  const float scale = (float)(2.0 / (double)nout);
  const double b1 = 0.9, b2 = 0.999;
  for (int ep = 0; ep < epochs; ++ep) {
    mlp_forward(s, P, M, X, act.p, pre.p, Y.p, st);
    launch_mlp_loss(Y.p, T, nout, scale, dY.p, part.p, st);
    if (ep == 0) loss0 = loss_sum(c, part.p, nb) / (double)nout;
    mlp_backward(s, P, M, X, act.p, pre.p, dY.p, work.p, G.p, st);
    const double f = cosine && epochs > 1 ? 0.1 + 0.45 * (1.0 + std::cos(M_PI * ep / (epochs - 1))) : 1.0;
    AdamStep a{(float)(lr * f), (float)b1, (float)b2, 1e-8f, (float)(1.0 - std::pow(b1, ep + 1)),
               (float)(1.0 - std::pow(b2, ep + 1))};
    launch_adam(P, G.p, m1.p, m2.p, (long long)np, a, st);
  }
  mlp_forward(s, P, M, X, act.p, pre.p, Y.p, st);
  launch_mlp_loss(Y.p, T, nout, scale, nullptr, part.p, st);
  loss1 = loss_sum(c, part.p, nb) / (double)nout;
  if (epochs == 0) loss0 = loss1;
  EWBEM_HIP_CHECK(hipGetLastError());
}

MlpShape mlp_shape(int n_layers, const int32_t* dims) {
  if (n_layers < 1 || n_layers > 16 || !dims) fail(EWBEM_EINVAL, "network: need 1..16 layers and their widths");
  MlpShape s;
  for (int l = 0; l <= n_layers; ++l) {
    if (dims[l] < 1 || dims[l] > 8192) fail(EWBEM_EINVAL, "network: widths must be 1..8192");
    s.dims.push_back(dims[l]);
  }
  return s;
}

// Serialised model: magic, then int32 version, n_dof, r, n_layers, dims,
// then fp64 energy, loss0, loss1, then the fp32 parameters, then the basis
// (n_dof x r complex128, column-major, caller dof order).
constexpr char kModelMagic[8] = {'E', 'W', 'B', 'G', 'U', 'E', 'S', 'S'};
constexpr int32_t kModelVersion = 2;  // 1: without the least-squares map (still read)

size_t model_bytes(const LearnedModel& m, long long N) {
  return 8 + 4 * (4 + m.shape.dims.size()) + 3 * 8 + 4 * m.params.size() + 16 * (size_t)N * m.r + 8 +
         16 * (m.rx.size() + m.rw.size());
}

}  // namespace

// ---- the allocation-free network evaluation's scratch
//
// One statically sized array per GPU, holding the activations, the
// pre-activations, the output gradient, the backward pass's work area and
// the loss partials of ewbem_mlp_eval_noalloc.  In host code its name is
// not a device address: every use goes through the address that
// hipGetSymbolAddress returned for the device (kept in g_scratch_addr).
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The scratch array's address on `device` (which must be current), looked
// up once per device.  Null when the lookup fails.
void* scratch_addr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_addr[device] = ptr;
  }
  return g_scratch_addr[device];
}

__global__ void k_zero_f32(float* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

void ewbem_default_op_opts(ewbem_op_opts* o) {
  if (!o) return;
  o->kind = EWBEM_OP_HMAT;
  o->leaf_size = 64;
  o->eta_adm = 1.0;
  o->aca_tol = 1e-5;
  o->far_store = EWBEM_STORE_C128;
  o->self_order = 24;
  o->aca_reuse = 1;
  o->autotune = 1;
  o->aca_batch_mb = 0;
  o->mv_mfma = 1;
  o->ws_keep = 1;
  o->ws_pivot_rel = 0.0;
}

void ewbem_default_solver_opts(ewbem_solver_opts* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->restart = 100;
  o->maxit = 2000;
  o->precond = EWBEM_PREC_LEAF;
  o->guess = EWBEM_GUESS_SEM;
  o->sem_k = 3;
  o->pipeline = 0;
}

int ewbem_create(ewbem_ctx** out, int32_t device, void* hip_stream) {
  if (!out) return EWBEM_EINVAL;
  *out = nullptr;
  ewbem_ctx* c = nullptr;
  try {
    c = new ewbem_ctx();
  } catch (...) {
    return EWBEM_ENOMEM;
  }
  ewbem_default_op_opts(&c->op);
  ewbem_default_solver_opts(&c->so);
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (device >= 0) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
      delete c;
      return EWBEM_ESTATE;
    }
    if (hipSetDevice(device) != hipSuccess) {
      delete c;
      return EWBEM_EHIP;
    }
    if (!scratch_addr(device)) {
      delete c;
      return EWBEM_EHIP;
    }
  }
  *out = c;
  return EWBEM_OK;
}

void ewbem_destroy(ewbem_ctx* ctx) {
  if (!ctx) return;
  if (ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->astream) {
      (void)hipStreamSynchronize(ctx->astream);
      (void)hipStreamDestroy(ctx->astream);
      ctx->astream = nullptr;
    }
    if (ctx->ws_side.stream) {
      (void)hipStreamSynchronize(ctx->ws_side.stream);
      (void)hipStreamDestroy(ctx->ws_side.stream);
      (void)hipEventDestroy(ctx->ws_side.fork);
      (void)hipEventDestroy(ctx->ws_side.join);
      ctx->ws_side = WsSide{};
    }
  }
  delete ctx;
}

const char* ewbem_last_error(const ewbem_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ewbem_set_mesh(ewbem_ctx* ctx, int64_t nv, const double* xyz, int64_t nt, const int32_t* tri,
                   int32_t exterior) {
  return guard(ctx, [&] {
    if (nv < 3 || nt < 1 || !xyz || !tri || nt > (1LL << 28) || nv > (1LL << 30))
      fail(EWBEM_EINVAL, "mesh: need nv >= 3, nt >= 1 and non-null arrays");
    if (!finite_all(xyz, 3 * (size_t)nv)) fail(EWBEM_EINVAL, "mesh: non-finite coordinates");
    for (int64_t i = 0; i < 3 * nt; ++i)
      if (tri[i] < 0 || tri[i] >= nv) fail(EWBEM_EINVAL, "mesh: vertex index out of range");
    for (int64_t t = 0; t < nt; ++t) {
      const double* a = xyz + 3 * tri[3 * t];
      const double* b = xyz + 3 * tri[3 * t + 1];
      const double* c = xyz + 3 * tri[3 * t + 2];
      double e1[3], e2[3];
      for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = c[k] - a[k];
      }
      const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                   cz = e1[0] * e2[1] - e1[1] * e2[0];
      if (!(cx * cx + cy * cy + cz * cz > 0)) fail(EWBEM_EINVAL, "mesh: zero-area triangle");
    }
    ctx->xyz.assign(xyz, xyz + 3 * nv);
    ctx->tri.assign(tri, tri + 3 * nt);
    ctx->nv = (int)nv;
    ctx->nt = (int)nt;
    ctx->exterior = exterior != 0;
    ctx->have_mesh = true;
    ctx->have_load = false;
    ctx->lm = LearnedModel{};  // its basis belongs to the old mesh
    ctx->lm_dev = false;
    ctx->structure_ok = false;
    ctx->device_ok = false;
    ctx->assembled_k = -1;
    return EWBEM_OK;
  });
}

int ewbem_set_material(ewbem_ctx* ctx, double rho, double mu, double nu) {
  return guard(ctx, [&] {
    if (!(rho > 0) || !(mu > 0) || !(nu > -1.0 && nu < 0.5) || !std::isfinite(rho) || !std::isfinite(mu))
      fail(EWBEM_EINVAL, "material: need rho > 0, mu > 0, -1 < nu < 1/2");
    ctx->rho = rho;
    ctx->mu = mu;
    ctx->nu = nu;
    ctx->have_mat = true;
    ctx->device_ok = false;
    ctx->assembled_k = -1;
    return EWBEM_OK;
  });
}

int ewbem_set_time(ewbem_ctx* ctx, double period, int32_t n_f, double sigma, int32_t window) {
  return guard(ctx, [&] {
    if (!(period > 0) || !std::isfinite(period) || n_f < 2 || (n_f % 2) != 0 || n_f > (1 << 20) ||
        !(sigma >= 0) || !std::isfinite(sigma) || window < 0 || window > 2)
      fail(EWBEM_EINVAL, "time: need T > 0, even N_f >= 2, sigma >= 0, window 0..2");
    ctx->period = period;
    ctx->n_f = n_f;
    ctx->sigma = sigma;
    ctx->window = window;
    ctx->have_time = true;
    ctx->have_load = false;
    ctx->device_ok = false;
    ctx->assembled_k = -1;
    return EWBEM_OK;
  });
}

static int set_load(ewbem_ctx* ctx, const double* v, size_t nv_, const double* history, bool pressure,
                    const int32_t* bc = nullptr) {
  return guard(ctx, [&] {
    if (!ctx->have_mesh || !ctx->have_time) fail(EWBEM_ESTATE, "load: set the mesh and time grid first");
    if (!v || !history) fail(EWBEM_EINVAL, "load: null array");
    if (!finite_all(v, nv_) || !finite_all(history, ctx->n_f)) fail(EWBEM_EINVAL, "load: non-finite values");
    if (bc) {
      for (int e = 0; e < ctx->nt; ++e) {
        if (bc[e] != 0 && bc[e] != 1) fail(EWBEM_EINVAL, "load: boundary-condition kind must be 0 or 1");
        if (bc[e] == 1 && (v[3 * e] != 0.0 || v[3 * e + 1] != 0.0 || v[3 * e + 2] != 0.0))
          fail(EWBEM_EINVAL, "load: prescribed displacements must be zero");
      }
      ctx->bc_caller.assign(bc, bc + ctx->nt);
    } else {
      ctx->bc_caller.clear();
    }
    ctx->load_caller.assign(v, v + nv_);
    ctx->history.assign(history, history + ctx->n_f);
    ctx->load_is_pressure = pressure;
    ctx->load_incident = false;
    ctx->inc_total = false;
    ctx->have_load = true;
    ctx->device_ok = false;
    ctx->assembled_k = -1;
    return EWBEM_OK;
  });
}

int ewbem_set_load_traction(ewbem_ctx* ctx, const double* t0, const double* history) {
  if (!ctx) return EWBEM_EINVAL;
  return set_load(ctx, t0, 3 * (size_t)ctx->nt, history, false);
}

int ewbem_set_load_pressure(ewbem_ctx* ctx, const double* p, const double* history) {
  if (!ctx) return EWBEM_EINVAL;
  return set_load(ctx, p, (size_t)ctx->nt, history, true);
}

int ewbem_set_load_mixed(ewbem_ctx* ctx, const int32_t* bc, const double* values, const double* history) {
  if (!ctx) return EWBEM_EINVAL;
  if (!bc) return guard(ctx, [&] {
    fail(EWBEM_EINVAL, "load: null boundary-condition array");
    return EWBEM_OK;
  });
  return set_load(ctx, values, 3 * (size_t)ctx->nt, history, false, bc);
}

static int set_incident(ewbem_ctx* ctx, const double* dir, const double* pol, double ricker_fc, double t0,
                        bool total) {
  return guard(ctx, [&] {
    if (!ctx->have_mesh || !ctx->have_time) fail(EWBEM_ESTATE, "load: set the mesh and time grid first");
    if (!dir || !pol) fail(EWBEM_EINVAL, "incident wave: null direction or polarisation");
    if (!finite_all(dir, 3) || !finite_all(pol, 3) || !std::isfinite(ricker_fc) || !std::isfinite(t0) ||
        !(ricker_fc > 0))
      fail(EWBEM_EINVAL, "incident wave: non-finite input or non-positive frequency");
    const double nd = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    const double np = std::sqrt(pol[0] * pol[0] + pol[1] * pol[1] + pol[2] * pol[2]);
    if (!(nd > 0) || !(np > 0)) fail(EWBEM_EINVAL, "incident wave: zero direction or polarisation");
    double dd[3], pp[3], dp = 0;
    for (int k = 0; k < 3; ++k) {
      dd[k] = dir[k] / nd;
      pp[k] = pol[k] / np;
      dp += dd[k] * pp[k];
    }
    if (std::fabs(dp) > 1e-9) fail(EWBEM_EINVAL, "incident S-wave: polarisation must be normal to the direction");
    const double dt = ctx->period / ctx->n_f;
    ctx->history.resize(ctx->n_f);
    for (int n = 0; n < ctx->n_f; ++n) {
      const double a = std::pow(M_PI * ricker_fc * (n * dt - t0), 2);
      ctx->history[n] = (1.0 - 2.0 * a) * std::exp(-a);
    }
    for (int k = 0; k < 3; ++k) {
      ctx->inc_dir[k] = dd[k];
      ctx->inc_pol[k] = pp[k];
    }
    ctx->inc_fc = ricker_fc;
    ctx->inc_t0 = t0;
    ctx->bc_caller.clear();
    ctx->load_caller.clear();
    ctx->load_is_pressure = false;
    ctx->load_incident = true;
    ctx->inc_total = total;
    ctx->have_load = true;
    ctx->device_ok = false;
    ctx->assembled_k = -1;
    return EWBEM_OK;
  });
}

int ewbem_set_load_incident_s(ewbem_ctx* ctx, const double* dir, const double* pol, double ricker_fc,
                              double t0) {
  return set_incident(ctx, dir, pol, ricker_fc, t0, false);
}

int ewbem_set_load_incident_s_total(ewbem_ctx* ctx, const double* dir, const double* pol, double ricker_fc,
                                    double t0) {
  return set_incident(ctx, dir, pol, ricker_fc, t0, true);
}

int ewbem_set_operator(ewbem_ctx* ctx, const ewbem_op_opts* o) {
  return guard(ctx, [&] {
    if (!o) fail(EWBEM_EINVAL, "operator options: null");
    if ((o->kind != EWBEM_OP_DENSE && o->kind != EWBEM_OP_HMAT) || o->leaf_size < 1 || o->leaf_size > 64 ||
        !(o->eta_adm > 0) || !(o->aca_tol > 0 && o->aca_tol < 1) ||
        (o->far_store != EWBEM_STORE_C128 && o->far_store != EWBEM_STORE_C64) || o->self_order < 4 ||
        o->self_order > MAX_SELF_ORDER || (o->aca_reuse != 0 && o->aca_reuse != 1) ||
        (o->autotune != 0 && o->autotune != 1) || (o->mv_mfma != 0 && o->mv_mfma != 1) || o->aca_batch_mb < 0 ||
        !(o->ws_pivot_rel >= 0 && o->ws_pivot_rel < 1) || (o->ws_keep != 0 && o->ws_keep != 1) ||
        (o->aca_batch_mb > 0 && (o->far_store != EWBEM_STORE_C64 || o->kind != EWBEM_OP_HMAT)))
      fail(EWBEM_EINVAL, "operator options out of range");
    ctx->op = *o;
    ctx->structure_ok = false;
    ctx->device_ok = false;
    ctx->assembled_k = -1;
    return EWBEM_OK;
  });
}

int ewbem_set_solver(ewbem_ctx* ctx, const ewbem_solver_opts* o) {
  return guard(ctx, [&] {
    if (!o) fail(EWBEM_EINVAL, "solver options: null");
    if (!(o->tol > 0) || o->restart < 1 || o->restart > 400 || o->maxit < 1 || o->precond < 0 ||
        o->precond > 2 || o->guess < 0 || o->guess > 3 || o->sem_k < 1 || o->sem_k > 8 ||
        (o->pipeline != 0 && o->pipeline != 1))
      fail(EWBEM_EINVAL, "solver options out of range");
    ctx->so = *o;
    ctx->device_ok = false;  // buffers depend on restart and sem_k
    ctx->assembled_k = -1;
    return EWBEM_OK;
  });
}

int ewbem_info(ewbem_ctx* ctx, ewbem_info_t* info) {
  return guard(ctx, [&] {
    if (!info) fail(EWBEM_EINVAL, "info: null");
    ensure_structure(ctx);
    info->n_elements = ctx->nt;
    info->n_dof = 3LL * ctx->nt;
    info->n_clusters = (int64_t)ctx->part.clusters.size();
    info->n_leaves = (int64_t)ctx->part.leaves.size();
    info->n_near = (int64_t)ctx->part.near.size();
    info->n_far = (int64_t)ctx->part.far.size();
    info->near_entries = ctx->near_entries;
    int mx = 0, mn = 1 << 30;
    for (int l : ctx->part.leaves) {
      mx = std::max(mx, ctx->part.clusters[l].size());
      mn = std::min(mn, ctx->part.clusters[l].size());
    }
    info->max_leaf = mx;
    info->min_leaf = mn;
    info->mv_cols = ctx->mv_cols;
    info->mv_task_div = ctx->mv_div;
    info->mv_tuned = ctx->mv_tuned ? 1 : 0;
    info->mv_tune_cached = ctx->mv_tuned && ctx->mv_tune_cached ? 1 : 0;
    info->mv_tune_best_ms = ctx->mv_tuned ? ctx->mv_best_ms : 0.0;
    info->mv_tune_default_ms = ctx->mv_tuned ? ctx->mv_default_ms : 0.0;
    info->lib_device_bytes = g_dev_bytes.load();
    long long fw = 0;
    for (int sl = 0; sl < 2; ++sl) {
      fw += (long long)(ctx->d_wsf[sl].n * sizeof(cd));
      for (const auto& r : ctx->d_retry[sl]) fw += (long long)(r->n * sizeof(cd));
    }
    fw += (long long)(ctx->d_f32.n * sizeof(cf));
    for (const auto& ch : ctx->d_f32s) fw += (long long)(ch->n * sizeof(cf));
    info->far_work_bytes = fw;
    info->aca_scratch_bytes = (long long)(ctx->d_cross.n * sizeof(cd) + ctx->d_wscoef.n * sizeof(cd) +
                                          ctx->d_wspart.n * sizeof(double) + ctx->d_aca_part.n * sizeof(double));
    return EWBEM_OK;
  });
}

int ewbem_get_partition(ewbem_ctx* ctx, int32_t* perm, int32_t* nearp, int32_t* farp) {
  return guard(ctx, [&] {
    ensure_structure(ctx);
    if (perm)
      for (int t = 0; t < ctx->nt; ++t) perm[t] = ctx->hg.perm[t];
    auto put = [&](const std::vector<BlockPair>& v, int32_t* o) {
      for (size_t i = 0; i < v.size(); ++i) {
        const Cluster& r = ctx->part.clusters[v[i].row];
        const Cluster& s = ctx->part.clusters[v[i].col];
        o[4 * i] = r.begin;
        o[4 * i + 1] = r.end;
        o[4 * i + 2] = s.begin;
        o[4 * i + 3] = s.end;
      }
    };
    if (nearp) put(ctx->part.near, nearp);
    if (farp) put(ctx->part.far, farp);
    return EWBEM_OK;
  });
}

int ewbem_load_spectrum(ewbem_ctx* ctx, ewbem_z* phat) {
  return guard(ctx, [&] {
    if (!phat) fail(EWBEM_EINVAL, "null output");
    ensure_device(ctx);
    EWBEM_HIP_CHECK(hipMemcpyAsync(phat, ctx->d_phat.p, (ctx->n_f / 2 + 1) * sizeof(cd),
                                   hipMemcpyDeviceToHost, ctx->stream));
    EWBEM_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return EWBEM_OK;
  });
}

int ewbem_kernel_eval(ewbem_ctx* ctx, ewbem_z s, int64_t n, const double* x, const double* y,
                      const double* nrm, ewbem_z* U, ewbem_z* T) {
  return guard(ctx, [&] {
    require_gpu(ctx);
    if (!ctx->have_mat) fail(EWBEM_ESTATE, "material not set");
    if (n < 0 || (n > 0 && (!x || !y || (T && !nrm)))) fail(EWBEM_EINVAL, "kernel_eval: bad arguments");
    EWBEM_HIP_CHECK(hipSetDevice(ctx->device));
    KParams P = make_params(ctx, cd{s.re, s.im});
    launch_kernel_eval(P, n, x, y, nrm, (cd*)U, (cd*)T, ctx->stream);
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return EWBEM_OK;
  });
}

int ewbem_assemble_dense(ewbem_ctx* ctx, ewbem_z s, ewbem_z* T, ewbem_z* U) {
  return guard(ctx, [&] {
    require_gpu(ctx);
    ensure_structure(ctx);
    if (!ctx->have_mat) fail(EWBEM_ESTATE, "material not set");
    EWBEM_HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const HostGeom& g = ctx->hg;
    ctx->d_cen.upload(g.cen, st);
    ctx->d_nrm.upload(g.nrm, st);
    ctx->d_qp.upload(g.qp, st);
    ctx->d_qw.upload(g.qw, st);
    ctx->d_vtx.upload(g.vtx, st);
    ctx->d_perm.upload(g.perm, st);
    ctx->d_selfT.reserve(9 * (size_t)ctx->nt);
    ctx->d_selfU.reserve(9 * (size_t)ctx->nt);
    SelfRule S{};
    S.nt = S.nr = ctx->op.self_order;
    gauss_legendre01(S.nt, S.t, S.wt);
    gauss_legendre01(S.nr, S.u, S.wu);
    KParams P = make_params(ctx, cd{s.re, s.im});
    DevGeom dg = dev_geom(ctx);
    dg.bc = nullptr;  // the raw T and U
    launch_self(dg, P, S, ctx->d_selfT.p, ctx->d_selfU.p, nullptr, st);
    launch_dense_pairs(dg, P, ctx->d_perm.p, (cd*)T, (cd*)U, st);
    launch_dense_self(ctx->d_selfT.p, ctx->d_selfU.p, ctx->d_perm.p, ctx->nt, (cd*)T, (cd*)U, st);
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    ctx->device_ok = false;  // geometry buffers were reused
    return EWBEM_OK;
  });
}

int ewbem_assemble(ewbem_ctx* ctx, int32_t k, ewbem_stats* stats) {
  return guard(ctx, [&] {
    begin_stats(ctx);
    assemble_k(ctx, k);
    end_stats(ctx, stats);
    return EWBEM_OK;
  });
}

int ewbem_apply(ewbem_ctx* ctx, const ewbem_z* x, ewbem_z* y) {
  return guard(ctx, [&] {
    require_gpu(ctx);
    if (ctx->assembled_k < 0 || !ctx->device_ok) fail(EWBEM_ESTATE, "apply: no assembled operator");
    if (!x || !y) fail(EWBEM_EINVAL, "apply: null vector");
    hipStream_t st = ctx->stream;
    launch_permute((const cd*)x, ctx->d_perm.p, ctx->nt, 1, ctx->d_tmp_in.p, st);
    apply_tree(ctx, ctx->d_tmp_in.p, ctx->d_tmp_out.p, nullptr);
    launch_permute(ctx->d_tmp_out.p, ctx->d_perm.p, ctx->nt, 0, (cd*)y, st);
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    return EWBEM_OK;
  });
}

int ewbem_apply_multi(ewbem_ctx* ctx, const ewbem_z* X, int32_t nrhs, ewbem_z* Y) {
  return guard(ctx, [&] {
    require_gpu(ctx);
    if (ctx->assembled_k < 0 || !ctx->device_ok) fail(EWBEM_ESTATE, "apply_multi: no assembled operator");
    if (!X || !Y) fail(EWBEM_EINVAL, "apply_multi: null matrix");
    if (nrhs < 1 || nrhs > HMV_MAXRHS) fail(EWBEM_EINVAL, "apply_multi: nrhs must be 1..8");
    hipStream_t st = ctx->stream;
    const long long N = 3LL * ctx->nt;
    ctx->d_amx.reserve(2 * (size_t)HMV_MAXRHS * N);
    cd* Xt = ctx->d_amx.p;
    cd* Yt = Xt + (size_t)HMV_MAXRHS * N;
    for (int j = 0; j < nrhs; ++j) launch_permute((const cd*)X + j * N, ctx->d_perm.p, ctx->nt, 1, Xt + j * N, st);
    apply_tree_multi(ctx, Xt, Yt, nrhs);
    for (int j = 0; j < nrhs; ++j) launch_permute(Yt + j * N, ctx->d_perm.p, ctx->nt, 0, (cd*)Y + j * N, st);
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    return EWBEM_OK;
  });
}

int ewbem_get_rhs(ewbem_ctx* ctx, ewbem_z* b) {
  return guard(ctx, [&] {
    require_gpu(ctx);
    if (ctx->assembled_k < 0 || !ctx->device_ok) fail(EWBEM_ESTATE, "get_rhs: no assembled operator");
    if (!b) fail(EWBEM_EINVAL, "get_rhs: null vector");
    launch_permute(ctx->d_b.p, ctx->d_perm.p, ctx->nt, 0, (cd*)b, ctx->stream);
    EWBEM_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return EWBEM_OK;
  });
}

int ewbem_solve_frequency(ewbem_ctx* ctx, int32_t k, const ewbem_z* x0, ewbem_z* a, ewbem_stats* stats) {
  return guard(ctx, [&] {
    if (!a) fail(EWBEM_EINVAL, "solve_frequency: null output");
    begin_stats(ctx);
    ensure_device(ctx);
    const int rc = solve_k(ctx, k, x0);
    launch_permute(ctx->d_x.p, ctx->d_perm.p, ctx->nt, 0, (cd*)a, ctx->stream);
    EWBEM_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    end_stats(ctx, stats);
    if (rc != EWBEM_OK) ctx->err = "GMRES did not reach the tolerance within maxit";
    return rc;
  });
}

int ewbem_solve_transient(ewbem_ctx* ctx, double* u, ewbem_z* spec, ewbem_stats* stats) {
  return guard(ctx, [&] {
    if (!u) fail(EWBEM_EINVAL, "solve_transient: null output");
    begin_stats(ctx);
    ensure_device(ctx);
    const int rc = frequency_loop(ctx);
    const auto tp = Clock::now();
    const long long N = 3LL * ctx->nt;
    launch_mft_inverse(ctx->d_spec.p, N, ctx->n_f, ctx->period, ctx->sigma, ctx->window, ctx->d_perm.p, u,
                       ctx->stream);
    if (spec)
      for (int k = 0; k <= ctx->n_f / 2; ++k)
        launch_permute(ctx->d_spec.p + (size_t)k * N, ctx->d_perm.p, ctx->nt, 0, (cd*)spec + (size_t)k * N,
                       ctx->stream);
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    ctx->acc.t_post_ms += ms_since(tp);
    end_stats(ctx, stats);
    if (rc != EWBEM_OK) ctx->err = "GMRES did not reach the tolerance within maxit at some frequency";
    return rc;
  });
}

int ewbem_batch_solve_transient(ewbem_ctx** ctxs, int32_t n, double** u_out, ewbem_stats* stats,
                                int32_t per_launch) {
  if (n < 0 || per_launch < 1 || (n > 0 && (!ctxs || !u_out))) return EWBEM_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !u_out[i]) return EWBEM_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return EWBEM_EINVAL;  // one context, one problem
  }
  std::vector<int> rc(n, EWBEM_OK);
  std::vector<ewbem_stats> st(n);
  std::atomic<int> next{0};
  auto worker = [&] {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) break;
      if (ctxs[i]->device >= 0 && hipSetDevice(ctxs[i]->device) != hipSuccess) {
        rc[i] = EWBEM_EHIP;
        continue;
      }
      rc[i] = ewbem_solve_transient(ctxs[i], u_out[i], nullptr, &st[i]);
    }
  };
  const int nth = std::min(n, (int)per_launch);
  std::vector<std::thread> th;
  for (int t = 1; t < nth; ++t) th.emplace_back(worker);
  if (nth > 0) worker();
  for (auto& t : th) t.join();
  if (stats) {
    ewbem_stats a{};
    for (int i = 0; i < n; ++i) {
      const ewbem_stats& b = st[i];
      a.n_solves += b.n_solves;
      a.iters_total += b.iters_total;
      a.iters_max = std::max(a.iters_max, b.iters_max);
      a.matvecs += b.matvecs;
      a.resid_max = std::max(a.resid_max, b.resid_max);
      a.guess_resid_sum += b.guess_resid_sum;
      a.t_assemble_ms += b.t_assemble_ms;
      a.t_guess_ms += b.t_guess_ms;
      a.t_gmres_ms += b.t_gmres_ms;
      a.t_post_ms += b.t_post_ms;
      a.t_matvec_ms += b.t_matvec_ms;
      a.matvec_bytes += b.matvec_bytes;
      a.stored_bytes += b.stored_bytes;
      a.n_near += b.n_near;
      a.n_far += b.n_far;
      a.rank_sum += b.rank_sum;
      a.rank_max = std::max(a.rank_max, b.rank_max);
      a.t_aca_ms += b.t_aca_ms;
      a.t_near_ms += b.t_near_ms;
      a.t_rhs_ms += b.t_rhs_ms;
      a.matvec_bytes_total += b.matvec_bytes_total;
      a.matvecs_timed += b.matvecs_timed;
      a.aca_warm_blocks += b.aca_warm_blocks;
      a.aca_cold_blocks += b.aca_cold_blocks;
      for (int cls = 0; cls < WS_NCLASS; ++cls) a.aca_core_blocks[cls] += b.aca_core_blocks[cls];
      a.aca_warm_pivots += b.aca_warm_pivots;
      a.aca_warm_kept += b.aca_warm_kept;
      a.aca_retries += b.aca_retries;
      a.aca_steps += b.aca_steps;
      a.aca_step_blocks += b.aca_step_blocks;
      a.aca_step_first += b.aca_step_first;
      a.guess_learned += b.guess_learned;
    }
    *stats = a;
  }
  int out = EWBEM_OK;
  for (int i = 0; i < n; ++i)
    if (rc[i] != EWBEM_OK && rc[i] != EWBEM_ENOCONV) return rc[i];
  for (int i = 0; i < n; ++i)
    if (rc[i] == EWBEM_ENOCONV) out = EWBEM_ENOCONV;
  return out;
}

// ---- several problems in lock-step: one concatenated matvec per Arnoldi step

namespace {

// The matvecs of several problems as one: their task tables concatenated,
// the vectors side by side (problem i's x at X + xo[i], its factor
// products at Z + zo[i]), the three launches captured as a graph that every
// Arnoldi step replays.  Each problem's tasks, and so its products, are its
// own launch's.
struct ConcatMatvec {
  DevBuf<VtTask> vt;
  DevBuf<Seg> seg;
  DevBuf<RowTask> rt;
  DevBuf<LeafRange> lr;
  DevBuf<cd> X, Y, Z, P;
  std::vector<long long> xo;
  int nvt = 0, nrt = 0, nlr = 0, cols = 2, c64 = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~ConcatMatvec() { drop(); }
  void drop() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  void build(const std::vector<ewbem_ctx*>& cs, hipStream_t s) {
    drop();
    std::vector<VtTask> v;
    std::vector<Seg> g;
    std::vector<RowTask> r;
    std::vector<LeafRange> l;
    xo.assign(cs.size(), 0);
    long long x = 0, z = 0;
    int far_kind = -1;
    cols = 2;
    for (size_t i = 0; i < cs.size(); ++i) {
      ewbem_ctx* c = cs[i];
      xo[i] = x;
      const long long segoff = (long long)g.size(), taskoff = (long long)r.size();
      if (!c->vt_h.empty()) {
        const int kind = c->store_c64_active ? 1 : 0;
        if (far_kind >= 0 && kind != far_kind)
          fail(EWBEM_EINVAL, "batch lock-step: every problem's far factors need the same store (c128 or c64)");
        far_kind = kind;
        cols = std::max(cols, c->vt_cols);
      }
      for (VtTask t : c->vt_h) {
        t.x0 += (int)x;
        t.zidx += z;
        v.push_back(t);
      }
      for (Seg q : c->seg_h) {
        q.src += (q.flags & SEG_FROM_Z) ? z : x;
        g.push_back(q);
      }
      for (RowTask t : c->rt_h) {
        t.row0 += (int)x;
        t.s0 += (int)segoff;
        t.s1 += (int)segoff;
        r.push_back(t);
      }
      for (LeafRange q : c->lr_h) {
        q.row0 += (int)x;
        q.t0 += (int)taskoff;
        q.t1 += (int)taskoff;
        l.push_back(q);
      }
      x += 3LL * c->nt;
      z += c->z_len;
      if (x > INT32_MAX / 2 || (long long)g.size() > INT32_MAX / 2 || (long long)r.size() > INT32_MAX / 2)
        fail(EWBEM_EINVAL, "batch lock-step: the problems together exceed the matvec's index range");
    }
    c64 = far_kind == 1;
    nvt = (int)v.size();
    nrt = (int)r.size();
    nlr = (int)l.size();
    vt.upload(v, s);
    seg.upload(g, s);
    rt.upload(r, s);
    lr.upload(l, s);
    X.reserve_grow(std::max<long long>(x, 1));
    Y.reserve_grow(std::max<long long>(x, 1));
    Z.reserve_grow(std::max<long long>(z, 1));
    P.reserve_grow((size_t)std::max(nrt, 1) * HMV_MAXROWS);
    EWBEM_HIP_CHECK(hipStreamSynchronize(s));  // the host tables go out of scope
    // the three launches as a graph (no memory set nodes: every output is
    // written by its kernel)
    EWBEM_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    launch_far_vt(vt.p, nvt, cols, c64, X.p, 0, 1, Z.p, 0, s);
    launch_hmv(rt.p, nrt, seg.p, X.p, 0, 1, Z.p, 0, P.p, 0, s);
    launch_hmv_reduce(lr.p, nlr, P.p, 0, 1, Y.p, 0, s);
    EWBEM_HIP_CHECK(hipStreamEndCapture(s, &graph));
    EWBEM_HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  void launch(hipStream_t s) { EWBEM_HIP_CHECK(hipGraphLaunch(exec, s)); }
};

// The host side of one Arnoldi step of a GMRES lane: column j of H from the
// Gram-Schmidt coefficients h (two passes) and |w| = hn, the earlier Givens
// rotations, a new one, and the residual estimate |g_{j+1}| / |b|.
double arnoldi_update(GmresLane& G, const cd* h, int m, double hn) {
  const int j = G.j;
  auto Hc = [&](int row) -> std::complex<double>& { return G.H[(size_t)j * (m + 1) + row]; };
  for (int q = 0; q <= j; ++q) Hc(q) = std::complex<double>(h[q].x + h[m + 2 + q].x, h[q].y + h[m + 2 + q].y);
  Hc(j + 1) = hn;
  for (int q = 0; q < j; ++q) {
    std::complex<double>& a = Hc(q);
    std::complex<double>& b = Hc(q + 1);
    const std::complex<double> t = std::conj(G.cs[q]) * a + std::conj(G.sn[q]) * b;
    b = -G.sn[q] * a + G.cs[q] * b;
    a = t;
  }
  const std::complex<double> a = Hc(j);
  const double den = std::sqrt(std::norm(a) + hn * hn);
  if (den == 0.0) {
    G.cs[j] = 1.0;
    G.sn[j] = 0.0;
  } else {
    G.cs[j] = a / den;
    G.sn[j] = hn / den;
  }
  Hc(j) = den;
  Hc(j + 1) = 0.0;
  G.g[j + 1] = -G.sn[j] * G.g[j];
  G.g[j] = std::conj(G.cs[j]) * G.g[j];
  return std::abs(G.g[j + 1]) / G.bnorm;
}

// y of the least-squares problem H y = g of a finished cycle (j columns).
std::vector<cd> cycle_coeffs(const GmresLane& G, int m) {
  const int j = G.j;
  std::vector<std::complex<double>> y(j);
  for (int i = j - 1; i >= 0; --i) {
    std::complex<double> sacc = G.g[i];
    for (int q = i + 1; q < j; ++q) sacc -= G.H[(size_t)q * (m + 1) + i] * y[q];
    y[i] = sacc / G.H[(size_t)i * (m + 1) + i];
  }
  std::vector<cd> out(j);
  for (int i = 0; i < j; ++i) out[i] = cd{y[i].real(), y[i].imag()};
  return out;
}

// Right-preconditioned GMRES of several problems (each with its own
// operator, restart, tolerance and iteration cap) in lock-step on stream s:
// every problem's context has s as its stream here; the operators are
// applied by one concatenated launch per step.  The arithmetic of each
// problem is that of gmres() on its own.  Returns each problem's iterations
// and final relative residual.
void gmres_lockstep(std::vector<ewbem_ctx*>& cs, hipStream_t s, ConcatMatvec& cm, std::vector<int>& its,
                    std::vector<double>& rel, std::vector<char>& conv) {
  const int nb = (int)cs.size();
  std::vector<GmresLane> L(nb);
  std::vector<int> lane_of(nb);  // position of problem i in the current launch, or -1
  const int hs_max = 4;          // cd entries per |.|^2 readback
  (void)hs_max;
  for (int i = 0; i < nb; ++i) {
    ewbem_ctx* c = cs[i];
    const int m = c->so.restart;
    GmresLane& G = L[i];
    G.b = c->d_b.p;
    G.x = c->d_x.p;
    G.r = c->d_r.p;
    G.V = c->d_V.p;
    G.hd = c->d_small.p;
    G.H.assign((size_t)(m + 1) * m, 0.0);
    G.cs.assign(m, 0.0);
    G.sn.assign(m, 0.0);
    G.g.assign(m + 1, 0.0);
  }
  auto norm_of = [&](ewbem_ctx* c, const cd* v) { return dev_norm(c, v); };
  for (int i = 0; i < nb; ++i) {
    GmresLane& G = L[i];
    G.bnorm = norm_of(cs[i], G.b);
    G.rnorm = norm_of(cs[i], G.r);
    if (G.bnorm == 0.0) {
      launch_axpby(cd{0.0, 0.0}, G.b, cd{0.0, 0.0}, G.x, 3LL * cs[i]->nt, s);
      G.relres = 0.0;
      G.done = true;
      continue;
    }
    G.relres = G.rnorm / G.bnorm;
    if (!(G.relres > cs[i]->so.tol)) G.done = true;
  }
  // the concatenated launch over the problems still iterating
  int built_for = -1;
  auto rebuild = [&] {
    std::vector<ewbem_ctx*> live;
    std::fill(lane_of.begin(), lane_of.end(), -1);
    for (int i = 0; i < nb; ++i)
      if (!L[i].done) {
        lane_of[i] = (int)live.size();
        live.push_back(cs[i]);
      }
    if (live.empty()) return;
    cm.build(live, s);
    built_for = (int)live.size();
  };
  std::vector<cd> hb;
  EventPair ev;
  for (;;) {
    int ndone = 0;
    for (const GmresLane& G : L) ndone += G.done ? 1 : 0;
    if (ndone == nb) break;
    if (built_for != nb - ndone) rebuild();
    // lanes starting a cycle
    for (int i = 0; i < nb; ++i) {
      GmresLane& G = L[i];
      if (G.done || G.arnoldi) continue;
      if (G.its >= cs[i]->so.maxit) {
        G.done = true;
        continue;
      }
      launch_axpby(cd{1.0 / G.rnorm, 0.0}, G.r, cd{0.0, 0.0}, G.V, 3LL * cs[i]->nt, s);
      std::fill(G.g.begin(), G.g.end(), 0.0);
      G.g[0] = G.rnorm;
      G.j = 0;
      G.arnoldi = true;
    }
    std::vector<int> act;
    for (int i = 0; i < nb; ++i)
      if (L[i].arnoldi && !L[i].done) act.push_back(i);
    if (act.empty()) continue;
    if (built_for != nb - ndone) continue;  // a lane hit its cap: the launch shrinks first
    // one Arnoldi step of each: w = A M^{-1} v_j, Gram-Schmidt twice, |w|
    for (int i : act) {
      ewbem_ctx* c = cs[i];
      const long long N = 3LL * c->nt;
      precond_apply(c, L[i].V + (size_t)L[i].j * N, cm.X.p + cm.xo[lane_of[i]]);
    }
    EWBEM_HIP_CHECK(hipEventRecord(ev.a, s));
    cm.launch(s);
    EWBEM_HIP_CHECK(hipEventRecord(ev.b, s));
    size_t hoff = 0;
    std::vector<size_t> at(nb);
    for (int i : act) {
      ewbem_ctx* c = cs[i];
      const int m = c->so.restart;
      const long long N = 3LL * c->nt;
      GmresLane& G = L[i];
      cd* w = cm.Y.p + cm.xo[lane_of[i]];
      cd* hd2 = G.hd + (m + 2);
      cd* nd = G.hd + 2 * (m + 2);
      launch_dots(G.V, N, G.j + 1, w, N, c->d_hpart.p, G.hd, s);
      launch_gemv_sub(G.V, N, G.j + 1, G.hd, w, N, s);
      launch_dots(G.V, N, G.j + 1, w, N, c->d_hpart.p, hd2, s);
      launch_gemv_sub(G.V, N, G.j + 1, hd2, w, N, s);
      launch_dots(w, N, 1, w, N, c->d_hpart.p, nd, s);
      at[i] = hoff;
      hoff += 2 * (m + 2) + 1;
    }
    hb.resize(hoff);
    for (int i : act) {
      const int m = cs[i]->so.restart;
      EWBEM_HIP_CHECK(hipMemcpyAsync(&hb[at[i]], L[i].hd, (2 * (m + 2) + 1) * sizeof(cd), hipMemcpyDeviceToHost, s));
    }
    EWBEM_HIP_CHECK(hipStreamSynchronize(s));
    {
      const float ms = ev.elapsed();
      for (int i : act) {
        cs[i]->acc.t_matvec_ms += ms / act.size();
        cs[i]->acc.matvec_bytes_total += cs[i]->matvec_bytes;
        cs[i]->acc.matvecs_timed += 1;
        cs[i]->acc.matvecs += 1;
      }
    }
    std::vector<int> ends;
    for (int i : act) {
      ewbem_ctx* c = cs[i];
      const int m = c->so.restart;
      const long long N = 3LL * c->nt;
      GmresLane& G = L[i];
      const cd* h = &hb[at[i]];
      ++G.its;
      const double hn = std::sqrt(std::max(0.0, h[2 * (m + 2)].x));
      const double est = arnoldi_update(G, h, m, hn);
      const int j = G.j;
      if (hn > 0.0 && j + 1 <= m)
        launch_axpby(cd{1.0 / hn, 0.0}, cm.Y.p + cm.xo[lane_of[i]], cd{0.0, 0.0}, G.V + (size_t)(j + 1) * N, N, s);
      G.j = j + 1;
      if (est <= c->so.tol || hn == 0.0 || G.j >= m || G.its >= c->so.maxit) ends.push_back(i);
    }
    if (ends.empty()) continue;
    // cycle ends: x += M^{-1} V y, then the true residuals in one launch
    std::vector<std::vector<cd>> yd(ends.size());
    for (size_t e = 0; e < ends.size(); ++e) {
      const int i = ends[e];
      ewbem_ctx* c = cs[i];
      const int m = c->so.restart;
      const long long N = 3LL * c->nt;
      GmresLane& G = L[i];
      yd[e] = cycle_coeffs(G, m);
      cd* u = cm.Y.p + cm.xo[lane_of[i]];
      cd* z = cm.X.p + cm.xo[lane_of[i]];
      EWBEM_HIP_CHECK(hipMemcpyAsync(G.hd, yd[e].data(), G.j * sizeof(cd), hipMemcpyHostToDevice, s));
      launch_gemv_acc(G.V, N, G.j, G.hd, cd{0.0, 0.0}, u, N, s);
      precond_apply(c, u, z);
      launch_axpby(cd{1.0, 0.0}, z, cd{1.0, 0.0}, G.x, N, s);
      EWBEM_HIP_CHECK(hipMemcpyAsync(z, G.x, N * sizeof(cd), hipMemcpyDeviceToDevice, s));
    }
    EWBEM_HIP_CHECK(hipEventRecord(ev.a, s));
    cm.launch(s);
    EWBEM_HIP_CHECK(hipEventRecord(ev.b, s));
    for (int i : ends) {
      ewbem_ctx* c = cs[i];
      const long long N = 3LL * c->nt;
      GmresLane& G = L[i];
      EWBEM_HIP_CHECK(hipMemcpyAsync(G.r, cm.Y.p + cm.xo[lane_of[i]], N * sizeof(cd), hipMemcpyDeviceToDevice, s));
      launch_axpby(cd{1.0, 0.0}, G.b, cd{-1.0, 0.0}, G.r, N, s);
    }
    EWBEM_HIP_CHECK(hipStreamSynchronize(s));  // yd lives on this frame
    {
      const float ms = ev.elapsed();
      for (int i : ends) {
        cs[i]->acc.t_matvec_ms += ms / ends.size();
        cs[i]->acc.matvec_bytes_total += cs[i]->matvec_bytes;
        cs[i]->acc.matvecs_timed += 1;
        cs[i]->acc.matvecs += 1;
      }
    }
    for (int i : ends) {
      GmresLane& G = L[i];
      G.rnorm = norm_of(cs[i], G.r);
      G.relres = G.rnorm / G.bnorm;
      G.arnoldi = false;
      if (!(G.relres > cs[i]->so.tol) || G.j == 0) G.done = true;
    }
  }
  its.assign(nb, 0);
  rel.assign(nb, 0.0);
  conv.assign(nb, 1);
  for (int i = 0; i < nb; ++i) {
    its[i] = L[i].its;
    rel[i] = L[i].relres;
    conv[i] = !(L[i].relres > cs[i]->so.tol);
  }
}

// The stream a context's calls enqueue on, swapped for the duration of a
// lock-step phase.
struct StreamSwap {
  ewbem_ctx* c;
  hipStream_t saved;
  StreamSwap(ewbem_ctx* cc, hipStream_t s) : c(cc), saved(cc->stream) { c->stream = s; }
  ~StreamSwap() { c->stream = saved; }
};

// Transients of one group of problems in lock-step over the frequency
// index: each problem assembles frequency k and forms its guess on its own
// library-owned stream (host threads, concurrently), then the group's GMRES
// run together on stream s with one concatenated matvec per step.
int lockstep_group(std::vector<ewbem_ctx*>& cs, double* const* u, hipStream_t s) {
  const int nb = (int)cs.size();
  int nk_max = 0;
  for (ewbem_ctx* c : cs) {
    ensure_device(c);
    if (c->so.pipeline) fail(EWBEM_EINVAL, "batch lock-step: not with the pipeline");
    nk_max = std::max(nk_max, c->n_f / 2 + 1);
  }
  // per-problem phases on each problem's second stream, in host threads
  auto each = [&](const std::vector<int>& who, const std::function<void(ewbem_ctx*)>& f) {
    std::vector<std::exception_ptr> err(who.size());
    std::vector<std::thread> th;
    for (size_t q = 0; q < who.size(); ++q)
      th.emplace_back([&, q] {
        try {
          ewbem_ctx* c = cs[who[q]];
          EWBEM_HIP_CHECK(hipSetDevice(c->device));
          StreamSwap sw(c, c->astream);
          f(c);
        } catch (...) {
          err[q] = std::current_exception();
        }
      });
    for (auto& t : th) t.join();
    for (auto& e : err)
      if (e) std::rethrow_exception(e);
  };
  std::vector<int> all(nb);
  for (int i = 0; i < nb; ++i) all[i] = i;
  each(all, [&](ewbem_ctx* c) {
    c->hist_n = 0;
    c->hist_slot.clear();
    c->hist_kidx.clear();
    c->lc_slot.clear();
    c->lc_kidx.clear();
    EventPair ev;
    const auto t0 = Clock::now();
    EWBEM_HIP_CHECK(hipEventRecord(ev.a, c->stream));
    rhs_precompute(c, dev_geom(c), 0, c->n_f / 2 + 1);
    EWBEM_HIP_CHECK(hipEventRecord(ev.b, c->stream));
    EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
    c->acc.t_rhs_ms += ev.elapsed();
    c->acc.t_assemble_ms += ms_since(t0);
  });
  int rc = EWBEM_OK;
  ConcatMatvec cm;
  for (int k = 0; k < nk_max; ++k) {
    std::vector<int> live;
    for (int i = 0; i < nb; ++i)
      if (k <= cs[i]->n_f / 2) live.push_back(i);
    each(live, [&](ewbem_ctx* c) {
      if (c->assembled_k != k) assemble_k(c, k);
      guess_k(c, k, nullptr);
      EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
    });
    std::vector<ewbem_ctx*> lc;
    for (int i : live) lc.push_back(cs[i]);
    std::vector<int> its;
    std::vector<double> rel;
    std::vector<char> conv;
    {
      std::vector<std::unique_ptr<StreamSwap>> sw;
      for (ewbem_ctx* c : lc) sw.emplace_back(new StreamSwap(c, s));
      const auto ts = Clock::now();
      gmres_lockstep(lc, s, cm, its, rel, conv);
      const double ms = ms_since(ts);
      for (size_t q = 0; q < lc.size(); ++q) {
        lc[q]->acc.t_gmres_ms += ms / lc.size();
        finish_k(lc[q], k, its[q], rel[q]);
        if (!conv[q]) rc = EWBEM_ENOCONV;
      }
      EWBEM_HIP_CHECK(hipStreamSynchronize(s));
    }
  }
  each(all, [&](ewbem_ctx* c) {
    const auto tp = Clock::now();
    size_t i = 0;
    while (cs[i] != c) ++i;
    launch_mft_inverse(c->d_spec.p, 3LL * c->nt, c->n_f, c->period, c->sigma, c->window, c->d_perm.p, u[i],
                       c->stream);
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(c->stream));
    c->acc.t_post_ms += ms_since(tp);
  });
  return rc;
}

}  // namespace

int ewbem_batch_solve_transient_lockstep(ewbem_ctx** ctxs, int32_t n, double** u_out, ewbem_stats* stats,
                                         int32_t per_launch) {
  if (n < 1 || per_launch < 1 || !ctxs || !u_out) return EWBEM_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !u_out[i]) return EWBEM_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return EWBEM_EINVAL;  // one context, one problem
    if (ctxs[i]->device != ctxs[0]->device) return EWBEM_EINVAL;
  }
  hipStream_t s = nullptr;
  std::vector<ewbem_stats> st(n);
  int rc = guard(ctxs[0], [&] {
    require_gpu(ctxs[0]);
    EWBEM_HIP_CHECK(hipSetDevice(ctxs[0]->device));
    EWBEM_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    for (int i = 0; i < n; ++i) begin_stats(ctxs[i]);
    int out = EWBEM_OK;
    for (int g0 = 0; g0 < n; g0 += per_launch) {
      const int g1 = std::min(n, g0 + per_launch);
      std::vector<ewbem_ctx*> cs(ctxs + g0, ctxs + g1);
      const int r = lockstep_group(cs, u_out + g0, s);
      if (r != EWBEM_OK) out = r;
    }
    for (int i = 0; i < n; ++i) end_stats(ctxs[i], &st[i]);
    return out;
  });
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  if (rc != EWBEM_OK && rc != EWBEM_ENOCONV) return rc;
  if (stats) {
    ewbem_stats a{};
    for (int i = 0; i < n; ++i) {
      const ewbem_stats& b = st[i];
      a.n_solves += b.n_solves;
      a.iters_total += b.iters_total;
      a.iters_max = std::max(a.iters_max, b.iters_max);
      a.matvecs += b.matvecs;
      a.resid_max = std::max(a.resid_max, b.resid_max);
      a.guess_resid_sum += b.guess_resid_sum;
      a.t_assemble_ms += b.t_assemble_ms;
      a.t_guess_ms += b.t_guess_ms;
      a.t_gmres_ms += b.t_gmres_ms;
      a.t_post_ms += b.t_post_ms;
      a.t_matvec_ms += b.t_matvec_ms;
      a.matvec_bytes += b.matvec_bytes;
      a.stored_bytes += b.stored_bytes;
      a.n_near += b.n_near;
      a.n_far += b.n_far;
      a.rank_sum += b.rank_sum;
      a.rank_max = std::max(a.rank_max, b.rank_max);
      a.t_aca_ms += b.t_aca_ms;
      a.t_near_ms += b.t_near_ms;
      a.t_rhs_ms += b.t_rhs_ms;
      a.matvec_bytes_total += b.matvec_bytes_total;
      a.matvecs_timed += b.matvecs_timed;
      a.aca_warm_blocks += b.aca_warm_blocks;
      a.aca_cold_blocks += b.aca_cold_blocks;
      for (int cls = 0; cls < WS_NCLASS; ++cls) a.aca_core_blocks[cls] += b.aca_core_blocks[cls];
      a.aca_warm_pivots += b.aca_warm_pivots;
      a.aca_warm_kept += b.aca_warm_kept;
      a.aca_retries += b.aca_retries;
      a.aca_steps += b.aca_steps;
      a.aca_step_blocks += b.aca_step_blocks;
      a.aca_step_first += b.aca_step_first;
      a.guess_learned += b.guess_learned;
    }
    *stats = a;
  }
  return rc;
}

int ewbem_solve_transient_loads(ewbem_ctx* ctx, int32_t n_loads, const double* loads, int32_t pressure, double* u,
                                ewbem_z* spec, ewbem_stats* stats) {
  return guard(ctx, [&] {
    if (n_loads < 1 || !loads || !u || (pressure != 0 && pressure != 1))
      fail(EWBEM_EINVAL, "solve_transient_loads: need n_loads >= 1, loads, u and pressure 0 or 1");
    if (!ctx->have_mesh || !ctx->have_time || !ctx->have_load)
      fail(EWBEM_ESTATE, "solve_transient_loads: set the mesh, time grid and a load (its history is used) first");
    if (ctx->load_incident || !ctx->bc_caller.empty())
      fail(EWBEM_ESTATE, "solve_transient_loads: needs a traction or pressure load (its history is used)");
    const size_t per = pressure ? (size_t)ctx->nt : 3 * (size_t)ctx->nt;
    if (!finite_all(loads, per * n_loads)) fail(EWBEM_EINVAL, "solve_transient_loads: non-finite load values");
    begin_stats(ctx);
    ensure_device(ctx);
    DevBuf<cd> sp;
    sp.reserve((size_t)n_loads * (ctx->n_f / 2 + 1) * 3 * ctx->nt);
    std::vector<LoadRun> runs = make_load_runs(ctx, n_loads, loads, pressure == 1, sp.p);
    return run_loads(ctx, runs, sp.p, u, spec, stats);
  });
}

int ewbem_solve_transient_incident_loads(ewbem_ctx* ctx, int32_t n_loads, const double* dirs, const double* pols,
                                         double* u, ewbem_z* spec, ewbem_stats* stats) {
  return guard(ctx, [&] {
    if (n_loads < 1 || !dirs || !pols || !u)
      fail(EWBEM_EINVAL, "solve_transient_incident_loads: need n_loads >= 1, directions, polarisations and u");
    if (ctx->inc_total)
      fail(EWBEM_ESTATE, "solve_transient_incident_loads: the scattered-field formulation only "
                         "(set the wave with ewbem_set_load_incident_s)");
    if (!ctx->have_mesh || !ctx->have_time || !ctx->have_load || !ctx->load_incident)
      fail(EWBEM_ESTATE, "solve_transient_incident_loads: set the mesh, time grid and an incident wave (its "
                         "wavelet is used) first");
    if (!finite_all(dirs, 3 * (size_t)n_loads) || !finite_all(pols, 3 * (size_t)n_loads))
      fail(EWBEM_EINVAL, "solve_transient_incident_loads: non-finite direction or polarisation");
    std::vector<double> dd(3 * (size_t)n_loads), pp(3 * (size_t)n_loads);
    for (int l = 0; l < n_loads; ++l) {
      const double* d = dirs + 3 * l;
      const double* q = pols + 3 * l;
      const double nd = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double np = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      if (!(nd > 0) || !(np > 0)) fail(EWBEM_EINVAL, "incident wave: zero direction or polarisation");
      double dp = 0;
      for (int k = 0; k < 3; ++k) {
        dd[3 * l + k] = d[k] / nd;
        pp[3 * l + k] = q[k] / np;
        dp += dd[3 * l + k] * pp[3 * l + k];
      }
      if (std::fabs(dp) > 1e-9) fail(EWBEM_EINVAL, "incident S-wave: polarisation must be normal to the direction");
    }
    begin_stats(ctx);
    ensure_device(ctx);
    DevBuf<cd> sp;
    sp.reserve((size_t)n_loads * (ctx->n_f / 2 + 1) * 3 * ctx->nt);
    std::vector<LoadRun> runs = make_incident_runs(ctx, n_loads, dd.data(), pp.data(), sp.p);
    return run_loads(ctx, runs, sp.p, u, spec, stats);
  });
}

void ewbem_default_train_opts(ewbem_train_opts* o) {
  if (!o) return;
  *o = ewbem_train_opts{};
  o->n_modes = 64;
  o->hidden = 256;
  o->n_hidden = 3;
  o->epochs = 2000;
  o->lr = 1e-3;
  o->power_iters = 2;
  o->load_kind = 0;
  o->seed = 1;
  o->augment = 4;
  o->unit_snapshots = 1;
  o->lsq_map = 1;
  o->lsq_reg = 1e-8;
}

int ewbem_guess_train(ewbem_ctx* ctx, int32_t n_cases, const double* loads, const ewbem_train_opts* o,
                      ewbem_stats* stats) {
  return guard(ctx, [&] {
    if (!o || !loads || n_cases < 1) fail(EWBEM_EINVAL, "guess_train: need options, loads and n_cases >= 1");
    if (o->n_modes < 1 || o->n_modes > 1024 || o->hidden < 1 || o->hidden > 4096 || o->n_hidden < 0 ||
        o->n_hidden > 8 || o->epochs < 0 || o->epochs > 1000000 || !(o->lr > 0) || !std::isfinite(o->lr) ||
        o->power_iters < 0 || o->power_iters > 10 || (o->load_kind != 0 && o->load_kind != 1) ||
        o->augment < 0 || o->augment > 64 || (o->unit_snapshots != 0 && o->unit_snapshots != 1) ||
        (o->lsq_map != 0 && o->lsq_map != 1) || !(o->lsq_reg > 0 && o->lsq_reg < 1))
      fail(EWBEM_EINVAL, "guess_train: options out of range");
    if (!ctx->have_mesh || !ctx->have_time || !ctx->have_load)
      fail(EWBEM_ESTATE, "guess_train: set the mesh, time grid and a load (its history is used) first");
    if (ctx->load_incident || !ctx->bc_caller.empty())
      fail(EWBEM_ESTATE, "guess_train: needs a traction or pressure load (its history is used)");
    const int nk = ctx->n_f / 2 + 1;
    if (nk < 4) fail(EWBEM_EINVAL, "guess_train: needs N_f >= 6 (three previous frequencies per sample)");
    const long long N = 3LL * ctx->nt;
    const long long Mll = (long long)n_cases * nk;
    if (Mll > 65535) fail(EWBEM_EINVAL, "guess_train: n_cases (N_f/2 + 1) must not exceed 65535 snapshots");
    const int M = (int)Mll;
    const int r = o->n_modes;
    if (r > M || r > N) fail(EWBEM_EINVAL, "guess_train: n_modes exceeds the number of snapshots or unknowns");
    const size_t per = o->load_kind == 1 ? (size_t)ctx->nt : 3 * (size_t)ctx->nt;
    if (!finite_all(loads, per * n_cases)) fail(EWBEM_EINVAL, "guess_train: non-finite load values");
    begin_stats(ctx);
    // data: every case's solutions at all frequencies, with the configured
    // solver (extrapolation instead of the model being replaced)
    const int saved_guess = ctx->so.guess;
    ctx->lm = LearnedModel{};
    ctx->lm_dev = false;
    if (ctx->so.guess == EWBEM_GUESS_LEARNED) ctx->so.guess = EWBEM_GUESS_SEM;
    DevBuf<cd> S;
    int rc = EWBEM_OK;
    try {
      ensure_device(ctx);
      S.reserve((size_t)N * M);
      // every frequency assembled once for all cases (snapshot m = case nk + k)
      std::vector<LoadRun> runs = make_load_runs(ctx, n_cases, loads, o->load_kind == 1, S.p);
      rc = multi_load_loop(ctx, runs);
    } catch (...) {
      ctx->so.guess = saved_guess;
      throw;
    }
    ctx->so.guess = saved_guess;
    hipStream_t st = ctx->stream;
    // reduced basis and every snapshot's coordinates
    DevBuf<cd> phi, coef, part;
    phi.reserve((size_t)N * r);
    // unit-norm snapshots weight every frequency alike; the raw ones are
    // dominated by the low frequencies, whose solutions are orders of
    // magnitude larger
    DevBuf<double> snorm;
    if (o->unit_snapshots) {
      snorm.reserve(M);
      launch_col_norms(S.p, N, M, N, snorm.p, st);
      launch_col_scale(S.p, N, M, N, snorm.p, 1, st);
    }
    const int l = std::min(M, r + 16);
    const double energy = pod_basis(ctx, S.p, N, M, r, l, o->power_iters, o->seed, phi.p);
    coef.reserve((size_t)M * r);
    part.reserve((size_t)dots_chunks(N) * r);
    for (int m = 0; m < M; ++m) launch_dots(phi.p, N, r, S.p + (size_t)m * N, N, part.p, coef.p + (size_t)m * r, st);
    if (o->unit_snapshots) launch_col_scale(coef.p, r, M, r, snorm.p, 0, st);  // the raw snapshots' coordinates
    S.release();
    // the least-squares map of each frequency over the training loads
    // (small dense algebra on the host: an n_cases x n_cases Gram matrix per
    // frequency), and its predictions of the training loads, the base the
    // network learns to correct (the map's own residual, lam W)
    std::vector<zc> rxh, rwh;
    int rn = 0;
    DevBuf<cd> base;
    if (o->lsq_map && n_cases >= 2) {
      const std::vector<zc> C = to_host(ctx, coef.p, (size_t)M * r);
      std::vector<cd> bh((size_t)M * r, cd{0.0, 0.0});
      std::vector<zc> X((size_t)3 * r * n_cases), Y((size_t)r * n_cases), W;
      std::vector<double> ad;
      double lam = 0.0;
      for (int k = 3; k < nk; ++k) {
        for (int i = 0; i < n_cases; ++i)
          for (int j = 0; j < r; ++j) {
            const size_t b = (size_t)i * nk;
            X[(size_t)i * 3 * r + j] = C[(b + k - 1) * r + j];
            X[(size_t)i * 3 * r + r + j] = C[(b + k - 2) * r + j];
            X[(size_t)i * 3 * r + 2 * r + j] = C[(b + k - 3) * r + j];
            Y[(size_t)i * r + j] = C[(b + k) * r + j];
          }
        if (!ridge_dual(X, Y, 3 * r, r, n_cases, o->lsq_reg, W, ad, lam))
          fail(EWBEM_EINVAL, "guess training: the training loads' histories are degenerate at some frequency");
        rxh.insert(rxh.end(), X.begin(), X.end());
        rwh.insert(rwh.end(), W.begin(), W.end());
        for (int i = 0; i < n_cases; ++i)
          for (int j = 0; j < r; ++j) {
            const zc v = Y[(size_t)i * r + j] - lam * W[(size_t)i * r + j];
            bh[((size_t)i * nk + k) * r + j] = cd{v.real(), v.imag()};
          }
      }
      rn = n_cases;
      base.upload(bh, st);
    }
    // the solutions depend linearly on the load, so any combination of the
    // cases' coordinate sequences is the sequence of the combined load:
    // augment virtual cases with complex Gaussian weights
    const int n_virt = o->augment * n_cases;
    const int n_all = n_cases + n_virt;
    if (n_virt > 0) {
      DevBuf<cd> tab, tabb, wv;
      tab.reserve((size_t)n_all * nk * r);
      EWBEM_HIP_CHECK(hipMemcpyAsync(tab.p, coef.p, (size_t)M * r * sizeof(cd), hipMemcpyDeviceToDevice, st));
      if (rn > 0) {
        tabb.reserve((size_t)n_all * nk * r);
        EWBEM_HIP_CHECK(hipMemcpyAsync(tabb.p, base.p, (size_t)M * r * sizeof(cd), hipMemcpyDeviceToDevice, st));
      }
      std::mt19937_64 rng(o->seed * 0x2545f4914f6cdd1dULL + 7);
      std::normal_distribution<double> nd(0.0, std::sqrt(0.5 / n_cases));
      std::vector<zc> w((size_t)n_virt * n_cases);
      for (auto& v : w) v = zc(nd(rng), nd(rng));
      wv.reserve(w.size());
      to_device(ctx, w, wv.p);
      const long long blk = (long long)nk * r;  // one case's coordinate sequence
      for (int v = 0; v < n_virt; ++v) {
        launch_gemv_acc(tab.p, blk, n_cases, wv.p + (size_t)v * n_cases, cd{0.0, 0.0},
                        tab.p + (size_t)(n_cases + v) * blk, blk, st);
        // the virtual case's base: the same combination of the leave-one-out
        // predictions
        if (rn > 0)
          launch_gemv_acc(tabb.p, blk, n_cases, wv.p + (size_t)v * n_cases, cd{0.0, 0.0},
                          tabb.p + (size_t)(n_cases + v) * blk, blk, st);
      }
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      std::swap(coef.p, tab.p);
      std::swap(coef.n, tab.n);
      if (rn > 0) {
        std::swap(base.p, tabb.p);
        std::swap(base.n, tabb.n);
      }
    }
    // samples: k = 3 .. N_f/2 of every case
    std::vector<int> idx;
    std::vector<float> kf;
    for (int cs = 0; cs < n_all; ++cs)
      for (int k = 3; k < nk; ++k) {
        const int b = cs * nk;
        idx.insert(idx.end(), {b + k - 1, b + k - 2, b + k - 3, b + k});
        kf.push_back((float)k / (float)(nk - 1));
      }
    const int ns = (int)kf.size();
    MlpShape shape;
    shape.dims.push_back(6 * r + 2);
    for (int h = 0; h < o->n_hidden; ++h) shape.dims.push_back(o->hidden);
    shape.dims.push_back(2 * r);
    DevBuf<int> d_idx;
    DevBuf<float> d_kf, X, T, P;
    d_idx.upload(idx, st);
    d_kf.upload(kf, st);
    X.reserve((size_t)ns * shape.dims[0]);
    T.reserve((size_t)ns * 2 * r);
    launch_learn_samples(coef.p, rn > 0 ? base.p : nullptr, r, d_idx.p, d_kf.p, ns, X.p, T.p, nullptr, st);
    // initial weights N(0, 1 / fan-in); the last layer starts at zero, so the
    // untrained network returns the quadratic extrapolation
    std::vector<float> p0(shape.n_params(), 0.f);
    {
      std::mt19937_64 rng(o->seed);
      for (int ly = 0; ly + 1 < shape.n_layers(); ++ly) {
        std::normal_distribution<double> nd(0.0, 1.0 / std::sqrt((double)shape.dims[ly]));
        const size_t w0 = shape.woff(ly), nw = (size_t)shape.dims[ly + 1] * shape.dims[ly];
        for (size_t i = 0; i < nw; ++i) p0[w0 + i] = (float)nd(rng);
      }
    }
    P.upload(p0, st);
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    LearnedModel m;
    train_mlp(ctx, shape, P.p, ns, X.p, T.p, o->epochs, o->lr, true, m.loss0, m.loss1);
    m.params.resize(p0.size());
    EWBEM_HIP_CHECK(hipMemcpyAsync(m.params.data(), P.p, p0.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    const std::vector<zc> pt = to_host(ctx, phi.p, (size_t)N * r);  // tree order
    m.phi.assign((size_t)N * r, 0.0);
    for (int j = 0; j < r; ++j)
      for (int t = 0; t < ctx->nt; ++t) {
        const size_t e = (size_t)ctx->hg.perm[t];
        for (int i = 0; i < 3; ++i) m.phi[(size_t)j * N + 3 * e + i] = pt[(size_t)j * N + 3 * (size_t)t + i];
      }
    m.ok = true;
    m.r = r;
    m.shape = shape;
    m.energy = energy;
    m.rn = rn;
    m.rk = rn > 0 ? nk : 0;
    m.rx = std::move(rxh);
    m.rw = std::move(rwh);
    ctx->lm = std::move(m);
    ctx->lm_dev = false;
    end_stats(ctx, stats);
    if (stats) {
      stats->pod_energy = ctx->lm.energy;
      stats->train_loss_first = ctx->lm.loss0;
      stats->train_loss_last = ctx->lm.loss1;
    }
    if (rc != EWBEM_OK) ctx->err = "GMRES did not reach the tolerance at some training frequency";
    return rc;
  });
}

int ewbem_guess_save(const ewbem_ctx* cctx, void* buf, size_t* len) {
  ewbem_ctx* ctx = const_cast<ewbem_ctx*>(cctx);  // only the error message changes
  return guard(ctx, [&] {
    if (!len) fail(EWBEM_EINVAL, "guess_save: null length");
    if (!ctx->lm.ok) fail(EWBEM_ESTATE, "guess_save: no trained or loaded model");
    const LearnedModel& m = ctx->lm;
    const long long N = (long long)m.phi.size() / m.r;
    const size_t need = model_bytes(m, N);
    if (!buf) {
      *len = need;
      return EWBEM_OK;
    }
    if (*len < need) {
      *len = need;
      fail(EWBEM_EINVAL, "guess_save: buffer too small");
    }
    char* p = (char*)buf;
    auto put = [&](const void* v, size_t n) {
      std::memcpy(p, v, n);
      p += n;
    };
    put(kModelMagic, 8);
    const int32_t hdr[4] = {kModelVersion, (int32_t)N, m.r, m.shape.n_layers()};
    put(hdr, sizeof(hdr));
    for (int d : m.shape.dims) {
      const int32_t v = d;
      put(&v, 4);
    }
    const double f[3] = {m.energy, m.loss0, m.loss1};
    put(f, sizeof(f));
    put(m.params.data(), 4 * m.params.size());
    put(m.phi.data(), 16 * m.phi.size());
    const int32_t rh[2] = {m.rn, m.rk};
    put(rh, sizeof(rh));
    put(m.rx.data(), 16 * m.rx.size());
    put(m.rw.data(), 16 * m.rw.size());
    *len = need;
    return EWBEM_OK;
  });
}

int ewbem_guess_load(ewbem_ctx* ctx, const void* buf, size_t len) {
  return guard(ctx, [&] {
    if (!buf) fail(EWBEM_EINVAL, "guess_load: null buffer");
    if (!ctx->have_mesh) fail(EWBEM_ESTATE, "guess_load: set the mesh first");
    const char* p = (const char*)buf;
    const char* end = p + len;
    auto get = [&](void* v, size_t n) {
      if ((size_t)(end - p) < n) fail(EWBEM_EINVAL, "guess_load: truncated model");
      std::memcpy(v, p, n);
      p += n;
    };
    char magic[8];
    get(magic, 8);
    if (std::memcmp(magic, kModelMagic, 8) != 0) fail(EWBEM_EINVAL, "guess_load: not a model");
    int32_t hdr[4];
    get(hdr, sizeof(hdr));
    if (hdr[0] != 1 && hdr[0] != kModelVersion) fail(EWBEM_EINVAL, "guess_load: unknown model version");
    const long long N = 3LL * ctx->nt;
    if (hdr[1] != N) fail(EWBEM_EINVAL, "guess_load: the model belongs to a mesh with another number of unknowns");
    const int r = hdr[2];
    if (r < 1 || r > 1024 || r > N) fail(EWBEM_EINVAL, "guess_load: bad basis size");
    std::vector<int32_t> dims(hdr[3] + 1 > 0 && hdr[3] <= 16 ? hdr[3] + 1 : 0);
    if (dims.empty()) fail(EWBEM_EINVAL, "guess_load: bad layer count");
    get(dims.data(), 4 * dims.size());
    LearnedModel m;
    m.shape = mlp_shape(hdr[3], dims.data());
    if (m.shape.dims[0] != 6 * r + 2 || m.shape.dims.back() != 2 * r)
      fail(EWBEM_EINVAL, "guess_load: network widths do not match the basis");
    double f[3];
    get(f, sizeof(f));
    m.params.resize(m.shape.n_params());
    get(m.params.data(), 4 * m.params.size());
    m.phi.resize((size_t)N * r);
    get(m.phi.data(), 16 * m.phi.size());
    if (hdr[0] >= 2) {
      int32_t rh[2];
      get(rh, sizeof(rh));
      if (rh[0] < 0 || rh[0] > 65535 || (rh[0] > 0 && (rh[1] < 4 || rh[1] > 65535)) || (rh[0] == 0 && rh[1] != 0))
        fail(EWBEM_EINVAL, "guess_load: bad least-squares map header");
      m.rn = rh[0];
      m.rk = rh[1];
      if (m.rn > 0) {
        const size_t nkk = (size_t)(m.rk - 3);
        const size_t want = 16 * nkk * (size_t)m.rn * 4 * (size_t)r;
        if ((size_t)(end - p) < want) fail(EWBEM_EINVAL, "guess_load: truncated model");
        m.rx.resize(nkk * 3 * (size_t)r * m.rn);
        m.rw.resize(nkk * (size_t)r * m.rn);
        get(m.rx.data(), 16 * m.rx.size());
        get(m.rw.data(), 16 * m.rw.size());
        if (!finite_all((const double*)m.rx.data(), 2 * m.rx.size()) ||
            !finite_all((const double*)m.rw.data(), 2 * m.rw.size()))
          fail(EWBEM_EINVAL, "guess_load: non-finite least-squares map");
      }
    }
    if (p != end) fail(EWBEM_EINVAL, "guess_load: trailing bytes");
    for (float v : m.params)
      if (!std::isfinite(v)) fail(EWBEM_EINVAL, "guess_load: non-finite parameters");
    if (!finite_all((const double*)m.phi.data(), 2 * m.phi.size())) fail(EWBEM_EINVAL, "guess_load: non-finite basis");
    m.ok = true;
    m.r = r;
    m.energy = f[0];
    m.loss0 = f[1];
    m.loss1 = f[2];
    ctx->lm = std::move(m);
    ctx->lm_dev = false;
    return EWBEM_OK;
  });
}

int ewbem_guess_basis(ewbem_ctx* ctx, int32_t* n_modes, ewbem_z* phi) {
  return guard(ctx, [&] {
    if (!ctx->lm.ok) fail(EWBEM_ESTATE, "guess_basis: no trained or loaded model");
    if (n_modes) *n_modes = ctx->lm.r;
    if (phi) {
      require_gpu(ctx);
      std::vector<cd> h(ctx->lm.phi.size());
      for (size_t i = 0; i < h.size(); ++i) h[i] = cd{ctx->lm.phi[i].real(), ctx->lm.phi[i].imag()};
      EWBEM_HIP_CHECK(hipMemcpyAsync(phi, h.data(), h.size() * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
      EWBEM_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    }
    return EWBEM_OK;
  });
}

int ewbem_mlp_eval(ewbem_ctx* ctx, int32_t n_layers, const int32_t* dims, const float* params, int64_t batch,
                   const float* x, const float* target, float* y, float* grad, double* loss) {
  return guard(ctx, [&] {
    require_gpu(ctx);
    const MlpShape s = mlp_shape(n_layers, dims);
    if (batch < 0 || batch > (1LL << 24)) fail(EWBEM_EINVAL, "mlp_eval: batch out of range");
    if (!params || (batch > 0 && (!x || !y))) fail(EWBEM_EINVAL, "mlp_eval: null array");
    if (batch > 0 && grad && !target) fail(EWBEM_EINVAL, "mlp_eval: the gradient needs a target");
    if (loss) *loss = 0.0;
    hipStream_t st = ctx->stream;
    const size_t np = s.n_params();
    if (batch == 0) {
      if (grad) EWBEM_HIP_CHECK(hipMemsetAsync(grad, 0, np * sizeof(float), st));
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      return EWBEM_OK;
    }
    const int dL = s.dims[n_layers];
    const long long nout = batch * dL;
    DevBuf<float> act, pre, dY, work;
    DevBuf<double> part;
    act.reserve(std::max<size_t>(1, s.hidden_sum() * batch));
    pre.reserve(std::max<size_t>(1, s.hidden_sum() * batch));
    mlp_forward(s, params, batch, x, act.p, pre.p, y, st);
    if (target) {
      const int nb = loss_blocks(nout);
      part.reserve(nb);
      dY.reserve(nout);
      launch_mlp_loss(y, target, nout, (float)(2.0 / (double)nout), dY.p, part.p, st);
      const double l = loss_sum(ctx, part.p, nb) / (double)nout;
      if (loss) *loss = l;
      if (grad) {
        work.reserve(2 * (size_t)s.max_width() * batch);
        mlp_backward(s, params, batch, x, act.p, pre.p, dY.p, work.p, grad, st);
      }
    }
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    return EWBEM_OK;
  });
}

int ewbem_mlp_eval_noalloc(ewbem_ctx* ctx, int32_t n_layers, const int32_t* dims, const float* params,
                           int64_t batch, const float* x, const float* target, float* y, float* grad,
                           double* loss) {
  return guard(ctx, [&] {
    require_gpu(ctx);
    const MlpShape s = mlp_shape(n_layers, dims);
    if (batch < 0 || batch > (1LL << 24)) fail(EWBEM_EINVAL, "mlp_eval_noalloc: batch out of range");
    if (!params || (batch > 0 && (!x || !y))) fail(EWBEM_EINVAL, "mlp_eval_noalloc: null array");
    if (batch > 0 && grad && !target) fail(EWBEM_EINVAL, "mlp_eval_noalloc: the gradient needs a target");
    // the same buffers as ewbem_mlp_eval, carved from the scratch array
    const int dL = s.dims[n_layers];
    const long long nout = batch * dL;
    const int nb = loss_blocks(nout);
    const size_t b_act = round256(sizeof(float) * std::max<size_t>(1, s.hidden_sum() * batch));
    const size_t b_dy = round256(sizeof(float) * std::max<long long>(1, nout));
    const size_t b_work = round256(sizeof(float) * 2 * (size_t)s.max_width() * batch);
    const size_t b_part = round256(sizeof(double) * nb);
    const size_t need = 2 * b_act + (target ? b_dy + b_part : 0) + (target && grad ? b_work : 0);
    if (need > kScratchBytes)
      fail(EWBEM_EINVAL, "mlp_eval_noalloc: batch x widths need " + std::to_string(need) +
                             " bytes of scratch, more than its " + std::to_string(kScratchBytes));
    void* base = scratch_addr(ctx->device);
    if (!base) fail(EWBEM_EHIP, "mlp_eval_noalloc: no scratch address on this device");
    if (loss) *loss = 0.0;
    hipStream_t st = ctx->stream;
    const size_t np = s.n_params();
    if (batch == 0) {
      if (grad)
        hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)std::min<size_t>((np + 255) / 256, 1024)), dim3(256), 0, st,
                           grad, (long long)np);
      EWBEM_HIP_CHECK(hipGetLastError());
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      return EWBEM_OK;
    }
    unsigned char* p = (unsigned char*)base;
    float* act = (float*)p;
    float* pre = (float*)(p + b_act);
    float* dY = (float*)(p + 2 * b_act);
    double* part = (double*)(p + 2 * b_act + b_dy);
    float* work = (float*)(p + 2 * b_act + b_dy + b_part);
    mlp_forward(s, params, batch, x, act, pre, y, st);
    if (target) {
      launch_mlp_loss(y, target, nout, (float)(2.0 / (double)nout), dY, part, st);
      double h[256];
      EWBEM_HIP_CHECK(hipMemcpyAsync(h, part, nb * sizeof(double), hipMemcpyDeviceToHost, st));
      EWBEM_HIP_CHECK(hipStreamSynchronize(st));
      double sum = 0.0;
      for (int i = 0; i < nb; ++i) sum += h[i];
      if (loss) *loss = sum / (double)nout;
      if (grad) mlp_backward(s, params, batch, x, act, pre, dY, work, grad, st);
    }
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    return EWBEM_OK;
  });
}

int ewbem_mlp_train(ewbem_ctx* ctx, int32_t n_layers, const int32_t* dims, float* params, int64_t batch,
                    const float* x, const float* target, int32_t epochs, double lr, double* loss_first,
                    double* loss_last) {
  return guard(ctx, [&] {
    require_gpu(ctx);
    const MlpShape s = mlp_shape(n_layers, dims);
    if (batch < 1 || batch > (1LL << 24) || epochs < 0 || epochs > 1000000 || !(lr > 0) || !std::isfinite(lr))
      fail(EWBEM_EINVAL, "mlp_train: need batch >= 1, epochs >= 0, lr > 0");
    if (!params || !x || !target) fail(EWBEM_EINVAL, "mlp_train: null array");
    double l0 = 0.0, l1 = 0.0;
    train_mlp(ctx, s, params, batch, x, target, epochs, lr, false, l0, l1);
    EWBEM_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    if (loss_first) *loss_first = l0;
    if (loss_last) *loss_last = l1;
    return EWBEM_OK;
  });
}

int ewbem_mft_inverse(ewbem_ctx* ctx, const ewbem_z* spec, double* u) {
  return guard(ctx, [&] {
    if (!spec || !u) fail(EWBEM_EINVAL, "mft_inverse: null array");
    ensure_device(ctx);
    const long long N = 3LL * ctx->nt;
    hipStream_t st = ctx->stream;
    // caller order -> tree order rows, then the inverse (which writes caller order)
    for (int k = 0; k <= ctx->n_f / 2; ++k)
      launch_permute((const cd*)spec + (size_t)k * N, ctx->d_perm.p, ctx->nt, 1, ctx->d_spec.p + (size_t)k * N,
                     st);
    launch_mft_inverse(ctx->d_spec.p, N, ctx->n_f, ctx->period, ctx->sigma, ctx->window, ctx->d_perm.p, u, st);
    EWBEM_HIP_CHECK(hipGetLastError());
    EWBEM_HIP_CHECK(hipStreamSynchronize(st));
    return EWBEM_OK;
  });
}

}  // extern "C"
