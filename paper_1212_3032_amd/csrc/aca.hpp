// Far-field (low-rank) blocks and the ACA / H-matrix matvec launchers.
#pragma once

#include "common.hpp"

namespace ewbem {

// Largest rank a far block may reach, and the largest number of row
// elements of one far block.
constexpr int ACA_KMAX = 1024;
constexpr int ACA_MAXM = 16384;

// Low-rank block A ~ U V^T between row elements [r0, r0+m) and column
// elements [c0, c0+n) (tree order).  U: 3m x kcap column-major (ld 3m),
// V: 3n x kcap column-major (ld 3n), complex128 workspace.  bitoff: first
// 32-bit word of the block's used-row bit set (ceil(m / 32) words).
struct FarBlk {
  int r0, m, c0, n;
  cd* U;
  cd* V;
  int kcap;
  int bitoff;
  int poff;  // pivot-element lists: rows at plist[poff..poff+m), columns at plist[poff+m..poff+2m)
  int pad;
};

// Per-block state of the lock-step cross approximation.
constexpr int ACA_ACTIVE = 0, ACA_DONE = 1, ACA_OVERFLOW = 2;
struct AcaState {
  int k;          // accepted rank so far
  int astar;      // current row element
  int bstar;      // pivot column element of the current step
  int status;     // ACA_ACTIVE / ACA_DONE / ACA_OVERFLOW
  int fails;      // consecutive rows found already represented
  int nacc;       // terms accepted in the current step
  int skip;       // the current step adds no terms
  int pad;
  double normS2;  // estimate of |S|_F^2 of the approximation so far
  double first_max;               // largest entry of the first residual row
  unsigned long long best;        // packed (score, column element): pivot search
  unsigned long long best_row;    // packed (score, row element): next-row search
};
// Weights of the current step's terms on the 3 cross columns / rows.
struct AcaPlan {
  cd alpha[3][3];
  cd beta[3][3];
};
// Row elements per wavefront in the column residual kernel (63 rows, so an
// element's three rows never straddle two wavefronts).
constexpr int ACA_ROWS_PER_WAVE = 21;

// Initialise the state, used-row bits and pivot lists of blocks ids[0..n).
void launch_aca_init(const int* ids, int n, const FarBlk* blks, AcaState* st, unsigned* used, int* nlist,
                     hipStream_t s);
// Active list act_out (count in *count, zeroed by the caller) of the blocks
// ids[0..n) whose state is ACA_ACTIVE.
void launch_aca_compact(const int* ids, int n, const AcaState* st, int* act_out, int* count, hipStream_t s);
// Exclusive scans over the *nact_dev active blocks in act, into offs (four
// arrays of nact + 1 entries, stride apart): element counts n and m,
// 64-column wavefront tasks ceil(3n / 64) and row wavefront tasks
// ceil(m / ACA_ROWS_PER_WAVE).  totals = {the four sums, nact}.
void launch_aca_scan(const int* act, const int* nact_dev, const FarBlk* blks, int* offs, int stride,
                     int* totals, hipStream_t s);
struct AcaLists {
  const int* act;
  int nact;
  int tot_n, tot_m, tot_wn, tot_wm;
  const int *offs_n, *offs_m, *offs_wn, *offs_wm;
};
// Device work areas of the lock-step approximation: part_v holds 3 doubles
// per 64-column task (tot_wn), part_u 3 per 21-row-element task (tot_wm).
struct AcaWork {
  const FarBlk* blks;
  AcaState* st;
  AcaPlan* plan;
  unsigned* used;
  double* part_u;
  double* part_v;
  int* plist;  // pivot row / column elements of each block's accepted steps
  int* nlist;  // per block: number of listed rows, columns (-1 rows: lists unusable)
};
// One lock-step iteration of every active block; blocks still active are
// appended to act_out, counted by *count (zeroed by the caller).
void launch_aca_step(const AcaLists& L, const AcaWork& W, const DevGeom& g, const KParams& P, double tol,
                     int* act_out, int* count, hipStream_t s);
// rank[b] = k, status[b] = 1 for blocks that ran out of capacity, else 0.
void launch_aca_finish(const int* ids, int n, const AcaState* st, int* rank, int* status, hipStream_t s);
void launch_to_c64(const FarBlk* blks, int nblk, const int* rank, const long long* uo,
                   const long long* vo, cf* out, hipStream_t st);
// The blocks ids[0..n): factors to complex64 at up[i], vp[i] (device arrays
// of device pointers).
void launch_to_c64_ptr(const FarBlk* blks, const int* ids, int n, const int* rank, cf* const* up, cf* const* vp,
                       hipStream_t st);

// ---- Warm start from the previous frequency's pivots.
// A block whose previous approximation accepted pivots in row elements
// rows[0..nr) and column elements cols[0..nc) starts from the cross
// approximation A(:, J) A(I, J)^+ A(I, :) on the rows I and columns J of
// those elements, evaluated at the new frequency, and continues with the
// ordinary steps until the stopping test holds.
constexpr int WS_MAXLIST = 256;  // longest pivot list used for a warm start
struct WsBlk {
  int blk;          // far block
  int nr, nc;       // listed row / column elements
  int rcap;         // 3 min(nr, nc): largest rank of the cross
  long long rr;     // Rr: 3n x 3nr column-major (column = cross row), offset in cross
  long long cc;     // Cc: 3m x 3nc column-major (column = cross column)
  long long w;      // W = A(I, J): 3nr x 3nc column-major, factored in place
  int pq;           // pivot order: p[rcap] (cross rows), q[rcap] (cross columns)
  int tu, tv;       // first U-forming and V-forming task (48-row tiles)
  int pad;
  long long pu, pv; // norm partials: (tasks of the block) x rcap doubles each
  long long co;     // substitution panels: U side, then V side, ws_panel_elems(rcap) each
};
struct WsArgs {
  const WsBlk* wb;
  int nwarm;
  const int* er_off;  // nwarm + 1: flattened (row element of the list, column element) offsets
  const int* ec_off;  // nwarm + 1: flattened (column element of the list, row element) offsets
  const int* tu_off;  // nwarm + 1: U-forming task offsets
  const int* tv_off;  // nwarm + 1: V-forming task offsets
  int tot_er, tot_ec, tot_tu, tot_tv;
  cd* cross;
  int* pq;
  int* rho;
  double* part;        // per-task squared norms of the terms (pu, pv of each block)
  cd* coef;            // substitution panels (co of each block)
  const int* lu_list;  // warm blocks by size class of W (n_lu[0..WS_NCLASS) entries)
  int n_lu[7];
  double stop2;        // the elimination stops at |pivot|^2 <= stop2 |first pivot|^2
  int keep_all;        // 1: keep every eliminated term, 0: up to the first meeting the stopping test
  unsigned long long* cnt;  // [0] += pivots eliminated, [1] += terms kept (zeroed by the caller)
};
constexpr int WS_LDS_TINY = 1024;   // entries of W held in LDS by the LDS classes (tiny: <= 64 rows)
constexpr int WS_LDS_SMALL = 2304;
constexpr int WS_LDS_MID = 4480;
constexpr int WS_LDS_LARGE = 8960;
// Substitutions on the matrix cores: 48-row tiles (16 row elements) per
// wavefront, chunks of 16 terms; panel k holds (16 + 16 k) x 16 complex.
constexpr int WS_TILE_ROWS = 48;
__host__ __device__ inline long long ws_panel_elems(int rcap) {
  const long long nk = (rcap + 15) / 16;
  return 256 * (nk * (nk + 1) / 2);
}
constexpr int WS_LU_NR_LDS = 2;     // LDS classes hold cores of at most 128 rows
// Size classes of the core elimination: 0..2 W in LDS (at most 2,304, 4,480,
// 8,960 entries), 3 in global memory, 4 tiny (at most 64 rows, 1,024 entries,
// two wavefronts), 5 in registers (at most 64 x 64), 6 in registers (at most
// 128 x 128).
constexpr int WS_NCLASS = 7;
constexpr int WS_REG_SMALL = 64, WS_REG_LARGE = 128;
// A second stream for the core eliminations outside registers (cores over
// 128 x 128 and the LDS classes: few, long workgroups), so that they overlap
// the register classes; null runs everything on the caller's stream.
struct WsSide {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;  // timing disabled
};
void launch_ws(const WsArgs& A, const AcaWork& W, const DevGeom& g, const KParams& P, double tol, hipStream_t s,
               const WsSide& side);

// ---- H-matrix matvec
// Phase 1 task: z[zidx + j] = sum_c V[c, j] x[x0 + c] for j < ncol, with V
// the column-major factor starting at column l0 (pointer already offset).
struct VtTask {
  const void* V;   // cd* or cf* (store type), first of ncol columns
  long long zidx;
  int C;           // column length 3n
  int x0;          // 3 * c0
  int ncol;        // <= the columns per wavefront of the launch (2, 4 or 8)
  int pad;
};

// Phase 2 segment: ncols columns of a column-major panel (ld rows) whose
// first row is the first row of the task's leaf; multiplies src[0..ncols).
struct Seg {
  const void* A;      // cd* (near, or far in c128) or cf* (far in c64)
  long long src;      // offset into x (near) or z (far)
  int ld;
  int ncols;
  int flags;          // bit 0: A is complex64; bit 1: source is z
  int pad;
};
constexpr int SEG_C64 = 1, SEG_FROM_Z = 2;

// One workgroup: rows [row0, row0+rows) (one leaf), segments [s0, s1).
struct RowTask {
  int row0, rows, s0, s1;
};

// Per leaf: tasks [t0, t1) whose partial results sum to the leaf's rows.
struct LeafRange {
  int row0, rows, t0, t1;
};

constexpr int HMV_MAXROWS = 192;

// nrhs = 1..4 right-hand sides: columns of x (stride ldx), z (ldz), the
// partial sums (ldp) and y (ldy).
// mfma (with nrhs = 8): tasks of up to HMV_MFMA_COLS columns on the matrix cores (k_far_vt_mfma8)
void launch_far_vt(const VtTask* tasks, int ntask, int cols_per_wave, int store_c64, const cd* x, long long ldx,
                   int nrhs, cd* z, long long ldz, hipStream_t st, int mfma = 0);
// mfma: eight right-hand sides on the matrix cores (k_hmv_mfma8)
void launch_hmv(const RowTask* tasks, int ntask, const Seg* segs, const cd* x, long long ldx, int nrhs,
                const cd* z, long long ldz, cd* partial, long long ldp, hipStream_t st, int mfma = 0);
void launch_hmv_reduce(const LeafRange* leaves, int nleaf, const cd* partial, long long ldp, int nrhs, cd* y,
                       long long ldy, hipStream_t st);
constexpr int HMV_MAXRHS = 8;  // right-hand sides of one multi-right-hand-side matvec
constexpr int HMV_MFMA_COLS = 16;  // factor columns per phase-1 task on the matrix cores

}  // namespace ewbem
