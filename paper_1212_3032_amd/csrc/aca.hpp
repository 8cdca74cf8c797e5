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

// Initialise the state and used-row bits of blocks ids[0..n).
void launch_aca_init(const int* ids, int n, const FarBlk* blks, AcaState* st, unsigned* used,
                     hipStream_t s);
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
};
// One lock-step iteration of every active block; blocks still active are
// appended to act_out, counted by *count (zeroed by the caller).
void launch_aca_step(const AcaLists& L, const AcaWork& W, const DevGeom& g, const KParams& P, double tol,
                     int* act_out, int* count, hipStream_t s);
// rank[b] = k, status[b] = 1 for blocks that ran out of capacity, else 0.
void launch_aca_finish(const int* ids, int n, const AcaState* st, int* rank, int* status, hipStream_t s);
void launch_to_c64(const FarBlk* blks, int nblk, const int* rank, const long long* uo,
                   const long long* vo, cf* out, hipStream_t st);

// ---- H-matrix matvec
// Phase 1 task: z[zidx + j] = sum_c V[c, j] x[x0 + c] for j < ncol, with V
// the column-major factor starting at column l0 (pointer already offset).
struct VtTask {
  const void* V;   // cd* or cf* (store type), first of ncol columns
  long long zidx;
  int C;           // column length 3n
  int x0;          // 3 * c0
  int ncol;        // <= 4
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

void launch_far_vt(const VtTask* tasks, int ntask, int store_c64, const cd* x, cd* z,
                   hipStream_t st);
void launch_hmv(const RowTask* tasks, int ntask, const Seg* segs, const cd* x, const cd* z,
                cd* partial, hipStream_t st);
void launch_hmv_reduce(const LeafRange* leaves, int nleaf, const cd* partial, cd* y,
                       hipStream_t st);

}  // namespace ewbem
