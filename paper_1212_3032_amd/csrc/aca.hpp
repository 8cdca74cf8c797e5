// Far-field (low-rank) blocks and the ACA / H-matrix matvec launchers.
#pragma once

#include "common.hpp"

namespace ewbem {

// Largest rank a far block may reach (per class of workgroup size), and the
// largest number of row elements of one far block.
constexpr int ACA_KMAX = 384;
constexpr int ACA_KMAX_SMALL = 96;
constexpr int ACA_MAXM = 16384;
// Blocks with at most this many row and column elements use 64-thread
// workgroups.
constexpr int ACA_SMALL = 64;

// Low-rank block A ~ U V^T between row elements [r0, r0+m) and column
// elements [c0, c0+n) (tree order).  U: 3m x kcap column-major (ld 3m),
// V: 3n x kcap column-major (ld 3n), complex128 workspace.
struct FarBlk {
  int r0, m, c0, n;
  cd* U;
  cd* V;
  int kcap;
  int pad;
};

void launch_aca(const FarBlk* blks, const int* order_small, int n_small, const int* order_big,
                int n_big, const DevGeom& g, const KParams& P, double tol, int* rank, int* status,
                hipStream_t st);
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
