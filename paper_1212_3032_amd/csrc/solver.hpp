// Krylov-solver vector kernels and the block-diagonal preconditioners.
#pragma once

#include "common.hpp"

namespace ewbem {

constexpr int HMV_MAXROWS_S = 192;  // largest leaf block (64 elements x 3)

int dots_chunks(long long n);
// out[c] = sum_r conj(V[r + c ld]) w[r], c < ncols (partial: ncols*dots_chunks(n))
void launch_dots(const cd* V, long long ld, int ncols, const cd* w, long long n, cd* partial,
                 cd* out, hipStream_t st);
// nrm[c] = |V(:, c)|_2; V(:, c) *= f[c] (inv: /= f[c], zero f leaves it)
void launch_col_norms(const cd* V, long long ld, int ncols, long long n, double* nrm, hipStream_t st);
void launch_col_scale(cd* V, long long ld, int ncols, long long n, const double* f, int inv, hipStream_t st);
void launch_gemv_sub(const cd* V, long long ld, int ncols, const cd* h, cd* w, long long n,
                     hipStream_t st);
void launch_gemv_acc(const cd* V, long long ld, int ncols, const cd* h, cd beta, cd* out, long long n,
                     hipStream_t st);
void launch_axpby(cd a, const cd* x, cd b, cd* y, long long n, hipStream_t st);
void launch_permute(const cd* in, const int* perm, int ne, int to_tree, cd* out, hipStream_t st);
void launch_inv3(const cd* A, int ne, cd* Ainv, hipStream_t st);
void launch_apply3(const cd* M, int ne, const cd* v, cd* z, hipStream_t st);
void launch_block_inv(const long long* offs, const int* dims, int nblk, cd* W, int* piv_fail,
                      hipStream_t st);
void launch_block_apply(const long long* offs, const int* dims, const int* row0s, int nblk,
                        const cd* W, const cd* v, cd* z, hipStream_t st);
void launch_copy_blocks(const long long* src_offs, const int* src_ld, const long long* dst_offs,
                        const int* dims, int nblk, const cd* D, cd* W, hipStream_t st);

}  // namespace ewbem
