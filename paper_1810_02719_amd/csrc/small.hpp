// Per-block small dense FP64 kernels of the orthonormalisation and the
// Rayleigh-Ritz step (one workgroup per block).
#pragma once

#include "dense.hpp"

namespace mis {

// Per-block state of the small kernels.
struct SmallDesc {
  int64_t m_off;    // ld x ld matrices (G, H, Rinv, A, Z, S)
  int64_t pk_off;   // packed upper-triangle scratch (q(q+1)/2)
  int64_t log_off;  // rotation log of one sweep ((q-1) * q/2 * 2)
  int64_t t_off;    // Ritz values / permutation (p entries)
  int32_t p, ld, q; // q = p rounded up to even
  int32_t blk;      // index into per-block arrays (status, a, b, flags)
};

constexpr int SMALL_THREADS = 1024;

// Cholesky of the column-scaled Gram G = R^T R and the inverse factor Rinv
// (upper, FP64, zeros elsewhere); optionally Rinv rounded to FP32 (S32) for
// the row product.  Sets MI_BLOCK_SHIFTED / _NOT_PD / _NONFINITE in status.
// ld <= 320 runs the FP64-MFMA kernel of chol.hip, wider blocks a 32-panel
// kernel with the working matrix Wk in global memory (ld x ld per block).
void launch_chol_blk(const SmallDesc* sd, int nb, const double* G, double* Wk, double* Rinv,
                     float* S32, int32_t* status, int max_ld, int lds_max, hipStream_t s);

// Blocked FP64-MFMA variant for ld <= 320 (chol.hip; above 192 part of its
// tiles live in Wk); false when max_ld is wider.  Same outputs and flags.
bool launch_chol_mfma(const SmallDesc* sd, int nb, const double* G, double* Wk, double* Rinv,
                      float* S32, int32_t* status, int max_ld, hipStream_t s);

// a[blk] <- max_j (Rinv^T H Rinv)_jj from T1 = H Rinv (largest Rayleigh
// quotient of the Cholesky-QR basis).
void launch_rq_max(const SmallDesc* sd, int nb, const double* Rinv, const double* T1,
                   double* a_lo, hipStream_t s);

// Packs the upper triangle of A (ld x ld) into the Jacobi scratch and sets Z
// to the identity; resets the per-block "converged" flag.
void launch_jacobi_init(const SmallDesc* sd, int nb, const double* A, double* pk, double* Z,
                        int32_t* conv, hipStream_t s);

// One cyclic sweep (q-1 rounds of q/2 disjoint rotations) of two-sided
// Jacobi on the packed matrix; rotations go to the log.
void launch_jacobi_sweep(const SmallDesc* sd, int nb, double* pk, double* log, int32_t* conv,
                         double tol, bool lds, size_t lds_bytes, hipStream_t s);

// Z <- Z * (rotations of the last sweep), rows in parallel.
void launch_apply_rot(const SmallDesc* sd, int nb, int max_q, const double* log,
                      const int32_t* conv, double* Z, int lds_max, hipStream_t s);

// Ritz values (diagonal) sorted ascending -> ritz[t_off..], permutation ->
// perm[t_off..]; a[blk] <- largest Ritz value when adapt; NOCONV flag when an
// off-diagonal entry still exceeds conv_tol * ||A||_F.
void launch_rr_finish(const SmallDesc* sd, int nb, const double* pk, const int32_t* conv,
                      double* ritz, int32_t* perm, double* a_lo, int adapt, int32_t* status,
                      double conv_tol, hipStream_t s);

// S32[i][j] = S64[i][perm[j]] for j < p, zero for padding columns.
void launch_perm_cast(const SmallDesc* sd, int nb, const double* S64, const int32_t* perm,
                      float* S32, double* S64out, hipStream_t s);


}  // namespace mis
