// Eigenspace tracking by orthogonal iteration (Section 4, Algorithm 1):
// host runtime that plans the waves, lays out the workspace, and enqueues
// (or captures into a HIP graph and replays) the kernel sequence.
//
// One iteration of a block, with Y the current basis (n_b x p_b, row-major):
//   filter pass (x passes):  Y <- T_m(t(L)) Y / T_m(t(0))       m SpMM steps
//     (between passes) Cholesky-QR: G = Y^T Y, Y <- Y R^-1       keeps Y well conditioned
//   Rayleigh-Ritz:           W = L Y;  G = Y^T Y, H = Y^T W        one dual Gram pass
//                            R^T R = G,  A = R^-T H R^-1,  A = Z Theta Z^T (Jacobi)
//                            V <- Y R^-1 Z   (columns ordered by Ritz value)
// and a final Cholesky-QR pass after the last iteration.  t(x) maps the
// damped interval [a, b] to [-1, 1]; b bounds the spectrum (Gershgorin), a
// tracks the largest Ritz value (the top of the tracked window).
#include <cstring>
#include <map>
#include <memory>

#include "eig.hpp"
#include "oi_plan.hpp"

namespace mis {

// ------------------------------------------------------------------ per-block scalar kernels

// b_hi[blk] = max_i sum_j |L_ij| (Gershgorin bound on lambda_max), one
// workgroup per block, deterministic.
__global__ void __launch_bounds__(256)
    k_gershgorin(const MatDesc* __restrict__ sets, const CsrDesc* __restrict__ csr,
                 const int32_t* __restrict__ row_ptr, const float* __restrict__ val,
                 double* __restrict__ b_hi) {
  __shared__ double red[4];
  const MatDesc d = sets[blockIdx.x];
  const CsrDesc c = csr[blockIdx.x];
  double mx = 0.0;
  for (int r = threadIdx.x; r < d.rows; r += 256) {
    double s = 0.0;
    for (int k = row_ptr[c.rp_off + r]; k < row_ptr[c.rp_off + r + 1]; ++k)
      s += fabs((double)val[c.nnz_off + k]);
    mx = fmax(mx, s);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) b_hi[d.blk] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void k_set_b(const MatDesc* __restrict__ sets, int nsets, double v, double* b_hi) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsets) b_hi[sets[i].blk] = v;
}

// Initial lower filter bound a of each block of a wave.
__global__ void k_init_a(const MatDesc* __restrict__ sets, int nsets,
                         const BlkInfo* __restrict__ info, int from_pred, int a_mode,
                         double a_value, const double* __restrict__ ritz_in,
                         double* __restrict__ a_lo, const double* __restrict__ b_hi) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsets) return;
  const int b = sets[i].blk;
  const BlkInfo bi = info[b];
  double a;
  if (from_pred && bi.pred >= 0) {
    const BlkInfo pi = info[bi.pred];
    a = a_lo[bi.pred] * (double)pi.n / (double)bi.n;
  } else if (a_mode == MI_A_ABS) {
    a = a_value;
  } else if (a_mode == MI_A_RITZ) {
    a = ritz_in[bi.t_off + bi.p - 1];
  } else {
    a = a_value * b_hi[b] * (double)bi.p / (double)bi.n;
  }
  a_lo[b] = a;
}

// Chebyshev coefficients of the scaled three-term recurrence (filter on
// [a, b], normalised at the bottom of the spectrum lambda = 0):
//   Y_1 = (s_1/e)(L - c0) Y_0,  Y_{k+1} = (2 s_{k+1}/e)(L - c0) Y_k - s_k s_{k+1} Y_{k-1}
//   e = (b-a)/2, c0 = (b+a)/2, s_1 = e/(0 - c0), s_{k+1} = 1/(2/s_1 - s_k).
// Stored as (alpha, beta, gamma) with Y_new = alpha L Y + beta Y + gamma Y_prev;
// slot m holds (1, 0, 0) for the plain product W = L Y.
__global__ void k_cheb_coef(const MatDesc* __restrict__ sets, int nsets,
                            const double* __restrict__ a_lo, const double* __restrict__ b_hi,
                            double* __restrict__ coef, int stride, int m) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsets) return;
  const int b = sets[i].blk;
  const double bb = b_hi[b];
  double a = a_lo[b];
  a = fmin(fmax(a, 1e-3 * bb), 0.95 * bb);
  const double e = 0.5 * (bb - a), c0 = 0.5 * (bb + a);
  const double s1 = e / (0.0 - c0);
  double* cf = coef + int64_t(b) * stride;
  double s = s1;
  cf[0] = s1 / e;
  cf[1] = -c0 * s1 / e;
  cf[2] = 0.0;
  for (int k = 1; k < m; ++k) {
    const double sn = 1.0 / (2.0 / s1 - s);
    const double al = 2.0 * sn / e;
    cf[3 * k] = al;
    cf[3 * k + 1] = -c0 * al;
    cf[3 * k + 2] = -s * sn;
    s = sn;
  }
  cf[3 * m] = 1.0;
  cf[3 * m + 1] = 0.0;
  cf[3 * m + 2] = 0.0;
}

// Warm start: block b's start is its predecessor's final basis, rows and
// columns index-aligned; rows past the predecessor's size are zero, columns
// past its width get the unit vector e_{(997 j) mod n_b}.
// The predecessor's basis is read from src (the caller's output), the start
// is written to dst (the same buffer outside the tolerance mode).
// (src and dst may differ in element type: FP32 output, BF16 working slab.)
template <typename TS, typename TD>
__global__ void __launch_bounds__(256)
    k_warm_copy(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                const MatDesc* __restrict__ psets, const TS* src, TD* dst) {
  typedef typename Acc<TD>::type A;
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set], pd = psets[t.set];
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  for (int e = threadIdx.x; e < rows * d.ld; e += 256) {
    const int r = t.row0 + e / d.ld, j = e % d.ld;
    A v = (A)0;
    if (j < d.cols) {
      if (j < pd.cols) {
        if (r < pd.rows) v = (A)Acc<TS>::load(src[pd.off + int64_t(r) * pd.ld + j]);
      } else if (r == int((997LL * j) % d.rows)) {
        v = (A)1;
      }
    }
    dst[d.off + int64_t(r) * d.ld + j] = Acc<TD>::store(v);
  }
}

// Seeded start of a block without predecessor (MI_RANDOM): entry (i, j) is
// 2u - 1, u uniform in [0, 1) from the SplitMix64 output function (Steele,
// Lea and Flood 2014) applied to the counter seed + golden (1 + key), key =
// b 2^40 + i 2^12 + j: independent of the slab layout and of the launch.
__device__ inline double splitmix_unit(uint64_t seed, uint64_t key) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (key + 1ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return double(z >> 11) * 0x1.0p-53;
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_random_start(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                   uint64_t seed, T* __restrict__ out) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  for (int e = threadIdx.x; e < rows * d.ld; e += 256) {
    const int r = t.row0 + e / d.ld, j = e % d.ld;
    const uint64_t key = (uint64_t(d.blk) << 40) + (uint64_t(r) << 12) + uint64_t(j);
    typedef typename Acc<T>::type A;
    out[d.off + int64_t(r) * d.ld + j] =
        Acc<T>::store(j < d.cols ? (A)(2.0 * splitmix_unit(seed, key) - 1.0) : (A)0);
  }
}

// ------------------------------------------------------------------ tolerance mode
// Residual norms r_j = ||L v_j - theta_j v_j||_2 of a wave's Ritz pairs.
// Stage 1, one workgroup per 16-row tile: each wavefront takes whole rows,
// gathers the neighbour rows, forms (L V)_row - theta V_row and accumulates
// its squares per column in FP64; the four wavefronts' sums are added in a
// fixed order into the tile's partial (global tile numbering).  Stage 2 adds
// a block's tile partials in tile order.
template <typename T>
__global__ void __launch_bounds__(256)
    k_resid_tile(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                 const CsrDesc* __restrict__ csr, const BlkInfo* __restrict__ info,
                 const int64_t* __restrict__ tile_base, int ldp,
                 const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                 const float* __restrict__ val, const T* __restrict__ V,
                 const double* __restrict__ ritz, double* __restrict__ part) {
  constexpr int MAXC = 1024 / 64;  // columns per lane for ld <= 1024
  __shared__ double wsum[4][1024];
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const CsrDesc c = csr[t.set];
  const double* th = ritz + info[d.blk].t_off;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  const T* Vb = V + d.off;
  const int32_t* cb = col + c.nnz_off;
  const float* vb = val + c.nnz_off;
  double acc[MAXC];
#pragma unroll
  for (int s = 0; s < MAXC; ++s) acc[s] = 0.0;
  for (int rr = wave; rr < rows; rr += 4) {
    const int r = t.row0 + rr;
    const int k0 = row_ptr[c.rp_off + r], k1 = row_ptr[c.rp_off + r + 1];
#pragma unroll
    for (int s = 0; s < MAXC; ++s) {
      const int j = lane + 64 * s;
      if (j >= d.ld) continue;
      double lv = 0.0;
      for (int k = k0; k < k1; ++k) lv = fma((double)vb[k], (double)Vb[int64_t(cb[k]) * d.ld + j], lv);
      const double th_j = j < d.cols ? th[j] : 0.0;
      const double res = fma(-th_j, (double)Vb[int64_t(r) * d.ld + j], lv);
      acc[s] = fma(res, res, acc[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < MAXC; ++s) {
    const int j = lane + 64 * s;
    if (j < d.ld) wsum[wave][j] = acc[s];
  }
  __syncthreads();
  double* out = part + (tile_base[d.blk] + t.row0 / SPMM_ROWS) * ldp;
  for (int j = threadIdx.x; j < d.ld; j += 256)
    out[j] = ((wsum[0][j] + wsum[1][j]) + wsum[2][j]) + wsum[3][j];
}

// Stage 2 and the test, one workgroup per block of the wave: resid[j] =
// sqrt(sum of the tile partials) for j < p; then thread 0 decides whether
// the block is converged (max_{j < c} r_j <= tol |theta_{p-1}|), or ends at
// the iteration cap, and if so freezes it now (fnow = 1): the iteration
// count, Ritz values and residuals go to the outputs.
__global__ void __launch_bounds__(256)
    k_tol_check(const MatDesc* __restrict__ sets, const BlkInfo* __restrict__ info,
                const int64_t* __restrict__ tile_base, int ldp, const double* __restrict__ part,
                double* __restrict__ resid_w, const double* __restrict__ ritz_w, double tol,
                int iter, int last, int32_t* __restrict__ frozen, int32_t* __restrict__ fnow,
                double* __restrict__ ritz_out, double* __restrict__ resid_out,
                int32_t* __restrict__ iters, int32_t* __restrict__ status) {
  __shared__ double red[4];
  const MatDesc d = sets[blockIdx.x];
  const BlkInfo bi = info[d.blk];
  const int nt = (d.rows + SPMM_ROWS - 1) / SPMM_ROWS;
  const int64_t base = tile_base[d.blk];
  double mx = 0.0;
  for (int j = threadIdx.x; j < bi.p; j += 256) {
    double s = 0.0;
    for (int k = 0; k < nt; ++k) s += part[(base + k) * ldp + j];
    const double r = sqrt(s);
    resid_w[bi.t_off + j] = r;
    if (j < bi.c) mx = fmax(mx, r);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const bool was = frozen[d.blk] != 0;
  const bool conv = mx <= tol * fabs(ritz_w[bi.t_off + bi.p - 1]);
  const bool now = !was && (conv || last);
  if (now) {
    for (int j = threadIdx.x; j < bi.p; j += 256) {
      ritz_out[bi.t_off + j] = ritz_w[bi.t_off + j];
      if (resid_out) resid_out[bi.t_off + j] = resid_w[bi.t_off + j];
    }
  }
  if (threadIdx.x == 0) {
    fnow[d.blk] = now ? 1 : 0;
    if (now) {
      frozen[d.blk] = 1;
      if (iters) iters[d.blk] = iter + 1;
      if (!conv) atomicOr(&status[d.blk], MI_BLOCK_UNCONVERGED);
    }
  }
}

// Rows of the blocks frozen in this iteration: working basis -> output.
template <typename T>
__global__ void __launch_bounds__(256)
    k_freeze_rows(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                  const int32_t* __restrict__ fnow, const T* __restrict__ src,
                  T* __restrict__ dst) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  if (!fnow[d.blk]) return;
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  for (int e = threadIdx.x; e < rows * d.ld; e += 256) {
    const int64_t o = d.off + int64_t(t.row0) * d.ld + e;
    dst[o] = src[o];
  }
}

// Fixed iteration counts: the residual norms of the final pairs (stage 2
// only) and the iteration count of every block of the wave.
__global__ void __launch_bounds__(256)
    k_resid_final(const MatDesc* __restrict__ sets, const BlkInfo* __restrict__ info,
                  const int64_t* __restrict__ tile_base, int ldp, const double* __restrict__ part,
                  double* __restrict__ resid, int T, int32_t* __restrict__ iters) {
  const MatDesc d = sets[blockIdx.x];
  const BlkInfo bi = info[d.blk];
  const int nt = (d.rows + SPMM_ROWS - 1) / SPMM_ROWS;
  const int64_t base = tile_base[d.blk];
  if (resid)
    for (int j = threadIdx.x; j < bi.p; j += 256) {
      double s = 0.0;
      for (int k = 0; k < nt; ++k) s += part[(base + k) * ldp + j];
      resid[bi.t_off + j] = sqrt(s);
    }
  if (iters && threadIdx.x == 0) iters[d.blk] = T;
}

// (with a conversion when the element types differ: FP32 <-> BF16)
template <typename TS, typename TD = TS>
__global__ void __launch_bounds__(256)
    k_copy_slab(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                const TS* __restrict__ src, TD* __restrict__ dst) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  for (int e = threadIdx.x; e < rows * d.ld; e += 256) {
    const int64_t o = d.off + int64_t(t.row0) * d.ld + e;
    dst[o] = Acc<TD>::store((typename Acc<TD>::type)Acc<TS>::load(src[o]));
  }
}

// Checkpoint copies of one wave's blocks (the recording for the adjoint):
// ld x ld matrices at m_off, and the filter coefficients of the blocks.
template <typename E>
__global__ void __launch_bounds__(256)
    k_copy_mats(const SmallDesc* __restrict__ sds, const E* __restrict__ src, E* __restrict__ dst) {
  const SmallDesc d = sds[blockIdx.x];
  const int64_t n = int64_t(d.ld) * d.ld;
  for (int64_t e = threadIdx.x; e < n; e += 256) dst[d.m_off + e] = src[d.m_off + e];
}

__global__ void k_copy_coef(const MatDesc* __restrict__ sets, int nsets, int stride,
                            const double* __restrict__ src, double* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsets * stride) return;
  const int64_t o = int64_t(sets[i / stride].blk) * stride + i % stride;
  dst[o] = src[o];
}

// ------------------------------------------------------------------ R^z (Section 4)
// The paper's operator R^z = (L + delta I)^-z, applied as z solves with
// (L + delta I), each by a fixed number of conjugate-gradient iterations on
// every column of the block at once (the columns are independent systems):
//   x = 0, r = p = b;  q = (L + delta I) p;  alpha = r.r / p.q;
//   x += alpha p;  r -= alpha q;  beta = r.r(new) / r.r(old);  p = r + beta p.
// q comes from the SpMM with the coefficients (1, delta, 0).  The other
// steps run over the SpMM's 16-row tiles (one wavefront per tile and 64
// columns); every column reduction is written as per-tile FP64 partials and
// summed by the consumer in tile order, so results are reproducible and
// the stream lanes never share a partial (slots are numbered per block).
constexpr int CG_COLS = 64;

// Coefficient rows of R^z: slot 0 = (1, delta, 0) for q = (L + delta I) p,
// slot m = (1, 0, 0) for the Rayleigh-Ritz product W = L Y.
__global__ void k_rz_coef(const MatDesc* __restrict__ sets, int nsets, double delta,
                          double* __restrict__ coef, int stride, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsets) return;
  double* cf = coef + int64_t(sets[i].blk) * stride;
  cf[0] = 1.0;
  cf[1] = delta;
  cf[2] = 0.0;
  cf[3 * m] = 1.0;
  cf[3 * m + 1] = 0.0;
  cf[3 * m + 2] = 0.0;
}

// Column j's sum over the block's tile partials (tile order).
__device__ inline double cg_sum(const double* __restrict__ part, int64_t base, int ntiles, int ldp,
                                int j) {
  double s = 0.0;
  for (int k = 0; k < ntiles; ++k) s += part[(base + k) * ldp + j];
  return s;
}

// Start of a solve: r = p = b, x = 0, partials of r.r.  b may be x itself
// (the previous solve's result): every element is read before it is cleared.
template <typename T>
__global__ void __launch_bounds__(64)
    k_cg_start(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
               const int64_t* __restrict__ tile_base, int ldp, const T* b, T* x,
               T* __restrict__ r, T* __restrict__ p, double* __restrict__ partR) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const int j = blockIdx.y * CG_COLS + threadIdx.x;
  if (j >= d.ld) return;
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  double s = 0.0;
  for (int i = 0; i < rows; ++i) {
    const int64_t o = d.off + int64_t(t.row0 + i) * d.ld + j;
    const T v = b[o];
    r[o] = v;
    p[o] = v;
    x[o] = (T)0;
    s += (double)v * (double)v;
  }
  partR[(tile_base[d.blk] + t.row0 / SPMM_ROWS) * ldp + j] = s;
}

// p.q partials of every tile (after q = (L + delta I) p).
template <typename T>
__global__ void __launch_bounds__(64)
    k_cg_pq(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
            const int64_t* __restrict__ tile_base, int ldp, const T* __restrict__ p,
            const T* __restrict__ q, double* __restrict__ partP) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const int j = blockIdx.y * CG_COLS + threadIdx.x;
  if (j >= d.ld) return;
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  double s = 0.0;
  for (int i = 0; i < rows; ++i) {
    const int64_t o = d.off + int64_t(t.row0 + i) * d.ld + j;
    s += (double)p[o] * (double)q[o];
  }
  partP[(tile_base[d.blk] + t.row0 / SPMM_ROWS) * ldp + j] = s;
}

// x += alpha p, r -= alpha q with alpha = r.r / p.q, and the partials of the
// new r.r (into the other buffer).
template <typename T>
__global__ void __launch_bounds__(64)
    k_cg_xr(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
            const int64_t* __restrict__ tile_base, int ldp, T* __restrict__ x, T* __restrict__ r,
            const T* __restrict__ p, const T* __restrict__ q, const double* __restrict__ partP,
            const double* __restrict__ partR, double* __restrict__ partR2) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const int j = blockIdx.y * CG_COLS + threadIdx.x;
  if (j >= d.ld) return;
  const int nt = (d.rows + SPMM_ROWS - 1) / SPMM_ROWS;
  const int64_t base = tile_base[d.blk];
  const double pq = cg_sum(partP, base, nt, ldp, j);
  const double rr = cg_sum(partR, base, nt, ldp, j);
  const double alpha = (j < d.cols && pq > 0.0) ? rr / pq : 0.0;
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  double s = 0.0;
  for (int i = 0; i < rows; ++i) {
    const int64_t o = d.off + int64_t(t.row0 + i) * d.ld + j;
    x[o] = (T)((double)x[o] + alpha * (double)p[o]);
    const double rn = (double)r[o] - alpha * (double)q[o];
    r[o] = (T)rn;
    s += rn * rn;
  }
  partR2[(base + t.row0 / SPMM_ROWS) * ldp + j] = s;
}

// p = r + beta p with beta = r.r(new) / r.r(old).
template <typename T>
__global__ void __launch_bounds__(64)
    k_cg_p(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
           const int64_t* __restrict__ tile_base, int ldp, const T* __restrict__ r,
           T* __restrict__ p, const double* __restrict__ partR, const double* __restrict__ partR2) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const int j = blockIdx.y * CG_COLS + threadIdx.x;
  if (j >= d.ld) return;
  const int nt = (d.rows + SPMM_ROWS - 1) / SPMM_ROWS;
  const int64_t base = tile_base[d.blk];
  const double r0 = cg_sum(partR, base, nt, ldp, j);
  const double r1 = cg_sum(partR2, base, nt, ldp, j);
  const double beta = (j < d.cols && r0 > 0.0) ? r1 / r0 : 0.0;
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  for (int i = 0; i < rows; ++i) {
    const int64_t o = d.off + int64_t(t.row0 + i) * d.ld + j;
    p[o] = (T)((double)r[o] + beta * (double)p[o]);
  }
}

// ------------------------------------------------------------------ dynamic OI (Alg. 2)
// The walk keeps c_b active columns at the front of the slab and zeros in
// the others.  The tracking kernels then act on the active columns alone:
// the filter maps zero columns to zero, and the Cholesky-QR of a basis with
// trailing zero columns yields the Cholesky-QR of its leading c_b columns
// (a Cholesky factor's leading block is the factor of the leading block;
// the zero columns come out as zero).  Each step computes the Eq. 6
// residual e = sum over x, y, z of (v - U U^T v) = s - U (U^T s), s_i =
// x_i + y_i + z_i, in FP64, and appends e/||e|| (Eq. 7), drops the last
// column, or stops; a stopped block's basis is frozen in a copy.
constexpr int DOI_THREADS = 256;
constexpr int DOI_CHUNK = 1024;   // rows of s staged in LDS at a time
constexpr int DOI_MAX_LD = 1024;  // slab stride the step kernel supports

// Start of the walk in the blocks of a wave: c_b is the predecessor's final
// size (warm waves) or the caller's start size, clamped to [1, min(c_max,
// p_b)]; columns >= c_b of the start basis are cleared; the trajectory is
// reset to -1 and the block marked running.
template <typename T>
__global__ void __launch_bounds__(DOI_THREADS)
    k_doi_init(const MatDesc* __restrict__ sets, const BlkInfo* __restrict__ info, int from_pred,
               int c_max, int t_max, int32_t* __restrict__ c, int32_t* __restrict__ done,
               double* __restrict__ traj, T* __restrict__ U) {
  const MatDesc d = sets[blockIdx.x];
  const int b = d.blk, pb = info[b].pred;
  int cb = (from_pred && pb >= 0) ? c[pb] : c[b];
  cb = max(1, min(cb, min(c_max, d.cols)));
  for (int64_t e = threadIdx.x; e < int64_t(d.rows) * d.ld; e += DOI_THREADS)
    if (int(e % d.ld) >= cb) U[d.off + e] = (T)0;
  for (int i = threadIdx.x; i < 2 * t_max; i += DOI_THREADS) traj[2 * int64_t(b) * t_max + i] = -1.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    c[b] = cb;
    done[b] = 0;
  }
}

// s_i = x_i + y_i + z_i of row i of a block (FP64)
__device__ inline double doi_s(const float* xb, int i) {
  return (double)xb[3 * i] + (double)xb[3 * i + 1] + (double)xb[3 * i + 2];
}

// e_i = s_i - sum_{j < cb} U_ij w_j for row i, one wavefront (lanes over j)
template <typename T>
__device__ inline double doi_e(const T* Ub, int ld, int cb, const double* w, const float* xb, int i,
                               int lane) {
  double acc = 0.0;
  for (int j = lane; j < cb; j += 64) acc += (double)Ub[int64_t(i) * ld + j] * w[j];
  return doi_s(xb, i) - wave_sum(acc);
}

// One decision of the walk per running block of a wave (one workgroup per
// block): the Eq. 6 residual of the current basis, recorded with c; then
// grow (||e|| > eps_h and c < min(c_max, p_b)), shrink (||e|| < eps_l and
// c > 1) or stop.  A stopping block, or every block at the last iteration,
// copies its basis into Vf.
template <typename T>
__global__ void __launch_bounds__(DOI_THREADS)
    k_doi_step(const MatDesc* __restrict__ sets, const int64_t* __restrict__ v_off,
               const float* __restrict__ X, T* __restrict__ U, T* __restrict__ Vf,
               int32_t* __restrict__ c, int32_t* __restrict__ done, int32_t* __restrict__ iters,
               double* __restrict__ traj, int t, int t_max, double eps_l, double eps_h, int c_max) {
  __shared__ double s_rows[DOI_CHUNK];
  __shared__ double w_col[DOI_MAX_LD];
  __shared__ double red[DOI_THREADS / 64];
  const MatDesc d = sets[blockIdx.x];
  const int b = d.blk;
  if (done[b]) return;  // uniform over the workgroup
  const int cb = c[b], n = d.rows, ld = d.ld;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float* xb = X + 3 * v_off[b];
  T* Ub = U + d.off;
  // w = U^T s over the active columns (threads over columns, rows staged)
  double wj[DOI_MAX_LD / DOI_THREADS];
#pragma unroll
  for (int q = 0; q < DOI_MAX_LD / DOI_THREADS; ++q) wj[q] = 0.0;
  for (int r0 = 0; r0 < n; r0 += DOI_CHUNK) {
    const int nr = min(DOI_CHUNK, n - r0);
    __syncthreads();
    for (int i = tid; i < nr; i += DOI_THREADS) s_rows[i] = doi_s(xb, r0 + i);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < DOI_MAX_LD / DOI_THREADS; ++q) {
      const int j = tid + DOI_THREADS * q;
      if (j < cb)
        for (int i = 0; i < nr; ++i) wj[q] += (double)Ub[int64_t(r0 + i) * ld + j] * s_rows[i];
    }
  }
#pragma unroll
  for (int q = 0; q < DOI_MAX_LD / DOI_THREADS; ++q) {
    const int j = tid + DOI_THREADS * q;
    if (j < DOI_MAX_LD) w_col[j] = j < cb ? wj[q] : 0.0;
  }
  __syncthreads();
  // ||e||^2, rows over wavefronts
  double ss = 0.0;
  for (int i = wv; i < n; i += DOI_THREADS / 64) {
    const double e = doi_e(Ub, ld, cb, w_col, xb, i, lane);
    ss += e * e;
  }
  if (lane == 0) red[wv] = ss;
  __syncthreads();
  double tot = 0.0;
  for (int k = 0; k < DOI_THREADS / 64; ++k) tot += red[k];
  const double ne = sqrt(tot);
  const int cmax_b = min(c_max, d.cols);
  const int dec = (ne > eps_h && cb < cmax_b && ne > 0.0) ? 1 : (ne < eps_l && cb > 1) ? -1 : 0;
  if (tid == 0) {
    traj[(int64_t(b) * t_max + t) * 2] = (double)cb;
    traj[(int64_t(b) * t_max + t) * 2 + 1] = ne;
  }
  if (dec == 1) {  // Eq. 7: the normalised residual becomes column cb
    for (int i = wv; i < n; i += DOI_THREADS / 64) {
      const double e = doi_e(Ub, ld, cb, w_col, xb, i, lane);
      if (lane == 0) Ub[int64_t(i) * ld + cb] = (T)(e / ne);
    }
  } else if (dec == -1) {
    for (int i = tid; i < n; i += DOI_THREADS) Ub[int64_t(i) * ld + cb - 1] = (T)0;
  }
  const bool stop = dec == 0 || t == t_max - 1;
  if (stop) {
    __syncthreads();  // the column update above before the copy
    for (int64_t e = tid; e < int64_t(n) * ld; e += DOI_THREADS) Vf[d.off + e] = Ub[e];
  }
  if (tid == 0) {
    c[b] = cb + dec;
    if (stop) {
      done[b] = 1;
      iters[b] = t + 1;
    }
  }
}

// The factorisations of the walk see the zero columns as rank deficiency
// and flag it; it is the walk's own layout, not a failure.
__global__ void k_doi_status(int B, int32_t* __restrict__ status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) status[b] &= ~MI_BLOCK_NOT_PD;
}

// ------------------------------------------------------------------ plan

static int q_of(int p) { return (p + 1) & ~1; }

// Blocks with a predecessor start from it (MI_WARM_PRED, and MI_RANDOM for
// the blocks that have one).
static bool chained(const mi_oi_params& prm) {
  return prm.warm == MI_WARM_PRED || prm.warm == MI_RANDOM;
}

// Waves: blocks whose predecessor finished in an earlier wave.  Under
// MI_WARM_GIVEN (or without predecessors) all blocks form one wave.  The
// predecessor forest's trees are independent: the trees are dealt to up to
// MAX_LANES stream lanes (by root block id), and each lane's waves run in
// level order on their own stream inside the captured graph, so the
// latency-bound small solves of one lane overlap the bandwidth-bound
// products of another.  The per-block reference path makes every block its
// own wave, in level order, on one lane.
constexpr int MAX_LANES = 4;

static mi_status build_waves(const HostBlocks& hb, const mi_oi_params& prm, bool per_block,
                             std::vector<std::vector<int>>* waves, std::vector<int>* level,
                             std::vector<int>* wave_lane = nullptr, int* n_lanes = nullptr) {
  const int B = hb.B;
  level->assign(B, 0);
  std::vector<int> root(B);
  for (int b = 0; b < B; ++b) root[b] = b;
  if (chained(prm)) {
    for (int b = 0; b < B; ++b) {
      int l = 0, x = b;
      while (hb.pred[x] >= 0) {
        x = hb.pred[x];
        if (++l > B) {
          set_error("predecessor chain of block %d has a cycle", b);
          return MI_ERR_ARG;
        }
      }
      (*level)[b] = l;
      root[b] = x;
    }
  }
  int maxl = 0;
  for (int b = 0; b < B; ++b) maxl = std::max(maxl, (*level)[b]);
  // lane of each block: its tree's rank among the roots, modulo MAX_LANES
  // (blocks that are all independent form one wave on one lane: lanes pay
  // off by overlapping the levels of different trees, and one launch over
  // every block fills the chip best)
  std::vector<int> lane(B, 0);
  int nl = 1;
  if (chained(prm) && !per_block && maxl > 0) {
    std::vector<int> rank(B, -1);
    int nr = 0;
    for (int b = 0; b < B; ++b)
      if (root[b] == b) rank[b] = nr++;
    for (int b = 0; b < B; ++b) lane[b] = rank[root[b]] % MAX_LANES;
    nl = std::min(nr, MAX_LANES);
  }
  waves->clear();
  if (wave_lane) wave_lane->clear();
  for (int ln = 0; ln < nl; ++ln)
    for (int l = 0; l <= maxl; ++l) {
      std::vector<int> w;
      for (int b = 0; b < B; ++b)
        if ((*level)[b] == l && lane[b] == ln) w.push_back(b);
      if (w.empty()) continue;
      if (per_block) {
        for (int b : w) {
          waves->push_back({b});
          if (wave_lane) wave_lane->push_back(0);
        }
      } else {
        waves->push_back(w);
        if (wave_lane) wave_lane->push_back(ln);
      }
    }
  if (n_lanes) *n_lanes = nl;
  return MI_OK;
}

// Output-column width of a row-product tile: the widest supported width that
// divides ld (all blocks of the wave alike), else 64 (masked tail).  Must be
// one of the widths launch_rowmul instantiates.
static int pick_nch(const std::vector<int>& lds_in_wave, bool dbl) {
  int mx = 0;
  bool same = true;
  for (int v : lds_in_wave) {
    same = same && v == lds_in_wave[0];
    mx = std::max(mx, v);
  }
  const int cap = dbl ? 128 : 256;
  if (same) {
    for (int c : {256, 192, 128, 96, 64, 32})
      if (c <= cap && mx % c == 0) return c;
  }
  return 64;
}

static WsLayout ws_layout(const HostBlocks& hb, const mi_oi_params& prm, size_t part_doubles,
                          int n_lanes) {
  const size_t es = prm.precision == MI_FP64 ? 8 : prm.precision == MI_BF16_IN ? 2 : 4;
  int64_t slab = hb.u_off[hb.B];
  int64_t mats = hb.m_off[hb.B];
  int64_t pk = 0, lg = 0, tp = hb.t_off[hb.B];
  for (int b = 0; b < hb.B; ++b) {
    const int64_t q = q_of(hb.p[b]);
    pk += q * (q + 1) / 2;
    lg += (q - 1) * (q / 2) * 2;
  }
  const int mmax = std::max(prm.m, prm.m0);
  WsLayout L;
  Carver c(nullptr);
  for (int i = 0; i < 4; ++i) L.slab[i] = c.used, c.take<char>(size_t(slab) * es);
  L.G = c.used, c.take<double>(mats);
  L.H = c.used, c.take<double>(mats);
  L.Rinv = c.used, c.take<double>(mats);
  L.T1 = c.used, c.take<double>(mats);
  L.A = c.used, c.take<double>(mats);
  L.Z = c.used, c.take<double>(mats);
  L.S64 = c.used, c.take<double>(mats);
  L.S32 = c.used, c.take<float>(mats);
  L.Wk = c.used, c.take<double>(mats);
  L.pk = c.used, c.take<double>(pk);
  L.log = c.used, c.take<double>(lg);
  L.perm = c.used, c.take<int32_t>(tp);
  L.tri = c.used, c.take<double>(4 * tp);
  L.part_lane = std::max<size_t>(part_doubles, 1);
  L.part = c.used, c.take<double>(L.part_lane * std::max(n_lanes, 1));
  L.queue = c.used, c.take<int32_t>(std::max(n_lanes, 1));
  L.a_lo = c.used, c.take<double>(hb.B);
  L.b_hi = c.used, c.take<double>(hb.B);
  L.coef_stride = 3 * (mmax + 1);
  L.coef = c.used, c.take<double>(size_t(hb.B) * L.coef_stride);
  L.conv = c.used, c.take<int32_t>(hb.B);
  // R^z: per-tile column partials (p.q and two generations of r.r)
  int64_t tiles = 0;
  L.cg_ldp = 0;
  for (int b = 0; b < hb.B; ++b) {
    tiles += (hb.v_off[b + 1] - hb.v_off[b] + SPMM_ROWS - 1) / SPMM_ROWS;
    L.cg_ldp = std::max(L.cg_ldp, hb.ld[b]);
  }
  L.cg_tiles = tiles;
  L.cg_part = c.used;
  if (prm.op == MI_OP_RZ) c.take<double>(3 * size_t(tiles) * L.cg_ldp);
  L.rpart = c.used, c.take<double>(size_t(tiles) * L.cg_ldp);
  const bool tolm = prm.tol > 0;
  L.slab_w = c.used, c.take<char>(tolm ? size_t(slab) * es : 0);
  L.ritz_w = c.used, c.take<double>(tolm ? tp : 0);
  L.resid_w = c.used, c.take<double>(tolm ? tp : 0);
  L.frozen = c.used, c.take<int32_t>(tolm ? hb.B : 0);
  L.fnow = c.used, c.take<int32_t>(tolm ? hb.B : 0);
  L.total = c.used;
  return L;
}

// Host-side tables of one wave (device pointers filled in by upload()).
struct WaveHost {
  std::vector<MatDesc> tall, ptall, small;
  std::vector<CsrDesc> csr;
  std::vector<SmallDesc> sd;
  std::vector<SpmmTile> spmm;
  std::vector<GramTile> gt, gts;
  std::vector<GramReduce> gr, grs;
  std::vector<RowTile> rt, rts;
  std::vector<int32_t> porder;
};

static void wave_host(const HostBlocks& hb, const std::vector<int64_t>& nnz_off,
                      const std::vector<int>& blocks, const mi_oi_params& prm, WaveTables* wt,
                      WaveHost* h, const std::vector<int64_t>& pk_off,
                      const std::vector<int64_t>& log_off, const WaveTune* tune = nullptr,
                      int spmm_force = -1) {
  const bool dbl = prm.precision == MI_FP64;
  std::vector<int> lds_list;
  for (int b : blocks) {
    const int n = int(hb.v_off[b + 1] - hb.v_off[b]);
    MatDesc d{hb.u_off[b], n, hb.ld[b], hb.p[b], b};
    h->tall.push_back(d);
    const int pb = hb.pred[b];
    if (pb >= 0)
      h->ptall.push_back(MatDesc{hb.u_off[pb], int(hb.v_off[pb + 1] - hb.v_off[pb]), hb.ld[pb],
                                 hb.p[pb], pb});
    else
      h->ptall.push_back(d);
    h->small.push_back(MatDesc{hb.m_off[b], hb.ld[b], hb.ld[b], hb.p[b], b});
    h->csr.push_back(CsrDesc{hb.v_off[b] + b, nnz_off[b]});
    SmallDesc s;
    s.m_off = hb.m_off[b];
    s.pk_off = pk_off[b];
    s.log_off = log_off[b];
    s.t_off = hb.t_off[b];
    s.p = hb.p[b];
    s.ld = hb.ld[b];
    s.q = q_of(hb.p[b]);
    s.blk = b;
    h->sd.push_back(s);
    lds_list.push_back(hb.ld[b]);
    wt->max_ld = std::max(wt->max_ld, hb.ld[b]);
    wt->max_q = std::max(wt->max_q, s.q);
    wt->max_p = std::max(wt->max_p, s.p);
  }
  wt->nb = (int)blocks.size();
  wt->nch = tune ? tune->nch : pick_nch(lds_list, dbl);
  wt->nchs = pick_nch(lds_list, true);
  spmm_tables(h->tall, &h->spmm);
  wt->epl = tune ? tune->epl : spmm_epl(h->tall);
  wt->spmm_var = tune ? tune->spmm_var : -1;
  if (spmm_force >= 0 && wt->epl > 0) wt->spmm_var = spmm_force;
  wt->gram_target = tune ? tune->gram_target : GRAM_TARGET;
  gram_tables(h->tall, true, &h->gt, &h->gr, wt->gram_target);
  wt->gram_direct = prm.precision != MI_BF16_IN && gram_unsplit(h->gr);
  // whole-block super-tiles (no partials) run largest block first, so that
  // the launch does not end on a long tile of a large block
  if (wt->gram_direct)
    std::stable_sort(h->gt.begin(), h->gt.end(), [](const GramTile& x, const GramTile& y) {
      return x.r1 - x.r0 > y.r1 - y.r0;
    });
  gram_tables(h->small, false, &h->gts, &h->grs);
  row_tables(h->tall, wt->nch, &h->rt);
  row_tables(h->small, wt->nchs, &h->rts);
  // persistent filter passes: blocks claimed largest first
  wt->persistent = prm.persistent == 1 && prm.op == MI_OP_CHEB && wt->epl > 0;
  h->porder.resize(h->tall.size());
  for (size_t i = 0; i < h->porder.size(); ++i) h->porder[i] = int32_t(i);
  std::stable_sort(h->porder.begin(), h->porder.end(),
                   [&](int32_t x, int32_t y) { return h->tall[x].rows > h->tall[y].rows; });
  wt->pgrid = 0;
  if (wt->persistent) {
    const int nb = (int)blocks.size();
    wt->pgrid = prm.precision == MI_FP64      ? cheb_pass_grid<double>(wt->epl, nb)
                : prm.precision == MI_BF16_IN ? cheb_pass_grid<bf16>(wt->epl, nb)
                                              : cheb_pass_grid<float>(wt->epl, nb);
    wt->persistent = wt->pgrid > 0;
  }
}

template <typename X>
static X* put(std::vector<char>& blob, const std::vector<X>& v, std::vector<size_t>* offs) {
  size_t off = align_up(blob.size());
  blob.resize(off + align_up(v.size() * sizeof(X)));
  if (!v.empty()) memcpy(blob.data() + off, v.data(), v.size() * sizeof(X));
  offs->push_back(off);
  return reinterpret_cast<X*>(off);  // relocated after upload
}

// Gram split-K targets and row-product widths the autotuner tries.
static const int kGramTargets[] = {192, 384, 768, 1536};
static const int kNchs[] = {64, 96, 128, 192, 256};

// Gram partial doubles of the largest split a tuned plan may choose.
static size_t tuned_part_max(const std::vector<MatDesc>& tall) {
  std::vector<GramTile> gt;
  std::vector<GramReduce> gr;
  gram_tables(tall, true, &gt, &gr, kGramTargets[3]);
  return gt.size() * 2 * GRAM_TILE * GRAM_TILE;
}

static mi_status make_plan(const HostBlocks& hb, const std::vector<int64_t>& nnz_off,
                           const mi_oi_params& prm, bool per_block, int lds_max,
                           int spmm_force, std::unique_ptr<OiPlan>* out, size_t* ws_need,
                           const std::vector<WaveTune>* tune = nullptr) {
  std::unique_ptr<OiPlan> P(new OiPlan());
  P->spmm_force = spmm_force;
  P->hb = hb;
  P->nnz_off = nnz_off;
  P->prm = prm;
  P->per_block = per_block;
  P->lds_max = lds_max;
  std::vector<std::vector<int>> waves;
  std::vector<int> level, wave_lane;
  mi_status st = build_waves(hb, prm, per_block, &waves, &level, &wave_lane, &P->n_lanes);
  if (st) return st;
  std::vector<int64_t> pk_off(hb.B), log_off(hb.B);
  int64_t pk = 0, lg = 0;
  for (int b = 0; b < hb.B; ++b) {
    const int64_t q = q_of(hb.p[b]);
    pk_off[b] = pk;
    log_off[b] = lg;
    pk += q * (q + 1) / 2;
    lg += (q - 1) * (q / 2) * 2;
  }
  std::vector<char> blob;
  std::vector<WaveHost> hosts(waves.size());
  P->waves.resize(waves.size());
  size_t part_max = 0;
  for (size_t w = 0; w < waves.size(); ++w) {
    WaveTables& wt = P->waves[w];
    const bool warm_wave = chained(prm) && level[waves[w][0]] > 0;
    wt.from_pred = warm_wave;
    wt.T = warm_wave ? prm.T : prm.T0;
    wt.m = warm_wave ? prm.m : prm.m0;
    wt.passes = warm_wave ? prm.passes : prm.passes0;
    wt.lane = wave_lane[w];
    wave_host(hb, nnz_off, waves[w], prm, &wt, &hosts[w], pk_off, log_off,
              tune ? &(*tune)[w] : nullptr, spmm_force);
    part_max = std::max(part_max, hosts[w].gt.size() * 2 * GRAM_TILE * GRAM_TILE);
    part_max = std::max(part_max, hosts[w].gts.size() * 2 * GRAM_TILE * GRAM_TILE);
    if (prm.autotune) part_max = std::max(part_max, tuned_part_max(hosts[w].tall));
    // BF16 slabs run only the wavefront-per-row SpMM (one width per wave)
    MI_CHECK_ARG(prm.precision != MI_BF16_IN || wt.epl > 0,
                 "MI_BF16_IN needs every block of a wave to share ld, a multiple of 64 up to 320");
  }
  P->L = ws_layout(hb, prm, part_max, P->n_lanes);
  *ws_need = P->L.total;
  // block info + whole-set tables for the per-call kernels
  std::vector<BlkInfo> info(hb.B);
  std::vector<MatDesc> all_tall;
  std::vector<CsrDesc> all_csr;
  for (int b = 0; b < hb.B; ++b) {
    info[b] = BlkInfo{hb.t_off[b], int(hb.v_off[b + 1] - hb.v_off[b]), hb.p[b], hb.pred[b],
                      hb.c[b]};
    all_tall.push_back(MatDesc{hb.u_off[b], info[b].n, hb.ld[b], hb.p[b], b});
    all_csr.push_back(CsrDesc{hb.v_off[b] + b, nnz_off[b]});
  }
  std::vector<size_t> offs;
  put(blob, info, &offs);
  put(blob, all_tall, &offs);
  put(blob, all_csr, &offs);
  put(blob, hb.v_off, &offs);
  std::vector<int64_t> tile_base(hb.B + 1, 0);
  for (int b = 0; b < hb.B; ++b)
    tile_base[b + 1] = tile_base[b] + (hb.v_off[b + 1] - hb.v_off[b] + SPMM_ROWS - 1) / SPMM_ROWS;
  put(blob, tile_base, &offs);
  for (auto& h : hosts) {
    put(blob, h.tall, &offs);
    put(blob, h.ptall, &offs);
    put(blob, h.small, &offs);
    put(blob, h.csr, &offs);
    put(blob, h.sd, &offs);
    put(blob, h.spmm, &offs);
    put(blob, h.gt, &offs);
    put(blob, h.gr, &offs);
    put(blob, h.gts, &offs);
    put(blob, h.grs, &offs);
    put(blob, h.rt, &offs);
    put(blob, h.rts, &offs);
    put(blob, h.porder, &offs);
  }
  MI_TRY_HIP(hipMalloc(&P->arena, std::max<size_t>(blob.size(), 256)));
  MI_TRY_HIP(hipMemcpy(P->arena, blob.data(), blob.size(), hipMemcpyHostToDevice));
  char* base = static_cast<char*>(P->arena);
  size_t k = 0;
  P->info = reinterpret_cast<BlkInfo*>(base + offs[k++]);
  P->all_tall = reinterpret_cast<MatDesc*>(base + offs[k++]);
  P->all_csr = reinterpret_cast<CsrDesc*>(base + offs[k++]);
  P->v_off = reinterpret_cast<int64_t*>(base + offs[k++]);
  P->tile_base = reinterpret_cast<int64_t*>(base + offs[k++]);
  for (size_t w = 0; w < waves.size(); ++w) {
    WaveTables& wt = P->waves[w];
    WaveHost& h = hosts[w];
    wt.tall = reinterpret_cast<MatDesc*>(base + offs[k++]);
    wt.ptall = reinterpret_cast<MatDesc*>(base + offs[k++]);
    wt.small = reinterpret_cast<MatDesc*>(base + offs[k++]);
    wt.csr = reinterpret_cast<CsrDesc*>(base + offs[k++]);
    wt.sd = reinterpret_cast<SmallDesc*>(base + offs[k++]);
    wt.spmm = reinterpret_cast<SpmmTile*>(base + offs[k++]);
    wt.n_spmm = (int)h.spmm.size();
    wt.gt = reinterpret_cast<GramTile*>(base + offs[k++]);
    wt.n_gt = (int)h.gt.size();
    wt.gr = reinterpret_cast<GramReduce*>(base + offs[k++]);
    wt.n_gr = (int)h.gr.size();
    wt.gts = reinterpret_cast<GramTile*>(base + offs[k++]);
    wt.n_gts = (int)h.gts.size();
    wt.grs = reinterpret_cast<GramReduce*>(base + offs[k++]);
    wt.n_grs = (int)h.grs.size();
    wt.rt = reinterpret_cast<RowTile*>(base + offs[k++]);
    wt.n_rt = (int)h.rt.size();
    wt.rts = reinterpret_cast<RowTile*>(base + offs[k++]);
    wt.n_rts = (int)h.rts.size();
    wt.porder = reinterpret_cast<int32_t*>(base + offs[k++]);
    wt.tall_host = h.tall;
  }
  *out = std::move(P);
  return MI_OK;
}

// ------------------------------------------------------------------ autotuner
// Per wave, times the candidate launch shapes of the tall-skinny kernels on
// the plan's own tables and workspace (operand values do not matter for the
// timing; every index stays inside the same buffers as in production) and
// keeps the fastest: the Gram's split-K target and the row product's output
// width.  Runs on a private stream at plan creation.

// Milliseconds per call of f: one warm-up, then three timed calls.
template <typename F>
static float time_calls(hipStream_t s, F&& f) {
  hipEvent_t a = nullptr, b = nullptr;
  float ms = 1e30f;
  if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
    f();
    (void)hipEventRecord(a, s);
    for (int r = 0; r < 3; ++r) f();
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess)
      ms /= 3.f;
    else
      ms = 1e30f;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return ms;
}

// Temporary device copy of a host table.
template <typename X>
struct DevTable {
  X* p = nullptr;
  explicit DevTable(const std::vector<X>& v) {
    if (!v.empty() && hipMalloc(&p, v.size() * sizeof(X)) == hipSuccess &&
        hipMemcpy(p, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(p);
      p = nullptr;
    }
  }
  ~DevTable() {
    if (p) (void)hipFree(p);
  }
};

template <typename T>
static void autotune_waves(const OiPlan& P, char* ws, hipStream_t s, const int32_t* row_ptr,
                           const int32_t* col, const float* val, std::vector<WaveTune>* tune) {
  const WsLayout& L = P.L;
  T* y0 = reinterpret_cast<T*>(ws + L.slab[0]);
  T* y1 = reinterpret_cast<T*>(ws + L.slab[1]);
  typedef typename Acc<T>::type TS;  // element type of the row product's S
  const TS* Sm = reinterpret_cast<const TS*>(ws + L.G);
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* G = reinterpret_cast<double*>(ws + L.H);
  const bool dbl = std::is_same<T, double>::value;
  tune->clear();
  for (const WaveTables& w : P.waves) {
    WaveTune best{w.gram_target, w.nch, w.epl, -1};
    float bt = 1e30f;
    for (int target : kGramTargets) {
      std::vector<GramTile> gt;
      std::vector<GramReduce> gr;
      gram_tables(w.tall_host, true, &gt, &gr, target);
      DevTable<GramTile> dgt(gt);
      DevTable<GramReduce> dgr(gr);
      if (!dgt.p || !dgr.p) continue;
      const bool direct = !std::is_same<T, bf16>::value && gram_unsplit(gr);
      const float t = time_calls(s, [&] {
        if constexpr (!std::is_same<T, bf16>::value) {
          if (direct) {
            launch_gram_direct<T>(dgt.p, (int)gt.size(), w.tall, w.small, y0, y0, nullptr, G,
                                  nullptr, s);
            return;
          }
        }
        launch_gram<T>(dgt.p, (int)gt.size(), w.tall, y0, y0, nullptr, part, s);
        launch_gram_reduce(dgr.p, (int)gr.size(), w.small, part, false, G, nullptr, s);
      });
      if (t < bt) bt = t, best.gram_target = target;
    }
    bool same = true;
    for (const MatDesc& d : w.tall_host) same = same && d.ld == w.tall_host[0].ld;
    bt = 1e30f;
    for (int nch : kNchs) {
      if (nch > (dbl ? 128 : 256)) continue;
      if (!(same && w.tall_host[0].ld % nch == 0) && nch != 64) continue;
      std::vector<RowTile> rt;
      row_tables(w.tall_host, nch, &rt);
      DevTable<RowTile> drt(rt);
      if (!drt.p) continue;
      const float t = time_calls(s, [&] {
        // most row products of a step multiply by a triangular R^-1
        launch_rowmul<T, TS>(drt.p, (int)rt.size(), w.tall, y0, w.small, Sm, w.tall, y1, nch, s,
                             true);
      });
      if (t < bt) bt = t, best.nch = nch;
    }
    // the SpMM keeps the row-per-wavefront kernel wherever it applies (the
    // faster one on every wave size measured) and times its variants: one
    // or two rows per wavefront, 8 or 4 neighbour rows gathered at a time,
    // 16- or 4-wavefront workgroups (one Chebyshev step with a previous
    // iterate, the common case)
    best.epl = spmm_epl(w.tall_host);
    if (best.epl > 0) {
      T* y2 = reinterpret_cast<T*>(ws + L.slab[2]);
      const double* coef = reinterpret_cast<const double*>(ws + L.coef);
      bt = 1e30f;
      for (int var = 0; var < SPMM_NVAR; ++var) {
        const float t = time_calls(s, [&] {
          launch_spmm<T>(w.spmm, w.n_spmm, w.tall, w.csr, row_ptr, col, val, y0, y1, y2, coef,
                         L.coef_stride, 1, s, best.epl, var);
        });
        if (t < bt) bt = t, best.spmm_var = var;
      }
    }
    tune->push_back(best);
  }
}

// ------------------------------------------------------------------ enqueue

// T: element type of the working slabs; TV: of the caller's V0 and V (the
// same, except for BF16 working slabs with an FP32 result).
template <typename T, typename TV = T>
static void enqueue(OiPlan& P, const Args& a, hipStream_t s) {
  constexpr bool same = std::is_same<T, TV>::value;
  typedef typename Acc<T>::type TS;  // the row products' S (FP32 or FP64)
  KClose kc_(a.tm);
  const mi_oi_params& prm = P.prm;
  const WsLayout& L = P.L;
  char* ws = a.ws;
  T* slab[4];
  for (int i = 0; i < 4; ++i) slab[i] = reinterpret_cast<T*>(ws + L.slab[i]);
  double* G = reinterpret_cast<double*>(ws + L.G);
  double* H = reinterpret_cast<double*>(ws + L.H);
  double* Rinv = reinterpret_cast<double*>(ws + L.Rinv);
  double* T1 = reinterpret_cast<double*>(ws + L.T1);
  double* Am = reinterpret_cast<double*>(ws + L.A);
  double* Z = reinterpret_cast<double*>(ws + L.Z);
  double* S64 = reinterpret_cast<double*>(ws + L.S64);
  float* S32 = reinterpret_cast<float*>(ws + L.S32);
  double* Wk = reinterpret_cast<double*>(ws + L.Wk);
  double* pk = reinterpret_cast<double*>(ws + L.pk);
  double* lg = reinterpret_cast<double*>(ws + L.log);
  int32_t* perm = reinterpret_cast<int32_t*>(ws + L.perm);
  double* tri = reinterpret_cast<double*>(ws + L.tri);
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* a_lo = reinterpret_cast<double*>(ws + L.a_lo);
  double* b_hi = reinterpret_cast<double*>(ws + L.b_hi);
  double* coef = reinterpret_cast<double*>(ws + L.coef);
  int32_t* conv = reinterpret_cast<int32_t*>(ws + L.conv);
  int32_t* queue0 = reinterpret_cast<int32_t*>(ws + L.queue);
  const bool dbl = std::is_same<T, double>::value;
  const int B = P.hb.B;
  const OiRecord* rec = a.rec;
  const DoiArgs* doi = a.doi;
  // tolerance mode: iterate in a working slab, copy each block out when it
  // meets the tolerance (or at the cap)
  const bool tolm = prm.tol > 0 && !doi && !rec;
  TV* Vout = static_cast<TV*>(a.V);
  TV* V = tolm ? reinterpret_cast<TV*>(ws + L.slab_w) : Vout;
  double* ritz_w = tolm ? reinterpret_cast<double*>(ws + L.ritz_w) : a.ritz;
  double* resid_w = reinterpret_cast<double*>(ws + L.resid_w);
  double* rpart = reinterpret_cast<double*>(ws + L.rpart);
  int32_t* frozen = reinterpret_cast<int32_t*>(ws + L.frozen);
  int32_t* fnow = reinterpret_cast<int32_t*>(ws + L.fnow);
  const TV* V0 = static_cast<const TV*>(a.V0);
  TV* Vf = doi ? reinterpret_cast<TV*>(ws + doi->off_vf) : nullptr;
  int32_t* doi_done = doi ? reinterpret_cast<int32_t*>(ws + doi->off_done) : nullptr;

  {
    KScope k_(a.tm, MI_K_SETUP, s);
    fill_i32(a.status, 0, B, s);
    if (tolm) fill_i32(frozen, 0, B, s);
  }
  {
    KScope k_(a.tm, MI_K_SETUP, s);
    if (prm.b_abs > 0)
      hipLaunchKernelGGL(k_set_b, dim3(ceil_div(B, 256)), dim3(256), 0, s, P.all_tall, B, prm.b_abs,
                         b_hi);
    else
      hipLaunchKernelGGL(k_gershgorin, dim3(B), dim3(256), 0, s, P.all_tall, P.all_csr, a.row_ptr,
                         a.val, b_hi);
  }

  // lanes: fork every lane stream from s, run each lane's waves on its own
  // stream, join them back into s at the end (graph capture only; eager runs
  // keep everything on s)
  const bool fork = a.fork && P.n_lanes > 1 && (int)P.lane_s.size() >= P.n_lanes;
  if (fork) {
    (void)hipEventRecord(P.fork_ev, s);
    for (int l = 0; l < P.n_lanes; ++l) (void)hipStreamWaitEvent(P.lane_s[l], P.fork_ev, 0);
  }
  double* part0 = part;
  const hipStream_t s_main = s;
  for (WaveTables& w : P.waves) {
    hipStream_t s = fork ? P.lane_s[w.lane] : s_main;
    int jp = 0;  // filter passes of this wave done (recording index)
    // checkpoints of this wave's blocks only (other waves' blocks hold their
    // own passes in the same recording slots)
    auto keep_slab = [&](void* dst, const T* src) {
      hipLaunchKernelGGL(k_copy_slab<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall, src,
                         static_cast<T*>(dst));
    };
    auto keep_mats = [&](void* dst, const void* src, bool f64) {
      if (f64)
        hipLaunchKernelGGL(k_copy_mats<double>, dim3(w.nb), dim3(256), 0, s, w.sd,
                           static_cast<const double*>(src), static_cast<double*>(dst));
      else
        hipLaunchKernelGGL(k_copy_mats<TS>, dim3(w.nb), dim3(256), 0, s, w.sd,
                           static_cast<const TS*>(src), static_cast<TS*>(dst));
    };
    double* part = part0 + (fork ? size_t(w.lane) * L.part_lane : 0);
    int32_t* queue = queue0 + (fork ? w.lane : 0);
    const size_t lds_jac = size_t(4 * (w.max_q / 2) + (size_t)w.max_q * (w.max_q + 1) / 2) * 8;
    const bool jac_lds = lds_jac <= (size_t)P.lds_max;
    const size_t lds_jac_use = jac_lds ? lds_jac : size_t(4 * (w.max_q / 2)) * 8;

    {
      KScope k_(a.tm, MI_K_SETUP, s);
      hipLaunchKernelGGL(k_init_a, dim3(ceil_div(w.nb, 256)), dim3(256), 0, s, w.tall, w.nb, P.info,
                         w.from_pred ? 1 : 0, prm.a_mode, prm.a_value, a.ritz, a_lo, b_hi);
    }
    // start basis X of the first iteration (in a working slab when the
    // working type differs from the caller's)
    const T* X = nullptr;
    int xslab = -1;  // slab holding X (-1: X lives in V0 / V)
    bool start_in_v = false;  // the start's Cholesky-QR wrote the output
    if constexpr (same) {
      X = V0;
    } else if (!w.from_pred && prm.warm != MI_RANDOM) {
      KScope k_(a.tm, MI_K_SETUP, s);
      hipLaunchKernelGGL((k_copy_slab<TV, T>), dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                         V0, slab[1]);
      X = slab[1];
      xslab = 1;
    }
    if (w.from_pred) {
      KScope k_(a.tm, MI_K_SETUP, s);
      if constexpr (same) {
        hipLaunchKernelGGL((k_warm_copy<T, T>), dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                           w.ptall, (const T*)Vout, V);
        X = V;
      } else {
        hipLaunchKernelGGL((k_warm_copy<TV, T>), dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                           w.ptall, (const TV*)Vout, slab[1]);
        X = slab[1];
        xslab = 1;
      }
    }
    // seeded start of the blocks without predecessor (MI_RANDOM)
    const bool rand_root = prm.warm == MI_RANDOM && !w.from_pred && !doi;
    if (rand_root) {
      KScope k_(a.tm, MI_K_SETUP, s);
      hipLaunchKernelGGL(k_random_start<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                         (uint64_t)prm.seed, slab[1]);
      X = slab[1];
    }
    if constexpr (same) if (doi) {
      // the walk edits its basis in place: roots start from a copy of V0
      if (!w.from_pred) {
        KScope k_(a.tm, MI_K_SETUP, s);
        hipLaunchKernelGGL(k_copy_slab<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall, V0, V);
      }
      X = V;
      KScope k_(a.tm, MI_K_DOI, s);
      hipLaunchKernelGGL(k_doi_init<T>, dim3(w.nb), dim3(DOI_THREADS), 0, s, w.tall, P.info,
                         w.from_pred ? 1 : 0, doi->c_max, doi->t_max, doi->c, doi_done, doi->traj,
                         V);
    }
    // Gram of the wave's slabs into G (and H for the dual product)
    auto gram = [&](const T* GA, const T* GW, double* Go, double* Ho) {
      if constexpr (!std::is_same<T, bf16>::value) {
        if (w.gram_direct) {
          KScope k_(a.tm, MI_K_GRAM, s);
          launch_gram_direct<T>(w.gt, w.n_gt, w.tall, w.small, GA, GA, GW, Go, Ho, s);
          return;
        }
      }
      {
        KScope k_(a.tm, MI_K_GRAM, s);
        launch_gram<T>(w.gt, w.n_gt, w.tall, GA, GA, GW, part, s);
      }
      KScope k_(a.tm, MI_K_GRAM_REDUCE, s);
      launch_gram_reduce(w.gr, w.n_gr, w.small, part, GW != nullptr, Go, Ho, s);
    };
    auto chol = [&](float* s32) {
      KScope k_(a.tm, MI_K_CHOL, s);
      launch_chol_blk(w.sd, w.nb, G, Wk, Rinv, s32, a.status, w.max_ld, P.lds_max, s);
    };
    if (w.from_pred || rand_root) {
      // The index-aligned warm start drops rows when the block is smaller
      // than its predecessor and can be badly conditioned (and a seeded
      // start is not orthonormal); one Cholesky-QR before the first filter
      // pass keeps the filtered basis of full rank in FP32.
      gram(X, nullptr, G, nullptr);
      chol(dbl ? nullptr : S32);
      const TS* Sr = dbl ? reinterpret_cast<const TS*>(Rinv) : reinterpret_cast<const TS*>(S32);
      KScope k_(a.tm, MI_K_ROWMUL, s);
      if (!same && w.T == 0 && !doi) {
        // no iteration follows: the orthonormalised start is the result,
        // written in the output type
        launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, X, w.small, Sr, w.tall, Vout, w.nch, s, true);
        start_in_v = true;
      } else {
        launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, X, w.small, Sr, w.tall, slab[0], w.nch, s,
                             true);
        X = slab[0];
        xslab = 0;
      }
    }
    const int n_iter = doi ? doi->t_max : w.T;
    bool wave_stopped = false;
    for (int t = 0; t < n_iter && !wave_stopped; ++t) {
      const bool last = !doi && t == w.T - 1;
      // an iteration that ends with the Rayleigh-Ritz step and the final
      // Cholesky-QR: the last one, or every one in the tolerance mode
      const bool fin = !doi && (last || tolm);
      const bool rr_now = !doi && (fin || prm.rr_every);
      int ycur = -1;
      for (int pass = 0; pass < w.passes; ++pass) {
        // the interval [a, b] changes only at the end of an iteration: the
        // first pass's coefficients serve every pass of the iteration
        if (pass == 0) {
          KScope k_(a.tm, MI_K_SETUP, s);
          if (prm.op == MI_OP_RZ)
            hipLaunchKernelGGL(k_rz_coef, dim3(ceil_div(w.nb, 256)), dim3(256), 0, s, w.tall, w.nb,
                               prm.delta, coef, L.coef_stride, w.m);
          else
            hipLaunchKernelGGL(k_cheb_coef, dim3(ceil_div(w.nb, 256)), dim3(256), 0, s, w.tall,
                               w.nb, a_lo, b_hi, coef, L.coef_stride, w.m);
        }
        if (rec) {
          if (pass == 0)
            hipLaunchKernelGGL(k_copy_coef, dim3(ceil_div(w.nb * L.coef_stride, 256)), dim3(256),
                               0, s, w.tall, w.nb, L.coef_stride, (const double*)coef,
                               rec->coef + size_t(t) * B * L.coef_stride);
          keep_slab(rec->X[jp], X);
        }
        int free_s[3], nf = 0;
        for (int i = 0; i < 4 && nf < 3; ++i)
          if (i != xslab) free_s[nf++] = i;
        if constexpr (same) if (prm.op == MI_OP_RZ) {
          // Y = R^z X: x, r, p in the free slabs; q in X's slab once the first
          // solve has read X (or in the fourth slab when X is outside them)
          int q_s = xslab;
          if (q_s < 0)
            for (int i = 0; i < 4; ++i)
              if (i != free_s[0] && i != free_s[1] && i != free_s[2]) q_s = i;
          T* xs = slab[free_s[0]];
          T* rs = slab[free_s[1]];
          T* ps = slab[free_s[2]];
          T* qs = slab[q_s];
          const size_t plane = size_t(L.cg_tiles) * L.cg_ldp;
          double* cgp = reinterpret_cast<double*>(ws + L.cg_part);
          double* partP = cgp;
          double* partR[2] = {cgp + plane, cgp + 2 * plane};
          const dim3 cg_grid(w.n_spmm, ceil_div(w.max_ld, CG_COLS));
          const int ldp = L.cg_ldp;
          for (int zz = 0; zz < prm.z; ++zz) {
            {
              KScope k_(a.tm, MI_K_CG, s);
              hipLaunchKernelGGL(k_cg_start<T>, cg_grid, dim3(CG_COLS), 0, s, w.spmm, w.tall,
                                 P.tile_base, ldp, zz == 0 ? X : (const T*)xs, xs, rs, ps,
                                 partR[0]);
            }
            for (int it = 0; it < prm.cg_iters; ++it) {
              double* r_old = partR[it & 1];
              double* r_new = partR[(it + 1) & 1];
              {
                KScope k_(a.tm, MI_K_SPMM, s);
                launch_spmm<T>(w.spmm, w.n_spmm, w.tall, w.csr, a.row_ptr, a.col, a.val, ps,
                               nullptr, qs, coef, L.coef_stride, 0, s, w.epl, w.spmm_var);
              }
              KScope k_(a.tm, MI_K_CG, s);
              hipLaunchKernelGGL(k_cg_pq<T>, cg_grid, dim3(CG_COLS), 0, s, w.spmm, w.tall,
                                 P.tile_base, ldp, (const T*)ps, (const T*)qs, partP);
              hipLaunchKernelGGL(k_cg_xr<T>, cg_grid, dim3(CG_COLS), 0, s, w.spmm, w.tall,
                                 P.tile_base, ldp, xs, rs, (const T*)ps, (const T*)qs,
                                 (const double*)partP, (const double*)r_old, r_new);
              hipLaunchKernelGGL(k_cg_p<T>, cg_grid, dim3(CG_COLS), 0, s, w.spmm, w.tall,
                                 P.tile_base, ldp, (const T*)rs, ps, (const double*)r_old,
                                 (const double*)r_new);
            }
          }
          ycur = free_s[0];
        }
        if (w.persistent && prm.op == MI_OP_CHEB && w.m > 0) {
          // the pass's m steps in one launch over a block work queue
          KScope k_(a.tm, MI_K_CHEB_PASS, s);
          launch_cheb_pass<T>(w.tall, w.csr, w.porder, w.nb, a.row_ptr, a.col, a.val, X,
                              slab[free_s[0]], slab[free_s[1]], slab[free_s[2]], coef,
                              L.coef_stride, w.m, queue, w.pgrid, w.epl, s);
          ycur = free_s[(w.m - 1) % 3];
        }
        const T* prev = nullptr;
        const T* cur = X;
        for (int k = 0; k < (prm.op == MI_OP_RZ || w.persistent ? 0 : w.m); ++k) {
          T* out = slab[free_s[k % 3]];
          {
            KScope k_(a.tm, MI_K_SPMM, s);
            launch_spmm<T>(w.spmm, w.n_spmm, w.tall, w.csr, a.row_ptr, a.col, a.val, cur, prev, out,
                           coef, L.coef_stride, k, s, w.epl, w.spmm_var);
          }
          prev = cur;
          cur = out;
          ycur = free_s[k % 3];
        }
        ++jp;
        if (pass < w.passes - 1) {
          // span-preserving Cholesky-QR between passes
          gram(slab[ycur], nullptr, G, nullptr);
          chol(dbl ? nullptr : S32);
          if (rec) keep_mats(rec->S[jp - 1], dbl ? (const void*)Rinv : (const void*)S32, false);
          int dst = -1;
          for (int i = 0; i < 4; ++i)
            if (i != ycur && i != xslab) dst = i;
          {
            KScope k_(a.tm, MI_K_ROWMUL, s);
            launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, slab[ycur], w.small,
                                 dbl ? reinterpret_cast<const TS*>(Rinv)
                                     : reinterpret_cast<const TS*>(S32),
                                 w.tall, slab[dst], w.nch, s, true);
          }
          X = slab[dst];
          xslab = dst;
        }
      }
      T* Y = slab[ycur];
      int wsl = -1;
      for (int i = 0; i < 4; ++i)
        if (i != ycur) wsl = i;
      T* Wm = slab[wsl];
      // BF16 slabs take the intermediate bound from the dual Gram (Y^T L Y
      // with R^-1 applied in FP64): a quotient of the BF16-rounded basis
      // would carry its rounding noise weighted by L
      const bool bf16_rq = std::is_same<T, bf16>::value && !rr_now && prm.adapt;
      if (rr_now || bf16_rq) {
        // W = L Y;  G = Y^T Y, H = Y^T W (one dual Gram pass);  R^T R = G
        {
          KScope k_(a.tm, MI_K_SPMM, s);
          launch_spmm<T>(w.spmm, w.n_spmm, w.tall, w.csr, a.row_ptr, a.col, a.val, Y, nullptr, Wm,
                         coef, L.coef_stride, w.m, s, w.epl, w.spmm_var);
        }
        gram(Y, Wm, G, H);
      }
      if (!rr_now) {
        // intermediate iteration: Cholesky-QR of Y, X = Y R^-1; the filter's
        // lower bound follows the largest Rayleigh quotient q_j^T L q_j of
        // the new basis, from W = L X (in Y's slab, free once X is formed)
        // column by column
        if (!bf16_rq) gram(Y, nullptr, G, nullptr);
        chol(dbl ? nullptr : S32);
        if (rec) keep_mats(rec->S[jp - 1], dbl ? (const void*)Rinv : (const void*)S32, false);
        if (bf16_rq) {
          {
            KScope k_(a.tm, MI_K_ROWMUL_SMALL, s);
            launch_rowmul<double, double>(w.rts, w.n_rts, w.small, H, w.small, Rinv, w.small, T1,
                                          w.nchs, s, true);
          }
          KScope k_(a.tm, MI_K_RQ_MAX, s);
          launch_rq_max(w.sd, w.nb, Rinv, T1, a_lo, s);
        }
        {
          KScope k_(a.tm, MI_K_ROWMUL, s);
          const TS* Sr = dbl ? reinterpret_cast<const TS*>(Rinv) : reinterpret_cast<const TS*>(S32);
          if constexpr (same) {
            launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, Y, w.small, Sr, w.tall, V, w.nch, s, true);
            X = V;
            xslab = -1;
          } else {
            launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, Y, w.small, Sr, w.tall, Wm, w.nch, s, true);
            X = Wm;
            xslab = wsl;
          }
        }
        if (prm.adapt && !bf16_rq) {
          {
            KScope k_(a.tm, MI_K_SPMM, s);
            launch_spmm<T>(w.spmm, w.n_spmm, w.tall, w.csr, a.row_ptr, a.col, a.val, X, nullptr, Y,
                           coef, L.coef_stride, w.m, s, w.epl, w.spmm_var);
          }
          KScope k_(a.tm, MI_K_RQ_MAX, s);
          launch_rq<T>(w.tall, w.small, w.nb, X, Y, H, a_lo, s);
        }
        if constexpr (same) if (doi) {
          KScope k_(a.tm, MI_K_DOI, s);
          hipLaunchKernelGGL(k_doi_step<T>, dim3(w.nb), dim3(DOI_THREADS), 0, s, w.tall, P.v_off,
                             doi->X, V, Vf, doi->c, doi_done, doi->iters, doi->traj, t, doi->t_max,
                             doi->eps_l, doi->eps_h, doi->c_max);
        }
        if (doi && doi->host_done) {
          // the walk runs eagerly: once every block of the wave has stopped,
          // the remaining iterations are skipped
          (void)hipMemcpyAsync(doi->host_done, doi_done, size_t(B) * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s);
          (void)hipStreamSynchronize(s);
          bool all = true;
          for (const MatDesc& d : w.tall_host) all = all && doi->host_done[d.blk] != 0;
          wave_stopped = all;
        }
        continue;
      }
      // Rayleigh-Ritz: A = Rinv^T H Rinv = Z Theta Z^T,  V = Y Rinv Z
      chol(nullptr);
      if (rec && last) {
        keep_mats(rec->Rrr, Rinv, true);
        keep_slab(rec->Y, Y);
      }
      {
        KScope k_(a.tm, MI_K_ROWMUL_SMALL, s);
        launch_rowmul<double, double>(w.rts, w.n_rts, w.small, H, w.small, Rinv, w.small, T1,
                                      w.nchs, s, true);
      }
      {
        // p x p: never split over rows
        KScope k_(a.tm, MI_K_GRAM_SMALL, s);
        launch_gram_direct<double>(w.gts, w.n_gts, w.small, w.small, Rinv, T1, nullptr, Am,
                                   nullptr, s);
      }
      const bool use_tri = prm.eig == MI_EIG_TRIDIAG && tri_eig_supported(w.max_ld);
      if (use_tri) {
        // Householder tridiagonalisation, multisection, inverse iteration;
        // Z / T1 / S64 double as per-thread scratch before Z is written
        {
          KScope k_(a.tm, MI_K_EIG_REDUCE, s);
          launch_tri_reduce(w.sd, w.nb, w.max_ld, Am, Wk, tri, a.status, s);
        }
        {
          KScope k_(a.tm, MI_K_EIG_VALUES, s);
          launch_tri_bisect(w.sd, w.nb, w.max_p, tri, ritz_w, perm, a_lo, prm.adapt, a.status, s);
        }
        {
          KScope k_(a.tm, MI_K_EIG_VECTORS, s);
          launch_tri_vectors(w.sd, w.nb, w.max_p, tri, Z, T1, S64, a.status, s);
        }
        {
          KScope k_(a.tm, MI_K_EIG_BACK, s);
          launch_tri_back(w.sd, w.nb, w.max_ld, S64, Wk, tri, Z, s);
        }
        if (rec && last) keep_mats(rec->Z, Z, true);
      } else {
        {
          KScope k_(a.tm, MI_K_JACOBI_INIT, s);
          launch_jacobi_init(w.sd, w.nb, Am, pk, Z, conv, s);
        }
        // the last iteration gets the requested tolerance; intermediate ones
        // (rr_every) only need a roughly Ritz-ordered basis of the span
        const double jtol = last ? prm.jacobi_tol : std::max(prm.jacobi_tol, 1e-8);
        for (int sw = 0; sw < prm.max_sweeps; ++sw) {
          {
            KScope k_(a.tm, MI_K_JACOBI_SWEEP, s);
            launch_jacobi_sweep(w.sd, w.nb, pk, lg, conv, jtol, jac_lds, lds_jac_use, s);
          }
          {
            KScope k_(a.tm, MI_K_APPLY_ROT, s);
            launch_apply_rot(w.sd, w.nb, w.max_q, lg, conv, Z, P.lds_max, s);
          }
        }
        {
          KScope k_(a.tm, MI_K_RR_FINISH, s);
          launch_rr_finish(w.sd, w.nb, pk, conv, ritz_w, perm, a_lo, prm.adapt, a.status,
                           std::max(1e-10, 10.0 * jtol), s);
        }
      }
      if (use_tri) {
        // already in ascending Ritz order: S = Rinv Z straight into the
        // operand of the row product (FP32 copy for FP32 slabs)
        KScope k_(a.tm, MI_K_ROWMUL_SMALL, s);
        if (dbl)
          launch_rowmul<double, double>(w.rts, w.n_rts, w.small, Rinv, w.small, Z, w.small, T1,
                                        w.nchs, s);
        else
          launch_rowmul<double, double>(w.rts, w.n_rts, w.small, Rinv, w.small, Z, w.small, S32,
                                       w.nchs, s);
      } else {
        {
          KScope k_(a.tm, MI_K_ROWMUL_SMALL, s);
          launch_rowmul<double, double>(w.rts, w.n_rts, w.small, Rinv, w.small, Z, w.small, S64,
                                        w.nchs, s);
        }
        // S <- columns of Rinv Z in ascending Ritz order (FP32 copy for FP32 products)
        KScope k_(a.tm, MI_K_PERM_CAST, s);
        launch_perm_cast(w.sd, w.nb, S64, perm, dbl ? nullptr : S32, dbl ? T1 : nullptr, s);
      }
      const TS* Sm = dbl ? reinterpret_cast<const TS*>(T1) : reinterpret_cast<const TS*>(S32);
      int dslab = -1;
      for (int i = 0; i < 4; ++i)
        if (i != ycur) dslab = i;
      if (!fin) {
        // an intermediate Rayleigh-Ritz step (rr_every): the rotated basis
        // is the next iteration's start
        KScope k_(a.tm, MI_K_ROWMUL, s);
        if constexpr (same) {
          launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, Y, w.small, Sm, w.tall, V, w.nch, s);
          X = V;
          xslab = -1;
        } else {
          launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, Y, w.small, Sm, w.tall, slab[dslab], w.nch,
                               s);
          X = slab[dslab];
          xslab = dslab;
        }
      } else {
        T* dstV = slab[dslab];
        {
          KScope k_(a.tm, MI_K_ROWMUL, s);
          launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, Y, w.small, Sm, w.tall, dstV, w.nch, s);
        }
        // final Cholesky-QR: V = Vtmp R^-1 (upper triangular: keeps the span of
        // every leading column set, hence the Ritz order)
        gram(dstV, nullptr, G, nullptr);
        chol(dbl ? nullptr : S32);
        {
          KScope k_(a.tm, MI_K_ROWMUL, s);
          launch_rowmul<T, TS>(w.rt, w.n_rt, w.tall, dstV, w.small,
                               dbl ? reinterpret_cast<const TS*>(Rinv)
                                   : reinterpret_cast<const TS*>(S32),
                               w.tall, V, w.nch, s, true);
        }
        if constexpr (same) {
          X = V;
          xslab = -1;
        }
        if constexpr (same) if (tolm) {
          // residuals of the new Ritz pairs, the test, and the copy-out of the
          // blocks that converge now (or reach the cap)
          {
            KScope k_(a.tm, MI_K_SETUP, s);
            hipLaunchKernelGGL(k_resid_tile<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                               w.csr, P.info, P.tile_base, L.cg_ldp, a.row_ptr, a.col, a.val,
                               (const T*)V, (const double*)ritz_w, rpart);
            hipLaunchKernelGGL(k_tol_check, dim3(w.nb), dim3(256), 0, s, w.tall, P.info,
                               P.tile_base, L.cg_ldp, (const double*)rpart, resid_w,
                               (const double*)ritz_w, prm.tol, t, last ? 1 : 0, frozen, fnow,
                               a.ritz, a.resid, a.iters, a.status);
            hipLaunchKernelGGL(k_freeze_rows<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                               (const int32_t*)fnow, (const T*)V, Vout);
          }
        }
      }
    }
    if (doi) {
      // the frozen bases become the wave's output (and the next waves' start)
      if (doi->t_max > 0) {
        KScope k_(a.tm, MI_K_SETUP, s);
        hipLaunchKernelGGL(k_copy_slab<TV>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                           (const TV*)Vf, V);
      }
    } else if (w.T == 0) {
      // no iteration: the start itself (after its Cholesky-QR for predecessor
      // and seeded starts) is the result
      KScope k_(a.tm, MI_K_SETUP, s);
      if (!start_in_v && static_cast<const void*>(X) != static_cast<const void*>(Vout))
        hipLaunchKernelGGL((k_copy_slab<T, TV>), dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                           X, Vout);
      if (a.iters)
        hipLaunchKernelGGL(k_resid_final, dim3(w.nb), dim3(256), 0, s, w.tall, P.info,
                           P.tile_base, L.cg_ldp, (const double*)rpart, (double*)nullptr, 0,
                           a.iters);
    } else if (!tolm && (a.resid || a.iters)) {
      KScope k_(a.tm, MI_K_SETUP, s);
      if (a.resid)
        hipLaunchKernelGGL(k_resid_tile<TV>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall,
                           w.csr, P.info, P.tile_base, L.cg_ldp, a.row_ptr, a.col, a.val,
                           (const TV*)Vout, (const double*)a.ritz, rpart);
      hipLaunchKernelGGL(k_resid_final, dim3(w.nb), dim3(256), 0, s, w.tall, P.info, P.tile_base,
                         L.cg_ldp, (const double*)rpart, a.resid, w.T, a.iters);
    }
  }
  if (doi) {
    KScope k_(a.tm, MI_K_DOI, s_main);
    hipLaunchKernelGGL(k_doi_status, dim3(ceil_div(B, 256)), dim3(256), 0, s_main, B, a.status);
  }
  if (fork) {
    for (int l = 0; l < P.n_lanes; ++l) {
      (void)hipEventRecord(P.lane_ev[l], P.lane_s[l]);
      (void)hipStreamWaitEvent(s, P.lane_ev[l], 0);
    }
  }
}

static bool same_key(const OiPlan& P, const HostBlocks& hb, const std::vector<int64_t>& nnz,
                     const mi_oi_params& prm, const std::vector<const void*>& ptrs,
                     size_t ws_bytes, bool per_block) {
  return P.per_block == per_block && P.hb.v_off == hb.v_off && P.hb.u_off == hb.u_off &&
         P.hb.p == hb.p && P.hb.ld == hb.ld && P.hb.pred == hb.pred && P.hb.c == hb.c &&
         P.nnz_off == nnz &&
         memcmp(&P.prm, &prm, sizeof(prm)) == 0 && P.ptrs == ptrs && P.ws_bytes == ws_bytes;
}

static mi_status check_params(const mi_oi_params* prm) {
  MI_CHECK_ARG(prm != nullptr, "params are NULL");
  MI_CHECK_ARG(prm->precision == MI_FP32 || prm->precision == MI_FP64 ||
                   prm->precision == MI_BF16_IN,
               "precision %d unsupported", prm->precision);
  MI_CHECK_ARG(prm->precision != MI_BF16_IN || (prm->op == MI_OP_CHEB && prm->tol == 0),
               "MI_BF16_IN supports the Chebyshev filter with fixed iteration counts only");
  MI_CHECK_ARG(prm->warm == MI_WARM_GIVEN || prm->warm == MI_WARM_PRED || prm->warm == MI_RANDOM,
               "warm mode %d unknown", prm->warm);
  MI_CHECK_ARG(prm->tol >= 0 && prm->tol < 1, "tol must be in [0, 1)");
  MI_CHECK_ARG(prm->tol == 0 || (prm->T >= 1 && prm->T0 >= 1),
               "the tolerance mode needs T, T0 >= 1 (the iteration caps)");
  MI_CHECK_ARG(prm->T >= 0 && prm->T0 >= 0 && prm->T <= 1000 && prm->T0 <= 1000, "T out of range");
  MI_CHECK_ARG(prm->m >= 1 && prm->m0 >= 1 && prm->m <= 256 && prm->m0 <= 256, "m out of range");
  MI_CHECK_ARG(prm->passes >= 1 && prm->passes0 >= 1, "passes must be >= 1");
  MI_CHECK_ARG(prm->max_sweeps >= 1 && prm->max_sweeps <= 100, "max_sweeps out of range");
  MI_CHECK_ARG(prm->a_mode >= 0 && prm->a_mode <= 2, "a_mode unknown");
  MI_CHECK_ARG(prm->rr_every == 0 || prm->rr_every == 1, "rr_every must be 0 or 1");
  MI_CHECK_ARG(prm->eig == MI_EIG_TRIDIAG || prm->eig == MI_EIG_JACOBI, "eig solver %d unknown",
               prm->eig);
  MI_CHECK_ARG(prm->jacobi_tol > 0 && prm->jacobi_tol < 1e-3, "jacobi_tol out of range");
  MI_CHECK_ARG(prm->autotune == 0 || prm->autotune == 1, "autotune must be 0 or 1");
  MI_CHECK_ARG(prm->op == MI_OP_CHEB || prm->op == MI_OP_RZ, "operator %d unknown", prm->op);
  if (prm->op == MI_OP_RZ) {
    MI_CHECK_ARG(prm->z >= 1 && prm->z <= 16, "z %d outside [1, 16]", prm->z);
    MI_CHECK_ARG(prm->cg_iters >= 1 && prm->cg_iters <= 100000, "cg_iters out of range");
    MI_CHECK_ARG(prm->delta > 0, "delta must be > 0");
  }
  return MI_OK;
}

// Dynamic LDS available to the small kernels: the per-workgroup maximum
// (160 KB on gfx950) less a margin for their static shared variables.
static int device_lds_max(int dev) {
  int v = 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    v = 65536;
  return v - 2048;
}

// The plan cached in *slot for this key, (re)built when the key changed.
static mi_status get_plan(mi_ctx* ctx, void** slot, const HostBlocks& hb,
                          const std::vector<int64_t>& nnz, const mi_oi_params& prm,
                          const std::vector<const void*>& ptrs, void* ws, size_t ws_bytes,
                          bool per_block, OiPlan** out) {
  OiPlan* P = static_cast<OiPlan*>(*slot);
  if (!P || !same_key(*P, hb, nnz, prm, ptrs, ws_bytes, per_block) ||
      P->spmm_force != ctx->spmm_force) {
    delete P;
    *slot = nullptr;
    std::unique_ptr<OiPlan> np;
    size_t need = 0;
    mi_status st = make_plan(hb, nnz, prm, per_block, device_lds_max(ctx->device),
                             ctx->spmm_force, &np, &need);
    if (st) return st;
    if (!ws || ws_bytes < need) {
      set_error("workspace %zu bytes < %zu required", ws_bytes, need);
      return MI_ERR_WORKSPACE;
    }
    if (prm.autotune) {
      if (!np->cap_stream)
        MI_TRY_HIP(hipStreamCreateWithFlags(&np->cap_stream, hipStreamNonBlocking));
      std::vector<WaveTune> tune;
      const int32_t* rp = static_cast<const int32_t*>(ptrs[0]);
      const int32_t* cl = static_cast<const int32_t*>(ptrs[1]);
      const float* vl = static_cast<const float*>(ptrs[2]);
      char* wsc = static_cast<char*>(ws);
      if (prm.precision == MI_FP64)
        autotune_waves<double>(*np, wsc, np->cap_stream, rp, cl, vl, &tune);
      else if (prm.precision == MI_BF16_IN)
        autotune_waves<bf16>(*np, wsc, np->cap_stream, rp, cl, vl, &tune);
      else
        autotune_waves<float>(*np, wsc, np->cap_stream, rp, cl, vl, &tune);
      MI_TRY_HIP(hipGetLastError());
      MI_TRY_HIP(hipStreamSynchronize(np->cap_stream));
      std::unique_ptr<OiPlan> tp;
      st = make_plan(hb, nnz, prm, per_block, device_lds_max(ctx->device), ctx->spmm_force, &tp,
                     &need, &tune);
      if (st) return st;
      tp->cap_stream = np->cap_stream;
      np->cap_stream = nullptr;
      np = std::move(tp);
    }
    np->ptrs = ptrs;
    np->ws_bytes = ws_bytes;
    P = np.release();
    *slot = P;
  }
  *out = P;
  return MI_OK;
}

mi_status oi_check_params(const mi_oi_params* prm) { return check_params(prm); }

size_t oi_ws_bytes(const HostBlocks& hb, const mi_oi_params& prm) {
  std::vector<std::vector<int>> waves;
  std::vector<int> level;
  int n_lanes = 1;
  if (build_waves(hb, prm, false, &waves, &level, nullptr, &n_lanes)) return 0;
  // the Gram partial buffer is sized for the largest wave
  size_t part_max = 0;
  std::vector<int64_t> pk_off(hb.B, 0), log_off(hb.B, 0), nnz(hb.B + 1, 0);
  for (auto& w : waves) {
    WaveTables wt;
    WaveHost h;
    wave_host(hb, nnz, w, prm, &wt, &h, pk_off, log_off);
    part_max = std::max(part_max, h.gt.size() * 2 * GRAM_TILE * GRAM_TILE);
    part_max = std::max(part_max, h.gts.size() * 2 * GRAM_TILE * GRAM_TILE);
    if (prm.autotune) part_max = std::max(part_max, tuned_part_max(h.tall));
  }
  return ws_layout(hb, prm, part_max, n_lanes).total;
}

mi_status oi_run_plan(mi_ctx* ctx, void** slot, const HostBlocks& hb,
                      const std::vector<int64_t>& nnz, const mi_oi_params& prm,
                      const int32_t* row_ptr, const int32_t* col, const float* val,
                      const void* V0, void* V, double* ritz, int32_t* status, void* ws,
                      size_t ws_bytes, const OiRecord* rec, hipStream_t s, OiPlan** plan_out) {
  std::vector<const void*> ptrs = {row_ptr, col, val, V0, V, ritz, status, ws};
  OiPlan* P = nullptr;
  mi_status st = get_plan(ctx, slot, hb, nnz, prm, ptrs, ws, ws_bytes, false, &P);
  if (st) return st;
  Args a{row_ptr, col, val, V0, V, ritz, status, static_cast<char*>(ws), ctx->timer, rec, false};
  if (prm.precision == MI_FP64)
    enqueue<double>(*P, a, s);
  else
    enqueue<float>(*P, a, s);
  MI_TRY_HIP(hipGetLastError());
  if (plan_out) *plan_out = P;
  return MI_OK;
}

static mi_status oi_run(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                        const int32_t* row_ptr, const int32_t* col, const float* val,
                        const int64_t* nnz_off, const void* V0, void* V, double* ritz,
                        double* resid, int32_t* iters, int32_t* status, void* ws,
                        size_t ws_bytes, void* stream, bool per_block) {
  begin_call();
  MI_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  mi_status st = check_params(prm);
  if (st) return st;
  HostBlocks hb;
  st = load_blocks(blk, &hb, true);
  if (st) return st;
  MI_CHECK_ARG(row_ptr && col && val && nnz_off && V && ritz && status, "NULL argument");
  std::vector<int64_t> nnz(nnz_off, nnz_off + hb.B + 1);
  bool needs_v0 = prm->warm == MI_WARM_GIVEN;
  for (int b = 0; b < hb.B; ++b) needs_v0 = needs_v0 || (prm->warm == MI_WARM_PRED && hb.pred[b] < 0);
  MI_CHECK_ARG(!needs_v0 || V0 != nullptr, "V0 is required");
  MI_CHECK_ARG(prm->tol == 0 || resid != nullptr, "the tolerance mode needs resid");
  if (prm->warm == MI_RANDOM)
    for (int b = 0; b < hb.B; ++b)
      MI_CHECK_ARG(b < (1 << 24) && hb.p[b] <= 4096 &&
                       hb.v_off[b + 1] - hb.v_off[b] <= (int64_t(1) << 28),
                   "MI_RANDOM covers b < 2^24, p_b <= 4096, n_b <= 2^28");
  MI_TRY_HIP(hipSetDevice(ctx->device));
  std::vector<const void*> ptrs = {row_ptr, col, val, V0, V, ritz, resid, iters, status, ws};
  OiPlan* P = nullptr;
  st = get_plan(ctx, &ctx->oi_plan, hb, nnz, *prm, ptrs, ws, ws_bytes, per_block, &P);
  if (st) return st;
  Args a{row_ptr, col, val, V0, V, ritz, status, static_cast<char*>(ws), ctx->timer, nullptr,
         false};
  a.resid = resid;
  a.iters = iters;
  hipStream_t s = (hipStream_t)stream;
  if (per_block || ctx->timer) {
    if (prm->precision == MI_FP64)
      enqueue<double>(*P, a, s);
    else if (prm->precision == MI_BF16_IN)
      enqueue<bf16, float>(*P, a, s);
    else
      enqueue<float>(*P, a, s);
    MI_TRY_HIP(hipGetLastError());
    return MI_OK;
  }
  if (!P->exec) {
    if (!P->cap_stream) MI_TRY_HIP(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    if (P->n_lanes > 1 && P->lane_s.empty()) {
      MI_TRY_HIP(hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming));
      for (int l = 0; l < P->n_lanes; ++l) {
        hipStream_t ls = nullptr;
        hipEvent_t le = nullptr;
        MI_TRY_HIP(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking));
        P->lane_s.push_back(ls);
        MI_TRY_HIP(hipEventCreateWithFlags(&le, hipEventDisableTiming));
        P->lane_ev.push_back(le);
      }
    }
    a.fork = true;
    MI_TRY_HIP(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    if (prm->precision == MI_FP64)
      enqueue<double>(*P, a, P->cap_stream);
    else if (prm->precision == MI_BF16_IN)
      enqueue<bf16, float>(*P, a, P->cap_stream);
    else
      enqueue<float>(*P, a, P->cap_stream);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamEndCapture(P->cap_stream, &P->graph);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      set_error("graph capture failed: %s / %s", hipGetErrorString(e1), hipGetErrorString(e2));
      return MI_ERR_HIP;
    }
    MI_TRY_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
  }
  MI_TRY_HIP(hipGraphLaunch(P->exec, s));
  return MI_OK;
}

// Workspace of the walk: the plan's layout, then the frozen bases (one slab)
// and the stop flags.
static void doi_layout(const HostBlocks& hb, const mi_oi_params& prm, size_t* off_vf,
                       size_t* off_done, size_t* total) {
  const size_t es = prm.precision == MI_FP64 ? 8 : 4;
  *off_vf = align_up(oi_ws_bytes(hb, prm));
  *off_done = *off_vf + align_up(size_t(hb.u_off[hb.B]) * es);
  *total = *off_done + align_up(size_t(std::max(hb.B, 1)) * sizeof(int32_t));
}

static mi_status doi_check(const HostBlocks& hb, const mi_oi_params* prm, const mi_doi_params* dp) {
  MI_CHECK_ARG(dp != nullptr, "walk parameters are NULL");
  MI_CHECK_ARG(prm->precision != MI_BF16_IN, "the dynamic walk supports MI_FP32 and MI_FP64");
  MI_CHECK_ARG(dp->eps_l >= 0 && dp->eps_h >= dp->eps_l, "need 0 <= eps_l <= eps_h");
  MI_CHECK_ARG(dp->t_max >= 0 && dp->t_max <= 10000, "t_max %d out of range", dp->t_max);
  MI_CHECK_ARG(dp->c_max >= 1, "c_max must be >= 1");
  MI_CHECK_ARG(prm->a_mode != MI_A_RITZ, "the walk takes no Ritz values: a_mode RITZ unsupported");
  MI_CHECK_ARG(prm->warm != MI_RANDOM && prm->tol == 0,
               "the walk takes given or predecessor starts and no tolerance (it has its own rule)");
  for (int b = 0; b < hb.B; ++b)
    MI_CHECK_ARG(hb.ld[b] <= DOI_MAX_LD, "block %d: ld %d above %d", b, hb.ld[b], DOI_MAX_LD);
  return MI_OK;
}

}  // namespace mis

using namespace mis;

extern "C" {

void mis_destroy_oi_plan(mi_ctx* ctx) {
  delete static_cast<OiPlan*>(ctx->oi_plan);
  ctx->oi_plan = nullptr;
  delete static_cast<OiPlan*>(ctx->doi_plan);
  ctx->doi_plan = nullptr;
  delete static_cast<OiPlan*>(ctx->adj_oi);
  ctx->adj_oi = nullptr;
}

mi_status mi_oi_workspace_size(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                               size_t* ws_bytes) {
  clear_error();
  MI_CHECK_ARG(ws_bytes != nullptr, "ws_bytes is NULL");
  (void)ctx;
  mi_status st = check_params(prm);
  if (st) return st;
  HostBlocks hb;
  st = load_blocks(blk, &hb, true);
  if (st) return st;
  std::vector<std::vector<int>> waves;
  std::vector<int> level;
  st = build_waves(hb, *prm, false, &waves, &level);
  if (st) return st;
  *ws_bytes = oi_ws_bytes(hb, *prm);
  return MI_OK;
}

mi_status mi_oi_tuning(mi_ctx* ctx, int32_t* out, int32_t cap, int32_t* n_waves) {
  clear_error();
  MI_CHECK_ARG(ctx && n_waves && (out || cap == 0) && cap >= 0, "NULL argument");
  const OiPlan* P = static_cast<const OiPlan*>(ctx->oi_plan);
  MI_CHECK_ARG(P != nullptr, "no tracking plan yet (call mi_oi_track first)");
  *n_waves = (int32_t)P->waves.size();
  for (int w = 0; w < (int)P->waves.size() && w < cap; ++w) {
    out[4 * w] = P->waves[w].gram_target;
    out[4 * w + 1] = P->waves[w].nch;
    out[4 * w + 2] = P->waves[w].epl;
    out[4 * w + 3] = P->waves[w].spmm_var;
  }
  return MI_OK;
}

mi_status mi_oi_track(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                      const int32_t* row_ptr, const int32_t* col, const float* val,
                      const int64_t* nnz_off, const void* V0, void* V, double* ritz,
                      double* resid, int32_t* iters, int32_t* status, void* ws,
                      size_t ws_bytes, void* stream) {
  return oi_run(ctx, blk, prm, row_ptr, col, val, nnz_off, V0, V, ritz, resid, iters, status, ws,
                ws_bytes, stream, false);
}

mi_status mi_doi_workspace_size(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                                const mi_doi_params* dp, size_t* ws_bytes) {
  clear_error();
  (void)ctx;
  MI_CHECK_ARG(ws_bytes != nullptr, "ws_bytes is NULL");
  mi_status st = check_params(prm);
  if (st) return st;
  HostBlocks hb;
  st = load_blocks(blk, &hb, true);
  if (st) return st;
  st = doi_check(hb, prm, dp);
  if (st) return st;
  std::vector<std::vector<int>> waves;
  std::vector<int> level;
  st = build_waves(hb, *prm, false, &waves, &level);
  if (st) return st;
  size_t a, b;
  doi_layout(hb, *prm, &a, &b, ws_bytes);
  return MI_OK;
}

mi_status mi_doi_track(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                       const mi_doi_params* dp, const int32_t* row_ptr, const int32_t* col,
                       const float* val, const int64_t* nnz_off, const float* X, const void* V0,
                       void* V, int32_t* c, double* traj, int32_t* iters, int32_t* status,
                       void* ws, size_t ws_bytes, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  mi_status st = check_params(prm);
  if (st) return st;
  HostBlocks hb;
  st = load_blocks(blk, &hb, true);
  if (st) return st;
  st = doi_check(hb, prm, dp);
  if (st) return st;
  MI_CHECK_ARG(row_ptr && col && val && nnz_off && X && V && c && iters && status,
               "NULL argument");
  MI_CHECK_ARG(dp->t_max == 0 || traj, "traj is required when t_max > 0");
  bool needs_v0 = prm->warm == MI_WARM_GIVEN;
  for (int b = 0; b < hb.B; ++b) needs_v0 = needs_v0 || hb.pred[b] < 0;
  MI_CHECK_ARG(!needs_v0 || V0 != nullptr, "V0 is required");
  MI_CHECK_ARG(V0 != V, "V0 and V must not alias (the walk edits V in place)");
  size_t off_vf, off_done, need;
  doi_layout(hb, *prm, &off_vf, &off_done, &need);
  MI_CHECK_ARG(ws && ws_bytes >= need, "workspace %zu bytes < %zu required", ws_bytes, need);
  std::vector<int64_t> nnz(nnz_off, nnz_off + hb.B + 1);
  MI_TRY_HIP(hipSetDevice(ctx->device));
  std::vector<const void*> ptrs = {row_ptr, col, val, V0, V, nullptr, status, ws};
  OiPlan* P = nullptr;
  st = get_plan(ctx, &ctx->doi_plan, hb, nnz, *prm, ptrs, ws, ws_bytes, false, &P);
  if (st) return st;
  DoiArgs d;
  d.X = X;
  d.c = c;
  d.traj = traj;
  d.iters = iters;
  d.eps_l = dp->eps_l;
  d.eps_h = dp->eps_h;
  d.c_max = dp->c_max;
  d.t_max = dp->t_max;
  d.off_vf = off_vf;
  d.off_done = off_done;
  MI_TRY_HIP(hipHostMalloc((void**)&d.host_done, size_t(std::max(hb.B, 1)) * sizeof(int32_t)));
  Args a{row_ptr, col, val, V0, V, nullptr, status, static_cast<char*>(ws), ctx->timer, nullptr,
         false, &d};
  hipStream_t s = (hipStream_t)stream;
  if (prm->precision == MI_FP64)
    enqueue<double>(*P, a, s);
  else
    enqueue<float>(*P, a, s);
  const hipError_t e = hipGetLastError();
  (void)hipStreamSynchronize(s);  // the last read of host_done is complete
  (void)hipHostFree(d.host_done);
  if (e != hipSuccess) {
    set_error("HIP: %s", hipGetErrorString(e));
    return MI_ERR_HIP;
  }
  return MI_OK;
}

mi_status mi_oi_track_per_block(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                                const int32_t* row_ptr, const int32_t* col, const float* val,
                                const int64_t* nnz_off, const void* V0, void* V, double* ritz,
                                double* resid, int32_t* iters, int32_t* status, void* ws,
                                size_t ws_bytes, void* stream) {
  return oi_run(ctx, blk, prm, row_ptr, col, val, nnz_off, V0, V, ritz, resid, iters, status, ws,
                ws_bytes, stream, true);
}

}  // extern "C"
