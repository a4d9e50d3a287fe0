// Small dense FP64 kernels, one workgroup per block (see small.hpp).
//
// Storage: symmetric / triangular p x p matrices are kept as a packed upper
// triangle, in LDS when it fits (p <= ~190 on gfx950's 160 KB) and in a
// per-block global scratch otherwise; the same code runs on either through a
// generic pointer.
#include "small.hpp"

namespace mis {

__device__ inline int64_t pidx(int i, int j, int q) {  // i <= j
  return int64_t(i) * q - (int64_t(i) * (i + 1)) / 2 + j;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// ------------------------------------------------------------------ Cholesky + inverse
// G -> column scaling D = diag(G)^-1/2, G^ = D G D = R^^T R^ (right-looking,
// pivots below piv_tol are raised to piv_tol and flagged), X = R^^-1 in
// place, Rinv = D X.
__global__ void __launch_bounds__(SMALL_THREADS)
    k_chol_inv(const SmallDesc* __restrict__ sds, const double* __restrict__ G,
               double* __restrict__ Rinv, float* __restrict__ S32, double* __restrict__ pks,
               int32_t* __restrict__ status, int use_lds) {
  extern __shared__ double smem[];
  __shared__ int flag;
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = SMALL_THREADS / 64;
  // dynamic LDS: [dsc | rdiag | tmp] (3 * pmax) then, in LDS mode, the packed factor
  double* dsc = smem;
  double* rdiag = smem + d.q;
  double* tmp = smem + 2 * d.q;
  double* W = use_lds ? smem + 3 * d.q : pks + d.pk_off;
  const double* Gb = G + d.m_off;
  const double piv_tol = 1e-13;
  if (tid == 0) flag = 0;
  __syncthreads();
  for (int i = tid; i < p; i += SMALL_THREADS) {
    const double g = Gb[int64_t(i) * ld + i];
    if (!isfinite(g)) atomicOr(&flag, MI_BLOCK_NONFINITE);
    if (!(g > 0.0)) atomicOr(&flag, MI_BLOCK_NOT_PD);
    dsc[i] = (g > 0.0 && isfinite(g)) ? 1.0 / sqrt(g) : 0.0;
  }
  __syncthreads();
  for (int i = wave; i < p; i += NW)
    for (int j = i + lane; j < p; j += 64)
      W[pidx(i, j, p)] = (i == j) ? 1.0 : Gb[int64_t(i) * ld + j] * dsc[i] * dsc[j];
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    double wkk = W[pidx(k, k, p)];
    if (!(wkk > piv_tol)) {
      if (tid == 0) atomicOr(&flag, isfinite(wkk) ? MI_BLOCK_SHIFTED : MI_BLOCK_NONFINITE);
      wkk = piv_tol;
    }
    const double rkk = sqrt(wkk), inv = 1.0 / rkk;
    if (tid == 0) rdiag[k] = rkk;
    for (int j = k + 1 + tid; j < p; j += SMALL_THREADS) W[pidx(k, j, p)] *= inv;
    __syncthreads();
    for (int i = k + 1 + wave; i < p; i += NW) {
      const double wki = W[pidx(k, i, p)];
      for (int j = i + lane; j < p; j += 64) W[pidx(i, j, p)] -= wki * W[pidx(k, j, p)];
    }
    __syncthreads();
  }
  // in-place inverse of the upper factor, column by column
  for (int j = 0; j < p; ++j) {
    const double xjj = 1.0 / rdiag[j];
    for (int i = wave; i < j; i += NW) {
      double acc = 0.0;
      for (int l = i + lane; l < j; l += 64) {
        const double xil = (l == i) ? W[pidx(i, i, p)] : W[pidx(i, l, p)];
        acc += xil * W[pidx(l, j, p)];
      }
      acc = wave_sum(acc);
      if (lane == 0) tmp[i] = acc;
    }
    __syncthreads();
    for (int i = tid; i < j; i += SMALL_THREADS) W[pidx(i, j, p)] = -tmp[i] * xjj;
    if (tid == 0) W[pidx(j, j, p)] = xjj;
    __syncthreads();
  }
  double* Rb = Rinv + d.m_off;
  for (int64_t e = tid; e < int64_t(ld) * ld; e += SMALL_THREADS) {
    const int i = int(e / ld), j = int(e % ld);
    double v = 0.0;
    if (i < p && j < p && i <= j) v = dsc[i] * W[pidx(i, j, p)];
    Rb[e] = v;
    if (S32) S32[d.m_off + e] = (float)v;
  }
  if (tid == 0 && flag) atomicOr(&status[d.blk], flag);
}

void launch_chol_inv(const SmallDesc* sd, int nb, const double* G, double* Rinv, float* S32,
                     double* pk_scratch, int32_t* status, bool lds, size_t lds_bytes,
                     hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_chol_inv, dim3(nb), dim3(SMALL_THREADS), lds_bytes, s, sd, G, Rinv, S32,
                     pk_scratch, status, lds ? 1 : 0);
}

// ------------------------------------------------------------------ Jacobi
__global__ void __launch_bounds__(256)
    k_jacobi_init(const SmallDesc* __restrict__ sds, const double* __restrict__ A,
                  double* __restrict__ pk, double* __restrict__ Z, int32_t* __restrict__ conv) {
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld, q = d.q;
  const double* Ab = A + d.m_off;
  double* P = pk + d.pk_off;
  for (int64_t e = threadIdx.x; e < int64_t(q) * q; e += 256) {
    const int i = int(e / q), j = int(e % q);
    if (i > j) continue;
    P[pidx(i, j, q)] = (i < p && j < p) ? Ab[int64_t(i) * ld + j] : 0.0;
  }
  double* Zb = Z + d.m_off;
  for (int64_t e = threadIdx.x; e < int64_t(ld) * ld; e += 256) {
    const int i = int(e / ld), j = int(e % ld);
    Zb[e] = (i == j && i < q) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) conv[d.blk] = 0;
}

void launch_jacobi_init(const SmallDesc* sd, int nb, const double* A, double* pk, double* Z,
                        int32_t* conv, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_jacobi_init, dim3(nb), dim3(256), 0, s, sd, A, pk, Z, conv);
}

// One sweep.  Round r pairs slot k with slot q-1-k of the circle
// arrangement; every 2x2 "pair block" A[{p_K,q_K},{p_K',q_K'}] is updated by
// exactly one thread as J_K^T M J_K' (J = [[c, s], [-s, c]]), the diagonal
// pair blocks by the closed form that zeroes their off-diagonal entry.
__global__ void __launch_bounds__(SMALL_THREADS)
    k_jacobi_sweep(const SmallDesc* __restrict__ sds, double* __restrict__ pk,
                   double* __restrict__ logbuf, int32_t* __restrict__ conv, double tol,
                   int use_lds) {
  extern __shared__ double smem[];
  __shared__ double red[SMALL_THREADS / 64];
  __shared__ double s_thresh;
  const SmallDesc d = sds[blockIdx.x];
  if (conv[d.blk]) return;
  const int q = d.q, h = q / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t npk = int64_t(q) * (q + 1) / 2;
  // dynamic LDS: rotation cosines, sines, tangents, pair indices, then (LDS
  // mode) the packed matrix
  double* rc = smem;
  double* rs = smem + h;
  double* rt = smem + 2 * h;
  int* pp = reinterpret_cast<int*>(smem + 3 * h);
  int* qq = pp + h;
  double* gP = pk + d.pk_off;
  double* A = use_lds ? smem + 3 * h + h : gP;
  if (use_lds)
    for (int64_t e = tid; e < npk; e += SMALL_THREADS) A[e] = gP[e];
  __syncthreads();
  // Frobenius norm of the packed symmetric matrix
  double f = 0.0;
  for (int i = wave; i < q; i += SMALL_THREADS / 64)
    for (int j = i + lane; j < q; j += 64) {
      const double v = A[pidx(i, j, q)];
      f += (i == j) ? v * v : 2.0 * v * v;
    }
  f = wave_sum(f);
  if (lane == 0) red[wave] = f;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < SMALL_THREADS / 64; ++w) t += red[w];
    s_thresh = tol * sqrt(t);
  }
  __syncthreads();
  const double thresh = s_thresh;
  double maxoff = 0.0;
  double* lg = logbuf + d.log_off;
  for (int r = 0; r < q - 1; ++r) {
    for (int k = tid; k < h; k += SMALL_THREADS) {
      int a = rr_index(k, r, q), b = rr_index(q - 1 - k, r, q);
      const int lo = min(a, b), hi = max(a, b);
      const double app = A[pidx(lo, lo, q)], aqq = A[pidx(hi, hi, q)], apq = A[pidx(lo, hi, q)];
      double c = 1.0, s = 0.0, t = 0.0;
      maxoff = fmax(maxoff, fabs(apq));
      if (fabs(apq) > thresh) {
        const double th = (aqq - app) / (2.0 * apq);
        t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
        c = 1.0 / sqrt(1.0 + t * t);
        s = t * c;
      }
      rc[k] = c;
      rs[k] = s;
      rt[k] = t;
      pp[k] = lo;
      qq[k] = hi;
      lg[(int64_t(r) * h + k) * 2] = c;
      lg[(int64_t(r) * h + k) * 2 + 1] = s;
    }
    __syncthreads();
    for (int e = tid; e < h * h; e += SMALL_THREADS) {
      const int K = e / h, K2 = e - K * h;
      if (K2 < K) continue;
      const double t1 = rt[K], t2 = rt[K2];
      if (t1 == 0.0 && t2 == 0.0) continue;
      if (K == K2) {
        const int lo = pp[K], hi = qq[K];
        const double apq = A[pidx(lo, hi, q)];
        A[pidx(lo, lo, q)] -= t1 * apq;
        A[pidx(hi, hi, q)] += t1 * apq;
        A[pidx(lo, hi, q)] = 0.0;
        continue;
      }
      const int x0 = pp[K], x1 = qq[K], y0 = pp[K2], y1 = qq[K2];
      const int64_t i00 = pidx(min(x0, y0), max(x0, y0), q), i01 = pidx(min(x0, y1), max(x0, y1), q);
      const int64_t i10 = pidx(min(x1, y0), max(x1, y0), q), i11 = pidx(min(x1, y1), max(x1, y1), q);
      const double m00 = A[i00], m01 = A[i01], m10 = A[i10], m11 = A[i11];
      const double c1 = rc[K], s1 = rs[K], c2 = rc[K2], s2 = rs[K2];
      const double n00 = c2 * m00 - s2 * m01, n01 = s2 * m00 + c2 * m01;
      const double n10 = c2 * m10 - s2 * m11, n11 = s2 * m10 + c2 * m11;
      A[i00] = c1 * n00 - s1 * n10;
      A[i10] = s1 * n00 + c1 * n10;
      A[i01] = c1 * n01 - s1 * n11;
      A[i11] = s1 * n01 + c1 * n11;
    }
    __syncthreads();
  }
  maxoff = wave_max(maxoff);
  if (lane == 0) red[wave] = maxoff;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int w = 0; w < SMALL_THREADS / 64; ++w) mx = fmax(mx, red[w]);
    // a sweep that found nothing above the threshold rotated nothing
    if (!(mx > thresh)) conv[d.blk] = 1;
  }
  if (use_lds)
    for (int64_t e = tid; e < npk; e += SMALL_THREADS) gP[e] = A[e];
}

void launch_jacobi_sweep(const SmallDesc* sd, int nb, double* pk, double* log, int32_t* conv,
                         double tol, bool lds, size_t lds_bytes, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_jacobi_sweep, dim3(nb), dim3(SMALL_THREADS), lds_bytes, s, sd, pk, log, conv,
                     tol, lds ? 1 : 0);
}

// Z <- Z J_1 ... J_R (the rotations of one sweep), ZROWS rows per workgroup.
constexpr int ZROWS = 8;
__global__ void __launch_bounds__(256)
    k_apply_rot(const SmallDesc* __restrict__ sds, const double* __restrict__ logbuf,
                const int32_t* __restrict__ conv, double* __restrict__ Z, int groups_per_block) {
  extern __shared__ double zs[];
  const int bi = blockIdx.x / groups_per_block, g = blockIdx.x % groups_per_block;
  const SmallDesc d = sds[bi];
  if (conv[d.blk]) return;
  const int q = d.q, h = q / 2, ld = d.ld;
  const int row0 = g * ZROWS;
  if (row0 >= q) return;
  const int nr = min(ZROWS, q - row0);
  const int zl = q + 1;
  double* Zb = Z + d.m_off;
  for (int e = threadIdx.x; e < nr * q; e += 256) {
    const int rr = e / q, cc = e % q;
    zs[rr * zl + cc] = Zb[int64_t(row0 + rr) * ld + cc];
  }
  __syncthreads();
  const double* lg = logbuf + d.log_off;
  for (int r = 0; r < q - 1; ++r) {
    for (int e = threadIdx.x; e < nr * h; e += 256) {
      const int rr = e / h, k = e % h;
      const double c = lg[(int64_t(r) * h + k) * 2], s = lg[(int64_t(r) * h + k) * 2 + 1];
      if (s == 0.0) continue;
      const int a = rr_index(k, r, q), b = rr_index(q - 1 - k, r, q);
      const int lo = min(a, b), hi = max(a, b);
      const double x = zs[rr * zl + lo], y = zs[rr * zl + hi];
      zs[rr * zl + lo] = c * x - s * y;
      zs[rr * zl + hi] = s * x + c * y;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nr * q; e += 256) {
    const int rr = e / q, cc = e % q;
    Zb[int64_t(row0 + rr) * ld + cc] = zs[rr * zl + cc];
  }
}

void launch_apply_rot(const SmallDesc* sd, int nb, int max_ld, const double* log,
                      const int32_t* conv, double* Z, hipStream_t s) {
  if (nb <= 0) return;
  const int gpb = ceil_div(max_ld, ZROWS);
  const size_t lds = size_t(ZROWS) * (max_ld + 1) * sizeof(double);
  hipLaunchKernelGGL(k_apply_rot, dim3(nb * gpb), dim3(256), lds, s, sd, log, conv, Z, gpb);
}

// ------------------------------------------------------------------ Ritz ordering
__global__ void __launch_bounds__(1024)
    k_rr_finish(const SmallDesc* __restrict__ sds, const double* __restrict__ pk,
                const int32_t* __restrict__ conv, double* __restrict__ ritz,
                int32_t* __restrict__ perm, double* __restrict__ a_lo, int adapt,
                int32_t* __restrict__ status) {
  __shared__ double th[1024];
  __shared__ double red[16];
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, q = d.q;
  const double* P = pk + d.pk_off;
  for (int i = threadIdx.x; i < p; i += 1024) th[i] = P[pidx(i, i, q)];
  __syncthreads();
  double mx = -1e308;
  for (int i = threadIdx.x; i < p; i += 1024) {
    const double v = th[i];
    int rank = 0;
    for (int j = 0; j < p; ++j) rank += (th[j] < v || (th[j] == v && j < i)) ? 1 : 0;
    perm[d.t_off + rank] = i;
    ritz[d.t_off + rank] = v;
    mx = fmax(mx, v);
  }
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = -1e308;
    for (int w = 0; w < 16; ++w) m = fmax(m, red[w]);
    if (adapt) a_lo[d.blk] = m;
  }
  // convergence: largest off-diagonal entry against the Frobenius norm
  double off = 0.0, fro = 0.0;
  for (int i = threadIdx.x >> 6; i < p; i += 16)
    for (int j = i + (threadIdx.x & 63); j < p; j += 64) {
      const double v = P[pidx(i, j, q)];
      fro += (i == j) ? v * v : 2.0 * v * v;
      if (i != j) off = fmax(off, fabs(v));
    }
  __syncthreads();
  fro = wave_sum(fro);
  off = wave_max(off);
  __shared__ double red2[32];
  if ((threadIdx.x & 63) == 0) {
    red2[threadIdx.x >> 6] = fro;
    red2[16 + (threadIdx.x >> 6)] = off;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double f = 0.0, o = 0.0;
    for (int w = 0; w < 16; ++w) {
      f += red2[w];
      o = fmax(o, red2[16 + w]);
    }
    if (!(o <= 1e-10 * sqrt(f))) atomicOr(&status[d.blk], MI_BLOCK_NOCONV);
  }
}

void launch_rr_finish(const SmallDesc* sd, int nb, const double* pk, const int32_t* conv,
                      double* ritz, int32_t* perm, double* a_lo, int adapt, int32_t* status,
                      hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_rr_finish, dim3(nb), dim3(1024), 0, s, sd, pk, conv, ritz, perm, a_lo, adapt,
                     status);
}

__global__ void __launch_bounds__(256)
    k_perm_cast(const SmallDesc* __restrict__ sds, const double* __restrict__ S64,
                const int32_t* __restrict__ perm, float* __restrict__ S32,
                double* __restrict__ S64out) {
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  const double* Sb = S64 + d.m_off;
  for (int64_t e = threadIdx.x; e < int64_t(ld) * ld; e += 256) {
    const int i = int(e / ld), j = int(e % ld);
    const double v = (j < p) ? Sb[int64_t(i) * ld + perm[d.t_off + j]] : 0.0;
    if (S32) S32[d.m_off + e] = (float)v;
    if (S64out) S64out[d.m_off + e] = v;
  }
}

void launch_perm_cast(const SmallDesc* sd, int nb, const double* S64, const int32_t* perm,
                      float* S32, double* S64out, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_perm_cast, dim3(nb), dim3(256), 0, s, sd, S64, perm, S32, S64out);
}

}  // namespace mis

namespace mis {
const void* k_chol_inv_ptr() { return reinterpret_cast<const void*>(&k_chol_inv); }
const void* k_jacobi_sweep_ptr() { return reinterpret_cast<const void*>(&k_jacobi_sweep); }
const void* k_apply_rot_ptr() { return reinterpret_cast<const void*>(&k_apply_rot); }
}  // namespace mis
