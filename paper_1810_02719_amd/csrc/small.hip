// Small dense FP64 kernels, one workgroup per block (see small.hpp).
//
// Storage: symmetric / triangular p x p matrices are kept as a packed upper
// triangle, in LDS when it fits (p <= ~190 on gfx950's 160 KB) and in a
// per-block global scratch otherwise; the same code runs on either through a
// generic pointer.
#include "small.hpp"

namespace mis {

// Packed upper-triangle index (i <= j); q <= 1024 keeps it in 32 bits.
__device__ __forceinline__ int pidx(int i, int j, int q) { return i * q - ((i * (i + 1)) >> 1) + j; }

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Cholesky of the scaled Gram and the inverse factor for blocks wider than
// 320 (narrower ones use the MFMA kernel in chol.hip), with 32-wide panels, so that only the 32 x 32
// diagonal tiles are factored step by step (inside one wavefront, one tile
// column per lane in registers, pivots and row entries broadcast by
// shuffles); the panel solves, trailing updates and the blocked inverse are
// parallel phases separated by ~40 barriers in total.  The working matrix
// lives in global memory (L2-resident, ld x ld per block), the current panel
// in LDS when PLDS.  Diagonal tiles of the working matrix end up holding the
// inverted tiles X_JJ; afterwards the off-diagonal blocks of X = R^^-1 are
// formed column block by column block in place.
constexpr int CB = 32;

template <bool PLDS>
__global__ void __launch_bounds__(256)
    k_chol_blk(const SmallDesc* __restrict__ sds, const double* __restrict__ G,
               double* __restrict__ Wk, double* __restrict__ Rinv, float* __restrict__ S32,
               int32_t* __restrict__ status) {
  extern __shared__ double dyn[];  // PLDS: panel / product scratch, CB x ld
  __shared__ double dsc[1024];
  __shared__ double Xt[CB][CB + 1];
  __shared__ int flag;
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Gb = G + d.m_off;
  double* W = Wk + d.m_off;
  double* P;  // CB x ld scratch
  if constexpr (PLDS)
    P = dyn;
  else
    P = Rinv + d.m_off;  // rows 0..CB-1 of the output serve as scratch until the end
  const double piv_tol = 1e-13;
  if (tid == 0) flag = 0;
  __syncthreads();
  for (int i = tid; i < p; i += 256) {
    const double g = Gb[int64_t(i) * ld + i];
    if (!isfinite(g)) atomicOr(&flag, MI_BLOCK_NONFINITE);
    if (!(g > 0.0)) atomicOr(&flag, MI_BLOCK_NOT_PD);
    dsc[i] = (g > 0.0 && isfinite(g)) ? 1.0 / sqrt(g) : 0.0;
  }
  __syncthreads();
  for (int i = wave; i < p; i += 4) {
    const double di = dsc[i];
    for (int j = i + lane; j < p; j += 64)
      W[int64_t(i) * ld + j] = (i == j) ? 1.0 + 2e-13 : Gb[int64_t(i) * ld + j] * di * dsc[j];
  }
  __syncthreads();
  const int nbk = (p + CB - 1) / CB;
  for (int J = 0; J < nbk; ++J) {
    const int j0 = J * CB, jb = min(CB, p - j0), r0 = j0 + jb;
    // (a) factor the diagonal tile in wave 0: lane l holds tile column l
    if (wave == 0) {
      double c[CB];
#pragma unroll
      for (int i = 0; i < CB; ++i)
        c[i] = (lane < jb && i <= lane) ? W[int64_t(j0 + i) * ld + j0 + lane] : 0.0;
#pragma unroll
      for (int k = 0; k < CB; ++k) {
        if (k < jb) {
          double piv = __shfl(c[k], k, 64);
          if (!(piv > 2e-12)) {  // within ten diagonal shifts of zero: flag
            if (lane == 0) atomicOr(&flag, isfinite(piv) ? MI_BLOCK_SHIFTED : MI_BLOCK_NONFINITE);
            if (!(piv > piv_tol)) piv = piv_tol;
          }
          const double r = sqrt(piv), inv = 1.0 / r;
          if (lane == k)
            c[k] = r;
          else if (lane > k)
            c[k] *= inv;
#pragma unroll
          for (int i = k + 1; i < CB; ++i) {
            const double rki = __shfl(c[k], i, 64);
            if (lane >= i && i < jb) c[i] -= rki * c[k];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < CB; ++i)
        if (lane < CB) Xt[i][lane] = (lane < jb && i <= lane) ? c[i] : 0.0;  // R tile, upper
    }
    __syncthreads();
    // (b) invert the tile: thread l < jb back-substitutes column l of X_JJ
    //     into registers; all reads of R finish before the barrier, the
    //     writes follow it
    double xcol[CB];
#pragma unroll
    for (int i = 0; i < CB; ++i) xcol[i] = 0.0;
    if (tid < jb) {
      const int l = tid;
#pragma unroll
      for (int i = CB - 1; i >= 0; --i) {
        if (i == l) xcol[i] = 1.0 / Xt[l][l];
        if (i < l) {
          double acc = 0.0;
#pragma unroll
          for (int k = i + 1; k < CB; ++k)
            if (k <= l) acc += Xt[i][k] * xcol[k];
          xcol[i] = -acc / Xt[i][i];
        }
      }
    }
    __syncthreads();
    if (tid < CB) {
#pragma unroll
      for (int i = 0; i < CB; ++i) Xt[i][tid] = (tid < jb) ? xcol[i] : 0.0;
    }
    __syncthreads();
    // the working matrix's diagonal tile keeps X_JJ for the inverse phase
    for (int e = tid; e < jb * jb; e += 256) {
      const int i = e / jb, l = e % jb;
      if (i <= l) W[int64_t(j0 + i) * ld + j0 + l] = Xt[i][l];
    }
    // (c) panel solve R[J, j] = X_JJ^T W[J, j] for j >= r0, into P
    for (int e = tid; e < jb * (p - r0); e += 256) {
      const int i = e % jb, j = r0 + e / jb;
      double acc = 0.0;
      for (int k = 0; k <= i; ++k) acc += Xt[k][i] * W[int64_t(j0 + k) * ld + j];
      P[i * ld + j] = acc;
    }
    __syncthreads();
    for (int e = tid; e < jb * (p - r0); e += 256) {
      const int i = e / (p - r0), j = r0 + e % (p - r0);
      W[int64_t(j0 + i) * ld + j] = P[i * ld + j];
    }
    // (d) trailing update W[i][j] -= sum_k P[k][i] P[k][j], r0 <= i <= j < p,
    //     4 x 4 register tiles
    {
      const int m = p - r0;
      const int nt = (m + 3) / 4;
      for (int e = tid; e < nt * nt; e += 256) {
        const int ti = e / nt, tj = e % nt;
        if (tj < ti) continue;
        const int i0 = r0 + 4 * ti, c0 = r0 + 4 * tj;
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        for (int k = 0; k < jb; ++k) {
          double pi[4], pj[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            pi[a] = (i0 + a < p) ? P[k * ld + i0 + a] : 0.0;
            pj[a] = (c0 + a < p) ? P[k * ld + c0 + a] : 0.0;
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += pi[a] * pj[b];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int i = i0 + a, j = c0 + b;
            if (i < p && j < p && i <= j) W[int64_t(i) * ld + j] -= acc[a][b];
          }
      }
    }
    __syncthreads();
  }
  // blocked inverse: X[0:j0, J] = -(X[0:j0, 0:j0] R[0:j0, J]) X_JJ, in place
  for (int J = 1; J < nbk; ++J) {
    const int j0 = J * CB, jb = min(CB, p - j0);
    // M[i][k] = sum_{l=i}^{j0-1} X[i][l] R[l][j0+k]  (into P as [i * CB + k])
    for (int e = tid; e < j0 * jb; e += 256) {
      const int i = e / jb, k = e % jb;
      double acc = 0.0;
      for (int l = i; l < j0; ++l) acc += W[int64_t(i) * ld + l] * W[int64_t(l) * ld + j0 + k];
      P[i * CB + k] = acc;
    }
    __syncthreads();
    // X[i][j0+k] = -sum_{k' <= k} M[i][k'] X_JJ[k'][k]
    for (int e = tid; e < j0 * jb; e += 256) {
      const int i = e / jb, k = e % jb;
      double acc = 0.0;
      for (int k2 = 0; k2 <= k; ++k2) acc += P[i * CB + k2] * W[int64_t(j0 + k2) * ld + j0 + k];
      W[int64_t(i) * ld + j0 + k] = -acc;
    }
    __syncthreads();
  }
  double* Rb = Rinv + d.m_off;
  for (int i = wave; i < ld; i += 4) {
    const double di = i < p ? dsc[i] : 0.0;
    for (int j = lane; j < ld; j += 64) {
      double v = 0.0;
      if (i < p && j < p && i <= j) v = di * W[int64_t(i) * ld + j];
      Rb[int64_t(i) * ld + j] = v;
      if (S32) S32[d.m_off + int64_t(i) * ld + j] = (float)v;
    }
  }
  if (tid == 0 && flag) atomicOr(&status[d.blk], flag);
}


void launch_chol_blk(const SmallDesc* sd, int nb, const double* G, double* Wk, double* Rinv,
                     float* S32, int32_t* status, int max_ld, int lds_max, hipStream_t s) {
  if (nb <= 0) return;
  if (launch_chol_mfma(sd, nb, G, Wk, Rinv, S32, status, max_ld, s)) return;  // ld <= 320
  const size_t pl = size_t(CB) * max_ld * sizeof(double);
  if (pl <= size_t(lds_max) - 40000)
    hipLaunchKernelGGL(k_chol_blk<true>, dim3(nb), dim3(256), pl, s, sd, G, Wk, Rinv, S32, status);
  else
    hipLaunchKernelGGL(k_chol_blk<false>, dim3(nb), dim3(256), 0, s, sd, G, Wk, Rinv, S32, status);
}

// a[blk] = max_j (Rinv^T H Rinv)_jj = max_j sum_{i<=j} Rinv[i][j] T1[i][j] with
// T1 = H Rinv: the largest Rayleigh quotient of the Cholesky-QR basis (a
// lower estimate of the top Ritz value, used as the filter's lower bound).
__global__ void __launch_bounds__(1024)
    k_rq_max(const SmallDesc* __restrict__ sds, const double* __restrict__ Rinv,
             const double* __restrict__ T1, double* __restrict__ a_lo) {
  __shared__ double colsum[4][256];
  __shared__ double red[16];
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  const double* R = Rinv + d.m_off;
  const double* T = T1 + d.m_off;
  // thread (g, c): rows i = g, g + 4, ... of columns c, c + 256, ...; the
  // four row groups are added in a fixed order
  const int g = threadIdx.x >> 8, c = threadIdx.x & 255;
  double mx = -1e308;
  for (int j0 = 0; j0 < p; j0 += 256) {
    const int j = j0 + c;
    double s = 0.0;
    if (j < p) {
#pragma unroll 4
      for (int i = g; i <= j; i += 4) s = fma(R[int64_t(i) * ld + j], T[int64_t(i) * ld + j], s);
    }
    colsum[g][c] = s;
    __syncthreads();
    if (g == 0 && j < p) mx = fmax(mx, ((colsum[0][c] + colsum[1][c]) + colsum[2][c]) + colsum[3][c]);
    __syncthreads();
  }
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < 16; ++w) m = fmax(m, red[w]);
    a_lo[d.blk] = m;
  }
}

void launch_rq_max(const SmallDesc* sd, int nb, const double* Rinv, const double* T1,
                   double* a_lo, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_rq_max, dim3(nb), dim3(1024), 0, s, sd, Rinv, T1, a_lo);
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
// exactly one lane as J_K^T M J_K' (J = [[c, s], [-s, c]]), the diagonal pair
// blocks by the closed form that zeroes their off-diagonal entry.  Waves own
// pair rows K, lanes walk K' >= K (no integer division in the loop).
template <bool LDS>
__global__ void __launch_bounds__(SMALL_THREADS)
    k_jacobi_sweep(const SmallDesc* __restrict__ sds, double* __restrict__ pk,
                   double* __restrict__ logbuf, int32_t* __restrict__ conv, double tol) {
  extern __shared__ double smem[];
  __shared__ double red[SMALL_THREADS / 64];
  __shared__ double s_thresh;
  const SmallDesc d = sds[blockIdx.x];
  if (conv[d.blk]) return;
  const int q = d.q, h = q / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = SMALL_THREADS / 64;
  const int npk = (q * (q + 1)) / 2;
  double* rc = smem;
  double* rs = smem + h;
  double* rt = smem + 2 * h;
  int* pp = reinterpret_cast<int*>(smem + 3 * h);
  int* qq = pp + h;
  double* gP = pk + d.pk_off;
  double* A;
  if constexpr (LDS) {
    A = smem + 4 * h;
    for (int e = tid; e < npk; e += SMALL_THREADS) A[e] = gP[e];
  } else {
    A = gP;
  }
  __syncthreads();
  double f = 0.0;
  for (int i = wave; i < q; i += NW) {
    const int ri = pidx(i, 0, q);
    for (int j = i + lane; j < q; j += 64) {
      const double v = A[ri + j];
      f += (i == j) ? v * v : 2.0 * v * v;
    }
  }
  f = wave_sum(f);
  if (lane == 0) red[wave] = f;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w];
    s_thresh = tol * sqrt(t);
  }
  __syncthreads();
  const double thresh = s_thresh;
  double maxoff = 0.0;
  double* lg = logbuf + d.log_off;
  for (int r = 0; r < q - 1; ++r) {
    for (int k = tid; k < h; k += SMALL_THREADS) {
      const int a = rr_index(k, r, q), b = rr_index(q - 1 - k, r, q);
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
      lg[(r * h + k) * 2] = c;
      lg[(r * h + k) * 2 + 1] = s;
    }
    __syncthreads();
    // lanes own pair columns K2 (their rotation data stays in registers),
    // waves walk the pair rows K <= K2
    for (int K2b = 0; K2b < h; K2b += 64) {
      const int K2 = K2b + lane;
      const bool live2 = K2 < h;
      const double t2 = live2 ? rt[K2] : 0.0;
      const double c2 = live2 ? rc[K2] : 1.0, s2 = live2 ? rs[K2] : 0.0;
      const int y0 = live2 ? pp[K2] : 0, y1 = live2 ? qq[K2] : 0;
      for (int K = wave; K < min(h, K2b + 64); K += NW) {
        if (!live2 || K > K2) continue;
        const double t1 = rt[K];
        if (t1 == 0.0 && t2 == 0.0) continue;
        const int x0 = pp[K], x1 = qq[K];
        if (K2 == K) {
          const int i01 = pidx(x0, x1, q);
          const double apq = A[i01];
          A[pidx(x0, x0, q)] -= t1 * apq;
          A[pidx(x1, x1, q)] += t1 * apq;
          A[i01] = 0.0;
          continue;
        }
        const double c1 = rc[K], s1 = rs[K];
        const int i00 = x0 < y0 ? pidx(x0, y0, q) : pidx(y0, x0, q);
        const int i01 = x0 < y1 ? pidx(x0, y1, q) : pidx(y1, x0, q);
        const int i10 = x1 < y0 ? pidx(x1, y0, q) : pidx(y0, x1, q);
        const int i11 = x1 < y1 ? pidx(x1, y1, q) : pidx(y1, x1, q);
        const double m00 = A[i00], m01 = A[i01], m10 = A[i10], m11 = A[i11];
        const double n00 = c2 * m00 - s2 * m01, n01 = s2 * m00 + c2 * m01;
        const double n10 = c2 * m10 - s2 * m11, n11 = s2 * m10 + c2 * m11;
        A[i00] = c1 * n00 - s1 * n10;
        A[i10] = s1 * n00 + c1 * n10;
        A[i01] = c1 * n01 - s1 * n11;
        A[i11] = s1 * n01 + c1 * n11;
      }
    }
    __syncthreads();
  }
  maxoff = wave_max(maxoff);
  if (lane == 0) red[wave] = maxoff;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int w = 0; w < NW; ++w) mx = fmax(mx, red[w]);
    // a sweep that found nothing above the threshold rotated nothing
    if (!(mx > thresh)) conv[d.blk] = 1;
  }
  if constexpr (LDS)
    for (int e = tid; e < npk; e += SMALL_THREADS) gP[e] = A[e];
}

void launch_jacobi_sweep(const SmallDesc* sd, int nb, double* pk, double* log, int32_t* conv,
                         double tol, bool lds, size_t lds_bytes, hipStream_t s) {
  if (nb <= 0) return;
  if (lds)
    hipLaunchKernelGGL(k_jacobi_sweep<true>, dim3(nb), dim3(SMALL_THREADS), lds_bytes, s, sd, pk, log,
                       conv, tol);
  else
    hipLaunchKernelGGL(k_jacobi_sweep<false>, dim3(nb), dim3(SMALL_THREADS), lds_bytes, s, sd, pk,
                       log, conv, tol);
}

// Z <- Z J_1 ... J_R (the rotations of one sweep), zrows rows per
// workgroup (32, or fewer when q is large, to fit LDS).  The log is staged
// through LDS RCH rounds at a time with coalesced loads; lane groups of zrows
// threads share one rotation and apply it to their rows.
constexpr int RCH = 16;
__global__ void __launch_bounds__(256)
    k_apply_rot(const SmallDesc* __restrict__ sds, const double* __restrict__ logbuf,
                const int32_t* __restrict__ conv, double* __restrict__ Z, int groups_per_block,
                int ZROWS) {
  extern __shared__ double zs[];
  const int bi = blockIdx.x / groups_per_block, g = blockIdx.x % groups_per_block;
  const SmallDesc d = sds[bi];
  if (conv[d.blk]) return;
  const int q = d.q, h = q / 2, ld = d.ld;
  const int row0 = g * ZROWS;
  if (row0 >= q) return;
  const int nr = min(ZROWS, q - row0);
  const int zl = q + 1;
  double* lgs = zs + ZROWS * zl;  // RCH rounds of (c, s) pairs
  double* Zb = Z + d.m_off;
  for (int rr = threadIdx.x / 64; rr < nr; rr += 4)
    for (int cc = threadIdx.x % 64; cc < q; cc += 64)
      zs[rr * zl + cc] = Zb[int64_t(row0 + rr) * ld + cc];
  const double* lg = logbuf + d.log_off;
  const int rr = threadIdx.x % ZROWS, kg = threadIdx.x / ZROWS;
  const int KG = 256 / ZROWS;
  for (int r0 = 0; r0 < q - 1; r0 += RCH) {
    const int nch = min(RCH, q - 1 - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < nch * h * 2; e += 256) lgs[e] = lg[int64_t(r0) * h * 2 + e];
    __syncthreads();
    for (int rl = 0; rl < nch; ++rl) {
      const int r = r0 + rl;
      if (rr < nr) {
        for (int k = kg; k < h; k += KG) {
          const double s = lgs[(rl * h + k) * 2 + 1];
          if (s == 0.0) continue;
          const double c = lgs[(rl * h + k) * 2];
          const int a = rr_index(k, r, q), b = rr_index(q - 1 - k, r, q);
          const int lo = min(a, b), hi = max(a, b);
          const double x = zs[rr * zl + lo], y = zs[rr * zl + hi];
          zs[rr * zl + lo] = c * x - s * y;
          zs[rr * zl + hi] = s * x + c * y;
        }
      }
      __syncthreads();
    }
  }
  for (int r2 = threadIdx.x / 64; r2 < nr; r2 += 4)
    for (int cc = threadIdx.x % 64; cc < q; cc += 64)
      Zb[int64_t(row0 + r2) * ld + cc] = zs[r2 * zl + cc];
}

void launch_apply_rot(const SmallDesc* sd, int nb, int max_q, const double* log,
                      const int32_t* conv, double* Z, int lds_max, hipStream_t s) {
  if (nb <= 0) return;
  const size_t logb = size_t(RCH) * (max_q / 2) * 2 * sizeof(double);
  int zrows = 32;
  while (zrows > 1 && size_t(zrows) * (max_q + 1) * sizeof(double) + logb > size_t(lds_max))
    zrows /= 2;
  const int gpb = ceil_div(max_q, zrows);
  const size_t lds = size_t(zrows) * (max_q + 1) * sizeof(double) + logb;
  hipLaunchKernelGGL(k_apply_rot, dim3(nb * gpb), dim3(256), lds, s, sd, log, conv, Z, gpb, zrows);
}

// ------------------------------------------------------------------ Ritz ordering
__global__ void __launch_bounds__(1024)
    k_rr_finish(const SmallDesc* __restrict__ sds, const double* __restrict__ pk,
                const int32_t* __restrict__ conv, double* __restrict__ ritz,
                int32_t* __restrict__ perm, double* __restrict__ a_lo, int adapt,
                int32_t* __restrict__ status, double conv_tol) {
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
    if (!(o <= conv_tol * sqrt(f))) atomicOr(&status[d.blk], MI_BLOCK_NOCONV);
  }
}

void launch_rr_finish(const SmallDesc* sd, int nb, const double* pk, const int32_t* conv,
                      double* ritz, int32_t* perm, double* a_lo, int adapt, int32_t* status,
                      double conv_tol, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_rr_finish, dim3(nb), dim3(1024), 0, s, sd, pk, conv, ritz, perm, a_lo, adapt,
                     status, conv_tol);
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


