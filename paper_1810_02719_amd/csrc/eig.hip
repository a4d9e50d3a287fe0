// Symmetric eigen-decomposition of the Rayleigh-Ritz matrices A (p x p,
// FP64, p <= 320) of a wave of blocks, in four launches:
//
//   1. k_tri_reduce   Householder tridiagonalisation T = Q^T A Q, one
//                     workgroup per block with A resident in registers
//                     (k_tri_reduce_g with A in global memory above 192).
//   2. k_tri_bisect   every eigenvalue of T by Sturm-count multisection
//                     (ascending, so the Ritz order comes for free).
//   3. k_tri_vectors  eigenvectors of T: the twisted factorisation of
//                     T - lambda I for isolated eigenvalues, inverse iteration
//                     with Gram-Schmidt inside clusters of close eigenvalues.
//   4. k_tri_back     back-transformation Z = Q Z_T, rows of Z_T^T spread
//                     over several workgroups per block.
//
// The eigenvalue problem itself is textbook linear algebra (Householder
// reduction, Sturm sequences, inverse iteration); the method only needs the
// Ritz pairs of its projected matrix.
#include <cfloat>

#include "eig.hpp"

namespace mis {

namespace {

constexpr int TRI_MAXIT = 24;         // multisection rounds (52 bits need at most 17)
constexpr int TRI_VC = 16;            // reflectors staged per LDS chunk
constexpr double TRI_TN_MIN = 1e-290; // floor of the matrix scale
constexpr double TRI_CLUSTER = 1e-8;  // relative gap below which vectors are
                                      // orthogonalised against each other

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double swz_xor16(double v) {
  // ds_swizzle bit mode within 32 lanes: and 0x1f, or 0, xor 0x10
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
  return __hiloint2double(hi, lo);
}

// Sum over the 32 lanes of a half-wavefront, in every lane: DPP quad
// permutations and row mirrors inside each 16-lane row, one swizzle across
// the two rows (all lanes must be active).
__device__ __forceinline__ double half_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v + swz_xor16(v);
}

// Sum over the 16 lanes of a DPP row, in every lane of the row.
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_d<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);        // row_half_mirror
  return v + dpp_d<0x140>(v);  // row_mirror
}

// Sum of 32 doubles in LDS, in every lane of the wavefront: one LDS read per
// lane (lane l reads x[l % 32]) and a half-wavefront DPP reduction.
__device__ __forceinline__ double sum32(const double* x) {
  return half_sum(x[threadIdx.x & 31]);
}

// A value that every lane holds identically, moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Square root of a normal positive x: hardware reciprocal square root, one
// Goldschmidt step for sqrt(x) and 1/(2 sqrt(x)), one Newton correction.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return fma(fma(-g, g, x), h, g);
}

// 1 / b by the hardware reciprocal and one Newton step (b nonzero and
// finite: the pivots are guarded away from zero).
__device__ __forceinline__ double recip(double b) {
  const double r = __builtin_amdgcn_rcp(b);
  return fma(r, fma(-b, r, 1.0), r);
}

__device__ __forceinline__ double guard(double t, double floor_) {
  return fabs(t) < floor_ ? -floor_ : t;
}

// Scale of T and the Sturm-count pivot floor (identical in every launch that
// needs them, so every kernel sees the same numbers).
struct TriScale {
  double lo, hi, tn, pivmin;
};

__device__ TriScale tri_scale(const double* __restrict__ dd, const double* __restrict__ ee, int p,
                              double* red /* LDS, >= 3 * (blockDim / 64) */) {
  double lo = DBL_MAX, hi = -DBL_MAX, e2 = 0.0;
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    const double el = i > 0 ? fabs(ee[i - 1]) : 0.0;
    const double er = i + 1 < p ? fabs(ee[i]) : 0.0;
    lo = fmin(lo, dd[i] - el - er);
    hi = fmax(hi, dd[i] + el + er);
    e2 = fmax(e2, er * er);
  }
  for (int o = 32; o > 0; o >>= 1) {
    if (o >= (int)blockDim.x) continue;  // workgroups narrower than a wavefront
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    e2 = fmax(e2, __shfl_xor(e2, o, 64));
  }
  const int nw = (blockDim.x + 63) >> 6, wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[wv] = lo;
    red[nw + wv] = hi;
    red[2 * nw + wv] = e2;
  }
  __syncthreads();
  TriScale s;
  s.lo = red[0];
  s.hi = red[nw];
  e2 = red[2 * nw];
  for (int w = 1; w < nw; ++w) {
    s.lo = fmin(s.lo, red[w]);
    s.hi = fmax(s.hi, red[nw + w]);
    e2 = fmax(e2, red[2 * nw + w]);
  }
  s.tn = fmax(fmax(fabs(s.lo), fabs(s.hi)), TRI_TN_MIN);
  s.pivmin = DBL_MIN * fmax(1.0, e2);
  s.lo -= 2.0 * DBL_EPSILON * s.tn + 2.0 * s.pivmin;
  s.hi += 2.0 * DBL_EPSILON * s.tn + 2.0 * s.pivmin;
  return s;
}

__device__ __forceinline__ double hash_unit(int i, int j) {
  uint32_t h = uint32_t(i) * 0x9E3779B1u + uint32_t(j) * 0x85EBCA77u + 0x165667B1u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return double(h) * (1.0 / 2147483648.0) - 1.0;
}

}  // namespace

// ------------------------------------------------------------------ 1. reduction
// TRI_THREADS threads per block.  Thread (tr, tc) = (tid / 16, tid % 16) holds
// A[tr + 32a][tc + 16b] (a < RT, b < 2 RT) in registers, both triangles.
// Step k: the owners of column k publish it below the diagonal (LDS) with
// partial squared norms; everyone forms the reflector H_k = I - beta v v^T
// (v zero up to k, v_{k+1} = x_{k+1} - alpha, alpha = -sign(x_{k+1}) ||x||),
// computes p = beta A v with sums inside 16-lane DPP rows, and applies
// A -= v w^T + w v^T with w = p - (beta/2)(v^T p) v.  v and w vanish at and
// above k, so finished rows and columns keep their values.  The step loop is
// split by the number KB of finished 16-column blocks, so each loop skips them
// (and the finished 32-row blocks) at compile time.  Two barriers per step;
// the LDS vectors are double-buffered by step parity; v_k is stored as row k
// of Hv as soon as it is known.
constexpr int TRI_THREADS = 512;

template <int RT>
__device__ __forceinline__ void tri_publish(const double (&w)[RT][2 * RT], double (*xcol)[32 * RT],
                                            double (*part)[32], double* sdd, int k, int tr,
                                            int tc) {
  const int par = k & 1, kb = k >> 4, kt = k & 15;
  if (tc == kt) {
    double ss = 0.0;
#pragma unroll
    for (int b = 0; b < 2 * RT; ++b)
      if (b == kb) {  // uniform: selects the register column
#pragma unroll
        for (int a = 0; a < RT; ++a) {
          const int i = tr + 32 * a;
          const double x = w[a][b];
          if (i == k) sdd[k] = x;
          const double xi = i <= k ? 0.0 : x;
          xcol[par][i] = xi;
          ss = fma(xi, xi, ss);
        }
      }
    part[par][tr] = ss;
  }
  __syncthreads();
}

// Step k after column k is published; KB = (k + 1) / 16 finished column
// blocks, KB / 2 finished row blocks.
template <int RT, int KB>
__device__ __forceinline__ void tri_step(double (&w)[RT][2 * RT], double (*xcol)[32 * RT],
                                         double (*pcol)[32 * RT], double (*part)[32],
                                         double (*vpart)[32], double* see, double* sbb,
                                         double* Hb, int k, int ld, int tr, int tc) {
  constexpr int CB = 2 * RT, KA = KB / 2;
  const int par = k & 1, k1 = k + 1;
  const double ss = sum32(part[par]);
  const double x1 = xcol[par][k1];
  double vc[CB], vr[RT];
#pragma unroll
  for (int b = KB; b < CB; ++b) vc[b] = xcol[par][tc + 16 * b];
#pragma unroll
  for (int a = KA; a < RT; ++a) vr[a] = xcol[par][tr + 32 * a];
  double al, be;
  if (ss <= DBL_MIN) {
    al = x1;
    be = 0.0;
  } else {
    al = -copysign(sqrt_pos(ss), x1);
    be = recip(al * (al - x1));
  }
  al = uniform(al);
  be = uniform(be);
  // element k+1 of v lies in column block KB and row block KA
  vc[KB] -= tc == (k1 & 15) ? al : 0.0;
  vr[KA] -= tr == (k1 & 31) ? al : 0.0;
  double vp = 0.0;
#pragma unroll
  for (int a = KA; a < RT; ++a) {
    double sa = 0.0;
#pragma unroll
    for (int b = KB; b < CB; ++b) sa = fma(w[a][b], vc[b], sa);
    const double pa = be * row_sum16(sa);
    vp = fma(vr[a], pa, vp);
    const int i = tr + 32 * a;
    if (tc == 0) pcol[par][i] = i <= k ? 0.0 : pa;
  }
  if (tc == 0) vpart[par][tr] = vp;
  if (threadIdx.x == 0) {
    see[k] = al;
    sbb[k] = be;
  }
  if ((int)threadIdx.x < ld)
    Hb[int64_t(k) * ld + threadIdx.x] = xcol[par][threadIdx.x] - ((int)threadIdx.x == k1 ? al : 0.0);
  __syncthreads();
  const double K = uniform(0.5 * be * sum32(vpart[par]));
  double wc[CB];
#pragma unroll
  for (int b = KB; b < CB; ++b) wc[b] = fma(-K, vc[b], pcol[par][tc + 16 * b]);
#pragma unroll
  for (int a = KA; a < RT; ++a) {
    const double wa = fma(-K, vr[a], pcol[par][tr + 32 * a]);
#pragma unroll
    for (int b = KB; b < CB; ++b) w[a][b] = fma(-vr[a], wc[b], fma(-wa, vc[b], w[a][b]));
  }
}

// Steps k with (k + 1) / 16 == KB, then the next column block.
template <int RT, int KB>
__device__ __forceinline__ void tri_steps(double (&w)[RT][2 * RT], double (*xcol)[32 * RT],
                                          double (*pcol)[32 * RT], double (*part)[32],
                                          double (*vpart)[32], double* sdd, double* see,
                                          double* sbb, double* Hb, int p, int ld, int tr, int tc) {
  if constexpr (KB < 2 * RT) {
    const int k_end = min(16 * KB + 15, p - 2);
    for (int k = max(16 * KB - 1, 0); k < k_end; ++k) {
      tri_publish<RT>(w, xcol, part, sdd, k, tr, tc);
      tri_step<RT, KB>(w, xcol, pcol, part, vpart, see, sbb, Hb, k, ld, tr, tc);
    }
    tri_steps<RT, KB + 1>(w, xcol, pcol, part, vpart, sdd, see, sbb, Hb, p, ld, tr, tc);
  }
}

template <int RT>
__global__ void __launch_bounds__(TRI_THREADS)
    k_tri_reduce(const SmallDesc* __restrict__ sds, const double* __restrict__ A,
                 double* __restrict__ Hv, double* __restrict__ tri, int32_t* __restrict__ status) {
  constexpr int LDM = 32 * RT, CB = 2 * RT;
  __shared__ double xcol[2][LDM];
  __shared__ double pcol[2][LDM];
  __shared__ double part[2][32];
  __shared__ double vpart[2][32];
  __shared__ double sdd[LDM], see[LDM], sbb[LDM];
  __shared__ int flag;
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const double* Ab = A + d.m_off;
  double* Hb = Hv + d.m_off;
  if (tid == 0) flag = 0;
  __syncthreads();
  double w[RT][CB];
  bool bad = false;
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int i = tr + 32 * a, j = tc + 16 * b;
      const double v = (i < p && j < p) ? Ab[int64_t(i) * ld + j] : 0.0;
      bad = bad || !isfinite(v);
      w[a][b] = v;
    }
  if (bad) atomicOr(&flag, MI_BLOCK_NONFINITE);
  __syncthreads();
  tri_steps<RT, 0>(w, xcol, pcol, part, vpart, sdd, see, sbb, Hb, p, ld, tr, tc);
  // the last 2 x 2 (or 1 x 1) block is already tridiagonal
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int i = tr + 32 * a, j = tc + 16 * b;
      if (p >= 2 && i == p - 2 && j == p - 2) sdd[p - 2] = w[a][b];
      if (i == p - 1 && j == p - 1) sdd[p - 1] = w[a][b];
      if (p >= 2 && i == p - 1 && j == p - 2) see[p - 2] = w[a][b];
    }
  if (tid == 0) {
    see[p - 1] = 0.0;
    if (p >= 2) sbb[p - 2] = 0.0;
    sbb[p - 1] = 0.0;
  }
  __syncthreads();
  double* dd = tri + 4 * d.t_off;
  for (int i = tid; i < p; i += TRI_THREADS) {
    dd[i] = sdd[i];
    dd[p + i] = see[i];
    dd[3 * p + i] = sbb[i];
  }
  if (tid == 0 && flag) atomicOr(&status[d.blk], flag);
}

// Wider blocks (192 < ld <= TRI_MAX_LD): the same reflectors with the
// matrix in global memory (the block's A, overwritten), one workgroup of
// TRI_G_THREADS per block.  Only the upper triangle of A is kept current,
// so column k below the diagonal is read as row k right of it (one
// coalesced row load), and each step moves half the trailing block.  The
// rank-2 update of step k - 1 is deferred and fused into step k's sweep,
// so the trailing triangle is read and written once per step:
//   A (one wavefront): row k with update k - 1 applied gives x, its norm,
//     alpha, beta and v (v_{k+1} = x_{k+1} - alpha, zero at and above k),
//     into LDS and row k of Hv;
//   B (all): every trailing row i > k gets update k - 1 (A -= v w^T + w v^T
//     with the previous v, w) on its columns j >= i, written back, and
//     p = beta A v from the symmetry: a_ij (j > i) adds a_ij v_j to p_i and
//     a_ij v_i to p_j.  One wavefront per row and lanes over the columns
//     (lane l owns columns l + 64 t), the p_i parts summed in the
//     wavefront, the p_j parts kept by the lane that owns column j over all
//     of its wavefront's rows and added over the wavefronts afterwards;
//   C: K = (beta/2) v^T p and w = p - K v.
// The last update is applied to the final 2 x 2 block at the end.  Every
// sum runs in a fixed order (wavefront tree, then the wavefront partials in
// order), so the result does not depend on the launch.
constexpr int TRI_G_THREADS = 1024;
constexpr int TRI_G_WAVES = TRI_G_THREADS / 64;
constexpr int TRI_G_PL = (TRI_MAX_LD + 63) / 64;  // row elements per lane

// Sum over the workgroup of one value per thread; every thread gets it.
__device__ __forceinline__ double tri_g_sum(double v, double* part) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < TRI_G_WAVES; ++w) t += part[w];
  return t;
}

__global__ void __launch_bounds__(TRI_G_THREADS, 8)
    k_tri_reduce_g(const SmallDesc* __restrict__ sds, double* __restrict__ A,
                   double* __restrict__ Hv, double* __restrict__ tri, int32_t* __restrict__ status) {
  __shared__ double vv[2][TRI_MAX_LD], ww[2][TRI_MAX_LD];
  __shared__ double sdd[TRI_MAX_LD], see[TRI_MAX_LD], sbb[TRI_MAX_LD];
  __shared__ double part[2][TRI_G_WAVES];
  __shared__ double rowp[TRI_MAX_LD];               // p_i from row i's own columns
  __shared__ double cpart[TRI_G_WAVES][TRI_MAX_LD];  // p_j parts of each wavefront
  __shared__ int flag;
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Ab = A + d.m_off;
  double* Hb = Hv + d.m_off;
  if (tid == 0) flag = 0;
  for (int i = tid; i < 2 * TRI_MAX_LD; i += TRI_G_THREADS) {
    (&vv[0][0])[i] = 0.0;
    (&ww[0][0])[i] = 0.0;
  }
  __syncthreads();
  {
    bool bad = false;
    for (int i = wave; i < p; i += TRI_G_WAVES)
      for (int j = lane; j < p; j += 64) bad = bad || !isfinite(Ab[int64_t(i) * ld + j]);
    if (bad) atomicOr(&flag, MI_BLOCK_NONFINITE);
  }
  for (int k = 0; k + 2 < p; ++k) {
    const int k1 = k + 1, cur = k & 1, prv = cur ^ 1;
    // A: the reflector of column k (row k with the pending update applied)
    if (wave == 0) {
      const double vk = vv[prv][k], wk = ww[prv][k];
      double xa[TRI_G_PL];
      double ss = 0.0;
#pragma unroll
      for (int t = 0; t < TRI_G_PL; ++t) {
        const int j = k + lane + 64 * t;
        double x = 0.0;
        if (j < p)
          x = fma(-vk, ww[prv][j], fma(-wk, vv[prv][j], Ab[int64_t(k) * ld + j]));
        xa[t] = x;
        if (j > k) ss = fma(x, x, ss);
      }
      ss = wave_sum(ss);
      const double dkk = __shfl(xa[0], 0, 64), x1 = __shfl(xa[0], 1, 64);
      double al, be;
      if (ss <= DBL_MIN) {
        al = x1;
        be = 0.0;
      } else {
        al = -copysign(sqrt_pos(ss), x1);
        be = recip(al * (al - x1));
      }
#pragma unroll
      for (int t = 0; t < TRI_G_PL; ++t) {
        const int j = k + lane + 64 * t;
        const double v = (j > k && j < p) ? xa[t] - (j == k1 ? al : 0.0) : 0.0;
        if (j < TRI_MAX_LD) vv[cur][j] = v;
        if (j < ld) Hb[int64_t(k) * ld + j] = v;
      }
      for (int j = lane; j <= k; j += 64) Hb[int64_t(k) * ld + j] = 0.0;
      if (lane == 0) {
        sdd[k] = dkk;
        see[k] = al;
        sbb[k] = be;
      }
    }
    __syncthreads();
    const double be = sbb[k];
    // B: pending update of the trailing upper triangle, written back, and
    // p = beta A v by rows (p_i) and by columns (p_j, per lane)
    double cacc[TRI_G_PL];
#pragma unroll
    for (int t = 0; t < TRI_G_PL; ++t) cacc[t] = 0.0;
    for (int i = k1 + wave; i < p; i += TRI_G_WAVES) {
      const double vi = vv[prv][i], wi = ww[prv][i], ni = vv[cur][i];
      double s1 = 0.0;
#pragma unroll
      for (int t = 0; t < TRI_G_PL; ++t) {
        const int j = lane + 64 * t;
        if (j >= i && j < p) {
          const int64_t o = int64_t(i) * ld + j;
          const double a = fma(-vi, ww[prv][j], fma(-wi, vv[prv][j], Ab[o]));
          Ab[o] = a;
          s1 = fma(a, vv[cur][j], s1);
          if (j > i) cacc[t] = fma(a, ni, cacc[t]);
        }
      }
      s1 = wave_sum(s1);
      if (lane == 0) rowp[i] = s1;
    }
#pragma unroll
    for (int t = 0; t < TRI_G_PL; ++t) {
      const int j = lane + 64 * t;
      if (j < TRI_MAX_LD) cpart[wave][j] = cacc[t];
    }
    __syncthreads();
    for (int j = tid; j < p; j += TRI_G_THREADS) {
      if (j > k) {
        double c = rowp[j];
        for (int w = 0; w < TRI_G_WAVES; ++w) c += cpart[w][j];
        ww[cur][j] = be * c;
      }
    }
    __syncthreads();
    // C: w = p - K v with K = (beta / 2) v^T p
    const double vp =
        tri_g_sum((tid > k && tid < p) ? vv[cur][tid] * ww[cur][tid] : 0.0, part[cur]);
    const double K = 0.5 * be * vp;
    if (tid > k && tid < p) ww[cur][tid] = fma(-K, vv[cur][tid], ww[cur][tid]);
    __syncthreads();
  }
  // the last 2 x 2 (or 1 x 1) block is already tridiagonal once the pending
  // update of the last step is applied
  if (tid == 0) {
    const int kl = p - 3, c = kl & 1;  // the last step and its buffers
    auto upd = [&](int i, int j) {
      const double a = Ab[int64_t(i) * ld + j];
      return kl >= 0 ? fma(-vv[c][i], ww[c][j], fma(-ww[c][i], vv[c][j], a)) : a;
    };
    if (p >= 2) {
      sdd[p - 2] = upd(p - 2, p - 2);
      see[p - 2] = upd(p - 2, p - 1);  // the upper triangle is the current one
      sbb[p - 2] = 0.0;
    }
    sdd[p - 1] = upd(p - 1, p - 1);
    see[p - 1] = 0.0;
    sbb[p - 1] = 0.0;
  }
  __syncthreads();
  double* dd = tri + 4 * d.t_off;
  for (int i = tid; i < p; i += TRI_G_THREADS) {
    dd[i] = sdd[i];
    dd[p + i] = see[i];
    dd[3 * p + i] = sbb[i];
  }
  if (tid == 0 && flag) atomicOr(&status[d.blk], flag);
}

// ------------------------------------------------------------------ 2. eigenvalues
// Count of eigenvalues of T below x = number of negative pivots of the
// LDL^T factorisation of T - x I (Sylvester's law of inertia); pivots
// smaller than pivmin are replaced by -pivmin.  Each eigenvalue j is owned
// by a group of G lanes that evaluate G equispaced points of its bracket
// [a, b] (count(a) <= j < count(b)) per round, one Sturm count per lane: a
// count is a chain of p dependent divisions, so one chain per lane keeps
// each round at the chain's latency, and more lanes per eigenvalue cut the
// number of rounds.
template <int G>
__global__ void __launch_bounds__(64)
    k_tri_bisect(const SmallDesc* __restrict__ sds, double* __restrict__ tri,
                 double* __restrict__ ritz, int32_t* __restrict__ perm, double* __restrict__ a_lo,
                 int adapt, int32_t* __restrict__ status) {
  extern __shared__ double smem[];
  __shared__ double red[3];
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p;
  const int j0 = blockIdx.y * (64 / G);
  if (j0 >= p) return;
  double* sd_ = smem;
  double* se2 = smem + p;
  const double* dd = tri + 4 * d.t_off;
  const double* ee = dd + p;
  double* lam = tri + 4 * d.t_off + 2 * p;
  for (int i = threadIdx.x; i < p; i += 64) {
    sd_[i] = dd[i];
    se2[i] = ee[i] * ee[i];
  }
  const TriScale sc = tri_scale(dd, ee, p, red);  // has a barrier
  const double atol = 4.0 * DBL_EPSILON * sc.tn + 2.0 * sc.pivmin;
  const int g = threadIdx.x / G, r = threadIdx.x % G;
  const int j = j0 + g;
  const bool live = j < p;
  double a = sc.lo, b = sc.hi;
  for (int it = 0; it < TRI_MAXIT; ++it) {
    const bool todo = live && (b - a > atol);
    if (!__any(todo)) break;
    double na = a, nb = b;
    if (todo) {
      const double x = a + (b - a) * (double(r + 1) * (1.0 / (G + 1)));
      double t = guard(sd_[0] - x, sc.pivmin);
      int c = t < 0.0;
      for (int i = 1; i < p; ++i) {
        // e2 / t by the hardware reciprocal and one Newton step: a count
        // only needs the pivot's sign, which a few ulps cannot flip except
        // within rounding distance of an eigenvalue
        t = guard((sd_[i] - x) - se2[i - 1] * recip(t), sc.pivmin);
        c += t < 0.0;
      }
      if (c <= j) na = x;
      else nb = x;
    }
    for (int o = 1; o < G; o <<= 1) {
      na = fmax(na, __shfl_xor(na, o, 64));
      nb = fmin(nb, __shfl_xor(nb, o, 64));
    }
    a = na;
    b = nb;
  }
  if (live && r == 0) {
    const double v = 0.5 * (a + b);
    lam[j] = v;
    ritz[d.t_off + j] = v;
    perm[d.t_off + j] = j;
    if (adapt && j == p - 1) a_lo[d.blk] = v;
    if (!isfinite(v)) atomicOr(&status[d.blk], MI_BLOCK_NONFINITE);
    else if (b - a > atol) atomicOr(&status[d.blk], MI_BLOCK_NOCONV);
  }
}

// ------------------------------------------------------------------ 3. eigenvectors of T
// One thread per eigenvalue; per-thread vectors live in columns of ld x ld
// scratch matrices (column j of thread j: coalesced across the threads).
// An isolated eigenvalue gets the twisted-factorisation vector: forward
// (dp) and backward (dm) pivots of T - lambda I, the twist index k with the
// smallest |dp_k + dm_k - (d_k - lambda)|, z_k = 1 and the two one-sided
// recurrences.  The first eigenvalue of a cluster (consecutive gaps below
// TRI_CLUSTER * ||T||) computes the whole cluster by inverse iteration (3
// rounds from a fixed pseudo-random start, LDL^T solves with pivots floored
// at eps ||T||, equal shifts separated by 10 eps ||T||, Gram-Schmidt twice
// against the cluster's earlier vectors).  Output: unit vectors in the
// columns of Zt (Zt[i][j] = component i of vector j).
__device__ void tri_inverse_iteration(const double* __restrict__ sd_, const double* __restrict__ se,
                                      const double* __restrict__ lam, int p, int ld, int j0,
                                      int j1, double tn, double* __restrict__ dp,
                                      double* __restrict__ y, double* __restrict__ Zt) {
  const double fl = DBL_EPSILON * tn;
  double sprev = 0.0;
  for (int jj = j0; jj <= j1; ++jj) {
    double s = lam[jj];
    if (jj > j0 && s <= sprev + 10.0 * fl) s = sprev + 10.0 * fl;
    sprev = s;
    double t = guard(sd_[0] - s, fl);
    dp[jj] = t;
    for (int i = 1; i < p; ++i) {
      t = guard((sd_[i] - s) - se[i - 1] * se[i - 1] / t, fl);
      dp[int64_t(i) * ld + jj] = t;
    }
    double* x = Zt + jj;
    for (int i = 0; i < p; ++i) x[int64_t(i) * ld] = hash_unit(i, jj);
    for (int it = 0; it < 3; ++it) {
      double mx = 0.0;
      for (int i = 0; i < p; ++i) mx = fmax(mx, fabs(x[int64_t(i) * ld]));
      const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
      // L y = x  (L unit lower, l_i = e_i / dp_i)
      double yi = x[0] * inv;
      y[jj] = yi;
      for (int i = 1; i < p; ++i) {
        yi = x[int64_t(i) * ld] * inv - se[i - 1] / dp[int64_t(i - 1) * ld + jj] * yi;
        y[int64_t(i) * ld + jj] = yi;
      }
      // D L^T z = y
      double zi = y[int64_t(p - 1) * ld + jj] / dp[int64_t(p - 1) * ld + jj];
      x[int64_t(p - 1) * ld] = zi;
      for (int i = p - 2; i >= 0; --i) {
        const double di = dp[int64_t(i) * ld + jj];
        zi = y[int64_t(i) * ld + jj] / di - se[i] / di * zi;
        x[int64_t(i) * ld] = zi;
      }
      for (int rep = 0; rep < 2; ++rep)
        for (int u = j0; u < jj; ++u) {
          double dot = 0.0;
          for (int i = 0; i < p; ++i) dot = fma(Zt[int64_t(i) * ld + u], x[int64_t(i) * ld], dot);
          for (int i = 0; i < p; ++i) x[int64_t(i) * ld] -= dot * Zt[int64_t(i) * ld + u];
        }
      double nrm = 0.0;
      for (int i = 0; i < p; ++i) nrm = fma(x[int64_t(i) * ld], x[int64_t(i) * ld], nrm);
      const double sc = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = 0; i < p; ++i) x[int64_t(i) * ld] *= sc;
    }
  }
}

// NT eigenvalues per workgroup (their pivots in LDS: 2 p NT doubles): 32
// up to p = 192, 16 for wider blocks.
template <int NT>
__global__ void __launch_bounds__(NT)
    k_tri_vectors(const SmallDesc* __restrict__ sds, const double* __restrict__ tri,
                  double* __restrict__ DP, double* __restrict__ DM, double* __restrict__ ZT,
                  int32_t* __restrict__ status) {
  extern __shared__ double smem[];
  __shared__ double red[3];
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  const int tx = threadIdx.x;
  const int j = blockIdx.y * NT + tx;
  if (blockIdx.y * NT >= p) return;
  double* sd_ = smem;
  double* se = smem + p;
  // forward / backward pivots of this workgroup's eigenvalues: pivot i of
  // thread tx at [i][tx] (consecutive threads in consecutive banks)
  double* ldp = smem + 2 * p;
  double* ldm = ldp + p * NT;
  const double* dd = tri + 4 * d.t_off;
  const double* ee = dd + p;
  const double* lam = dd + 2 * p;
  for (int i = tx; i < p; i += NT) {
    sd_[i] = dd[i];
    se[i] = ee[i];
  }
  const TriScale sc = tri_scale(dd, ee, p, red);  // has a barrier
  if (j >= p) return;
  const double ctol = TRI_CLUSTER * sc.tn;
  if (j > 0 && !(lam[j] - lam[j - 1] > ctol)) return;  // inside a cluster led by an earlier j
  int j1 = j;
  while (j1 + 1 < p && !(lam[j1 + 1] - lam[j1] > ctol)) ++j1;
  double* Zt = ZT + d.m_off;
  if (j1 > j) {
    tri_inverse_iteration(sd_, se, lam, p, ld, j, j1, sc.tn, DP + d.m_off, DM + d.m_off, Zt);
    return;
  }
  const double lj = lam[j];
  const double pm = sc.pivmin;
  // the two pivot recurrences only store (no loads on their chains)
  double t = guard(sd_[0] - lj, pm);
  ldp[tx] = t;
  for (int i = 1; i < p; ++i) {
    t = guard((sd_[i] - lj) - se[i - 1] * se[i - 1] * recip(t), pm);
    ldp[i * NT + tx] = t;
  }
  t = guard(sd_[p - 1] - lj, pm);
  ldm[(p - 1) * NT + tx] = t;
  for (int i = p - 2; i >= 0; --i) {
    t = guard((sd_[i] - lj) - se[i] * se[i] * recip(t), pm);
    ldm[i * NT + tx] = t;
  }
  // twist index: smallest |dp_k + dm_k - (d_k - lambda)| (independent terms)
  int kmin = p - 1;
  double gmin = fabs(ldp[(p - 1) * NT + tx] + ldm[(p - 1) * NT + tx] - (sd_[p - 1] - lj));
  for (int i = p - 2; i >= 0; --i) {
    const double gam = fabs(ldp[i * NT + tx] + ldm[i * NT + tx] - (sd_[i] - lj));
    if (gam < gmin) {
      gmin = gam;
      kmin = i;
    }
  }
  // the two one-sided recurrences from z_k = 1; z_i replaces the pivot it
  // consumed (ldp[i] for i < k, ldm[i] read and ldp[i] written for i > k),
  // so the vector stays in LDS until it is scaled on the way out
  double nrm = 1.0;
  ldp[kmin * NT + tx] = 1.0;
  double z = 1.0;
  for (int i = kmin - 1; i >= 0; --i) {
    z *= -se[i] * recip(ldp[i * NT + tx]);
    ldp[i * NT + tx] = z;
    nrm = fma(z, z, nrm);
  }
  z = 1.0;
  for (int i = kmin + 1; i < p; ++i) {
    z *= -se[i - 1] * recip(ldm[i * NT + tx]);
    ldp[i * NT + tx] = z;
    nrm = fma(z, z, nrm);
  }
  if (!isfinite(nrm)) {  // overflow in the recurrences: fall back to inverse iteration
    tri_inverse_iteration(sd_, se, lam, p, ld, j, j, sc.tn, DP + d.m_off, DM + d.m_off, Zt);
    return;
  }
  const double inv = 1.0 / sqrt(nrm);
  for (int i = 0; i < p; ++i) Zt[int64_t(i) * ld + j] = ldp[i * NT + tx] * inv;
  (void)status;
}

// ------------------------------------------------------------------ 4. back-transformation
// Z^T = Z_T^T H_{p-3} ... H_0: every row of Z_T^T (an eigenvector of T) is
// updated independently, so a block splits into ld / 32 workgroups of 32
// rows.  A row is held by 8 lanes, lane q holding components 16b + 2q and
// 16b + 2q + 1: its dot product with a reflector is reduced in three DPP
// steps, and the reflector is read from LDS as 128-bit pairs.  The
// reflectors stream through LDS TRI_VC at a time; the next chunk is loaded
// into registers while the current one is applied.  Output Z[i][j] =
// component i of the j-th eigenvector (ascending), zero outside p x p.
constexpr int TRI_BACK_THREADS = 256;

// Sum over the 8 lanes of each aligned lane octet, in every lane.
__device__ __forceinline__ double oct_sum(double v) {
  v += dpp_d<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);         // quad_perm [2,3,0,1]
  return v + dpp_d<0x141>(v);  // row_half_mirror: lane l <-> 7 - l of each octet
}

template <int RT>
__global__ void __launch_bounds__(TRI_BACK_THREADS)
    k_tri_back(const SmallDesc* __restrict__ sds, const double* __restrict__ ZT,
               const double* __restrict__ Hv, const double* __restrict__ tri,
               double* __restrict__ Z) {
  constexpr int LDM = 32 * RT, NB = 2 * RT;
  constexpr int PF = TRI_VC * LDM / TRI_BACK_THREADS;  // chunk values per thread
  static_assert(PF * TRI_BACK_THREADS == TRI_VC * LDM, "chunk must split evenly");
  __shared__ __align__(16) double vb[TRI_VC * LDM];
  __shared__ double bt[TRI_VC];
  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  if (int(blockIdx.y) * 32 >= ld) return;
  const int tid = threadIdx.x, g = tid >> 3, q = tid & 7;
  const int j = blockIdx.y * 32 + g;
  const double* Zt = ZT + d.m_off;
  const double* Hb = Hv + d.m_off;
  const double* bb = tri + 4 * d.t_off + 3 * p;
  double w[NB][2];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int i = 16 * b + 2 * q + s;
      w[b][s] = (i < p && j < p) ? Zt[int64_t(i) * ld + j] : 0.0;
    }
  // reflectors kl .. k0 of one chunk, element e = kk * LDM + i
  double pf[PF], pfb = 0.0;
  auto fetch = [&](int k0) {
    const int kl = max(0, k0 - TRI_VC + 1), cnt = k0 - kl + 1;
#pragma unroll
    for (int m = 0; m < PF; ++m) {
      const int e = tid + TRI_BACK_THREADS * m, kk = e / LDM, i = e % LDM;
      pf[m] = (kk < cnt && i < p) ? Hb[int64_t(kl + kk) * ld + i] : 0.0;
    }
    pfb = tid < cnt ? bb[kl + tid] : 0.0;
  };
  if (p >= 3) fetch(p - 3);
  for (int k0 = p - 3; k0 >= 0; k0 -= TRI_VC) {
    const int cnt = k0 - max(0, k0 - TRI_VC + 1) + 1;
    __syncthreads();  // the previous chunk is consumed
#pragma unroll
    for (int m = 0; m < PF; ++m) vb[tid + TRI_BACK_THREADS * m] = pf[m];
    if (tid < TRI_VC) bt[tid] = pfb;
    __syncthreads();
    if (k0 >= TRI_VC) fetch(k0 - TRI_VC);
    for (int kk = cnt - 1; kk >= 0; --kk) {
      const double be = bt[kk];
      double v[NB][2];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double2 t = *reinterpret_cast<const double2*>(&vb[kk * LDM + 16 * b + 2 * q]);
        v[b][0] = t.x;
        v[b][1] = t.y;
      }
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        s0 = fma(w[b][0], v[b][0], s0);
        s1 = fma(w[b][1], v[b][1], s1);
      }
      const double sc = be * oct_sum(s0 + s1);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        w[b][0] = fma(-sc, v[b][0], w[b][0]);
        w[b][1] = fma(-sc, v[b][1], w[b][1]);
      }
    }
  }
  double* Zb = Z + d.m_off;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int i = 16 * b + 2 * q + s;
      if (i < ld && j < ld) Zb[int64_t(i) * ld + j] = (i < p && j < p) ? w[b][s] : 0.0;
    }
}

// ------------------------------------------------------------------ launch
bool tri_eig_supported(int max_ld) { return max_ld <= TRI_MAX_LD; }

#define MI_TRI_CASE(R)                                                                           \
  case R:                                                                                        \
    hipLaunchKernelGGL(k_tri_reduce<R>, dim3(nb), dim3(TRI_THREADS), 0, s, sd, A, Hv, tri, status); \
    break;

#define MI_TRI_BACK_CASE(R)                                                                      \
  case R:                                                                                        \
    hipLaunchKernelGGL(k_tri_back<R>, dim3(nb, max_ld / 32), dim3(TRI_BACK_THREADS), 0, s, sd, ZT, Hv, tri, Z); \
    break;

void launch_tri_reduce(const SmallDesc* sd, int nb, int max_ld, double* A, double* Hv,
                       double* tri, int32_t* status, hipStream_t s) {
  if (nb <= 0) return;
  if (max_ld > 32 * 6) {
    // Two workgroups per CU (64 registers, 62 KB of LDS each): with only the
    // upper triangle swept (about 400 KB touched per block at ld = 320),
    // the blocks in flight still fit the 256 MB infinity cache (16.5 against
    // 19.2 ms for 1,024 blocks of ld 320 at one per CU; when the full square
    // was swept, two per CU overflowed it: 34.0 against 27.7 ms)
    hipLaunchKernelGGL(k_tri_reduce_g, dim3(nb), dim3(TRI_G_THREADS), 0, s, sd, A, Hv, tri,
                       status);
    return;
  }
  switch ((max_ld + 31) / 32) {
    MI_TRI_CASE(1)
    MI_TRI_CASE(2)
    MI_TRI_CASE(3)
    MI_TRI_CASE(4)
    MI_TRI_CASE(5)
    MI_TRI_CASE(6)
    default: break;
  }
}

void launch_tri_bisect(const SmallDesc* sd, int nb, int max_p, double* tri, double* ritz,
                       int32_t* perm, double* a_lo, int adapt, int32_t* status, hipStream_t s) {
  if (nb <= 0) return;
  // 16 lanes per eigenvalue while the launch leaves most CUs idle, 8 once it
  // holds more blocks (more rounds, but half the waves)
  const size_t shm = size_t(2 * max_p) * sizeof(double);
  if (nb <= 16)
    hipLaunchKernelGGL(k_tri_bisect<16>, dim3(nb, ceil_div(max_p, 4)), dim3(64), shm, s, sd, tri,
                       ritz, perm, a_lo, adapt, status);
  else
    hipLaunchKernelGGL(k_tri_bisect<8>, dim3(nb, ceil_div(max_p, 8)), dim3(64), shm, s, sd, tri,
                       ritz, perm, a_lo, adapt, status);
}

void launch_tri_vectors(const SmallDesc* sd, int nb, int max_p, const double* tri, double* DP,
                        double* DM, double* ZT, int32_t* status, hipStream_t s) {
  if (nb <= 0) return;
  if (max_p <= 192)
    hipLaunchKernelGGL(k_tri_vectors<32>, dim3(nb, ceil_div(max_p, 32)), dim3(32),
                       size_t(2 * max_p + 2 * max_p * 32) * sizeof(double), s, sd, tri, DP, DM,
                       ZT, status);
  else
    hipLaunchKernelGGL(k_tri_vectors<16>, dim3(nb, ceil_div(max_p, 16)), dim3(16),
                       size_t(2 * max_p + 2 * max_p * 16) * sizeof(double), s, sd, tri, DP, DM,
                       ZT, status);
}

void launch_tri_back(const SmallDesc* sd, int nb, int max_ld, const double* ZT, const double* Hv,
                     const double* tri, double* Z, hipStream_t s) {
  if (nb <= 0) return;
  switch ((max_ld + 31) / 32) {
    MI_TRI_BACK_CASE(1)
    MI_TRI_BACK_CASE(2)
    MI_TRI_BACK_CASE(3)
    MI_TRI_BACK_CASE(4)
    MI_TRI_BACK_CASE(5)
    MI_TRI_BACK_CASE(6)
    MI_TRI_BACK_CASE(7)
    MI_TRI_BACK_CASE(8)
    MI_TRI_BACK_CASE(9)
    MI_TRI_BACK_CASE(10)
    default: break;
  }
}

}  // namespace mis
