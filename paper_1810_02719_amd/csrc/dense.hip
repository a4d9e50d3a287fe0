// Tall-skinny kernels (see dense.hpp).
#include "dense.hpp"

namespace mis {

typedef double d4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ SpMM
// Yout = alpha * (L Yin) + beta * Yin + gamma * Yprev for the rows of one
// tile; (alpha, beta, gamma) per block and step.  Each wavefront takes whole
// rows: the row's CSR entries are wave-uniform (scalar loads, read once),
// lanes cover the row's ld coefficients with 16-byte vectors, and the
// neighbour rows are gathered four at a time so that several coalesced
// loads are in flight per lane.
template <typename T>
__global__ void __launch_bounds__(256)
    k_spmm(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
           const CsrDesc* __restrict__ csr, const int32_t* __restrict__ row_ptr,
           const int32_t* __restrict__ col, const float* __restrict__ val,
           const T* __restrict__ Yin, const T* __restrict__ Yprev, T* __restrict__ Yout,
           const double* __restrict__ coef, int coef_stride, int step) {
  typedef typename VecOf<T>::type V;
  constexpr int W = VecOf<T>::W;
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const CsrDesc c = csr[t.set];
  const double* cf = coef + int64_t(d.blk) * coef_stride + 3 * step;
  const T alpha = (T)cf[0], beta = (T)cf[1], gamma = (T)cf[2];
  const int nvec = d.ld / W;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  const T* yb = Yin + d.off;
  const int32_t* cb = col + c.nnz_off;
  const float* vb = val + c.nnz_off;
  for (int rr = wave; rr < rows; rr += 4) {
    const int r = t.row0 + rr;
    const int k0 = row_ptr[c.rp_off + r], k1 = row_ptr[c.rp_off + r + 1];
    for (int v = lane; v < nvec; v += 64) {
      const T* yv = yb + v * W;
      V acc = (V)(T)0;
      int k = k0;
      for (; k + 4 <= k1; k += 4) {
        const int j0 = cb[k], j1 = cb[k + 1], j2 = cb[k + 2], j3 = cb[k + 3];
        const V y0 = *reinterpret_cast<const V*>(yv + int64_t(j0) * d.ld);
        const V y1 = *reinterpret_cast<const V*>(yv + int64_t(j1) * d.ld);
        const V y2 = *reinterpret_cast<const V*>(yv + int64_t(j2) * d.ld);
        const V y3 = *reinterpret_cast<const V*>(yv + int64_t(j3) * d.ld);
        acc += (T)vb[k] * y0;
        acc += (T)vb[k + 1] * y1;
        acc += (T)vb[k + 2] * y2;
        acc += (T)vb[k + 3] * y3;
      }
      for (; k < k1; ++k) acc += (T)vb[k] * *reinterpret_cast<const V*>(yv + int64_t(cb[k]) * d.ld);
      const int64_t o = d.off + int64_t(r) * d.ld + v * W;
      V out = alpha * acc + beta * *reinterpret_cast<const V*>(Yin + o);
      if (Yprev) out += gamma * *reinterpret_cast<const V*>(Yprev + o);
      *reinterpret_cast<V*>(Yout + o) = out;
    }
  }
}

// Same product when every block of the launch has ld = 64 * EPL: one
// wavefront per row (16 per workgroup, one tile), every lane owns EPL
// consecutive elements of the row, and the row's neighbour rows are
// gathered SPMM_GATHER at a time with clamped indices (zero weight past the
// row end), so all of those loads are issued before the first use.
// Workgroups are dealt to the 8 XCDs in turn; workgroup i takes tile
// (i mod 8) * per + i / 8, so each XCD works through one contiguous eighth
// of the tiles and the neighbour rows a row gathers (nearby in the BFS
// vertex order) are mostly already in that XCD's L2.
constexpr int SPMM_GATHER = 8;
constexpr int NUM_XCD = 8;

// With STRIDED, lane l owns the row's columns l, l + 64, ..., so that each
// of its EPL loads is one coalesced 256-byte (FP32) wavefront access; used
// for EPL = 5 (320-wide slabs), where EPL consecutive elements would not
// form 16-byte vectors.
// With WPG = 4 a tile's 16 rows are split over four workgroups of four
// wavefronts (same XCD, consecutive), so that more workgroups fit a CU when
// the kernel's registers allow more wavefronts than one 16-wavefront group.
template <typename T, int EPL, bool STRIDED = false, int G = SPMM_GATHER, int WPG = SPMM_ROWS>
__global__ void __launch_bounds__(64 * WPG)
    k_spmm_row(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
               const CsrDesc* __restrict__ csr, const int32_t* __restrict__ row_ptr,
               const int32_t* __restrict__ col, const float* __restrict__ val,
               const T* __restrict__ Yin, const T* __restrict__ Yprev, T* __restrict__ Yout,
               const double* __restrict__ coef, int coef_stride, int step, int ntiles) {
  static_assert(SPMM_ROWS % WPG == 0, "workgroup split");
  constexpr int SPLIT = SPMM_ROWS / WPG;
  const int per = (ntiles + NUM_XCD - 1) / NUM_XCD;
  const int k = blockIdx.x / NUM_XCD;  // index within this workgroup's XCD
  const int ti = (blockIdx.x % NUM_XCD) * per + k / SPLIT;
  if (ti >= ntiles) return;
  const SpmmTile t = tiles[ti];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const MatDesc d = sets[t.set];
  const int r = t.row0 + (k % SPLIT) * WPG + wave;
  if (r >= d.rows) return;  // wave-uniform
  const CsrDesc c = csr[t.set];
  const int lane = threadIdx.x & 63;
  typedef Acc<T> AC;  // arithmetic in AC::type (FP32 for BF16 slabs)
  typedef typename AC::type A;
  const double* cf = coef + int64_t(d.blk) * coef_stride + 3 * step;
  const A alpha = (A)cf[0], beta = (A)cf[1], gamma = (A)cf[2];
  constexpr int ES = STRIDED ? 64 : 1;  // element stride of a lane
  const int l0 = STRIDED ? lane : lane * EPL;
  const T* yv = Yin + d.off + l0;
  const int32_t* cb = col + c.nnz_off;
  const float* vb = val + c.nnz_off;
  // the row's own terms first: their loads overlap the row pointer ->
  // column -> neighbour chain of the gather (without a previous iterate the
  // third term reads the current one with weight 0, so both loads are
  // unconditional and issued here)
  const int64_t o = d.off + int64_t(r) * d.ld + l0;
  const T* yp = Yprev ? Yprev : Yin;
  const A g3 = Yprev ? gamma : (A)0;
  A yin[EPL], ypr[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    yin[e] = AC::load(Yin[o + e * ES]);
    ypr[e] = AC::load(yp[o + e * ES]);
  }
  const int k0 = row_ptr[c.rp_off + r], k1 = row_ptr[c.rp_off + r + 1];
  A acc[EPL], base[EPL];
  {
    // first chunk of the row, unconditional (entries past the row gather the
    // row itself with weight 0), so that the row's own terms are consumed
    // in the same block and their loads stay ahead of the gather
    A y[G][EPL];
    A w[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const bool in = k0 + u < k1;
      w[u] = in ? (A)vb[k0 + u] : (A)0;
      const T* src = yv + int64_t(in ? cb[k0 + u] : r) * d.ld;
#pragma unroll
      for (int e = 0; e < EPL; ++e) y[u][e] = AC::load(src[e * ES]);
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      base[e] = beta * yin[e] + g3 * ypr[e];
      acc[e] = (A)0;
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int e = 0; e < EPL; ++e) acc[e] = fma(w[u], y[u][e], acc[e]);
    // pin base here: otherwise the compiler sinks its loads past the loop
#pragma unroll
    for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(base[e]));
  }
  for (int k = k0 + G; k < k1; k += G) {
    A y[G][EPL];
    A w[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int kk = min(k + u, k1 - 1);
      w[u] = k + u < k1 ? (A)vb[kk] : (A)0;
      const T* src = yv + int64_t(cb[kk]) * d.ld;
#pragma unroll
      for (int e = 0; e < EPL; ++e) y[u][e] = AC::load(src[e * ES]);
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int e = 0; e < EPL; ++e) acc[e] = fma(w[u], y[u][e], acc[e]);
  }
  A out[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) out[e] = alpha * acc[e] + base[e];
#pragma unroll
  for (int e = 0; e < EPL; ++e) Yout[o + e * ES] = AC::store(out[e]);
}

// The same product with R rows per wavefront taken one after the other, the
// row pointers, column indices and weights of all R rows loaded first (into
// scalar registers: they are wave-uniform), so that the chain row pointer ->
// columns -> neighbour rows is paid once per R rows and each row then costs
// one round of gathers.  A workgroup of 16 wavefronts covers R consecutive
// tiles of its XCD's range; entries past a row's first SPMM_GATHER are
// gathered afterwards in chunks (rows of high degree).
template <typename T, int EPL, bool STRIDED, int R, int WPG = SPMM_ROWS>
__global__ void __launch_bounds__(64 * WPG)
    k_spmm_rows(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                const CsrDesc* __restrict__ csr, const int32_t* __restrict__ row_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val,
                const T* __restrict__ Yin, const T* __restrict__ Yprev, T* __restrict__ Yout,
                const double* __restrict__ coef, int coef_stride, int step, int ntiles) {
  typedef Acc<T> AC;
  typedef typename AC::type A;
  constexpr int G = SPMM_GATHER;
  constexpr int ES = STRIDED ? 64 : 1;
  constexpr int SPLIT = SPMM_ROWS / WPG;  // workgroups per group of R tiles
  const int ngroups = (ntiles + R - 1) / R;
  const int per = (ngroups + NUM_XCD - 1) / NUM_XCD;
  const int kx = blockIdx.x / NUM_XCD;
  const int g = (blockIdx.x % NUM_XCD) * per + kx / SPLIT;
  if (g >= ngroups) return;
  const int wave = (kx % SPLIT) * WPG + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int l0 = STRIDED ? lane : lane * EPL;
  // indices of the R rows (wave-uniform)
  int rr[R], sset[R], k0[R], k1[R], cj[R][G];
  A wj[R][G];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int ti = g * R + j;
    rr[j] = -1;
    sset[j] = 0;
    k0[j] = k1[j] = 0;
    if (ti < ntiles) {
      const SpmmTile t = tiles[ti];
      const MatDesc d = sets[t.set];
      const int r = t.row0 + wave;
      if (r < d.rows) {
        rr[j] = r;
        sset[j] = t.set;
        const CsrDesc c = csr[t.set];
        k0[j] = row_ptr[c.rp_off + r];
        k1[j] = row_ptr[c.rp_off + r + 1];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const CsrDesc c = csr[sset[j]];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const bool in = k0[j] + u < k1[j];
      cj[j][u] = in ? col[c.nnz_off + k0[j] + u] : max(rr[j], 0);
      wj[j][u] = in ? (A)val[c.nnz_off + k0[j] + u] : (A)0;
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (rr[j] < 0) continue;  // wave-uniform
    const MatDesc d = sets[sset[j]];
    const CsrDesc c = csr[sset[j]];
    const double* cf = coef + int64_t(d.blk) * coef_stride + 3 * step;
    const A alpha = (A)cf[0], beta = (A)cf[1], gamma = (A)cf[2];
    const T* yv = Yin + d.off + l0;
    const int64_t o = d.off + int64_t(rr[j]) * d.ld + l0;
    const T* yp = Yprev ? Yprev : Yin;
    const A g3 = Yprev ? gamma : (A)0;
    A y[G][EPL], yin[EPL], ypr[EPL], acc[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      yin[e] = AC::load(Yin[o + e * ES]);
      ypr[e] = AC::load(yp[o + e * ES]);
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const T* src = yv + int64_t(cj[j][u]) * d.ld;
#pragma unroll
      for (int e = 0; e < EPL; ++e) y[u][e] = AC::load(src[e * ES]);
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) acc[e] = (A)0;
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int e = 0; e < EPL; ++e) acc[e] = fma(wj[j][u], y[u][e], acc[e]);
    const int32_t* cb = col + c.nnz_off;
    const float* vb = val + c.nnz_off;
    for (int k = k0[j] + G; k < k1[j]; k += G) {
      A w[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int kk = min(k + u, k1[j] - 1);
        w[u] = k + u < k1[j] ? (A)vb[kk] : (A)0;
        const T* src = yv + int64_t(cb[kk]) * d.ld;
#pragma unroll
        for (int e = 0; e < EPL; ++e) y[u][e] = AC::load(src[e * ES]);
      }
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[e] = fma(w[u], y[u][e], acc[e]);
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e)
      Yout[o + e * ES] = AC::store(alpha * acc[e] + (beta * yin[e] + g3 * ypr[e]));
  }
}

// Non-temporal element load and store (the previous iterate is read once and
// the output is not read again by the launch, so neither should displace the
// gathered neighbour rows from the caches).
template <typename T>
__device__ inline T ld_nt(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <>
__device__ inline bf16 ld_nt<bf16>(const bf16* p) {
  return bf16{__builtin_nontemporal_load(&p->u)};
}
template <typename T>
__device__ inline void st_nt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}
template <>
__device__ inline void st_nt<bf16>(bf16* p, bf16 v) {
  __builtin_nontemporal_store(v.u, &p->u);
}

// A lane's EPL elements of a row (consecutive, or strided by 64 with
// STRIDED), widened to the arithmetic type.  Two or four consecutive BF16
// values move as one 4- or 8-byte access (element-wise 2-byte accesses,
// non-temporal ones especially, cost more than the bytes they move).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <typename T, int EPL, bool STRIDED, bool NT>
__device__ __forceinline__ void row_load(const T* p, typename Acc<T>::type* v) {
  constexpr int ES = STRIDED ? 64 : 1;
  if constexpr (std::is_same<T, bf16>::value && !STRIDED && EPL == 8) {
    const u32x4 w = NT ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p))
                       : *reinterpret_cast<const u32x4*>(p);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      v[2 * h] = __uint_as_float(w[h] << 16);
      v[2 * h + 1] = __uint_as_float(w[h] & 0xFFFF0000u);
    }
  } else if constexpr (std::is_same<T, float>::value && !STRIDED && EPL % 4 == 0) {
#pragma unroll
    for (int h = 0; h < EPL / 4; ++h) {
      const f32x4 w = NT ? __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p) + h)
                         : reinterpret_cast<const f32x4*>(p)[h];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[4 * h + e] = w[e];
    }
  } else if constexpr (std::is_same<T, bf16>::value && !STRIDED && EPL == 4) {
    const u32x2 w = NT ? __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p))
                       : *reinterpret_cast<const u32x2*>(p);
    v[0] = __uint_as_float(w.x << 16);
    v[1] = __uint_as_float(w.x & 0xFFFF0000u);
    v[2] = __uint_as_float(w.y << 16);
    v[3] = __uint_as_float(w.y & 0xFFFF0000u);
  } else if constexpr (std::is_same<T, bf16>::value && !STRIDED && EPL == 2) {
    const uint32_t w = NT ? __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p))
                          : *reinterpret_cast<const uint32_t*>(p);
    v[0] = __uint_as_float(w << 16);
    v[1] = __uint_as_float(w & 0xFFFF0000u);
  } else {
#pragma unroll
    for (int e = 0; e < EPL; ++e) v[e] = Acc<T>::load(NT ? ld_nt(p + e * ES) : p[e * ES]);
  }
}
template <typename T, int EPL, bool STRIDED, bool NT>
__device__ __forceinline__ void row_store(T* p, const typename Acc<T>::type* v) {
  constexpr int ES = STRIDED ? 64 : 1;
  if constexpr (std::is_same<T, bf16>::value && !STRIDED && EPL == 8) {
    u32x4 x;
#pragma unroll
    for (int h = 0; h < 4; ++h)
      x[h] = uint32_t(f32_to_bf16(v[2 * h]).u) | (uint32_t(f32_to_bf16(v[2 * h + 1]).u) << 16);
    if (NT)
      __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(p));
    else
      *reinterpret_cast<u32x4*>(p) = x;
  } else if constexpr (std::is_same<T, float>::value && !STRIDED && EPL % 4 == 0) {
#pragma unroll
    for (int h = 0; h < EPL / 4; ++h) {
      const f32x4 x = {v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]};
      if (NT)
        __builtin_nontemporal_store(x, reinterpret_cast<f32x4*>(p) + h);
      else
        reinterpret_cast<f32x4*>(p)[h] = x;
    }
  } else if constexpr (std::is_same<T, bf16>::value && !STRIDED && (EPL == 2 || EPL == 4)) {
    uint32_t w[2];
#pragma unroll
    for (int h = 0; h < EPL / 2; ++h)
      w[h] = uint32_t(f32_to_bf16(v[2 * h]).u) | (uint32_t(f32_to_bf16(v[2 * h + 1]).u) << 16);
    if constexpr (EPL == 4) {
      const u32x2 x = {w[0], w[1]};
      if (NT)
        __builtin_nontemporal_store(x, reinterpret_cast<u32x2*>(p));
      else
        *reinterpret_cast<u32x2*>(p) = x;
    } else {
      if (NT)
        __builtin_nontemporal_store(w[0], reinterpret_cast<uint32_t*>(p));
      else
        *reinterpret_cast<uint32_t*>(p) = w[0];
    }
  } else {
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const T x = Acc<T>::store(v[e]);
      if (NT)
        st_nt(p + e * ES, x);
      else
        p[e * ES] = x;
    }
  }
}

// One row per wavefront gathering exactly the row's off-diagonal entries
// (wave-uniform branches, no padded loads), with the product in difference
// form:
//   (L Y)_r = sum_{j != r} L_rj (Y_j - Y_r) + (sum_j L_rj) Y_r,
//   W_r = alpha (L Y)_r + beta Y_r + gamma Yprev_r.
// For a Laplacian the row sum is zero (exactly, for combinatorial weights)
// and the differences of a smooth iterate are small and exact in floating
// point, so the low-frequency components of L Y lose nothing to the
// cancellation of a degree-sized diagonal term against its neighbours: their
// rounding error scales with lambda |Y| instead of ||L|| |Y|.  The row's own
// values are loaded anyway; the diagonal entry itself is never gathered.
// The WPG rows of a workgroup are consecutive, so the neighbour rows they
// share are fetched once into the CU's L1 for all of them; with NT the
// previous iterate and the output stream past the caches.  The gather
// volume per row drops from ceil(nnz/8)*8 rows to nnz - 1 (the seven-entry
// rows of a triangle mesh: 8 to 6), which is what bounds this kernel once
// the HBM bytes are right.
template <typename T, int EPL, bool STRIDED, bool NT>
__device__ __forceinline__ void rowx_row(const MatDesc& d, const CsrDesc& c, int r, int lane,
                                         const int32_t* __restrict__ row_ptr,
                                         const int32_t* __restrict__ col,
                                         const float* __restrict__ val, const T* Yin,
                                         const T* Yprev, T* Yout,
                                         typename Acc<T>::type alpha, typename Acc<T>::type beta,
                                         typename Acc<T>::type gamma) {
  typedef typename Acc<T>::type A;
  constexpr int G = SPMM_GATHER;
  const int l0 = STRIDED ? lane : lane * EPL;
  const T* yv = Yin + d.off + l0;
  const int64_t o = d.off + int64_t(r) * d.ld + l0;
  A yin[EPL], ypr[EPL];
  row_load<T, EPL, STRIDED, false>(Yin + o, yin);
  if (Yprev) {
    row_load<T, EPL, STRIDED, NT>(Yprev + o, ypr);
  } else {
#pragma unroll
    for (int e = 0; e < EPL; ++e) ypr[e] = (A)0;
  }
  const A g3 = Yprev ? gamma : (A)0;
  const int k0 = row_ptr[c.rp_off + r], k1 = row_ptr[c.rp_off + r + 1];
  const int32_t* cb = col + c.nnz_off;
  const float* vb = val + c.nnz_off;
  A acc[EPL], rs = (A)0;  // rs: the row's entry sum (zero for a Laplacian)
#pragma unroll
  for (int e = 0; e < EPL; ++e) acc[e] = (A)0;
  for (int k = k0; k < k1; k += G) {
    // the group's column indices and weights in one vector load (lane u
    // holds entry k + u), read out lane by lane: one memory round trip per
    // group instead of a dependent scalar load per entry
    int cjv = 0;
    float wvv = 0.0f;
    if (lane < G && k + lane < k1) {
      cjv = cb[k + lane];
      wvv = vb[k + lane];
    }
    A y[G][EPL];
    A w[G];
    bool has[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      has[u] = false;
      w[u] = (A)0;
      if (k + u < k1) {
        const int cj = __builtin_amdgcn_readlane(cjv, u);
        const A wv = (A)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(wvv), u));
        rs += wv;
        if (cj != r) {
          has[u] = true;
          w[u] = wv;
          row_load<T, EPL, STRIDED, false>(yv + int64_t(cj) * d.ld, y[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
      if (has[u])
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[e] = fma(w[u], y[u][e] - yin[e], acc[e]);
  }
  A out[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const A ly = fma(rs, yin[e], acc[e]);  // (L Y)_r in difference form
    out[e] = alpha * ly + (beta * yin[e] + g3 * ypr[e]);
  }
  row_store<T, EPL, STRIDED, NT>(Yout + o, out);
}

template <typename T, int EPL, bool STRIDED, int WPG, bool NT>
__global__ void __launch_bounds__(64 * WPG)
    k_spmm_rowx(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                const CsrDesc* __restrict__ csr, const int32_t* __restrict__ row_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val,
                const T* __restrict__ Yin, const T* __restrict__ Yprev, T* __restrict__ Yout,
                const double* __restrict__ coef, int coef_stride, int step, int ntiles) {
  static_assert(SPMM_ROWS % WPG == 0, "workgroup split");
  typedef typename Acc<T>::type A;
  constexpr int SPLIT = SPMM_ROWS / WPG;
  const int per = (ntiles + NUM_XCD - 1) / NUM_XCD;
  const int kx = blockIdx.x / NUM_XCD;
  const int ti = (blockIdx.x % NUM_XCD) * per + kx / SPLIT;
  if (ti >= ntiles) return;
  const SpmmTile t = tiles[ti];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const MatDesc d = sets[t.set];
  const CsrDesc c = csr[t.set];
  const int r = t.row0 + (kx % SPLIT) * WPG + wave;
  if (r >= d.rows) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  const double* cf = coef + int64_t(d.blk) * coef_stride + 3 * step;
  rowx_row<T, EPL, STRIDED, NT>(d, c, r, lane, row_ptr, col, val, Yin, Yprev, Yout, (A)cf[0],
                                (A)cf[1], (A)cf[2]);
}

// The same rows with half a wavefront per row (two rows per wavefront, the
// WPG wavefronts of a workgroup on 2 WPG consecutive rows): a lane holds
// 2 EPL consecutive elements, so each of its loads and stores moves twice
// the bytes (16 bytes for 256-wide BF16 or 128-wide FP32 rows), and a
// wavefront has both rows' gathers in flight.  Each element sees the same
// operations in the same order as in k_spmm_rowx, so the results are
// bit-identical to it (the neighbour rows are gathered 4 at a time instead
// of 8, which changes only how many loads are in flight together, and keeps
// the doubled rows within the registers of 6 wavefronts per SIMD).  Rows of
// up to 256 columns (not strided).
template <typename T, int EPL, int WPG, bool NT>
__global__ void __launch_bounds__(64 * WPG)
    k_spmm_rowh(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                const CsrDesc* __restrict__ csr, const int32_t* __restrict__ row_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val,
                const T* __restrict__ Yin, const T* __restrict__ Yprev, T* __restrict__ Yout,
                const double* __restrict__ coef, int coef_stride, int step, int ntiles) {
  static_assert(SPMM_ROWS % (2 * WPG) == 0, "workgroup split");
  typedef typename Acc<T>::type A;
  constexpr int H = 2 * EPL;  // elements per lane
  constexpr int G = 4;
  constexpr int SPLIT = SPMM_ROWS / (2 * WPG);
  const int per = (ntiles + NUM_XCD - 1) / NUM_XCD;
  const int kx = blockIdx.x / NUM_XCD;
  const int ti = (blockIdx.x % NUM_XCD) * per + kx / SPLIT;
  if (ti >= ntiles) return;
  const SpmmTile t = tiles[ti];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const MatDesc d = sets[t.set];
  const CsrDesc c = csr[t.set];
  const int r0 = t.row0 + (kx % SPLIT) * 2 * WPG + 2 * wave;
  if (r0 >= d.rows) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  const int r = r0 + (lane >> 5);
  const bool act = r < d.rows;  // the second half of the last row pair may be past the block
  const double* cf = coef + int64_t(d.blk) * coef_stride + 3 * step;
  const A alpha = (A)cf[0], beta = (A)cf[1], gamma = (A)cf[2];
  const int l0 = (lane & 31) * H;
  const T* yv = Yin + d.off + l0;
  const int64_t o = d.off + int64_t(r) * d.ld + l0;
  A yin[H], ypr[H];
#pragma unroll
  for (int e = 0; e < H; ++e) yin[e] = ypr[e] = (A)0;
  int k0 = 0, k1 = 0;
  if (act) {
    row_load<T, H, false, false>(Yin + o, yin);
    if (Yprev) row_load<T, H, false, NT>(Yprev + o, ypr);
    k0 = row_ptr[c.rp_off + r];
    k1 = row_ptr[c.rp_off + r + 1];
  }
  const A g3 = Yprev ? gamma : (A)0;
  // entries of the longer of the two rows, for the wavefront's loop bound
  const int deg = k1 - k0;
  const int dmax = max(__builtin_amdgcn_readlane(deg, 0), __builtin_amdgcn_readlane(deg, 32));
  const int32_t* cb = col + c.nnz_off;
  const float* vb = val + c.nnz_off;
  A acc[H], rs = (A)0;
#pragma unroll
  for (int e = 0; e < H; ++e) acc[e] = (A)0;
  for (int j = 0; j < dmax; j += G) {
    A y[G][H];
    A w[G];
    bool has[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      has[u] = false;
      w[u] = (A)0;
      if (j + u < deg) {
        const int cj = cb[k0 + j + u];
        const A wv = (A)vb[k0 + j + u];
        rs += wv;
        if (cj != r) {
          has[u] = true;
          w[u] = wv;
          row_load<T, H, false, false>(yv + int64_t(cj) * d.ld, y[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
      if (has[u])
#pragma unroll
        for (int e = 0; e < H; ++e) acc[e] = fma(w[u], y[u][e] - yin[e], acc[e]);
  }
  if (!act) return;
  A out[H];
#pragma unroll
  for (int e = 0; e < H; ++e) {
    const A ly = fma(rs, yin[e], acc[e]);
    out[e] = alpha * ly + (beta * yin[e] + g3 * ypr[e]);
  }
  row_store<T, H, false, NT>(Yout + o, out);
}

// A whole filter pass (the m Chebyshev steps) in one persistent launch:
// each workgroup claims a block from the queue head (blocks in the order of
// `order`, largest first) and runs the pass's m steps on it, its wavefronts
// taking the block's rows in turn with the row product above, with a
// workgroup barrier between steps (a step reads only its own block's rows
// of the previous one).  Step k writes out[k mod 3], reading out[k-1] and
// out[k-2] (X for step 0, nothing before it), as the launch sequence of the
// separate steps does, so the result is bit-identical to it.  Every
// workgroup leaves once the queue head passes the last block.
template <typename T, int EPL, bool STRIDED>
__global__ void __launch_bounds__(64 * PASS_WAVES)
    k_cheb_pass(const MatDesc* __restrict__ sets, const CsrDesc* __restrict__ csr,
                const int32_t* __restrict__ order, int nsets, const int32_t* __restrict__ row_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val, const T* X,
                T* o0, T* o1, T* o2, const double* __restrict__ coef, int coef_stride, int m,
                int32_t* queue) {
  typedef typename Acc<T>::type A;
  __shared__ int job_s;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  for (;;) {
    if (threadIdx.x == 0) job_s = atomicAdd(queue, 1);
    __syncthreads();
    const int job = job_s;
    __syncthreads();  // every thread has read job_s before the next claim
    if (job >= nsets) break;  // workgroup-uniform
    const int si = order[job];
    const MatDesc d = sets[si];
    const CsrDesc c = csr[si];
    const double* cf = coef + int64_t(d.blk) * coef_stride;
    const T* cur = X;
    const T* prev = nullptr;
    for (int k = 0; k < m; ++k) {
      T* out = k % 3 == 0 ? o0 : k % 3 == 1 ? o1 : o2;
      const A alpha = (A)cf[3 * k], beta = (A)cf[3 * k + 1], gamma = (A)cf[3 * k + 2];
      // ordinary (cached) loads and stores: the workgroup's wavefronts share
      // the CU's L1, and the barrier makes every row of the step visible to
      // all of them before the next step reads it
      for (int r = wave; r < d.rows; r += PASS_WAVES)
        rowx_row<T, EPL, STRIDED, false>(d, c, r, lane, row_ptr, col, val, cur, prev, out, alpha,
                                         beta, gamma);
      __syncthreads();
      prev = cur;
      cur = out;
    }
  }
}

// The same product with two rows per wavefront: both rows' loads are in
// flight together, so a launch holds twice the rows per wavefront slot.
template <typename T, int EPL, bool STRIDED = false>
__global__ void __launch_bounds__(512)
    k_spmm_row2(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                const CsrDesc* __restrict__ csr, const int32_t* __restrict__ row_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val,
                const T* __restrict__ Yin, const T* __restrict__ Yprev, T* __restrict__ Yout,
                const double* __restrict__ coef, int coef_stride, int step, int ntiles) {
  const int per = (ntiles + NUM_XCD - 1) / NUM_XCD;
  const int ti = (blockIdx.x % NUM_XCD) * per + blockIdx.x / NUM_XCD;
  if (ti >= ntiles) return;
  const SpmmTile t = tiles[ti];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const MatDesc d = sets[t.set];
  const int ra = t.row0 + 2 * wave;
  if (ra >= d.rows) return;  // wave-uniform
  const bool two = ra + 1 < d.rows;
  const int rw[2] = {ra, two ? ra + 1 : ra};
  const CsrDesc c = csr[t.set];
  const int lane = threadIdx.x & 63;
  typedef Acc<T> AC;
  typedef typename AC::type A;
  const double* cf = coef + int64_t(d.blk) * coef_stride + 3 * step;
  const A alpha = (A)cf[0], beta = (A)cf[1], gamma = (A)cf[2];
  constexpr int ES = STRIDED ? 64 : 1;  // element stride of a lane
  const int l0 = STRIDED ? lane : lane * EPL;
  const T* yv = Yin + d.off + l0;
  const int32_t* cb = col + c.nnz_off;
  const float* vb = val + c.nnz_off;
  const T* yp = Yprev ? Yprev : Yin;
  const A g3 = Yprev ? gamma : (A)0;
  int64_t o[2];
  A yin[2][EPL], ypr[2][EPL];
  int k0[2], k1[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    o[h] = d.off + int64_t(rw[h]) * d.ld + l0;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      yin[h][e] = AC::load(Yin[o[h] + e * ES]);
      ypr[h][e] = AC::load(yp[o[h] + e * ES]);
    }
    k0[h] = row_ptr[c.rp_off + rw[h]];
    k1[h] = row_ptr[c.rp_off + rw[h] + 1];
  }
  A acc[2][EPL], base[2][EPL];
  {
    // first chunk of both rows (entries past a row gather the row itself
    // with weight 0)
    A y[2][SPMM_GATHER][EPL];
    A w[2][SPMM_GATHER];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < SPMM_GATHER; ++u) {
        const bool in = k0[h] + u < k1[h];
        w[h][u] = in ? (A)vb[k0[h] + u] : (A)0;
        const T* src = yv + int64_t(in ? cb[k0[h] + u] : rw[h]) * d.ld;
#pragma unroll
        for (int e = 0; e < EPL; ++e) y[h][u][e] = AC::load(src[e * ES]);
      }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        base[h][e] = beta * yin[h][e] + g3 * ypr[h][e];
        acc[h][e] = (A)0;
      }
#pragma unroll
      for (int u = 0; u < SPMM_GATHER; ++u)
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[h][e] = fma(w[h][u], y[h][u][e], acc[h][e]);
#pragma unroll
      for (int e = 0; e < EPL; ++e) asm volatile("" : "+v"(base[h][e]));
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
    for (int k = k0[h] + SPMM_GATHER; k < k1[h]; k += SPMM_GATHER) {
      A y[SPMM_GATHER][EPL];
      A w[SPMM_GATHER];
#pragma unroll
      for (int u = 0; u < SPMM_GATHER; ++u) {
        const int kk = min(k + u, k1[h] - 1);
        w[u] = k + u < k1[h] ? (A)vb[kk] : (A)0;
        const T* src = yv + int64_t(cb[kk]) * d.ld;
#pragma unroll
        for (int e = 0; e < EPL; ++e) y[u][e] = AC::load(src[e * ES]);
      }
#pragma unroll
      for (int u = 0; u < SPMM_GATHER; ++u)
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[h][e] = fma(w[u], y[u][e], acc[h][e]);
    }
#pragma unroll
  for (int e = 0; e < EPL; ++e) Yout[o[0] + e * ES] = AC::store(alpha * acc[0][e] + base[0][e]);
  if (two) {
#pragma unroll
    for (int e = 0; e < EPL; ++e)
      Yout[o[1] + e * ES] = AC::store(alpha * acc[1][e] + base[1][e]);
  }
}

template <typename T, int EPL, bool ST>
static void launch_spmm_rows(int var, const SpmmTile* tiles, int ntiles, const MatDesc* sets,
                             const CsrDesc* csr, const int32_t* row_ptr, const int32_t* col,
                             const float* val, const T* Yin, const T* Yprev, T* Yout,
                             const double* coef, int coef_stride, int step, hipStream_t s) {
  const dim3 grid(NUM_XCD * ceil_div(ntiles, NUM_XCD));
  if (var == SPMM_VAR_ROW2)
    hipLaunchKernelGGL((k_spmm_row2<T, EPL, ST>), grid, dim3(32 * SPMM_ROWS), 0, s, tiles, sets,
                       csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride, step, ntiles);
  else if (var == SPMM_VAR_ROW_G4)
    hipLaunchKernelGGL((k_spmm_row<T, EPL, ST, 4>), grid, dim3(64 * SPMM_ROWS), 0, s, tiles,
                       sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride, step,
                       ntiles);
  else if (var == SPMM_VAR_ROWS2)
    hipLaunchKernelGGL((k_spmm_rows<T, EPL, ST, 2>),
                       dim3(NUM_XCD * ceil_div(ceil_div(ntiles, 2), NUM_XCD)), dim3(1024), 0, s,
                       tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride,
                       step, ntiles);
  else if (var == SPMM_VAR_ROWS4)
    hipLaunchKernelGGL((k_spmm_rows<T, EPL, ST, 4>),
                       dim3(NUM_XCD * ceil_div(ceil_div(ntiles, 4), NUM_XCD)), dim3(1024), 0, s,
                       tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride,
                       step, ntiles);
  else if (var == SPMM_VAR_ROWS2_W4)
    hipLaunchKernelGGL((k_spmm_rows<T, EPL, ST, 2, 4>),
                       dim3(4 * NUM_XCD * ceil_div(ceil_div(ntiles, 2), NUM_XCD)), dim3(256), 0,
                       s, tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef,
                       coef_stride, step, ntiles);
  else if (var == SPMM_VAR_X8_NT)
    hipLaunchKernelGGL((k_spmm_rowx<T, EPL, ST, 8, true>), dim3(2 * grid.x), dim3(512), 0, s,
                       tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride,
                       step, ntiles);
  else if (var == SPMM_VAR_X16_NT) {
    // FP64 rows of 320 would spill in 16-wavefront workgroups: 8 instead
    if constexpr (sizeof(typename Acc<T>::type) * EPL > 32)
      hipLaunchKernelGGL((k_spmm_rowx<T, EPL, ST, 8, true>), dim3(2 * grid.x), dim3(512), 0, s,
                         tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef,
                         coef_stride, step, ntiles);
    else
      hipLaunchKernelGGL((k_spmm_rowx<T, EPL, ST, 16, true>), grid, dim3(1024), 0, s, tiles,
                         sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride, step,
                         ntiles);
  }
  else if (var == SPMM_VAR_X8)
    hipLaunchKernelGGL((k_spmm_rowx<T, EPL, ST, 8, false>), dim3(2 * grid.x), dim3(512), 0, s,
                       tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride,
                       step, ntiles);
  else if (var == SPMM_VAR_XH8_NT || var == SPMM_VAR_XH4_NT) {
    // half a wavefront per row: rows of up to 256 columns; wider (strided)
    // rows take the one-wavefront kernel, which gives the same bits
    if constexpr (!ST && EPL <= 4) {
      if (var == SPMM_VAR_XH8_NT)
        hipLaunchKernelGGL((k_spmm_rowh<T, EPL, 8, true>), grid, dim3(512), 0, s, tiles, sets,
                           csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride, step,
                           ntiles);
      else
        hipLaunchKernelGGL((k_spmm_rowh<T, EPL, 4, true>), dim3(2 * grid.x), dim3(256), 0, s,
                           tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef,
                           coef_stride, step, ntiles);
    } else {
      hipLaunchKernelGGL((k_spmm_rowx<T, EPL, ST, 8, true>), dim3(2 * grid.x), dim3(512), 0, s,
                         tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride,
                         step, ntiles);
    }
  }
  else if (var == SPMM_VAR_X4_NT)
    hipLaunchKernelGGL((k_spmm_rowx<T, EPL, ST, 4, true>), dim3(4 * grid.x), dim3(256), 0, s,
                       tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride,
                       step, ntiles);
  else if (var == SPMM_VAR_ROW_W4)
    hipLaunchKernelGGL((k_spmm_row<T, EPL, ST, SPMM_GATHER, 4>), dim3(4 * grid.x), dim3(256), 0,
                       s, tiles, sets, csr, row_ptr, col, val, Yin, Yprev, Yout, coef,
                       coef_stride, step, ntiles);
  else
    hipLaunchKernelGGL((k_spmm_row<T, EPL, ST>), grid, dim3(64 * SPMM_ROWS), 0, s, tiles, sets,
                       csr, row_ptr, col, val, Yin, Yprev, Yout, coef, coef_stride, step, ntiles);
}

// Without the autotuner: the exact-gather kernel in 8-wavefront workgroups
// with non-temporal streams (the fastest on slabs far beyond the caches).
int spmm_default_var(int) { return SPMM_VAR_X8_NT; }

template <typename T>
void launch_spmm(const SpmmTile* tiles, int ntiles, const MatDesc* sets, const CsrDesc* csr,
                 const int32_t* row_ptr, const int32_t* col, const float* val, const T* Yin,
                 const T* Yprev, T* Yout, const double* coef, int coef_stride, int step,
                 hipStream_t s, int epl, int var) {
  if (ntiles <= 0) return;
  if (var < 0) var = spmm_default_var(epl);
#define MI_SPMM_ROWS(E, ST)                                                                    \
  case E:                                                                                      \
    launch_spmm_rows<T, E, ST>(var, tiles, ntiles, sets, csr, row_ptr, col, val, Yin, Yprev,   \
                               Yout, coef, coef_stride, step, s);                              \
    return;
  switch (epl) {
    MI_SPMM_ROWS(1, false)
    MI_SPMM_ROWS(2, false)
    MI_SPMM_ROWS(3, false)
    MI_SPMM_ROWS(4, false)
    MI_SPMM_ROWS(5, true)
    default:
      break;
  }
#undef MI_SPMM_ROWS
  // the vector kernel for waves of mixed widths (FP32 and FP64 slabs only: the
  // plan refuses BF16 slabs without a uniform width)
  if constexpr (!std::is_same<T, bf16>::value)
    hipLaunchKernelGGL(k_spmm<T>, dim3(ntiles), dim3(256), 0, s, tiles, sets, csr, row_ptr, col,
                       val, Yin, Yprev, Yout, coef, coef_stride, step);
}

template void launch_spmm<float>(const SpmmTile*, int, const MatDesc*, const CsrDesc*,
                                 const int32_t*, const int32_t*, const float*, const float*,
                                 const float*, float*, const double*, int, int, hipStream_t, int,
                                 int);
template void launch_spmm<double>(const SpmmTile*, int, const MatDesc*, const CsrDesc*,
                                  const int32_t*, const int32_t*, const float*, const double*,
                                  const double*, double*, const double*, int, int, hipStream_t,
                                  int, int);
template void launch_spmm<bf16>(const SpmmTile*, int, const MatDesc*, const CsrDesc*,
                                const int32_t*, const int32_t*, const float*, const bf16*,
                                const bf16*, bf16*, const double*, int, int, hipStream_t, int,
                                int);

template <typename T>
void launch_cheb_pass(const MatDesc* sets, const CsrDesc* csr, const int32_t* order, int nsets,
                      const int32_t* row_ptr, const int32_t* col, const float* val, const T* X,
                      T* o0, T* o1, T* o2, const double* coef, int coef_stride, int m,
                      int32_t* queue, int grid, int epl, hipStream_t s) {
  if (nsets <= 0 || m <= 0 || grid <= 0) return;
  fill_i32(queue, 0, 1, s);
#define MI_PASS(E, ST)                                                                          \
  case E:                                                                                       \
    hipLaunchKernelGGL((k_cheb_pass<T, E, ST>), dim3(grid), dim3(64 * PASS_WAVES), 0, s, sets,  \
                       csr, order, nsets, row_ptr, col, val, X, o0, o1, o2, coef, coef_stride, \
                       m, queue);                                                               \
    return;
  switch (epl) {
    MI_PASS(1, false)
    MI_PASS(2, false)
    MI_PASS(3, false)
    MI_PASS(4, false)
    MI_PASS(5, true)
    default:
      return;
  }
#undef MI_PASS
}

template <typename T>
int cheb_pass_grid(int epl, int nsets) {
  int per_cu = 0;
#define MI_OCC(E, ST)                                                                           \
  case E:                                                                                       \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cheb_pass<T, E, ST>,           \
                                                     64 * PASS_WAVES, 0) != hipSuccess)         \
      per_cu = 0;                                                                               \
    break;
  switch (epl) {
    MI_OCC(1, false)
    MI_OCC(2, false)
    MI_OCC(3, false)
    MI_OCC(4, false)
    MI_OCC(5, true)
    default:
      return 0;
  }
#undef MI_OCC
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return std::min(nsets, std::max(per_cu, 1) * std::max(cus, 1));
}

#define MI_PASS_INST(T)                                                                         \
  template void launch_cheb_pass<T>(const MatDesc*, const CsrDesc*, const int32_t*, int,       \
                                    const int32_t*, const int32_t*, const float*, const T*,    \
                                    T*, T*, T*, const double*, int, int, int32_t*, int, int,   \
                                    hipStream_t);                                               \
  template int cheb_pass_grid<T>(int, int);
MI_PASS_INST(float)
MI_PASS_INST(double)
MI_PASS_INST(bf16)
#undef MI_PASS_INST

// ------------------------------------------------------------------ Rayleigh quotients
// q_j^T L q_j for the columns of an orthonormalised basis X from W = L X:
// sums over RQ_CHUNKS row chunks of each block (a workgroup per block and
// chunk, threads over the columns, rows in order) into the block's p x p
// matrix slot (RQ_CHUNKS rows of ld doubles), then per block the chunks in
// order and the largest quotient over its p columns.
constexpr int RQ_CHUNKS = 8;

template <typename T>
__global__ void __launch_bounds__(256)
    k_rq_part(const MatDesc* __restrict__ sets, const MatDesc* __restrict__ osets,
              const T* __restrict__ X, const T* __restrict__ W, double* __restrict__ part) {
  const int b = blockIdx.x / RQ_CHUNKS, c = blockIdx.x % RQ_CHUNKS;
  const MatDesc d = sets[b];
  const int per = (d.rows + RQ_CHUNKS - 1) / RQ_CHUNKS;
  const int r0 = c * per, r1 = min(d.rows, r0 + per);
  double* out = part + osets[b].off + int64_t(c) * d.ld;
  for (int j = threadIdx.x; j < d.ld; j += 256) {
    double s = 0.0;
#pragma unroll 4
    for (int r = r0; r < r1; ++r) {
      const int64_t e = d.off + int64_t(r) * d.ld + j;
      s = fma((double)Acc<T>::load(X[e]), (double)Acc<T>::load(W[e]), s);
    }
    out[j] = s;
  }
}

__global__ void __launch_bounds__(256)
    k_rq_final(const MatDesc* __restrict__ sets, const MatDesc* __restrict__ osets,
               const double* __restrict__ part, double* __restrict__ a_lo) {
  __shared__ double red[4];
  const MatDesc d = sets[blockIdx.x];
  const double* pb = part + osets[blockIdx.x].off;
  double mx = -1e308;
  for (int j = threadIdx.x; j < d.cols; j += 256) {
    double s = 0.0;
    for (int c = 0; c < RQ_CHUNKS; ++c) s += pb[int64_t(c) * d.ld + j];
    mx = fmax(mx, s);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) a_lo[d.blk] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

template <typename T>
void launch_rq(const MatDesc* sets, const MatDesc* osets, int nb, const T* X, const T* W,
               double* part, double* a_lo, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_rq_part<T>, dim3(nb * RQ_CHUNKS), dim3(256), 0, s, sets, osets, X, W,
                     part);
  hipLaunchKernelGGL(k_rq_final, dim3(nb), dim3(256), 0, s, sets, osets, (const double*)part,
                     a_lo);
}
template void launch_rq<float>(const MatDesc*, const MatDesc*, int, const float*, const float*,
                               double*, double*, hipStream_t);
template void launch_rq<double>(const MatDesc*, const MatDesc*, int, const double*, const double*,
                                double*, double*, hipStream_t);
template void launch_rq<bf16>(const MatDesc*, const MatDesc*, int, const bf16*, const bf16*,
                              double*, double*, hipStream_t);

// ------------------------------------------------------------------ Gram
// One workgroup: a 64 x 64 super-tile of A^T B (and A^T W when DUAL) over a
// row range, staged through LDS 32 rows at a time from 16-byte vector loads
// (the next chunk is fetched while the current one is multiplied).  Four
// waves, each a 32 x 32 quadrant as 2 x 2 tiles of the 16x16x4 FP64 MFMA.  Operands are promoted to FP64 exactly, so every
// product is exact and only the FP64 accumulation rounds.
// MFMA operand layout (16x16x4): lane l supplies A(m = l%16, k = l/16) and
// B(k = l/16, n = l%16).  Result element (m, n = l%16) sits in register q of
// lane l with m = l/16 + 4q for the FP64 instruction and m = 4(l/16) + q for
// the FP32 one (measured lane layouts).
// Workgroups are dealt to the 8 XCDs in contiguous tile ranges (workgroup i
// takes tile (i mod 8) * per + i / 8): tiles that read the same rows (a row
// product's output-column chunks, neighbours in its table) then run on one
// XCD and read those rows through its L2 once, instead of once per tile
// from HBM (5% off the row product on the 1,024-disk slab; the Gram's
// super-tile pairs measured 3% slower dealt this way and keep the plain
// order).
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int per = (ntiles + NUM_XCD - 1) / NUM_XCD;
  return int(blockIdx.x % NUM_XCD) * per + int(blockIdx.x / NUM_XCD);
}
inline dim3 xcd_grid(int ntiles) { return dim3(NUM_XCD * ceil_div(ntiles, NUM_XCD)); }

// With G non-null the tile is the whole super-tile (no split over row
// chunks): its upper triangle and the mirror go straight into the p x p
// outputs G (and H) described by outsets, and no partial is written.
template <typename T, bool DUAL>
__global__ void __launch_bounds__(256)
    k_gram(const GramTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
           const T* __restrict__ A, const T* __restrict__ B, const T* __restrict__ Wm,
           double* __restrict__ part, const MatDesc* __restrict__ outsets, double* __restrict__ G,
           double* __restrict__ H) {
  typedef typename VecOf<T>::type V;
  constexpr int W = VecOf<T>::W;
  constexpr int RC = 32;                            // rows per staged chunk
  constexpr int NV = RC * GRAM_TILE / W / 256;      // vectors per operand and thread
  constexpr int LDT = GRAM_TILE + 16;               // row offset of a quarter (FP32) /
                                                    // half (FP64) of the banks
  constexpr int NOP = DUAL ? 3 : 2;
  __shared__ __attribute__((aligned(16))) T St[NOP][RC * LDT];
  const int ti = blockIdx.x;  // partial slot = table position
  const GramTile t = tiles[ti];
  const MatDesc d = sets[t.set];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int kq = lane >> 4, mi = lane & 15;
  d4v acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
  d4v w00 = acc00, w01 = acc00, w10 = acc00, w11 = acc00;
  const T* src[3] = {A + d.off, B + d.off, DUAL ? Wm + d.off : nullptr};
  const int c0[3] = {t.I0, t.J0, t.J0};
  V reg[NOP][NV];
  // rows [r, r + RC) of the three column panels -> registers (zero outside)
  auto fetch = [&](int r) {
#pragma unroll
    for (int o = 0; o < NOP; ++o)
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        const int e = threadIdx.x + 256 * j;
        const int rr = e / (GRAM_TILE / W), cv = e % (GRAM_TILE / W);
        const int row = r + rr, col = c0[o] + cv * W;
        reg[o][j] = (row < t.r1 && col < d.ld)
                        ? *reinterpret_cast<const V*>(src[o] + int64_t(row) * d.ld + col)
                        : (V)(T)0;
      }
  };
  fetch(t.r0);
  for (int r = t.r0; r < t.r1; r += RC) {
#pragma unroll
    for (int o = 0; o < NOP; ++o)
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        const int e = threadIdx.x + 256 * j;
        *reinterpret_cast<V*>(&St[o][(e / (GRAM_TILE / W)) * LDT + (e % (GRAM_TILE / W)) * W]) =
            reg[o][j];
      }
    __syncthreads();
    if (r + RC < t.r1) fetch(r + RC);  // in flight during the MFMAs
#pragma unroll
    for (int ks = 0; ks < RC; ks += 4) {
      const T* ar = &St[0][(ks + kq) * LDT];
      const T* br = &St[1][(ks + kq) * LDT];
      const double a0 = (double)ar[wi * 32 + mi], a1 = (double)ar[wi * 32 + 16 + mi];
      const double b0 = (double)br[wj * 32 + mi], b1 = (double)br[wj * 32 + 16 + mi];
      acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
      if (DUAL) {
        const T* xr = &St[DUAL ? 2 : 0][(ks + kq) * LDT];
        const double x0 = (double)xr[wj * 32 + mi], x1 = (double)xr[wj * 32 + 16 + mi];
        w00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x0, w00, 0, 0, 0);
        w01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x1, w01, 0, 0, 0);
        w10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x0, w10, 0, 0, 0);
        w11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x1, w11, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int kk = kq, mm = mi;
  const int n = mm;
  if (G) {
    const MatDesc o = outsets[t.set];
    auto put = [&](double* M, int li, int lj, double v) {
      const int gi = t.I0 + li, gj = t.J0 + lj;
      if (gi <= gj && gj < o.ld) {
        M[o.off + int64_t(gi) * o.ld + gj] = v;
        M[o.off + int64_t(gj) * o.ld + gi] = v;
      }
    };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = kk + 4 * q;  // FP64 result layout
      const int i0 = wi * 32 + m, i1 = i0 + 16;
      const int j0 = wj * 32 + n, j1 = j0 + 16;
      put(G, i0, j0, acc00[q]);
      put(G, i0, j1, acc01[q]);
      put(G, i1, j0, acc10[q]);
      put(G, i1, j1, acc11[q]);
      if (DUAL) {
        put(H, i0, j0, w00[q]);
        put(H, i0, j1, w01[q]);
        put(H, i1, j0, w10[q]);
        put(H, i1, j1, w11[q]);
      }
    }
    return;
  }
  double* out = part + int64_t(ti) * (DUAL ? 2 : 1) * GRAM_TILE * GRAM_TILE;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = kk + 4 * q;  // FP64 result layout
    const int i0 = wi * 32 + m, i1 = i0 + 16;
    const int j0 = wj * 32 + n, j1 = j0 + 16;
    out[i0 * GRAM_TILE + j0] = acc00[q];
    out[i0 * GRAM_TILE + j1] = acc01[q];
    out[i1 * GRAM_TILE + j0] = acc10[q];
    out[i1 * GRAM_TILE + j1] = acc11[q];
    if (DUAL) {
      double* o2 = out + GRAM_TILE * GRAM_TILE;
      o2[i0 * GRAM_TILE + j0] = w00[q];
      o2[i0 * GRAM_TILE + j1] = w01[q];
      o2[i1 * GRAM_TILE + j0] = w10[q];
      o2[i1 * GRAM_TILE + j1] = w11[q];
    }
  }
}

// The same super-tiles for BF16 slabs on the BF16 MFMA (16x16x16, FP32
// accumulation): products of two BF16 values are exact in FP32, so only the
// FP32 sums over one staged chunk of 32 rows round; each chunk's sums are
// added into FP64 accumulators, and the partials in FP64 like the other
// Grams (an FP32 sum over all of a workgroup's rows would cost the
// Cholesky-QR its orthogonality on ill-conditioned iterates).  Each 32-row chunk of the three column
// panels is staged through LDS transposed (a column's rows contiguous), so
// that a lane's four consecutive-row operands are one 64-bit LDS read.
// Operand layout (16x16x16 BF16): lane l supplies A(m = l%16, k = 4(l/16) +
// i) and B(k = 4(l/16) + i, n = l%16), i < 4; result (m = 4(l/16) + q, n =
// l%16) in register q.
typedef short s4v __attribute__((ext_vector_type(4)));

template <bool DUAL>
__global__ void __launch_bounds__(256)
    k_gram_bf16(const GramTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                const bf16* __restrict__ A, const bf16* __restrict__ B,
                const bf16* __restrict__ Wm, double* __restrict__ part) {
  constexpr int RC = 32;           // rows per staged chunk
  constexpr int LDT = RC + 8;      // LDS stride of a column (bf16 elements)
  constexpr int NOP = DUAL ? 3 : 2;
  __shared__ __attribute__((aligned(16))) uint16_t St[NOP][GRAM_TILE * LDT];
  const int ti = blockIdx.x;  // partial slot = table position
  const GramTile t = tiles[ti];
  const MatDesc d = sets[t.set];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int kq = lane >> 4, mi = lane & 15;
  d4v acc[2][2], accw[2][2];  // FP64 sums over the chunks
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = accw[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
  const bf16* src[3] = {A + d.off, B + d.off, DUAL ? Wm + d.off : nullptr};
  const int c0[3] = {t.I0, t.J0, t.J0};
  // thread e stages 8 consecutive columns of one row of each panel
  const int srow = threadIdx.x >> 3, scol = (threadIdx.x & 7) * 8;
  uint4 reg[NOP];
  auto fetch = [&](int r) {
#pragma unroll
    for (int o = 0; o < NOP; ++o) {
      const int row = r + srow, col = c0[o] + scol;
      reg[o] = (row < t.r1 && col < d.ld)
                   ? *reinterpret_cast<const uint4*>(src[o] + int64_t(row) * d.ld + col)
                   : uint4{0u, 0u, 0u, 0u};
    }
  };
  fetch(t.r0);
  for (int r = t.r0; r < t.r1; r += RC) {
#pragma unroll
    for (int o = 0; o < NOP; ++o) {
      const uint32_t w4[4] = {reg[o].x, reg[o].y, reg[o].z, reg[o].w};
#pragma unroll
      for (int j = 0; j < 8; ++j)
        St[o][(scol + j) * LDT + srow] = uint16_t(w4[j >> 1] >> (16 * (j & 1)));
    }
    __syncthreads();
    if (r + RC < t.r1) fetch(r + RC);  // in flight during the MFMAs
    f4v c32[2][2], w32[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) c32[i][j] = w32[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < RC; ks += 16) {
      s4v a[2], b[2], x[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        a[h] = *reinterpret_cast<const s4v*>(&St[0][(wi * 32 + h * 16 + mi) * LDT + ks + 4 * kq]);
        b[h] = *reinterpret_cast<const s4v*>(&St[1][(wj * 32 + h * 16 + mi) * LDT + ks + 4 * kq]);
        if (DUAL)
          x[h] = *reinterpret_cast<const s4v*>(
              &St[DUAL ? 2 : 0][(wj * 32 + h * 16 + mi) * LDT + ks + 4 * kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], c32[i][j], 0, 0, 0);
          if (DUAL)
            w32[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], x[j], w32[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[i][j][q] += (double)c32[i][j][q];
          if (DUAL) accw[i][j][q] += (double)w32[i][j][q];
        }
    __syncthreads();
  }
  double* out = part + int64_t(ti) * (DUAL ? 2 : 1) * GRAM_TILE * GRAM_TILE;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = wi * 32 + i * 16 + 4 * kq + q, n = wj * 32 + j * 16 + mi;
        out[m * GRAM_TILE + n] = acc[i][j][q];
        if (DUAL) out[GRAM_TILE * GRAM_TILE + m * GRAM_TILE + n] = accw[i][j][q];
      }
}

template <>
void launch_gram<bf16>(const GramTile* tiles, int ntiles, const MatDesc* sets, const bf16* A,
                       const bf16* B, const bf16* W, double* part, hipStream_t s) {
  if (ntiles <= 0) return;
  if (W)
    hipLaunchKernelGGL(k_gram_bf16<true>, dim3(ntiles), dim3(256), 0, s, tiles, sets, A, B,
                       W, part);
  else
    hipLaunchKernelGGL(k_gram_bf16<false>, dim3(ntiles), dim3(256), 0, s, tiles, sets, A, B,
                       W, part);
}

template <typename T>
void launch_gram(const GramTile* tiles, int ntiles, const MatDesc* sets, const T* A, const T* B,
                 const T* W, double* part, hipStream_t s) {
  if (ntiles <= 0) return;
  if (W)
    hipLaunchKernelGGL((k_gram<T, true>), dim3(ntiles), dim3(256), 0, s, tiles, sets, A, B,
                       W, part, nullptr, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_gram<T, false>), dim3(ntiles), dim3(256), 0, s, tiles, sets, A, B,
                       W, part, nullptr, nullptr, nullptr);
}
template void launch_gram<float>(const GramTile*, int, const MatDesc*, const float*, const float*,
                                 const float*, double*, hipStream_t);
template void launch_gram<double>(const GramTile*, int, const MatDesc*, const double*,
                                  const double*, const double*, double*, hipStream_t);

template <typename T>
void launch_gram_direct(const GramTile* tiles, int ntiles, const MatDesc* sets,
                        const MatDesc* outsets, const T* A, const T* B, const T* W, double* G,
                        double* H, hipStream_t s) {
  if (ntiles <= 0) return;
  if (W)
    hipLaunchKernelGGL((k_gram<T, true>), dim3(ntiles), dim3(256), 0, s, tiles, sets, A, B,
                       W, nullptr, outsets, G, H);
  else
    hipLaunchKernelGGL((k_gram<T, false>), dim3(ntiles), dim3(256), 0, s, tiles, sets, A, B,
                       W, nullptr, outsets, G, H);
}
template void launch_gram_direct<float>(const GramTile*, int, const MatDesc*, const MatDesc*,
                                        const float*, const float*, const float*, double*,
                                        double*, hipStream_t);
template void launch_gram_direct<double>(const GramTile*, int, const MatDesc*, const MatDesc*,
                                         const double*, const double*, const double*, double*,
                                         double*, hipStream_t);

bool gram_unsplit(const std::vector<GramReduce>& jobs) {
  for (const GramReduce& g : jobs)
    if (g.count != 1) return false;
  return true;
}

// Sum the split-K partials of one super-tile in chunk order (deterministic)
// and write the upper triangle and its mirror.  GRAM_RED_SPLIT workgroups
// per super-tile, one element per thread, partial loads issued together.
constexpr int GRAM_RED_SPLIT = GRAM_TILE * GRAM_TILE / 256;
__global__ void __launch_bounds__(256)
    k_gram_reduce(const GramReduce* __restrict__ jobs, const MatDesc* __restrict__ outsets,
                  const double* __restrict__ part, int dual, double* __restrict__ G,
                  double* __restrict__ H) {
  const GramReduce j = jobs[blockIdx.x / GRAM_RED_SPLIT];
  const MatDesc o = outsets[j.set];
  const int64_t stride = int64_t(dual ? 2 : 1) * GRAM_TILE * GRAM_TILE;
  const int e = (blockIdx.x % GRAM_RED_SPLIT) * 256 + threadIdx.x;
  const int il = e / GRAM_TILE, jl = e % GRAM_TILE;
  const int gi = j.I0 + il, gj = j.J0 + jl;
  if (gi >= o.ld || gj >= o.ld || gi > gj) return;
  const double* pp = part + int64_t(j.first) * stride + e;
  const int64_t cs = int64_t(j.stride) * stride;  // from one chunk's partial to the next
  double sg = 0.0, sh = 0.0;
  int c = 0;
  for (; c + 4 <= j.count; c += 4) {
    const double g0 = pp[(c + 0) * cs], g1 = pp[(c + 1) * cs];
    const double g2 = pp[(c + 2) * cs], g3 = pp[(c + 3) * cs];
    sg += g0;
    sg += g1;
    sg += g2;
    sg += g3;
    if (dual) {
      const double h0 = pp[(c + 0) * cs + GRAM_TILE * GRAM_TILE];
      const double h1 = pp[(c + 1) * cs + GRAM_TILE * GRAM_TILE];
      const double h2 = pp[(c + 2) * cs + GRAM_TILE * GRAM_TILE];
      const double h3 = pp[(c + 3) * cs + GRAM_TILE * GRAM_TILE];
      sh += h0;
      sh += h1;
      sh += h2;
      sh += h3;
    }
  }
  for (; c < j.count; ++c) {
    sg += pp[c * cs];
    if (dual) sh += pp[c * cs + GRAM_TILE * GRAM_TILE];
  }
  G[o.off + int64_t(gi) * o.ld + gj] = sg;
  G[o.off + int64_t(gj) * o.ld + gi] = sg;
  if (dual) {
    H[o.off + int64_t(gi) * o.ld + gj] = sh;
    H[o.off + int64_t(gj) * o.ld + gi] = sh;
  }
}

void launch_gram_reduce(const GramReduce* jobs, int njobs, const MatDesc* outsets,
                        const double* part, bool dual, double* G, double* H, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_gram_reduce, dim3(njobs * GRAM_RED_SPLIT), dim3(256), 0, s, jobs, outsets,
                     part, dual ? 1 : 0, G, H);
}

// ------------------------------------------------------------------ A * S
// Out rows [row0, row0+64) x columns [n0, n0+NCH) = A rows x S.  Per K-chunk
// of 32, the A row tile and the S panel are staged through LDS from 16-byte
// vector loads; the next chunk is fetched into registers while the MFMAs of
// the current one run.  Each wave owns 16 rows and NCH/16 MFMA tiles.
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef f4v acc_t;
  __device__ static acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};
template <>
struct Mfma<double> {
  typedef d4v acc_t;
  __device__ static acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};

// A may be a BF16 slab (TA = bf16, T = float): its chunk is widened to FP32
// on the way into LDS and the product runs on the FP32 MFMA.
template <typename TA, typename T, typename TO, int NCH>
__global__ void __launch_bounds__(256)
    k_rowmul(const RowTile* __restrict__ tiles, const MatDesc* __restrict__ asets,
             const TA* __restrict__ A, const MatDesc* __restrict__ ssets, const T* __restrict__ S,
             const MatDesc* __restrict__ osets, TO* __restrict__ Out, int ntiles, int upper) {
  typedef typename VecOf<T>::type V;
  typedef typename VecOf<TA>::type VA;
  constexpr int W = VecOf<T>::W;           // elements per 16-byte vector
  constexpr int WA = VecOf<TA>::W;
  constexpr int KC = 32;
  constexpr int NT = NCH / 16;
  constexpr int AV = ROW_TILE * KC / WA / 256;  // A vectors per thread and chunk
  constexpr int SV = KC * NCH / W / 256;        // S vectors per thread and chunk
  constexpr int LDA = KC + W;                   // keeps vector rows aligned, spreads banks
  constexpr int LDS_ = NCH + (sizeof(T) == 4 ? 16 : 16);  // row offset of half the banks
  static_assert(AV * WA * 256 == ROW_TILE * KC && SV * W * 256 == KC * NCH, "tile shape");
  static_assert(std::is_same<TA, T>::value || (std::is_same<TA, bf16>::value &&
                                              std::is_same<T, float>::value), "A type");
  __shared__ __attribute__((aligned(16))) T As[ROW_TILE * LDA];
  __shared__ __attribute__((aligned(16))) T Ss[KC * LDS_];
  typedef typename Mfma<T>::acc_t acc_t;
  const int ti = xcd_tile(ntiles);
  if (ti >= ntiles) return;
  const RowTile t = tiles[ti];
  const MatDesc da = asets[t.set], ds = ssets[t.set], dout = osets[t.set];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // an upper triangular S has no entries below row n in column n: the
  // output columns [n0, n0 + NCH) need only its rows k < n0 + NCH (the
  // chunks skipped would add products with exact zeros)
  const int K = upper ? min(ds.rows, t.n0 + NCH) : ds.rows;
  acc_t acc[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) acc[i] = (acc_t)(T)0;
  VA ra[AV];
  V rs[SV];
  // chunk k0 -> registers (rows past the block and columns past S read as 0)
  auto fetch = [&](int k0) {
#pragma unroll
    for (int j = 0; j < AV; ++j) {
      const int e = threadIdx.x + 256 * j;
      const int rr = e / (KC / WA), kv = e % (KC / WA);
      const int row = t.row0 + rr;
      if (row < da.rows)
        ra[j] = *reinterpret_cast<const VA*>(A + da.off + int64_t(row) * da.ld + k0 + kv * WA);
      else
        __builtin_memset(&ra[j], 0, sizeof(VA));
    }
#pragma unroll
    for (int j = 0; j < SV; ++j) {
      const int e = threadIdx.x + 256 * j;
      const int kr = e / (NCH / W), nv = e % (NCH / W);
      const int n = t.n0 + nv * W;
      rs[j] = (n < ds.ld)
                  ? *reinterpret_cast<const V*>(S + ds.off + int64_t(k0 + kr) * ds.ld + n)
                  : (V)(T)0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
    for (int j = 0; j < AV; ++j) {
      const int e = threadIdx.x + 256 * j;
      T* dst = &As[(e / (KC / WA)) * LDA + (e % (KC / WA)) * WA];
      if constexpr (std::is_same<TA, T>::value) {
        *reinterpret_cast<V*>(dst) = ra[j];
      } else {
        const uint32_t w4[4] = {ra[j].x, ra[j].y, ra[j].z, ra[j].w};
        f4v lo, hi;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          lo[2 * q] = bf16_to_f32(bf16{uint16_t(w4[q])});
          lo[2 * q + 1] = bf16_to_f32(bf16{uint16_t(w4[q] >> 16)});
          hi[2 * q] = bf16_to_f32(bf16{uint16_t(w4[2 + q])});
          hi[2 * q + 1] = bf16_to_f32(bf16{uint16_t(w4[2 + q] >> 16)});
        }
        *reinterpret_cast<f4v*>(dst) = lo;
        *reinterpret_cast<f4v*>(dst + 4) = hi;
      }
    }
#pragma unroll
    for (int j = 0; j < SV; ++j) {
      const int e = threadIdx.x + 256 * j;
      *reinterpret_cast<V*>(&Ss[(e / (NCH / W)) * LDS_ + (e % (NCH / W)) * W]) = rs[j];
    }
    __syncthreads();
    if (k0 + KC < K) fetch(k0 + KC);  // in flight while the MFMAs run
#pragma unroll 2
    for (int ks = 0; ks < KC; ks += 4) {
      const T a = As[(wave * 16 + (lane & 15)) * LDA + ks + (lane >> 4)];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const T b = Ss[(ks + (lane >> 4)) * LDS_ + nt * 16 + (lane & 15)];
        acc[nt] = Mfma<T>::op(a, b, acc[nt]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = t.n0 + nt * 16 + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = t.row0 + wave * 16 + Mfma<T>::row(lane, q);
      if (row < dout.rows && n < dout.ld)
        Out[dout.off + int64_t(row) * dout.ld + n] = Acc<TO>::store((typename Acc<TO>::type)acc[nt][q]);
    }
  }
}

template <typename TA, typename T, typename TO>
void launch_rowmul(const RowTile* tiles, int ntiles, const MatDesc* asets, const TA* A,
                   const MatDesc* ssets, const T* S, const MatDesc* osets, TO* Out, int nch,
                   hipStream_t s, bool upper) {
  if (ntiles <= 0) return;
  switch (nch) {
#define MI_ROWMUL_CASE(N)                                                                       \
  case N:                                                                                       \
    hipLaunchKernelGGL((k_rowmul<TA, T, TO, N>), xcd_grid(ntiles), dim3(256), 0, s, tiles,     \
                       asets, A, ssets, S, osets, Out, ntiles, upper ? 1 : 0);                  \
    break;
    MI_ROWMUL_CASE(32)
    MI_ROWMUL_CASE(64)
    MI_ROWMUL_CASE(96)
    MI_ROWMUL_CASE(128)
    MI_ROWMUL_CASE(192)
    MI_ROWMUL_CASE(256)
#undef MI_ROWMUL_CASE
    default:
      break;  // the tile planner only produces the widths above
  }
}

template void launch_rowmul<float, float, float>(const RowTile*, int, const MatDesc*,
                                                 const float*, const MatDesc*, const float*,
                                                 const MatDesc*, float*, int, hipStream_t, bool);
template void launch_rowmul<double, double, double>(const RowTile*, int, const MatDesc*,
                                                    const double*, const MatDesc*, const double*,
                                                    const MatDesc*, double*, int, hipStream_t, bool);
template void launch_rowmul<double, double, float>(const RowTile*, int, const MatDesc*,
                                                   const double*, const MatDesc*, const double*,
                                                   const MatDesc*, float*, int, hipStream_t, bool);
template void launch_rowmul<bf16, float, bf16>(const RowTile*, int, const MatDesc*, const bf16*,
                                               const MatDesc*, const float*, const MatDesc*, bf16*,
                                               int, hipStream_t, bool);
template void launch_rowmul<bf16, float, float>(const RowTile*, int, const MatDesc*, const bf16*,
                                                const MatDesc*, const float*, const MatDesc*,
                                                float*, int, hipStream_t, bool);

// ------------------------------------------------------------------ tile tables

int gram_chunks(int nsets, int npairs, int rows, int target) {
  // target: workgroups per launch (enough to fill the chip, few partials)
  int ch = ceil_div(target, std::max(1, nsets * npairs));
  ch = std::min(ch, std::max(1, rows / 64));
  return std::max(ch, 1);
}

// Gram tile table for a list of per-block matrices with `rows` rows each:
// per block, its row chunks in order, and per chunk every super-tile pair
// (I <= J), so that a chunk's pairs are neighbours in the table (and on one
// XCD, see gram_tile_of); a pair's partials are npairs tiles apart.
void gram_tables(const std::vector<MatDesc>& sets, bool split,
                 std::vector<GramTile>* tiles, std::vector<GramReduce>* red, int target) {
  for (int si = 0; si < (int)sets.size(); ++si) {
    const MatDesc& d = sets[si];
    const int nsup = ceil_div(d.ld, GRAM_TILE);
    const int npairs = nsup * (nsup + 1) / 2;
    const int ch = split ? gram_chunks((int)sets.size(), npairs, d.rows, target) : 1;
    int rows_per = ceil_div(d.rows, ch);
    rows_per = ((rows_per + 15) / 16) * 16;
    const int base = (int)tiles->size();
    int nch = 0;
    for (int r0 = 0; r0 < d.rows; r0 += rows_per, ++nch)
      for (int I = 0; I < nsup; ++I)
        for (int J = I; J < nsup; ++J)
          tiles->push_back(GramTile{si, I * GRAM_TILE, J * GRAM_TILE, r0,
                                    std::min(d.rows, r0 + rows_per)});
    int pidx = 0;
    for (int I = 0; I < nsup; ++I)
      for (int J = I; J < nsup; ++J, ++pidx)
        red->push_back(GramReduce{si, I * GRAM_TILE, J * GRAM_TILE, base + pidx, nch, npairs});
  }
}

void row_tables(const std::vector<MatDesc>& sets, int nch, std::vector<RowTile>* tiles) {
  for (int si = 0; si < (int)sets.size(); ++si) {
    const MatDesc& d = sets[si];
    for (int r0 = 0; r0 < d.rows; r0 += ROW_TILE)
      for (int n0 = 0; n0 < d.ld; n0 += nch) tiles->push_back(RowTile{si, r0, n0});
  }
}

int spmm_epl(const std::vector<MatDesc>& sets) {
  if (sets.empty()) return 0;
  const int ld = sets[0].ld;
  for (const MatDesc& d : sets)
    if (d.ld != ld) return 0;
  return (ld % 64 == 0 && ld <= 320) ? ld / 64 : 0;
}

void spmm_tables(const std::vector<MatDesc>& sets, std::vector<SpmmTile>* tiles) {
  for (int si = 0; si < (int)sets.size(); ++si)
    for (int r0 = 0; r0 < sets[si].rows; r0 += SPMM_ROWS) tiles->push_back(SpmmTile{si, r0});
}

}  // namespace mis
