// Adjoint of a block's encode/decode X~ = U_c U_c^T X (Section 3 GFT and its
// inverse, Section 7.1 truncation) with respect to the vertex coordinates X
// and the Laplacian edge weights w (L = sum_e w_e (e_a - e_b)(e_a - e_b)^T,
// Section 3, Eq. 1-2), through the unrolled orthogonal iteration of Section 4
// (Alg. 1 with the Chebyshev operator) that produced U_c.
//
// The forward is replayed with checkpoints (the input basis of every filter
// pass, the Cholesky-QR factors, the Rayleigh-Ritz basis and rotation); the
// reverse sweep then runs, per block and batched over all blocks:
//   projection     Xbar = U_c U_c^T Gbar,  Ubar = Gbar E^T + X F^T
//   Rayleigh-Ritz  Q = Y R^-1, A = Q^T L Q = Z Theta Z^T, U_c = Q Z_c:
//                  Abar = sum_{i<c<=j} z_j z_i^T (z_j^T Q^T Ubar_i)/(theta_i - theta_j),
//                  Qbar = Ubar Z_c^T + 2 L Q sym(Abar),
//                  wbar_e += d_e(Q)^T sym(Abar) d_e(Q)   (d_e: row a minus row b)
//   Cholesky-QR    the loss depends on span(Q) only, so Ybar = (I - Q Q^T) Qbar R^-T
//   filter pass    Y = p(L) X by the three-term recurrence; its reverse
//                  recurrence gives Xbar = p(L) Ybar and, per step,
//                  wbar_e += alpha_k d_e(ybar_{k+1}) . d_e(y_k)
// and stops at each block's start basis (the given or seeded start, or the
// predecessor's result: a constant).  The filter interval of every iteration
// (recorded in the forward, adaptive or not) is a constant too, so no
// gradient flows into it.  Distance weights chain into X.
#include <cstring>

#include "eig.hpp"
#include "oi_plan.hpp"

namespace mis {

namespace {

struct AdjBlock {
  int64_t v_off, u_off, t_off, m_off, nnz_off, rp_off, e_off, part_off;
  int32_t n, p, ld, ne;
};

constexpr int ADJ_CHUNKS = 8;  // row ranges of the Q^T [X | Gbar] partial sums

struct AdjPlan {
  std::vector<int64_t> v_off, u_off, nnz, eoff;
  std::vector<int32_t> p, ld;
  AdjBlock* dev = nullptr;
  int max_ne = 0;
  int64_t part_doubles = 0;
  // block ids of the tracking plan's waves, wave after wave (woff[w] .. woff[w + 1])
  std::vector<int32_t> ids, woff;
  int32_t* ids_dev = nullptr;
  ~AdjPlan() {
    if (dev) (void)hipFree(dev);
    if (ids_dev) (void)hipFree(ids_dev);
  }
};

// Passes and iterations of the longest wave: the roots run T0 iterations of
// passes0 passes; blocks warm-started from a predecessor run T of passes.
void adj_counts(const HostBlocks& hb, const mi_oi_params& prm, int* npass, int* n_iter) {
  bool warm = false;
  if (prm.warm == MI_WARM_PRED)
    for (int b = 0; b < hb.B; ++b) warm = warm || hb.pred[b] >= 0;
  *npass = std::max(prm.T0 * prm.passes0, warm ? prm.T * prm.passes : 0);
  *n_iter = std::max(prm.T0, warm ? prm.T : 0);
}

// Workspace of one adjoint call (element type T of the slabs).
struct AdjWs {
  size_t oi, V, ritz, status, recX, recS, recY, Rrr, Z, coef;
  size_t Q, W, Qb, Tm, yb, ys, acc, part, EF, ZEF, PP, T1, S2d, S2, M, Hm, RT, MRT, Rc;
  size_t total;
};

AdjWs adj_layout(const HostBlocks& hb, const mi_oi_params& prm, int64_t nnz, int64_t part) {
  const size_t es = prm.precision == MI_FP64 ? 8 : 4;
  const int B = hb.B;
  const int64_t slab = hb.u_off[B], mats = hb.m_off[B], tp = hb.t_off[B];
  int npass = 0, n_iter = 0;
  adj_counts(hb, prm, &npass, &n_iter);
  Carver c(nullptr);
  AdjWs L;
  auto take = [&](size_t bytes) {
    size_t o = c.used;
    c.take<char>(bytes);
    return o;
  };
  L.oi = take(oi_ws_bytes(hb, prm));
  L.V = take(slab * es);
  L.ritz = take(tp * 8);
  L.status = take(B * 4);
  L.recX = take(size_t(npass) * slab * es);
  L.recS = take(size_t(std::max(npass - 1, 1)) * mats * es);
  L.recY = take(slab * es);
  L.Rrr = take(mats * 8);
  L.Z = take(mats * 8);
  L.coef = take(size_t(n_iter) * B * 3 * (std::max(prm.m, prm.m0) + 1) * 8);
  L.Q = take(slab * es);
  L.W = take(slab * es);
  L.Qb = take(slab * es);
  L.Tm = take(slab * es);
  L.yb = take(3 * slab * es);
  L.ys = take(size_t(std::max(std::max(prm.m0, prm.m) - 1, 1)) * slab * es);
  L.acc = take(std::max<int64_t>(nnz, 1) * 8);
  L.part = take(std::max<int64_t>(part, 1) * 8);
  L.EF = take(6 * tp * 8);
  L.ZEF = take(6 * tp * 8);
  L.PP = take(6 * tp * 8);
  L.T1 = take(mats * 8);
  L.S2d = take(mats * 8);
  L.S2 = take(mats * es);
  L.M = take(mats * 8);
  L.Hm = take(mats * 8);
  L.RT = take(mats * es);
  L.MRT = take(mats * es);
  L.Rc = take(mats * es);
  L.total = c.used;
  return L;
}

int64_t adj_part_doubles(const HostBlocks& hb, std::vector<int64_t>* off) {
  int64_t t = 0;
  for (int b = 0; b < hb.B; ++b) {
    if (off) off->push_back(t);
    t += int64_t(ADJ_CHUNKS) * hb.ld[b] * 6;
  }
  return t;
}

}  // namespace

// ------------------------------------------------------------------ reverse SpMM
// One reverse step of the filter recurrence for the rows of a tile:
//   out = alpha_k L yb + beta_k yb + gamma_{k+1} ybp      (coef != null)
// and, for every stored off-diagonal entry (r, j) of the row,
//   acc[entry] += s * sum_cols (yb[r] - yb[j]) (yf[r] - yf[j])
// with s = alpha_k (coef != null) or acc_scale (accumulation only, out null).
// A wavefront per row; each entry's column sum is a wavefront reduction, and
// every entry is owned by its row's wavefront, so the accumulation is
// deterministic.  Products and sums in FP64.
template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_spmm(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
               const CsrDesc* __restrict__ csr, const int32_t* __restrict__ row_ptr,
               const int32_t* __restrict__ col, const float* __restrict__ val,
               const T* __restrict__ yb, const T* __restrict__ ybp, const T* __restrict__ yf,
               T* __restrict__ out, double* __restrict__ acc, const double* __restrict__ coef,
               int stride, int step, double acc_scale) {
  typedef typename VecOf<T>::type V;
  constexpr int W = VecOf<T>::W;
  constexpr int MAXV = 1024 / W / 64;
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const CsrDesc c = csr[t.set];
  double al = acc_scale, be = 0.0, ga = 0.0;
  if (coef) {
    const double* cf = coef + int64_t(d.blk) * stride;
    al = cf[3 * step];
    be = cf[3 * step + 1];
    ga = cf[3 * step + 5];  // gamma of step k+1 (slot m holds gamma = 0)
  }
  const int nvec = d.ld / W;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  const T* ybb = yb + d.off;
  const T* yfb = yf ? yf + d.off : nullptr;
  for (int rr = wave; rr < rows; rr += 4) {
    const int r = t.row0 + rr;
    const int k0 = row_ptr[c.rp_off + r], k1 = row_ptr[c.rp_off + r + 1];
    V yi[MAXV], fi[MAXV];
    double lv[MAXV][W];
#pragma unroll
    for (int s = 0; s < MAXV; ++s) {
      const int v = lane + 64 * s;
#pragma unroll
      for (int e = 0; e < W; ++e) lv[s][e] = 0.0;
      yi[s] = (V)(T)0;
      fi[s] = (V)(T)0;
      if (v < nvec) {
        yi[s] = *reinterpret_cast<const V*>(ybb + int64_t(r) * d.ld + v * W);
        if (yfb) fi[s] = *reinterpret_cast<const V*>(yfb + int64_t(r) * d.ld + v * W);
      }
    }
    for (int k = k0; k < k1; ++k) {
      const int j = col[c.nnz_off + k];
      const double w = val[c.nnz_off + k];
      const bool edge = acc && j != r;
      double dot = 0.0;
#pragma unroll
      for (int s = 0; s < MAXV; ++s) {
        const int v = lane + 64 * s;
        if (v < nvec) {
          const V yj = *reinterpret_cast<const V*>(ybb + int64_t(j) * d.ld + v * W);
#pragma unroll
          for (int e = 0; e < W; ++e) lv[s][e] = fma(w, (double)yj[e], lv[s][e]);
          if (edge) {
            const V fj = *reinterpret_cast<const V*>(yfb + int64_t(j) * d.ld + v * W);
#pragma unroll
            for (int e = 0; e < W; ++e)
              dot = fma((double)yi[s][e] - (double)yj[e], (double)fi[s][e] - (double)fj[e], dot);
          }
        }
      }
      if (edge) {
        dot = wave_sum(dot);
        if (lane == 0) acc[c.nnz_off + k] += al * dot;
      }
    }
    if (out) {
#pragma unroll
      for (int s = 0; s < MAXV; ++s) {
        const int v = lane + 64 * s;
        if (v >= nvec) continue;
        const int64_t o = d.off + int64_t(r) * d.ld + v * W;
        V pv = (V)(T)0;
        if (ybp) pv = *reinterpret_cast<const V*>(ybp + o);
        V res;
#pragma unroll
        for (int e = 0; e < W; ++e)
          res[e] = (T)(al * lv[s][e] + be * (double)yi[s][e] + ga * (double)pv[e]);
        *reinterpret_cast<V*>(out + o) = res;
      }
    }
  }
}

// ------------------------------------------------------------------ Q^T [X | Gbar]
// EF[t_off + k][0..2] = sum_i Q[i][k] X[i][:], EF[..][3..5] = sum_i Q[i][k] Gbar[i][:]:
// workgroup (block, chunk) sums one row range into an FP64 partial; the
// second kernel adds the partials in chunk order.
template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_tall6(const AdjBlock* __restrict__ blks, const int32_t* __restrict__ ids,
                const T* __restrict__ Q, const T* __restrict__ X, const T* __restrict__ G,
                double* __restrict__ part) {
  constexpr int KPT = 4;  // ld <= 1024
  const AdjBlock b = blks[ids[blockIdx.x]];
  const int chunk = blockIdx.y;
  const int rows_per = (b.n + ADJ_CHUNKS - 1) / ADJ_CHUNKS;
  const int r0 = chunk * rows_per, r1 = min(b.n, r0 + rows_per);
  double a[KPT][6];
#pragma unroll
  for (int s = 0; s < KPT; ++s)
#pragma unroll
    for (int d = 0; d < 6; ++d) a[s][d] = 0.0;
  const T* Qb = Q + b.u_off;
  const T* Xb = X + 3 * b.v_off;
  const T* Gb = G + 3 * b.v_off;
  for (int i = r0; i < r1; ++i) {
    double xg[6];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xg[d] = (double)Xb[3 * i + d];
      xg[3 + d] = (double)Gb[3 * i + d];
    }
#pragma unroll
    for (int s = 0; s < KPT; ++s) {
      const int k = threadIdx.x + 256 * s;
      if (k < b.p) {
        const double q = (double)Qb[int64_t(i) * b.ld + k];
#pragma unroll
        for (int d = 0; d < 6; ++d) a[s][d] = fma(q, xg[d], a[s][d]);
      }
    }
  }
  double* pb = part + b.part_off + int64_t(chunk) * b.ld * 6;
#pragma unroll
  for (int s = 0; s < KPT; ++s) {
    const int k = threadIdx.x + 256 * s;
    if (k < b.ld)
#pragma unroll
      for (int d = 0; d < 6; ++d) pb[6 * k + d] = a[s][d];
  }
}

__global__ void __launch_bounds__(256)
    k_adj_sum6(const AdjBlock* __restrict__ blks, const int32_t* __restrict__ ids,
               const double* __restrict__ part, double* __restrict__ EF) {
  const AdjBlock b = blks[ids[blockIdx.x]];
  for (int e = threadIdx.x; e < 6 * b.p; e += 256) {
    double v = 0.0;
    for (int ch = 0; ch < ADJ_CHUNKS; ++ch) v += part[b.part_off + int64_t(ch) * b.ld * 6 + e];
    EF[6 * b.t_off + e] = v;
  }
}

// ------------------------------------------------------------------ Rayleigh-Ritz adjoint
// ZEF[j][:] = sum_k Z[k][j] EF[k][:]  (Z^T Q^T X | Z^T Q^T Gbar), j < p.
__global__ void __launch_bounds__(256)
    k_rr_zef(const AdjBlock* __restrict__ blks, const int32_t* __restrict__ ids,
             const double* __restrict__ Z, const double* __restrict__ EF,
             double* __restrict__ ZEF) {
  const AdjBlock b = blks[ids[blockIdx.x]];
  const double* Zb = Z + b.m_off;
  const double* ef = EF + 6 * b.t_off;
  for (int e = threadIdx.x; e < 6 * b.p; e += 256) {
    const int j = e / 6, d = e % 6;
    double s = 0.0;
    for (int k = 0; k < b.p; ++k) s = fma(Zb[int64_t(k) * b.ld + j], ef[6 * k + d], s);
    ZEF[6 * b.t_off + e] = s;
  }
}

// PP[k][0..2] = sum_{i<c} Z[k][i] ZEF[i][0..2]  (Pe = Z_c Z_c^T Q^T X),
// PP[k][3..5] likewise from ZEF[..][3..5]     (Pf = Z_c Z_c^T Q^T Gbar),
// T1[k][i] = sum_{c<=j<p} Z[k][j] K_ji, K_ji = z_j^T Q^T Ubar_i / (theta_i - theta_j)
//          = (ZF_j . ZE_i + ZE_j . ZF_i) / (theta_i - theta_j)   for i < c.
__global__ void __launch_bounds__(256)
    k_rr_pk(const AdjBlock* __restrict__ blks, const int32_t* __restrict__ ids,
            const int32_t* __restrict__ cvec, const double* __restrict__ Z,
            const double* __restrict__ theta, const double* __restrict__ ZEF,
            double* __restrict__ PP, double* __restrict__ T1) {
  const int bi = ids[blockIdx.x];
  const AdjBlock b = blks[bi];
  const int c = min(max(cvec[bi], 1), b.p);
  const double* Zb = Z + b.m_off;
  const double* ze = ZEF + 6 * b.t_off;
  const double* th = theta + b.t_off;
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e < 6 * b.p) {
    const int k = e / 6, d = e % 6;
    double s = 0.0;
    for (int i = 0; i < c; ++i) s = fma(Zb[int64_t(k) * b.ld + i], ze[6 * i + d], s);
    PP[6 * b.t_off + e] = s;
  }
  if (e < b.p * c) {
    const int k = e / c, i = e % c;
    double s = 0.0;
    for (int j = c; j < b.p; ++j) {
      const double num = ze[6 * j + 3] * ze[6 * i] + ze[6 * j + 4] * ze[6 * i + 1] +
                         ze[6 * j + 5] * ze[6 * i + 2] + ze[6 * j] * ze[6 * i + 3] +
                         ze[6 * j + 1] * ze[6 * i + 4] + ze[6 * j + 2] * ze[6 * i + 5];
      s = fma(Zb[int64_t(k) * b.ld + j], num / (th[i] - th[j]), s);
    }
    T1[b.m_off + int64_t(k) * b.ld + i] = s;
  }
}

// S2 = 2 sym(Abar) = Abar + Abar^T with Abar = T1 Z_c^T (zero outside p x p),
// in FP64 and in the slab element type.
template <typename T>
__global__ void __launch_bounds__(256)
    k_rr_abar(const AdjBlock* __restrict__ blks, const int32_t* __restrict__ ids,
              const int32_t* __restrict__ cvec, const double* __restrict__ Z,
              const double* __restrict__ T1, double* __restrict__ S2d, T* __restrict__ S2) {
  const int bi = ids[blockIdx.x];
  const AdjBlock b = blks[bi];
  const int c = min(max(cvec[bi], 1), b.p);
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= b.ld * b.ld) return;
  const int k = e / b.ld, l = e % b.ld;
  double s = 0.0;
  if (k < b.p && l < b.p) {
    const double* Zb = Z + b.m_off;
    const double* Tb = T1 + b.m_off;
    for (int i = 0; i < c; ++i)
      s += Tb[int64_t(k) * b.ld + i] * Zb[int64_t(l) * b.ld + i] +
           Tb[int64_t(l) * b.ld + i] * Zb[int64_t(k) * b.ld + i];
  }
  S2d[b.m_off + e] = s;
  S2[b.m_off + e] = (T)s;
}

// Qbar[i][k] += Gbar[i] . Pe[k] + X[i] . Pf[k]   (k < p): the projection part
// Ubar Z_c^T = Gbar (Z_c E)^T + X (Z_c F)^T.
template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_lowrank(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
                  const AdjBlock* __restrict__ blks, const double* __restrict__ PP,
                  const T* __restrict__ X, const T* __restrict__ G, T* __restrict__ Qb) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const AdjBlock b = blks[d.blk];
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  const double* pp = PP + 6 * b.t_off;
  for (int e = threadIdx.x; e < rows * b.p; e += 256) {
    const int i = t.row0 + e / b.p, k = e % b.p;
    const T* xi = X + 3 * (b.v_off + i);
    const T* gi = G + 3 * (b.v_off + i);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) s += (double)gi[q] * pp[6 * k + q] + (double)xi[q] * pp[6 * k + 3 + q];
    T* o = Qb + d.off + int64_t(i) * d.ld + k;
    *o = (T)((double)*o + s);
  }
}

// ------------------------------------------------------------------ Cholesky-QR adjoint helpers
// RT = R^T and MRT = M R^T (ld x ld per block); M FP64, R in the slab type.
template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_prep(const AdjBlock* __restrict__ blks, const int32_t* __restrict__ ids,
               const double* __restrict__ M, const T* __restrict__ R, T* __restrict__ RT,
               T* __restrict__ MRT) {
  const AdjBlock b = blks[ids[blockIdx.x]];
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= b.ld * b.ld) return;
  const int k = e / b.ld, l = e % b.ld;
  const T* Rb = R + b.m_off;
  const double* Mb = M + b.m_off;
  double s = 0.0;
  for (int j = 0; j < b.ld; ++j) s = fma(Mb[int64_t(k) * b.ld + j], (double)Rb[int64_t(l) * b.ld + j], s);
  RT[b.m_off + e] = Rb[int64_t(l) * b.ld + k];
  MRT[b.m_off + e] = (T)s;
}

// out = a - b over the rows of a wave's tiles.
template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_sub(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
              const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ out) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  for (int e = threadIdx.x; e < rows * d.ld; e += 256) {
    const int64_t o = d.off + int64_t(t.row0) * d.ld + e;
    out[o] = a[o] - b[o];
  }
}

template <typename T>
__global__ void k_adj_cast(int64_t n, const double* __restrict__ a, T* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) out[i] = (T)a[i];
}

// ------------------------------------------------------------------ outputs
// Xbar[i] = sum_{k<p} Q[i][k] Pf[k] (= U_c U_c^T Gbar) plus, for distance
// weights, sum_j wbar_ij dw_ij/dx_i with w = |x_i - x_j|^-2 (dw/dx_i =
// -2 (x_i - x_j)/|.|^4) or |x_i - x_j|^-1 (dw/dx_i = -(x_i - x_j)/|.|^3).
// A wavefront per row.
template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_xbar(const SpmmTile* __restrict__ tiles, const MatDesc* __restrict__ sets,
               const CsrDesc* __restrict__ csr, const AdjBlock* __restrict__ blks,
               const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
               const double* __restrict__ acc, const T* __restrict__ Q,
               const double* __restrict__ PP, const T* __restrict__ X, int mode,
               double* __restrict__ Xbar) {
  const SpmmTile t = tiles[blockIdx.x];
  const MatDesc d = sets[t.set];
  const CsrDesc c = csr[t.set];
  const AdjBlock b = blks[d.blk];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows = min(SPMM_ROWS, d.rows - t.row0);
  const double* pp = PP + 6 * b.t_off;
  for (int rr = wave; rr < rows; rr += 4) {
    const int r = t.row0 + rr;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = lane; k < b.p; k += 64) {
      const double q = (double)Q[d.off + int64_t(r) * d.ld + k];
      s0 = fma(q, pp[6 * k + 3], s0);
      s1 = fma(q, pp[6 * k + 4], s1);
      s2 = fma(q, pp[6 * k + 5], s2);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      if (mode == MI_W_INV_SQ_DIST || mode == MI_W_INV_DIST) {
        const T* xr = X + 3 * (b.v_off + r);
        for (int k = row_ptr[c.rp_off + r]; k < row_ptr[c.rp_off + r + 1]; ++k) {
          const int j = col[c.nnz_off + k];
          if (j == r) continue;
          const T* xj = X + 3 * (b.v_off + j);
          const double d0 = (double)xr[0] - (double)xj[0], d1 = (double)xr[1] - (double)xj[1],
                       d2 = (double)xr[2] - (double)xj[2];
          const double q = d0 * d0 + d1 * d1 + d2 * d2;
          const double f = mode == MI_W_INV_SQ_DIST ? -2.0 / (q * q) : -1.0 / (q * sqrt(q));
          const double g = acc[c.nnz_off + k] * f;
          s0 = fma(g, d0, s0);
          s1 = fma(g, d1, s1);
          s2 = fma(g, d2, s2);
        }
      }
      double* o = Xbar + 3 * (b.v_off + r);
      o[0] = s0;
      o[1] = s1;
      o[2] = s2;
    }
  }
}

// wbar[e] = acc at the CSR entry (a, b) of canonical edge e = (a < b).
__global__ void __launch_bounds__(256)
    k_adj_edges(const AdjBlock* __restrict__ blks, const int32_t* __restrict__ row_ptr,
                const int32_t* __restrict__ col, const int32_t* __restrict__ edges,
                const double* __restrict__ acc, double* __restrict__ wbar) {
  const AdjBlock b = blks[blockIdx.x];
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= b.ne) return;
  const int a = edges[2 * (b.e_off + e)], bb = edges[2 * (b.e_off + e) + 1];
  int lo = row_ptr[b.rp_off + a], hi = row_ptr[b.rp_off + a + 1] - 1;
  const int32_t* cb = col + b.nnz_off;
  while (lo < hi) {  // first entry with col >= bb
    const int mid = (lo + hi) >> 1;
    if (cb[mid] < bb)
      lo = mid + 1;
    else
      hi = mid;
  }
  wbar[b.e_off + e] = cb[lo] == bb ? acc[b.nnz_off + lo] : 0.0;
}

// ------------------------------------------------------------------ driver

template <typename T>
static void reverse(const OiPlan& P, const AdjPlan& A, const AdjWs& L, char* ws,
                    const OiRecord& rec, const int32_t* row_ptr, const int32_t* col,
                    const float* val, const int32_t* edges, const int32_t* c, const T* X,
                    const T* G, int mode, double* Xbar, double* wbar, hipStream_t s) {
  const HostBlocks& hb = P.hb;
  const int B = hb.B;
  const int64_t slab = hb.u_off[B], mats = hb.m_off[B];
  const int stride = P.L.coef_stride;
  auto S = [&](size_t off) { return reinterpret_cast<T*>(ws + off); };
  auto D = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
  T* Q = S(L.Q);
  T* Wl = S(L.W);
  T* Qb = S(L.Qb);
  T* Tm = S(L.Tm);
  T* yb[3] = {S(L.yb), S(L.yb) + slab, S(L.yb) + 2 * slab};
  double* acc = D(L.acc);
  double* part = D(L.part);
  double* EF = D(L.EF);
  double* ZEF = D(L.ZEF);
  double* PP = D(L.PP);
  double* T1 = D(L.T1);
  double* S2d = D(L.S2d);
  T* S2 = S(L.S2);
  double* M = D(L.M);
  double* Hm = D(L.Hm);
  T* RT = S(L.RT);
  T* MRT = S(L.MRT);
  T* ys = S(L.ys);
  const double* ritz = D(L.ritz);
  double* gpart = D(L.oi + P.L.part);  // Gram partials (the tracking workspace's buffer)
  fill_f64(acc, 0.0, int64_t(P.nnz_off[B]), s);
  // R^-1 of every block's Rayleigh-Ritz step in the slab type
  const T* Rc;
  if (std::is_same<T, double>::value) {
    Rc = reinterpret_cast<const T*>(rec.Rrr);
  } else {
    hipLaunchKernelGGL(k_adj_cast<T>, dim3(ceil_div(mats, 256)), dim3(256), 0, s, mats, rec.Rrr,
                       S(L.Rc));
    Rc = S(L.Rc);
  }
  // Every block's reverse sweep ends at its own start basis (the given
  // start, or its predecessor's result, held constant), so the waves are
  // reversed one after the other, each with its own pass count and degree.
  for (size_t wi = 0; wi < P.waves.size(); ++wi) {
    const WaveTables& w = P.waves[wi];
    const int32_t* ids = A.ids_dev + A.woff[wi];
    const int nbw = A.woff[wi + 1] - A.woff[wi];
    if (nbw <= 0 || w.T <= 0) continue;
    const int m = w.m, npass = w.T * w.passes;
    auto coef_of = [&](int j) { return rec.coef + size_t(j / w.passes) * B * stride; };
    const int gsm = ceil_div(int64_t(w.max_ld) * w.max_ld, 256);

    // Q = Y R^-1 of the Rayleigh-Ritz step; W = L Q (slot m: the plain product)
    launch_rowmul<T, T>(w.rt, w.n_rt, w.tall, static_cast<const T*>(rec.Y), w.small, Rc, w.tall,
                        Q, w.nch, s, true);
    launch_spmm<T>(w.spmm, w.n_spmm, w.tall, w.csr, row_ptr, col, val, Q, nullptr, Wl,
                   coef_of(npass - 1), stride, m, s, w.epl, w.spmm_var);
    // projection and Rayleigh-Ritz adjoint
    hipLaunchKernelGGL(k_adj_tall6<T>, dim3(nbw, ADJ_CHUNKS), dim3(256), 0, s, A.dev, ids, Q, X,
                       G, part);
    hipLaunchKernelGGL(k_adj_sum6, dim3(nbw), dim3(256), 0, s, A.dev, ids, part, EF);
    hipLaunchKernelGGL(k_rr_zef, dim3(nbw), dim3(256), 0, s, A.dev, ids, rec.Z, EF, ZEF);
    hipLaunchKernelGGL(k_rr_pk, dim3(nbw, gsm), dim3(256), 0, s, A.dev, ids, c, rec.Z, ritz, ZEF,
                       PP, T1);
    hipLaunchKernelGGL(k_rr_abar<T>, dim3(nbw, gsm), dim3(256), 0, s, A.dev, ids, c, rec.Z, T1,
                       S2d, S2);
    launch_rowmul<T, T>(w.rt, w.n_rt, w.tall, Wl, w.small, S2, w.tall, Qb, w.nch, s);
    hipLaunchKernelGGL(k_adj_lowrank<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall, A.dev,
                       PP, X, G, Qb);
    // wbar_e += d_e(Q S2/2) . d_e(Q)
    launch_rowmul<T, T>(w.rt, w.n_rt, w.tall, Q, w.small, S2, w.tall, Tm, w.nch, s);
    hipLaunchKernelGGL(k_adj_spmm<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall, w.csr,
                       row_ptr, col, val, Tm, nullptr, Q, nullptr, acc, nullptr, 0, 0, 0.5);

    // Ybar = (I - B B^T) Bbar R^-T for the basis B = Y R^-1 (span-only loss)
    auto cholqr_adj = [&](const T* Bm, const T* Bbar, const T* R, T* out) {
      if (w.gram_direct) {
        launch_gram_direct<T>(w.gt, w.n_gt, w.tall, w.small, Bm, Bm, Bbar, M, Hm, s);
      } else {
        launch_gram<T>(w.gt, w.n_gt, w.tall, Bm, Bm, Bbar, gpart, s);
        launch_gram_reduce(w.gr, w.n_gr, w.small, gpart, true, M, Hm, s);
      }
      hipLaunchKernelGGL(k_adj_prep<T>, dim3(nbw, gsm), dim3(256), 0, s, A.dev, ids, Hm, R, RT,
                         MRT);
      launch_rowmul<T, T>(w.rt, w.n_rt, w.tall, Bm, w.small, MRT, w.tall, Tm, w.nch, s);
      launch_rowmul<T, T>(w.rt, w.n_rt, w.tall, Bbar, w.small, RT, w.tall, out, w.nch, s);
      hipLaunchKernelGGL(k_adj_sub<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall, out, Tm,
                         out);
    };
    cholqr_adj(Q, Qb, Rc, yb[0]);
    int cur = 0;  // yb slab holding the gradient of the current pass output
    for (int j = npass - 1; j >= 0; --j) {
      const double* cf = coef_of(j);
      // forward intermediates y_0 .. y_{m-1} of pass j from its checkpointed input
      const T* xin = static_cast<const T*>(rec.X[j]);
      auto y_at = [&](int k) -> const T* { return k == 0 ? xin : ys + int64_t(k - 1) * slab; };
      for (int k = 0; k + 1 < m; ++k)
        launch_spmm<T>(w.spmm, w.n_spmm, w.tall, w.csr, row_ptr, col, val, y_at(k),
                       k > 0 ? y_at(k - 1) : nullptr, ys + int64_t(k) * slab, cf, stride, k, s,
                       w.epl, w.spmm_var);
      // reverse recurrence
      int nxt = cur, prv = -1;
      for (int k = m - 1; k >= 0; --k) {
        int o = 0;
        while (o == nxt || o == prv) ++o;
        hipLaunchKernelGGL(k_adj_spmm<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall, w.csr,
                           row_ptr, col, val, yb[nxt], prv >= 0 ? yb[prv] : nullptr, y_at(k),
                           yb[o], acc, cf, stride, k, 0.0);
        prv = nxt;
        nxt = o;
      }
      cur = nxt;  // gradient of the pass input
      if (j > 0) {
        int o = 0;
        while (o == cur) ++o;
        cholqr_adj(xin, yb[cur], static_cast<const T*>(rec.S[j - 1]), yb[o]);
        cur = o;
      }
    }
    hipLaunchKernelGGL(k_adj_xbar<T>, dim3(w.n_spmm), dim3(256), 0, s, w.spmm, w.tall, w.csr,
                       A.dev, row_ptr, col, acc, Q, PP, X, mode, Xbar);
  }
  if (A.max_ne > 0)
    hipLaunchKernelGGL(k_adj_edges, dim3(B, ceil_div(A.max_ne, 256)), dim3(256), 0, s, A.dev,
                       row_ptr, col, edges, acc, wbar);
}

static mi_status adj_check(const mi_oi_params* prm, const HostBlocks& hb) {
  mi_status st = oi_check_params(prm);
  if (st) return st;
  MI_CHECK_ARG(prm->precision != MI_BF16_IN, "the adjoint supports MI_FP32 and MI_FP64");
  MI_CHECK_ARG(prm->tol == 0, "the adjoint differentiates fixed iteration counts (tol = 0)");
  MI_CHECK_ARG(prm->op == MI_OP_CHEB, "the adjoint differentiates the Chebyshev filter only");
  MI_CHECK_ARG(prm->rr_every == 0, "the adjoint needs rr_every = 0");
  MI_CHECK_ARG(prm->eig == MI_EIG_TRIDIAG, "the adjoint needs eig = MI_EIG_TRIDIAG");
  MI_CHECK_ARG(prm->T0 >= 1, "the adjoint needs T0 >= 1");
  bool warm = false;
  if (prm->warm == MI_WARM_PRED)
    for (int b = 0; b < hb.B; ++b) warm = warm || hb.pred[b] >= 0;
  MI_CHECK_ARG(!warm || prm->T >= 1, "the adjoint needs T >= 1 for warm-started blocks");
  int max_ld = 0;
  for (int b = 0; b < hb.B; ++b) max_ld = std::max(max_ld, hb.ld[b]);
  // the widths the reverse sweep is tested at
  constexpr int ADJ_MAX_LD = 192;
  MI_CHECK_ARG(max_ld <= ADJ_MAX_LD, "the adjoint supports ld <= %d", ADJ_MAX_LD);
  return MI_OK;
}

}  // namespace mis

using namespace mis;

extern "C" {

void mis_destroy_adj_plan(mi_ctx* ctx) {
  delete static_cast<AdjPlan*>(ctx->adj_plan);
  ctx->adj_plan = nullptr;
}

mi_status mi_adjoint_workspace_size(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                                    const int64_t* nnz_off, size_t* ws_bytes) {
  clear_error();
  (void)ctx;
  MI_CHECK_ARG(ws_bytes && nnz_off, "NULL argument");
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  st = adj_check(prm, hb);
  if (st) return st;
  *ws_bytes = adj_layout(hb, *prm, nnz_off[hb.B], adj_part_doubles(hb, nullptr)).total;
  return MI_OK;
}

mi_status mi_encdec_adjoint(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                            int32_t mode, const int32_t* row_ptr, const int32_t* col,
                            const float* val, const int64_t* nnz_off, const int32_t* edges,
                            const int64_t* edge_off, const void* V0, const void* X,
                            const int32_t* c, const void* Gbar, double* Xbar, double* wbar,
                            void* ws, size_t ws_bytes, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && prm && row_ptr && col && val && nnz_off && edges && edge_off && X && c &&
                   Gbar && Xbar && wbar,
               "NULL argument");
  MI_CHECK_ARG(V0 || prm->warm == MI_RANDOM, "V0 is NULL (needed unless warm = MI_RANDOM)");
  MI_CHECK_ARG(mode == MI_W_COMBINATORIAL || mode == MI_W_INV_SQ_DIST || mode == MI_W_INV_DIST ||
                   mode == MI_W_USER,
               "weight mode %d unknown", mode);
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  st = adj_check(prm, hb);
  if (st) return st;
  std::vector<int64_t> nnz(nnz_off, nnz_off + hb.B + 1), eoff(edge_off, edge_off + hb.B + 1);
  for (int b = 0; b < hb.B; ++b)
    MI_CHECK_ARG(nnz[b + 1] >= nnz[b] && eoff[b + 1] >= eoff[b], "offsets must be non-decreasing");
  std::vector<int64_t> poff;
  const int64_t part = adj_part_doubles(hb, &poff);
  const AdjWs L = adj_layout(hb, *prm, nnz[hb.B], part);
  if (!ws || ws_bytes < L.total) {
    set_error("workspace %zu bytes < %zu required", ws_bytes, L.total);
    return MI_ERR_WORKSPACE;
  }
  MI_TRY_HIP(hipSetDevice(ctx->device));
  AdjPlan* A = static_cast<AdjPlan*>(ctx->adj_plan);
  if (!A || A->v_off != hb.v_off || A->u_off != hb.u_off || A->p != hb.p || A->ld != hb.ld ||
      A->nnz != nnz || A->eoff != eoff) {
    delete A;
    ctx->adj_plan = nullptr;
    A = new AdjPlan();
    A->v_off = hb.v_off;
    A->u_off = hb.u_off;
    A->p = hb.p;
    A->ld = hb.ld;
    A->nnz = nnz;
    A->eoff = eoff;
    A->part_doubles = part;
    std::vector<AdjBlock> h(hb.B);
    for (int b = 0; b < hb.B; ++b) {
      h[b] = AdjBlock{hb.v_off[b], hb.u_off[b], hb.t_off[b], hb.m_off[b], nnz[b],
                      hb.v_off[b] + b, eoff[b], poff[b], int(hb.v_off[b + 1] - hb.v_off[b]),
                      hb.p[b], hb.ld[b], int(eoff[b + 1] - eoff[b])};
      A->max_ne = std::max(A->max_ne, h[b].ne);
    }
    if (hipMalloc(&A->dev, std::max(hb.B, 1) * sizeof(AdjBlock)) != hipSuccess) {
      delete A;
      set_error("device allocation for the adjoint tables failed");
      return MI_ERR_HIP;
    }
    ctx->adj_plan = A;
    MI_TRY_HIP(hipMemcpy(A->dev, h.data(), hb.B * sizeof(AdjBlock), hipMemcpyHostToDevice));
  }
  hipStream_t s = (hipStream_t)stream;
  char* w = static_cast<char*>(ws);
  const size_t es = prm->precision == MI_FP64 ? 8 : 4;
  int npass = 0, n_iter = 0;
  adj_counts(hb, *prm, &npass, &n_iter);
  std::vector<void*> xs(npass), ss(std::max(npass - 1, 1));
  for (int j = 0; j < npass; ++j) xs[j] = w + L.recX + size_t(j) * hb.u_off[hb.B] * es;
  for (int j = 0; j + 1 < npass; ++j) ss[j] = w + L.recS + size_t(j) * hb.m_off[hb.B] * es;
  OiRecord rec;
  rec.X = xs.data();
  rec.S = ss.data();
  rec.Y = w + L.recY;
  rec.Rrr = reinterpret_cast<double*>(w + L.Rrr);
  rec.Z = reinterpret_cast<double*>(w + L.Z);
  rec.coef = reinterpret_cast<double*>(w + L.coef);
  rec.npass = npass;
  rec.n_iter = n_iter;
  OiPlan* P = nullptr;
  st = oi_run_plan(ctx, &ctx->adj_oi, hb, nnz, *prm, row_ptr, col, val, V0, w + L.V,
                   reinterpret_cast<double*>(w + L.ritz), reinterpret_cast<int32_t*>(w + L.status),
                   w + L.oi, oi_ws_bytes(hb, *prm), &rec, s, &P);
  if (st) return st;
  // the plan's waves, as block id lists (wave after wave)
  std::vector<int32_t> ids, woff{0};
  for (const WaveTables& wt : P->waves) {
    for (const MatDesc& d : wt.tall_host) ids.push_back(d.blk);
    woff.push_back((int32_t)ids.size());
  }
  if (ids != A->ids || woff != A->woff) {
    if (!A->ids_dev && hipMalloc(&A->ids_dev, std::max(hb.B, 1) * sizeof(int32_t)) != hipSuccess) {
      A->ids_dev = nullptr;
      set_error("device allocation for the adjoint tables failed");
      return MI_ERR_HIP;
    }
    MI_CHECK_ARG((int)ids.size() == hb.B, "every block must belong to one wave");
    MI_TRY_HIP(hipMemcpy(A->ids_dev, ids.data(), ids.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    A->ids = ids;
    A->woff = woff;
  }
  if (prm->precision == MI_FP64)
    reverse<double>(*P, *A, L, w, rec, row_ptr, col, val, edges, c, static_cast<const double*>(X),
                    static_cast<const double*>(Gbar), mode, Xbar, wbar, s);
  else
    reverse<float>(*P, *A, L, w, rec, row_ptr, col, val, edges, c, static_cast<const float*>(X),
                   static_cast<const float*>(Gbar), mode, Xbar, wbar, s);
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

}  // extern "C"
