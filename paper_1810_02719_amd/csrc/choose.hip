// Choice of the subspace size c per block (Section 5: the smallest
// subspace meeting a reconstruction-quality target) with the NMSVE of
// Section 8, Eq. 16 as the quality measure.
//
// With U the Ritz basis (ascending), E = U^T X, G the GL operator of the
// original mesh (G v = (L_d v) / diag(L_d), L_d the 1/d-weighted Laplacian),
// Z = G U, F = Z^T (G X) and M = Z^T Z, every c costs O(c) from prefix sums:
//   ||X - U_c E_c||^2    = ||X||^2 - sum_{k<c} |E_k|^2
//   ||G X - G U_c E_c||^2 = ||GX||^2 - 2 sum_{k<c} F_k.E_k + sum_{k,l<c} (E_k.E_l) M_kl
//   NMSVE(c) = (sqrt(first) + sqrt(second)) / (2 n)
#include <cstring>

#include "dense.hpp"

namespace mis {

struct CcBlock {
  int64_t v_off, u_off, t_off, m_off, nnz_off, rp_off;
  int32_t n, p, ld, pad;
};

struct CcPlan {
  HostBlocks hb;
  std::vector<int64_t> nnz_off;
  void* arena = nullptr;
  CcBlock* blocks = nullptr;
  MatDesc* tall = nullptr;
  MatDesc* small = nullptr;
  GramTile* gt = nullptr;
  int n_gt = 0;
  GramReduce* gr = nullptr;
  int n_gr = 0;
  bool gram_direct = false;  // no super-tile split: the Gram writes M itself
  size_t z_off = 0, gx_off = 0, ef_off = 0, efp_off = 0, m_off = 0, part_off = 0, nrm_off = 0,
         total = 0;
  ~CcPlan() {
    if (arena) (void)hipFree(arena);
  }
};

// Z = G U (row-scaled SpMM over the 1/d Laplacian); one thread per (row, 4 columns).
__global__ void __launch_bounds__(256)
    k_gl_apply(const CcBlock* __restrict__ blks, const SpmmTile* __restrict__ tiles,
               const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
               const float* __restrict__ val, const float* __restrict__ U, float* __restrict__ Z) {
  const SpmmTile t = tiles[blockIdx.x];
  const CcBlock b = blks[t.set];
  const int nvec = b.ld / 4;
  const int rows = min(SPMM_ROWS, b.n - t.row0);
  for (int idx = threadIdx.x; idx < rows * nvec; idx += 256) {
    const int r = t.row0 + idx / nvec, v = idx % nvec;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    float diag = 0.f;
    for (int k = row_ptr[b.rp_off + r]; k < row_ptr[b.rp_off + r + 1]; ++k) {
      const int j = col[b.nnz_off + k];
      const float w = val[b.nnz_off + k];
      if (j == r) diag = w;
      const float4 u = *reinterpret_cast<const float4*>(U + b.u_off + int64_t(j) * b.ld + 4 * v);
      acc.x += w * u.x;
      acc.y += w * u.y;
      acc.z += w * u.z;
      acc.w += w * u.w;
    }
    float4 out;
    if (diag > 0.f) {
      const float inv = 1.f / diag;
      out = make_float4(acc.x * inv, acc.y * inv, acc.z * inv, acc.w * inv);
    } else {  // isolated vertex: GL is the identity on it
      out = *reinterpret_cast<const float4*>(U + b.u_off + int64_t(r) * b.ld + 4 * v);
    }
    *reinterpret_cast<float4*>(Z + b.u_off + int64_t(r) * b.ld + 4 * v) = out;
  }
}

// The same product for blocks of one width ld = 64 EPL (up to 320): one
// wavefront per row (lanes over the columns, strided by 64 at 320), the
// row's column indices and weights in one vector load read out by lane, the
// off-diagonal rows gathered together and summed in difference form,
// (L U)_r = sum_{j != r} L_rj (U_j - U_r) + (sum_j L_rj) U_r, then scaled
// by 1 / L_rr; 8 consecutive rows per workgroup.
template <int EPL, bool STRIDED>
__global__ void __launch_bounds__(512)
    k_gl_apply_rows(const CcBlock* __restrict__ blks, const SpmmTile* __restrict__ tiles,
                    int ntiles, const int32_t* __restrict__ row_ptr,
                    const int32_t* __restrict__ col, const float* __restrict__ val,
                    const float* __restrict__ U, float* __restrict__ Z) {
  constexpr int G = 8, ES = STRIDED ? 64 : 1;
  const int ti = blockIdx.x / 2;
  if (ti >= ntiles) return;
  const SpmmTile t = tiles[ti];
  const CcBlock b = blks[t.set];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = t.row0 + (blockIdx.x % 2) * 8 + wave;
  if (r >= b.n) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  const int l0 = STRIDED ? lane : lane * EPL;
  const float* uv = U + b.u_off + l0;
  const int64_t o = b.u_off + int64_t(r) * b.ld + l0;
  float yin[EPL], acc[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    yin[e] = U[o + e * ES];
    acc[e] = 0.f;
  }
  const int k0 = row_ptr[b.rp_off + r], k1 = row_ptr[b.rp_off + r + 1];
  float rs = 0.f, diag = 0.f;
  for (int k = k0; k < k1; k += G) {
    int cjv = 0;
    float wvv = 0.f;
    if (lane < G && k + lane < k1) {
      cjv = col[b.nnz_off + k + lane];
      wvv = val[b.nnz_off + k + lane];
    }
    float y[G][EPL], w[G];
    bool has[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      has[u] = false;
      w[u] = 0.f;
      if (k + u < k1) {
        const int cj = __builtin_amdgcn_readlane(cjv, u);
        const float wv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wvv), u));
        rs += wv;
        if (cj == r) {
          diag = wv;
        } else {
          has[u] = true;
          w[u] = wv;
#pragma unroll
          for (int e = 0; e < EPL; ++e) y[u][e] = uv[int64_t(cj) * b.ld + e * ES];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
      if (has[u])
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[e] = fmaf(w[u], y[u][e] - yin[e], acc[e]);
  }
  const float inv = diag > 0.f ? 1.f / diag : 0.f;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    // an isolated vertex (no entries): GL is the identity on it
    const float out = diag > 0.f ? fmaf(rs, yin[e], acc[e]) * inv : yin[e];
    Z[o + e * ES] = out;
  }
}

// GX = G X in FP64, and the norms ||X||^2, ||GX||^2 per block (one workgroup
// per block, fixed-order reduction).
__global__ void __launch_bounds__(256)
    k_gl_coords(const CcBlock* __restrict__ blks, const int32_t* __restrict__ row_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val,
                const float* __restrict__ X, double* __restrict__ GX, double* __restrict__ nrm) {
  __shared__ double red[2][256];
  const CcBlock b = blks[blockIdx.x];
  double sx = 0.0, sg = 0.0;
  for (int r = threadIdx.x; r < b.n; r += 256) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, diag = 0.0;
    for (int k = row_ptr[b.rp_off + r]; k < row_ptr[b.rp_off + r + 1]; ++k) {
      const int j = col[b.nnz_off + k];
      const double w = val[b.nnz_off + k];
      if (j == r) diag = w;
      const float* xj = X + 3 * (b.v_off + j);
      a0 += w * xj[0];
      a1 += w * xj[1];
      a2 += w * xj[2];
    }
    const float* xr = X + 3 * (b.v_off + r);
    double g0, g1, g2;
    if (diag > 0.0) {
      g0 = a0 / diag;
      g1 = a1 / diag;
      g2 = a2 / diag;
    } else {
      g0 = xr[0];
      g1 = xr[1];
      g2 = xr[2];
    }
    double* gx = GX + 3 * (b.v_off + r);
    gx[0] = g0;
    gx[1] = g1;
    gx[2] = g2;
    sx += double(xr[0]) * xr[0] + double(xr[1]) * xr[1] + double(xr[2]) * xr[2];
    sg += g0 * g0 + g1 * g1 + g2 * g2;
  }
  red[0][threadIdx.x] = sx;
  red[1][threadIdx.x] = sg;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    nrm[2 * blockIdx.x] = red[0][0];
    nrm[2 * blockIdx.x + 1] = red[1][0];
  }
}

// E = U^T X and F = Z^T GX (p x 3 each, FP64): sums over EF_CHUNKS row
// chunks of each block (a workgroup per block and chunk, threads over the
// columns, rows in order), then per block the chunks added in order.
constexpr int EF_CHUNKS = 8;

__global__ void __launch_bounds__(256)
    k_proj_ef_part(const CcBlock* __restrict__ blks, const float* __restrict__ U,
                   const float* __restrict__ Z, const float* __restrict__ X,
                   const double* __restrict__ GX, double* __restrict__ EFP) {
  constexpr int KPT = 4;
  const int c = blockIdx.x % EF_CHUNKS;
  const CcBlock b = blks[blockIdx.x / EF_CHUNKS];
  const int per = (b.n + EF_CHUNKS - 1) / EF_CHUNKS;
  const int r0 = c * per, r1 = min(b.n, r0 + per);
  double e[KPT][3], f[KPT][3];
  for (int s = 0; s < KPT; ++s)
    for (int d = 0; d < 3; ++d) e[s][d] = f[s][d] = 0.0;
  for (int i = r0; i < r1; ++i) {
    const float* x = X + 3 * (b.v_off + i);
    const double* g = GX + 3 * (b.v_off + i);
    const double x0 = x[0], x1 = x[1], x2 = x[2], g0 = g[0], g1 = g[1], g2 = g[2];
#pragma unroll
    for (int s = 0; s < KPT; ++s) {
      const int k = threadIdx.x + 256 * s;
      if (k < b.p) {
        const double u = U[b.u_off + int64_t(i) * b.ld + k];
        const double z = Z[b.u_off + int64_t(i) * b.ld + k];
        e[s][0] += u * x0;
        e[s][1] += u * x1;
        e[s][2] += u * x2;
        f[s][0] += z * g0;
        f[s][1] += z * g1;
        f[s][2] += z * g2;
      }
    }
  }
  double* o0 = EFP + 6 * (int64_t(EF_CHUNKS) * b.t_off + int64_t(c) * b.p);
  for (int s = 0; s < KPT; ++s) {
    const int k = threadIdx.x + 256 * s;
    if (k < b.p) {
      double* o = o0 + 6 * k;
      o[0] = e[s][0];
      o[1] = e[s][1];
      o[2] = e[s][2];
      o[3] = f[s][0];
      o[4] = f[s][1];
      o[5] = f[s][2];
    }
  }
}

__global__ void __launch_bounds__(256)
    k_proj_ef_sum(const CcBlock* __restrict__ blks, const double* __restrict__ EFP,
                  double* __restrict__ EF) {
  const CcBlock b = blks[blockIdx.x];
  const double* pb = EFP + 6 * int64_t(EF_CHUNKS) * b.t_off;
  for (int e = threadIdx.x; e < 6 * b.p; e += 256) {
    double s = 0.0;
    for (int c = 0; c < EF_CHUNKS; ++c) s += pb[6 * int64_t(c) * b.p + e];
    EF[6 * b.t_off + e] = s;
  }
}

// Per block: the NMSVE curve by prefix sums, then the choice rule.
__global__ void __launch_bounds__(256)
    k_choose(const CcBlock* __restrict__ blks, const int32_t* __restrict__ c_max,
             const double* __restrict__ EF, const double* __restrict__ M,
             const double* __restrict__ nrm, const double* __restrict__ ritz, double target,
             double g_min, int32_t* __restrict__ c_out, double* __restrict__ metric) {
  __shared__ double red[256];
  const CcBlock b = blks[blockIdx.x];
  const int cm = min(max(c_max[blockIdx.x], 1), b.p);
  const double* ef = EF + 6 * b.t_off;
  const double* Mb = M + b.m_off;
  const double X2 = nrm[2 * blockIdx.x], GX2 = nrm[2 * blockIdx.x + 1];
  double l2 = X2, lin = 0.0, Q = 0.0;
  for (int k = 0; k < cm; ++k) {
    const double ek0 = ef[6 * k], ek1 = ef[6 * k + 1], ek2 = ef[6 * k + 2];
    double part = 0.0;
    for (int l = threadIdx.x; l < k; l += 256) {
      const double dot = ek0 * ef[6 * l] + ek1 * ef[6 * l + 1] + ek2 * ef[6 * l + 2];
      part += dot * Mb[int64_t(k) * b.ld + l];
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    const double cross = red[0];
    __syncthreads();
    const double ee = ek0 * ek0 + ek1 * ek1 + ek2 * ek2;
    l2 -= ee;
    lin += ek0 * ef[6 * k + 3] + ek1 * ef[6 * k + 4] + ek2 * ef[6 * k + 5];
    Q += 2.0 * cross + ee * Mb[int64_t(k) * b.ld + k];
    const double gl2 = GX2 - 2.0 * lin + Q;
    if (threadIdx.x == 0)
      metric[b.t_off + k] = (sqrt(fmax(l2, 0.0)) + sqrt(fmax(gl2, 0.0))) / (2.0 * b.n);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = cm;
    for (int k = 0; k < cm; ++k)
      if (metric[b.t_off + k] <= target) {
        c = k + 1;
        break;
      }
    const double* th = ritz + b.t_off;
    while (c < cm && c < b.p) {
      if (th[c] - th[c - 1] >= g_min * fabs(th[c])) break;
      ++c;
    }
    c_out[blockIdx.x] = c;
  }
}

static mi_status cc_plan(mi_ctx* ctx, const HostBlocks& hb, const std::vector<int64_t>& nnz,
                         CcPlan** out) {
  CcPlan* P = static_cast<CcPlan*>(ctx->cc_plan);
  if (P && P->hb.v_off == hb.v_off && P->hb.u_off == hb.u_off && P->hb.p == hb.p &&
      P->hb.ld == hb.ld && P->nnz_off == nnz) {
    *out = P;
    return MI_OK;
  }
  delete P;
  ctx->cc_plan = nullptr;
  P = new CcPlan();
  P->hb = hb;
  P->nnz_off = nnz;
  std::vector<CcBlock> cb(hb.B);
  std::vector<MatDesc> tall(hb.B), small(hb.B);
  for (int b = 0; b < hb.B; ++b) {
    const int n = int(hb.v_off[b + 1] - hb.v_off[b]);
    cb[b] = CcBlock{hb.v_off[b], hb.u_off[b], hb.t_off[b], hb.m_off[b], nnz[b], hb.v_off[b] + b,
                    n, hb.p[b], hb.ld[b], 0};
    tall[b] = MatDesc{hb.u_off[b], n, hb.ld[b], hb.p[b], b};
    small[b] = MatDesc{hb.m_off[b], hb.ld[b], hb.ld[b], hb.p[b], b};
  }
  std::vector<GramTile> gt;
  std::vector<GramReduce> gr;
  gram_tables(tall, true, &gt, &gr);
  // whole-block super-tiles (no partials) run largest block first
  if (gram_unsplit(gr))
    std::stable_sort(gt.begin(), gt.end(), [](const GramTile& x, const GramTile& y) {
      return x.r1 - x.r0 > y.r1 - y.r0;
    });
  std::vector<SpmmTile> st;
  spmm_tables(tall, &st);
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  const size_t ob = put(cb.size() * sizeof(CcBlock)), ot = put(tall.size() * sizeof(MatDesc)),
               os = put(small.size() * sizeof(MatDesc)), og = put(gt.size() * sizeof(GramTile)),
               orr = put(gr.size() * sizeof(GramReduce)), osp = put(st.size() * sizeof(SpmmTile));
  MI_TRY_HIP(hipMalloc(&P->arena, o));
  char* a = static_cast<char*>(P->arena);
  MI_TRY_HIP(hipMemcpy(a + ob, cb.data(), cb.size() * sizeof(CcBlock), hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(a + ot, tall.data(), tall.size() * sizeof(MatDesc), hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(a + os, small.data(), small.size() * sizeof(MatDesc), hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(a + og, gt.data(), gt.size() * sizeof(GramTile), hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(a + orr, gr.data(), gr.size() * sizeof(GramReduce), hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(a + osp, st.data(), st.size() * sizeof(SpmmTile), hipMemcpyHostToDevice));
  P->blocks = reinterpret_cast<CcBlock*>(a + ob);
  P->tall = reinterpret_cast<MatDesc*>(a + ot);
  P->small = reinterpret_cast<MatDesc*>(a + os);
  P->gt = reinterpret_cast<GramTile*>(a + og);
  P->n_gt = (int)gt.size();
  P->gr = reinterpret_cast<GramReduce*>(a + orr);
  P->n_gr = (int)gr.size();
  P->gram_direct = gram_unsplit(gr);
  // spmm tile table kept right after the reduce table
  static_assert(sizeof(SpmmTile) == 8, "");
  // workspace layout
  Carver c(nullptr);
  P->z_off = c.used, c.take<float>(hb.u_off[hb.B]);
  P->gx_off = c.used, c.take<double>(3 * hb.v_off[hb.B]);
  P->ef_off = c.used, c.take<double>(6 * hb.t_off[hb.B]);
  P->efp_off = c.used, c.take<double>(6 * EF_CHUNKS * hb.t_off[hb.B]);
  P->m_off = c.used, c.take<double>(hb.m_off[hb.B]);
  P->part_off = c.used, c.take<double>(gt.size() * GRAM_TILE * GRAM_TILE);
  P->nrm_off = c.used, c.take<double>(2 * hb.B);
  P->total = c.used;
  ctx->cc_plan = P;
  *out = P;
  (void)osp;
  return MI_OK;
}

}  // namespace mis

using namespace mis;

extern "C" {

void mis_destroy_cc_plan(mi_ctx* ctx) {
  delete static_cast<CcPlan*>(ctx->cc_plan);
  ctx->cc_plan = nullptr;
}

mi_status mi_choose_c_workspace_size(mi_ctx* ctx, const mi_blocks* blk, size_t* ws_bytes) {
  clear_error();
  MI_CHECK_ARG(ws_bytes != nullptr, "ws_bytes is NULL");
  (void)ctx;
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  std::vector<MatDesc> tall(hb.B);
  for (int b = 0; b < hb.B; ++b)
    tall[b] = MatDesc{hb.u_off[b], int(hb.v_off[b + 1] - hb.v_off[b]), hb.ld[b], hb.p[b], b};
  std::vector<GramTile> gt;
  std::vector<GramReduce> gr;
  gram_tables(tall, true, &gt, &gr);
  Carver c(nullptr);
  c.take<float>(hb.u_off[hb.B]);
  c.take<double>(3 * hb.v_off[hb.B]);
  // the same regions as the plan's layout, in the same order
  c.take<double>(6 * hb.t_off[hb.B]);
  c.take<double>(6 * EF_CHUNKS * hb.t_off[hb.B]);
  c.take<double>(hb.m_off[hb.B]);
  c.take<double>(gt.size() * GRAM_TILE * GRAM_TILE);
  c.take<double>(2 * hb.B);
  *ws_bytes = c.used;
  return MI_OK;
}

mi_status mi_choose_c(mi_ctx* ctx, const mi_blocks* blk, const int32_t* c_max, double target,
                      double g_min, const float* U, const double* ritz, const float* X,
                      const int32_t* gl_row_ptr, const int32_t* gl_col, const float* gl_val,
                      const int64_t* nnz_off, int32_t* c_out, double* metric_out, void* ws,
                      size_t ws_bytes, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && c_max && U && ritz && X && gl_row_ptr && gl_col && gl_val && nnz_off &&
                   c_out && metric_out,
               "NULL argument");
  MI_CHECK_ARG(target >= 0 && g_min >= 0, "target and g_min must be >= 0");
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  std::vector<int64_t> nnz(nnz_off, nnz_off + hb.B + 1);
  MI_TRY_HIP(hipSetDevice(ctx->device));
  CcPlan* P = nullptr;
  st = cc_plan(ctx, hb, nnz, &P);
  if (st) return st;
  if (!ws || ws_bytes < P->total) {
    set_error("workspace %zu bytes < %zu required", ws_bytes, P->total);
    return MI_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  char* w = static_cast<char*>(ws);
  float* Z = reinterpret_cast<float*>(w + P->z_off);
  double* GX = reinterpret_cast<double*>(w + P->gx_off);
  double* EF = reinterpret_cast<double*>(w + P->ef_off);
  double* M = reinterpret_cast<double*>(w + P->m_off);
  double* part = reinterpret_cast<double*>(w + P->part_off);
  double* nrm = reinterpret_cast<double*>(w + P->nrm_off);
  // the SpMM tile table sits after the Gram reduce table in the arena
  char* a = static_cast<char*>(P->arena);
  const size_t osp = reinterpret_cast<char*>(P->gr) - a + align_up(P->n_gr * sizeof(GramReduce));
  const SpmmTile* tiles = reinterpret_cast<const SpmmTile*>(a + osp);
  int ntiles = 0;
  for (int b = 0; b < hb.B; ++b) ntiles += ceil_div(hb.v_off[b + 1] - hb.v_off[b], SPMM_ROWS);
  // one width for every block (a multiple of 64 up to 320): a wavefront per
  // row; otherwise a thread per row and 4 columns
  int epl = hb.B > 0 && hb.ld[0] % 64 == 0 && hb.ld[0] <= 320 ? hb.ld[0] / 64 : 0;
  for (int b = 0; b < hb.B && epl; ++b)
    if (hb.ld[b] != hb.ld[0]) epl = 0;
  switch (epl) {
#define MI_GL_ROWS(E, ST)                                                                       \
  case E:                                                                                       \
    hipLaunchKernelGGL((k_gl_apply_rows<E, ST>), dim3(2 * ntiles), dim3(512), 0, s, P->blocks,  \
                       tiles, ntiles, gl_row_ptr, gl_col, gl_val, U, Z);                        \
    break;
    MI_GL_ROWS(1, false)
    MI_GL_ROWS(2, false)
    MI_GL_ROWS(3, false)
    MI_GL_ROWS(4, false)
    MI_GL_ROWS(5, true)
#undef MI_GL_ROWS
    default:
      hipLaunchKernelGGL(k_gl_apply, dim3(ntiles), dim3(256), 0, s, P->blocks, tiles, gl_row_ptr,
                         gl_col, gl_val, U, Z);
  }
  hipLaunchKernelGGL(k_gl_coords, dim3(hb.B), dim3(256), 0, s, P->blocks, gl_row_ptr, gl_col,
                     gl_val, X, GX, nrm);
  double* EFP = reinterpret_cast<double*>(w + P->efp_off);
  hipLaunchKernelGGL(k_proj_ef_part, dim3(hb.B * EF_CHUNKS), dim3(256), 0, s, P->blocks, U, Z, X,
                     GX, EFP);
  hipLaunchKernelGGL(k_proj_ef_sum, dim3(hb.B), dim3(256), 0, s, P->blocks, (const double*)EFP,
                     EF);
  if (P->gram_direct) {
    launch_gram_direct<float>(P->gt, P->n_gt, P->tall, P->small, Z, Z, nullptr, M, nullptr, s);
  } else {
    launch_gram<float>(P->gt, P->n_gt, P->tall, Z, Z, nullptr, part, s);
    launch_gram_reduce(P->gr, P->n_gr, P->small, part, false, M, nullptr, s);
  }
  hipLaunchKernelGGL(k_choose, dim3(hb.B), dim3(256), 0, s, P->blocks, c_max, EF, M, nrm, ritz,
                     target, g_min, c_out, metric_out);
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

}  // extern "C"
