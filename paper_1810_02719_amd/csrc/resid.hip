// Residual norms of the tracked Ritz pairs, || L v_j - theta_j v_j ||_2, for
// the iteration control of the orthogonal iteration (Section 4: the number
// of iterations; a caller stops when every kept pair is accurate enough).
//
// Stage 1 (one workgroup per 16-row tile): each wavefront takes whole rows,
// gathers the neighbour rows like the filter's SpMM (wave-uniform CSR reads,
// 16-byte vectors), forms r = (L V)_row - theta * V_row and accumulates r^2
// per column in FP64; the four wavefronts' sums are added in a fixed order
// and written as the tile's partial.  Stage 2 adds a block's tile partials
// in tile order and takes the square root, so results are reproducible.
#include <vector>

#include "common.hpp"
#include "dense.hpp"
#include "kernels_util.hpp"

namespace mis {

namespace {

struct ResTile {
  int32_t blk;
  int32_t row0;
};

struct ResBlock {
  int64_t v_off, u_off, t_off, nnz_off, part_off;  // part_off: first tile's partial
  int32_t n, p, ld, ntiles;
};

struct ResPlan {
  std::vector<int64_t> v_off, u_off, nnz;
  std::vector<int32_t> p, ld;
  ResTile* tiles = nullptr;
  ResBlock* blocks = nullptr;
  int ntiles = 0;
  int64_t part_doubles = 0;
  ~ResPlan() {
    if (tiles) (void)hipFree(tiles);
    if (blocks) (void)hipFree(blocks);
  }
};

int64_t part_layout(const HostBlocks& hb, std::vector<ResBlock>* blocks, std::vector<ResTile>* tiles,
                    const std::vector<int64_t>* nnz_off) {
  int64_t part = 0;
  for (int b = 0; b < hb.B; ++b) {
    const int n = int(hb.v_off[b + 1] - hb.v_off[b]);
    const int nt = ceil_div(n, SPMM_ROWS);
    if (blocks)
      blocks->push_back(ResBlock{hb.v_off[b], hb.u_off[b], hb.t_off[b],
                                 nnz_off ? (*nnz_off)[b] : 0, part, n, hb.p[b], hb.ld[b], nt});
    if (tiles)
      for (int t = 0; t < nt; ++t) tiles->push_back(ResTile{b, t * SPMM_ROWS});
    part += int64_t(nt) * hb.ld[b];
  }
  return part;
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(256)
    k_resid_part(const ResTile* __restrict__ tiles, const ResBlock* __restrict__ blks,
                 const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                 const float* __restrict__ val, const T* __restrict__ V,
                 const double* __restrict__ ritz, double* __restrict__ part) {
  typedef typename VecOf<T>::type Vv;
  constexpr int W = VecOf<T>::W;
  constexpr int MAXV = 1024 / W / 64;  // vectors per lane for ld <= 1024
  __shared__ double wsum[4][1024];
  const ResTile t = tiles[blockIdx.x];
  const ResBlock b = blks[t.blk];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nvec = b.ld / W;
  const int rows = min(SPMM_ROWS, b.n - t.row0);
  const T* Vb = V + b.u_off;
  const int32_t* rp = row_ptr + b.v_off + t.blk;
  const int32_t* cb = col + b.nnz_off;
  const float* vb = val + b.nnz_off;
  double acc[MAXV][W];
#pragma unroll
  for (int s = 0; s < MAXV; ++s)
#pragma unroll
    for (int e = 0; e < W; ++e) acc[s][e] = 0.0;
  for (int rr = wave; rr < rows; rr += 4) {
    const int r = t.row0 + rr;
    const int k0 = rp[r], k1 = rp[r + 1];
#pragma unroll
    for (int s = 0; s < MAXV; ++s) {
      const int v = lane + 64 * s;
      if (v >= nvec) continue;
      double lv[W];
#pragma unroll
      for (int e = 0; e < W; ++e) lv[e] = 0.0;
      for (int k = k0; k < k1; ++k) {
        const Vv y = *reinterpret_cast<const Vv*>(Vb + int64_t(cb[k]) * b.ld + v * W);
        const double w = vb[k];
#pragma unroll
        for (int e = 0; e < W; ++e) lv[e] = fma(w, (double)y[e], lv[e]);
      }
      const Vv x = *reinterpret_cast<const Vv*>(Vb + int64_t(r) * b.ld + v * W);
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const int j = v * W + e;
        const double th = j < b.p ? ritz[b.t_off + j] : 0.0;
        const double res = fma(-th, (double)x[e], lv[e]);
        acc[s][e] = fma(res, res, acc[s][e]);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < MAXV; ++s) {
    const int v = lane + 64 * s;
    if (v < nvec)
#pragma unroll
      for (int e = 0; e < W; ++e) wsum[wave][v * W + e] = acc[s][e];
  }
  __syncthreads();
  double* out = part + b.part_off + int64_t(t.row0 / SPMM_ROWS) * b.ld;
  for (int j = threadIdx.x; j < b.ld; j += 256)
    out[j] = ((wsum[0][j] + wsum[1][j]) + wsum[2][j]) + wsum[3][j];
}

__global__ void __launch_bounds__(256)
    k_resid_sum(const ResBlock* __restrict__ blks, const double* __restrict__ part,
                double* __restrict__ resid) {
  const ResBlock b = blks[blockIdx.x];
  for (int j = threadIdx.x; j < b.p; j += 256) {
    double s = 0.0;
    for (int t = 0; t < b.ntiles; ++t) s += part[b.part_off + int64_t(t) * b.ld + j];
    resid[b.t_off + j] = sqrt(s);
  }
}

}  // namespace mis

using namespace mis;

extern "C" {

void mis_destroy_res_plan(mi_ctx* ctx) {
  delete static_cast<ResPlan*>(ctx->res_plan);
  ctx->res_plan = nullptr;
}

mi_status mi_residual_workspace_size(mi_ctx* ctx, const mi_blocks* blk, size_t* ws_bytes) {
  clear_error();
  (void)ctx;
  MI_CHECK_ARG(ws_bytes != nullptr, "ws_bytes is NULL");
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  *ws_bytes = size_t(part_layout(hb, nullptr, nullptr, nullptr)) * sizeof(double);
  return MI_OK;
}

mi_status mi_ritz_residuals(mi_ctx* ctx, const mi_blocks* blk, int32_t precision,
                            const int32_t* row_ptr, const int32_t* col, const float* val,
                            const int64_t* nnz_off, const void* V, const double* ritz,
                            double* resid, void* ws, size_t ws_bytes, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && row_ptr && col && val && nnz_off && V && ritz && resid, "NULL argument");
  MI_CHECK_ARG(precision == MI_FP32 || precision == MI_FP64, "precision %d unsupported", precision);
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  std::vector<int64_t> nnz(nnz_off, nnz_off + hb.B + 1);
  for (int b = 0; b < hb.B; ++b)
    MI_CHECK_ARG(nnz[b + 1] >= nnz[b], "nnz_off must be non-decreasing");
  const int64_t need = part_layout(hb, nullptr, nullptr, nullptr);
  if (!ws || ws_bytes < size_t(need) * sizeof(double)) {
    set_error("workspace %zu bytes < %zu required", ws_bytes, size_t(need) * sizeof(double));
    return MI_ERR_WORKSPACE;
  }
  MI_TRY_HIP(hipSetDevice(ctx->device));
  ResPlan* P = static_cast<ResPlan*>(ctx->res_plan);
  if (!P || P->v_off != hb.v_off || P->u_off != hb.u_off || P->p != hb.p || P->ld != hb.ld ||
      P->nnz != nnz) {
    delete P;
    ctx->res_plan = nullptr;
    P = new ResPlan();
    P->v_off = hb.v_off;
    P->u_off = hb.u_off;
    P->p = hb.p;
    P->ld = hb.ld;
    P->nnz = nnz;
    std::vector<ResBlock> bl;
    std::vector<ResTile> tl;
    P->part_doubles = part_layout(hb, &bl, &tl, &nnz);
    P->ntiles = (int)tl.size();
    if (hipMalloc(&P->blocks, bl.size() * sizeof(ResBlock)) != hipSuccess ||
        hipMalloc(&P->tiles, std::max<size_t>(tl.size(), 1) * sizeof(ResTile)) != hipSuccess) {
      delete P;
      set_error("device allocation for the residual tables failed");
      return MI_ERR_HIP;
    }
    ctx->res_plan = P;
    MI_TRY_HIP(hipMemcpy(P->blocks, bl.data(), bl.size() * sizeof(ResBlock), hipMemcpyHostToDevice));
    if (!tl.empty())
      MI_TRY_HIP(hipMemcpy(P->tiles, tl.data(), tl.size() * sizeof(ResTile), hipMemcpyHostToDevice));
  }
  hipStream_t s = (hipStream_t)stream;
  double* part = static_cast<double*>(ws);
  KClose kc_(ctx->timer);
  KScope k_(ctx->timer, MI_K_SETUP, s);
  if (P->ntiles > 0) {
    if (precision == MI_FP64)
      hipLaunchKernelGGL(k_resid_part<double>, dim3(P->ntiles), dim3(256), 0, s, P->tiles,
                         P->blocks, row_ptr, col, val, (const double*)V, ritz, part);
    else
      hipLaunchKernelGGL(k_resid_part<float>, dim3(P->ntiles), dim3(256), 0, s, P->tiles,
                         P->blocks, row_ptr, col, val, (const float*)V, ritz, part);
  }
  hipLaunchKernelGGL(k_resid_sum, dim3(hb.B), dim3(256), 0, s, P->blocks, part, resid);
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

}  // extern "C"
