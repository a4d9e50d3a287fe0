// Merge of overlapped submeshes (Section 6.1, Alg. 3): every mesh vertex
// gets the average of its reconstructions in the submeshes that hold it,
// each weighted by the vertex's degree in that submesh (the off-diagonal
// entry count of its row of the submesh Laplacian).
//
// The occurrences of every mesh vertex (block rows that hold it) are listed
// once per (blocks, vertex map) on the host, in ascending block order; one
// thread per mesh vertex then gathers its occurrences and sums them in FP64
// in that order, so the result is bitwise reproducible.  The kernel is a
// gather bound by HBM latency and traffic: per occurrence 12 bytes of
// coordinates, two row pointers and the occurrence entry; per vertex the
// occurrence offsets and 12 bytes of output.
#include <algorithm>
#include <cstring>
#include <memory>

#include "common.hpp"

namespace mis {

struct MergePlan {
  std::vector<int64_t> v_off;
  std::vector<int32_t> gid;
  int64_t n_vertices = 0;
  int64_t* occ_off = nullptr;   // [n_vertices + 1]
  int32_t* occ_row = nullptr;   // block row (v_off[b] + i) of every occurrence
  int32_t* occ_blk = nullptr;   // its block b
  ~MergePlan() {
    if (occ_off) (void)hipFree(occ_off);
    if (occ_row) (void)hipFree(occ_row);
    if (occ_blk) (void)hipFree(occ_blk);
  }
};

__global__ void __launch_bounds__(256)
    k_merge(const int64_t* __restrict__ occ_off, const int32_t* __restrict__ occ_row,
            const int32_t* __restrict__ occ_blk, const int32_t* __restrict__ row_ptr,
            const float* __restrict__ X, float* __restrict__ out, int64_t nv) {
  const int64_t v = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (v >= nv) return;
  const int64_t o0 = occ_off[v], o1 = occ_off[v + 1];
  double sx = 0.0, sy = 0.0, sz = 0.0, sw = 0.0;
  for (int64_t k = o0; k < o1; ++k) {
    const int64_t r = occ_row[k];
    const int64_t rp = r + occ_blk[k];  // the block's row pointers start at v_off[b] + b
    // degree: entries of the row minus the stored diagonal; w * x is exact
    // in FP64, so each step rounds once, like the plain sum
    const double w = double(row_ptr[rp + 1] - row_ptr[rp] - 1);
    sx = fma(w, double(X[3 * r]), sx);
    sy = fma(w, double(X[3 * r + 1]), sy);
    sz = fma(w, double(X[3 * r + 2]), sz);
    sw += w;
  }
  if (!(sw > 0.0) && o1 > o0) {  // isolated in every submesh: plain mean
    sx = sy = sz = 0.0;
    for (int64_t k = o0; k < o1; ++k) {
      const int64_t r = occ_row[k];
      sx += double(X[3 * r]);
      sy += double(X[3 * r + 1]);
      sz += double(X[3 * r + 2]);
    }
    sw = double(o1 - o0);
  }
  if (sw > 0.0) {
    out[3 * v] = float(sx / sw);
    out[3 * v + 1] = float(sy / sw);
    out[3 * v + 2] = float(sz / sw);
  } else {  // in no submesh
    out[3 * v] = 0.0f;
    out[3 * v + 1] = 0.0f;
    out[3 * v + 2] = 0.0f;
  }
}

static mi_status merge_plan(mi_ctx* ctx, const HostBlocks& hb, const int32_t* gid, int64_t nv,
                            MergePlan** out) {
  const int64_t N = hb.v_off[hb.B];
  MergePlan* P = static_cast<MergePlan*>(ctx->merge_plan);
  if (P && P->n_vertices == nv && P->v_off == hb.v_off &&
      std::memcmp(P->gid.data(), gid, size_t(N) * sizeof(int32_t)) == 0) {
    *out = P;
    return MI_OK;
  }
  delete P;
  ctx->merge_plan = nullptr;
  std::unique_ptr<MergePlan> np(new MergePlan());
  np->v_off = hb.v_off;
  np->gid.assign(gid, gid + N);
  np->n_vertices = nv;
  // counting sort of the block rows by mesh vertex; rows are visited in
  // ascending order, hence blocks in ascending order within every vertex
  std::vector<int64_t> off(nv + 1, 0);
  for (int64_t r = 0; r < N; ++r) {
    const int32_t g = gid[r];
    if (g < 0 || g >= nv) {
      set_error("row %lld: vertex %d outside [0, %lld)", (long long)r, g, (long long)nv);
      return MI_ERR_INDEX;
    }
    ++off[g + 1];
  }
  for (int64_t v = 0; v < nv; ++v) off[v + 1] += off[v];
  std::vector<int32_t> row(N), blk(N);
  std::vector<int64_t> fill(off.begin(), off.end() - 1);
  for (int b = 0; b < hb.B; ++b)
    for (int64_t r = hb.v_off[b]; r < hb.v_off[b + 1]; ++r) {
      const int64_t k = fill[gid[r]]++;
      row[k] = int32_t(r);
      blk[k] = b;
    }
  MI_TRY_HIP(hipMalloc(&np->occ_off, size_t(nv + 1) * sizeof(int64_t)));
  MI_TRY_HIP(hipMalloc(&np->occ_row, std::max<size_t>(N, 1) * sizeof(int32_t)));
  MI_TRY_HIP(hipMalloc(&np->occ_blk, std::max<size_t>(N, 1) * sizeof(int32_t)));
  MI_TRY_HIP(hipMemcpy(np->occ_off, off.data(), size_t(nv + 1) * sizeof(int64_t),
                       hipMemcpyHostToDevice));
  if (N > 0) {
    MI_TRY_HIP(hipMemcpy(np->occ_row, row.data(), size_t(N) * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    MI_TRY_HIP(hipMemcpy(np->occ_blk, blk.data(), size_t(N) * sizeof(int32_t),
                         hipMemcpyHostToDevice));
  }
  P = np.release();
  ctx->merge_plan = P;
  *out = P;
  return MI_OK;
}

}  // namespace mis

using namespace mis;

extern "C" {

void mis_destroy_merge_plan(mi_ctx* ctx) {
  delete static_cast<MergePlan*>(ctx->merge_plan);
  ctx->merge_plan = nullptr;
}

mi_status mi_merge_overlapped(mi_ctx* ctx, const mi_blocks* blk, const int32_t* gid,
                              int64_t n_vertices, const int32_t* row_ptr, const float* Xr,
                              float* Xout, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && gid && row_ptr && Xr && Xout, "NULL argument");
  MI_CHECK_ARG(n_vertices >= 0 && n_vertices < (int64_t(1) << 31), "n_vertices %lld out of range",
               (long long)n_vertices);
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, false);
  if (st) return st;
  MI_CHECK_ARG(hb.v_off[hb.B] < (int64_t(1) << 31), "more than 2^31 block rows");
  MI_TRY_HIP(hipSetDevice(ctx->device));
  MergePlan* P = nullptr;
  st = merge_plan(ctx, hb, gid, n_vertices, &P);
  if (st) return st;
  if (n_vertices == 0) return MI_OK;
  KClose kc_(ctx->timer);
  KScope k_(ctx->timer, MI_K_MERGE, (hipStream_t)stream);
  hipLaunchKernelGGL(k_merge, dim3(ceil_div(n_vertices, 256)), dim3(256), 0, (hipStream_t)stream,
                     P->occ_off, P->occ_row, P->occ_blk, row_ptr, Xr, Xout, n_vertices);
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

}  // extern "C"
