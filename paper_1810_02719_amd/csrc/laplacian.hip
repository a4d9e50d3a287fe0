// Graph Laplacian of every block (Section 3, Eq. 1-2), built on the GPU.
//
// Work plan (all blocks in the same launches):
//   1. every primitive emits its edges as two half-edges; a per-row counter
//      (atomic, integer: order independent) gives the row's half-edge count;
//   2. exclusive scan -> slot offsets; the half-edges are scattered into the
//      slots (slot order depends on atomics, the next step removes that);
//   3. one thread per row sorts its neighbour list (insertion sort; rows of a
//      triangle mesh hold ~12 entries) and removes duplicates;
//   4. scans of the unique counts give the CSR offsets and the canonical
//      edge numbering (upper-triangle entries in row-major order);
//   5. one thread per row writes columns (diagonal merged in order), values
//      and its canonical edges.
// The result does not depend on scheduling: structure is bit-exact.
#include "common.hpp"
#include "kernels_util.hpp"

namespace mis {

struct LapWs {
  int32_t* cnt;      // [N] half-edges per row (with duplicates)
  int32_t* fillpos;  // [N]
  int64_t* slot;     // [N+1]
  int32_t* adj;      // [H]
  int32_t* ucnt;     // [N] unique neighbours + 1 (diagonal)
  int32_t* upcnt;    // [N] unique neighbours > row
  int64_t* nnzs;     // [N+1]
  int64_t* edges_s;  // [N+1]
  int64_t* scratch;  // scan scratch
  int32_t* err;      // [1]
  int64_t* dev_voff; // [B+1]
  int64_t* dev_poff; // [B+1]
  int64_t* gather;   // [2*(B+1)]
};

static size_t lap_ws(int64_t N, int64_t H, int B, LapWs* w, void* base) {
  Carver c(base);
  LapWs t;
  t.cnt = c.take<int32_t>(N);
  t.fillpos = c.take<int32_t>(N);
  t.slot = c.take<int64_t>(N + 1);
  t.adj = c.take<int32_t>(std::max<int64_t>(H, 1));
  t.ucnt = c.take<int32_t>(N);
  t.upcnt = c.take<int32_t>(N);
  t.nnzs = c.take<int64_t>(N + 1);
  t.edges_s = c.take<int64_t>(N + 1);
  t.scratch = c.take<int64_t>(scan_scratch_bytes(N + 1) / sizeof(int64_t) + 1);
  t.err = c.take<int32_t>(1);
  t.dev_voff = c.take<int64_t>(B + 1);
  t.dev_poff = c.take<int64_t>(B + 1);
  t.gather = c.take<int64_t>(2 * (B + 1));
  if (w) *w = t;
  return c.used;
}

static int64_t half_edges(int64_t nprims, int arity) { return nprims * (arity == 3 ? 6 : 2); }

// Pass 1 (count) and pass 2 (scatter) share the traversal.
template <bool SCATTER>
__global__ void k_emit(const int32_t* __restrict__ prims, int arity, int64_t nprims,
                       const int64_t* __restrict__ poff, const int64_t* __restrict__ voff, int B,
                       int32_t* __restrict__ cnt, int32_t* __restrict__ fillpos,
                       const int64_t* __restrict__ slot, int32_t* __restrict__ adj,
                       int32_t* __restrict__ err) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nprims) return;
  int b = find_block(poff, B, q);
  int64_t v0 = voff[b];
  int32_t n = (int32_t)(voff[b + 1] - v0);
  int32_t c[3];
  for (int k = 0; k < arity; ++k) {
    c[k] = prims[q * arity + k];
    if (c[k] < -1 || c[k] >= n) {
      atomicExch(err, (int)MI_ERR_INDEX);
      return;
    }
  }
  const int ne = (arity == 3) ? 3 : 1;
  for (int k = 0; k < ne; ++k) {
    int32_t u = c[k], v = c[(k + 1) % arity];
    if (u < 0 || v < 0 || u == v) continue;
    if (!SCATTER) {
      atomicAdd(&cnt[v0 + u], 1);
      atomicAdd(&cnt[v0 + v], 1);
    } else {
      int32_t pu = atomicAdd(&fillpos[v0 + u], 1);
      adj[slot[v0 + u] + pu] = v;
      int32_t pv = atomicAdd(&fillpos[v0 + v], 1);
      adj[slot[v0 + v] + pv] = u;
    }
  }
}

__global__ void k_sort_unique(const int64_t* __restrict__ voff, int B, int64_t N,
                              const int32_t* __restrict__ cnt, const int64_t* __restrict__ slot,
                              int32_t* __restrict__ adj, int32_t* __restrict__ ucnt,
                              int32_t* __restrict__ upcnt) {
  int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int b = find_block(voff, B, r);
  int32_t i = (int32_t)(r - voff[b]);
  int32_t* a = adj + slot[r];
  int32_t d = cnt[r];
  for (int x = 1; x < d; ++x) {  // insertion sort
    int32_t key = a[x];
    int y = x - 1;
    while (y >= 0 && a[y] > key) {
      a[y + 1] = a[y];
      --y;
    }
    a[y + 1] = key;
  }
  int32_t u = 0, up = 0;
  for (int x = 0; x < d; ++x) {
    if (x == 0 || a[x] != a[x - 1]) {
      a[u++] = a[x];
      if (a[x] > i) ++up;
    }
  }
  ucnt[r] = u + 1;
  upcnt[r] = up;
}

__global__ void k_gather_offsets(const int64_t* __restrict__ voff, int B,
                                 const int64_t* __restrict__ nnzs, const int64_t* __restrict__ es,
                                 int64_t* __restrict__ out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > B) return;
  out[b] = nnzs[voff[b]];
  out[B + 1 + b] = es[voff[b]];
}

__device__ inline double edge_weight(int mode, const float* __restrict__ X, int64_t gi, int64_t gj,
                                     const float* __restrict__ user_w, int64_t eidx,
                                     int32_t* __restrict__ err) {
  if (mode == MI_W_COMBINATORIAL) return 1.0;
  if (mode == MI_W_USER) return (double)user_w[eidx];
  double dx = (double)X[3 * gi] - (double)X[3 * gj];
  double dy = (double)X[3 * gi + 1] - (double)X[3 * gj + 1];
  double dz = (double)X[3 * gi + 2] - (double)X[3 * gj + 2];
  double d2 = dx * dx + dy * dy + dz * dz;
  if (d2 == 0.0) {
    if (err) atomicExch(err, (int)MI_ERR_DEGENERATE);
    return 0.0;
  }
  return mode == MI_W_INV_SQ_DIST ? 1.0 / d2 : 1.0 / sqrt(d2);
}

// Canonical index of edge (lo, hi), lo < hi, of the row-global block rows:
// edge_start(lo) + rank of hi among lo's neighbours greater than lo.
__device__ inline int64_t edge_index(int64_t rlo, int32_t lo_local, int32_t hi,
                                     const int64_t* __restrict__ slot,
                                     const int32_t* __restrict__ ucnt,
                                     const int32_t* __restrict__ adj,
                                     const int64_t* __restrict__ es) {
  const int32_t* a = adj + slot[rlo];
  int32_t u = ucnt[rlo] - 1;
  // first position with a[pos] > lo_local
  int l = 0, h = u;
  while (l < h) {
    int m = (l + h) >> 1;
    if (a[m] > lo_local) h = m; else l = m + 1;
  }
  int first_up = l;
  l = first_up;
  h = u;
  while (l < h) {
    int m = (l + h) >> 1;
    if (a[m] < hi) l = m + 1; else h = m;
  }
  return es[rlo] + (l - first_up);
}

__global__ void k_fill_csr(const int64_t* __restrict__ voff, int B, int64_t N, int mode,
                           const float* __restrict__ X, const float* __restrict__ user_w,
                           const int64_t* __restrict__ slot, const int32_t* __restrict__ adj,
                           const int32_t* __restrict__ ucnt, const int64_t* __restrict__ nnzs,
                           const int64_t* __restrict__ es, int32_t* __restrict__ row_ptr,
                           int32_t* __restrict__ col, float* __restrict__ val,
                           int32_t* __restrict__ edges, float* __restrict__ edge_w,
                           int32_t* __restrict__ err) {
  int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int b = find_block(voff, B, r);
  int64_t v0 = voff[b];
  int32_t i = (int32_t)(r - v0);
  int32_t n = (int32_t)(voff[b + 1] - v0);
  int64_t nbase = nnzs[v0];
  int64_t start = nnzs[r];
  row_ptr[v0 + b + i] = (int32_t)(start - nbase);
  if (i == n - 1) row_ptr[v0 + b + n] = (int32_t)(nnzs[r + 1] - nbase);
  const int32_t* a = adj + slot[r];
  int32_t u = ucnt[r] - 1;
  double diag = 0.0;
  int64_t pos = start;
  int64_t dpos = -1;
  int64_t ecount = 0;
  for (int x = 0; x <= u; ++x) {
    if (dpos < 0 && (x == u || a[x] > i)) {
      dpos = pos++;
      col[dpos] = i;
    }
    if (x == u) break;
    int32_t j = a[x];
    int64_t eidx;
    if (j > i) {
      eidx = es[r] + ecount;
      ++ecount;
    } else {
      eidx = edge_index(v0 + j, j, i, slot, ucnt, adj, es);
    }
    double w = edge_weight(mode, X, v0 + i, v0 + j, user_w, eidx, err);
    col[pos] = j;
    val[pos] = (float)(-w);
    ++pos;
    diag += w;
    if (j > i) {
      edges[2 * eidx] = i;
      edges[2 * eidx + 1] = j;
      if (edge_w) edge_w[eidx] = (float)w;
    }
  }
  val[dpos] = (float)diag;
}

// Values on a fixed structure: one thread per row.
__global__ void k_values(const int64_t* __restrict__ voff, int B, int64_t N, int mode,
                         const float* __restrict__ X, const float* __restrict__ user_w,
                         const int64_t* __restrict__ nnz_off, const int64_t* __restrict__ e_off,
                         const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                         const int32_t* __restrict__ edges, float* __restrict__ val,
                         float* __restrict__ edge_w, int32_t* __restrict__ err) {
  int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int b = find_block(voff, B, r);
  int64_t v0 = voff[b];
  int32_t i = (int32_t)(r - v0);
  const int32_t* rp = row_ptr + v0 + b;
  int64_t e0 = e_off[b], ne = e_off[b + 1] - e0;
  const int32_t* eb = edges + 2 * e0;
  double diag = 0.0;
  int64_t dpos = -1;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    int64_t kk = nnz_off[b] + k;
    int32_t j = col[kk];
    if (j == i) {
      dpos = kk;
      continue;
    }
    int32_t lo = min(i, j), hi = max(i, j);
    int64_t l = 0, h = ne;  // lexicographic binary search
    while (l < h) {
      int64_t m = (l + h) >> 1;
      int32_t a0 = eb[2 * m], a1 = eb[2 * m + 1];
      if (a0 < lo || (a0 == lo && a1 < hi)) l = m + 1; else h = m;
    }
    int64_t eidx = e0 + l;
    double w = edge_weight(mode, X, v0 + i, v0 + j, user_w, eidx, err);
    val[kk] = (float)(-w);
    diag += w;
    if (j > i && edge_w) edge_w[eidx] = (float)w;
  }
  if (dpos >= 0) val[dpos] = (float)diag;
}

static mi_status lap_common(const mi_blocks* blk, const int64_t* prim_off, int arity,
                            HostBlocks* hb, int64_t* N, int64_t* H) {
  mi_status st = load_blocks(blk, hb, false);
  if (st) return st;
  MI_CHECK_ARG(prim_off != nullptr, "prim_off is NULL");
  MI_CHECK_ARG(arity == 2 || arity == 3, "arity must be 2 or 3 (got %d)", arity);
  MI_CHECK_ARG(prim_off[0] == 0, "prim_off[0] must be 0");
  for (int b = 0; b < hb->B; ++b)
    MI_CHECK_ARG(prim_off[b + 1] >= prim_off[b], "prim_off not ascending at %d", b);
  *N = hb->v_off[hb->B];
  *H = half_edges(prim_off[hb->B], arity);
  return MI_OK;
}

// Runs passes 1-4 into the workspace.  Returns a status read back after a sync.
static mi_status lap_structure(const HostBlocks& hb, const int64_t* prim_off, const int32_t* prims,
                               int arity, int64_t N, int64_t H, const LapWs& w, hipStream_t s) {
  const int B = hb.B;
  const int64_t P = prim_off[B];
  MI_TRY_HIP(hipMemcpyAsync(w.dev_voff, hb.v_off.data(), (B + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
  MI_TRY_HIP(hipMemcpyAsync(w.dev_poff, prim_off, (B + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
  fill_i32(w.cnt, 0, N, s);
  fill_i32(w.fillpos, 0, N, s);
  fill_i32(w.err, 0, 1, s);
  if (P > 0) {
    MI_CHECK_ARG(prims != nullptr, "prims is NULL");
    hipLaunchKernelGGL(k_emit<false>, dim3(ceil_div(P, 256)), dim3(256), 0, s, prims, arity, P,
                       w.dev_poff, w.dev_voff, B, w.cnt, w.fillpos, w.slot, w.adj, w.err);
  }
  exclusive_scan(w.cnt, w.slot, N, w.scratch, s);
  if (P > 0)
    hipLaunchKernelGGL(k_emit<true>, dim3(ceil_div(P, 256)), dim3(256), 0, s, prims, arity, P,
                       w.dev_poff, w.dev_voff, B, w.cnt, w.fillpos, w.slot, w.adj, w.err);
  hipLaunchKernelGGL(k_sort_unique, dim3(ceil_div(N, 256)), dim3(256), 0, s, w.dev_voff, B, N,
                     w.cnt, w.slot, w.adj, w.ucnt, w.upcnt);
  exclusive_scan(w.ucnt, w.nnzs, N, w.scratch, s);
  exclusive_scan(w.upcnt, w.edges_s, N, w.scratch, s);
  MI_TRY_HIP(hipGetLastError());
  (void)H;
  return MI_OK;
}

static mi_status read_err(const LapWs& w, hipStream_t s) {
  int32_t e = 0;
  MI_TRY_HIP(hipMemcpyAsync(&e, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MI_TRY_HIP(hipStreamSynchronize(s));
  if (e == MI_ERR_INDEX) {
    set_error("a primitive references a vertex id outside its block");
    return MI_ERR_INDEX;
  }
  if (e == MI_ERR_DEGENERATE) {
    set_error("zero-length edge under a distance weight");
    return MI_ERR_DEGENERATE;
  }
  return MI_OK;
}

}  // namespace mis

using namespace mis;

extern "C" {

mi_status mi_laplacian_workspace_size(const mi_blocks* blk, const int64_t* prim_off,
                                      int32_t arity, size_t* ws_bytes) {
  clear_error();
  MI_CHECK_ARG(ws_bytes != nullptr, "ws_bytes is NULL");
  HostBlocks hb;
  int64_t N, H;
  mi_status st = lap_common(blk, prim_off, arity, &hb, &N, &H);
  if (st) return st;
  *ws_bytes = lap_ws(N, H, hb.B, nullptr, nullptr);
  return MI_OK;
}

mi_status mi_build_laplacian_count(mi_ctx* ctx, const mi_blocks* blk, const int64_t* prim_off,
                                   const int32_t* prims, int32_t arity, int64_t* nnz_off,
                                   int64_t* edge_off, void* ws, size_t ws_bytes, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  MI_CHECK_ARG(nnz_off && edge_off, "nnz_off / edge_off are NULL");
  HostBlocks hb;
  int64_t N, H;
  mi_status st = lap_common(blk, prim_off, arity, &hb, &N, &H);
  if (st) return st;
  size_t need = lap_ws(N, H, hb.B, nullptr, nullptr);
  if (!ws || ws_bytes < need) {
    set_error("workspace %zu bytes < %zu required", ws_bytes, need);
    return MI_ERR_WORKSPACE;
  }
  MI_TRY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  LapWs w;
  lap_ws(N, H, hb.B, &w, ws);
  st = lap_structure(hb, prim_off, prims, arity, N, H, w, s);
  if (st) return st;
  hipLaunchKernelGGL(k_gather_offsets, dim3(ceil_div(hb.B + 1, 256)), dim3(256), 0, s, w.dev_voff,
                     hb.B, w.nnzs, w.edges_s, w.gather);
  std::vector<int64_t> h(2 * (hb.B + 1));
  MI_TRY_HIP(hipMemcpyAsync(h.data(), w.gather, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  st = read_err(w, s);
  if (st) return st;
  for (int b = 0; b <= hb.B; ++b) {
    nnz_off[b] = h[b];
    edge_off[b] = h[hb.B + 1 + b];
  }
  return MI_OK;
}

mi_status mi_build_laplacian(mi_ctx* ctx, const mi_blocks* blk, const int64_t* prim_off,
                             const int32_t* prims, int32_t arity, const int64_t* nnz_off,
                             const int64_t* edge_off, int32_t weight_mode, const float* coords,
                             const float* user_w, int32_t* row_ptr, int32_t* col, float* val,
                             int32_t* edges, float* edge_w, void* ws, size_t ws_bytes,
                             void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  HostBlocks hb;
  int64_t N, H;
  mi_status st = lap_common(blk, prim_off, arity, &hb, &N, &H);
  if (st) return st;
  MI_CHECK_ARG(weight_mode >= 0 && weight_mode <= 3, "weight_mode %d unknown", weight_mode);
  MI_CHECK_ARG(weight_mode == MI_W_COMBINATORIAL || weight_mode == MI_W_USER || coords,
               "coords required for distance weights");
  MI_CHECK_ARG(weight_mode != MI_W_USER || user_w, "user_w required for MI_W_USER");
  MI_CHECK_ARG(row_ptr && col && val && edges, "row_ptr, col, val and edges are required");
  MI_CHECK_ARG(nnz_off && edge_off, "nnz_off / edge_off are NULL");
  size_t need = lap_ws(N, H, hb.B, nullptr, nullptr);
  if (!ws || ws_bytes < need) {
    set_error("workspace %zu bytes < %zu required", ws_bytes, need);
    return MI_ERR_WORKSPACE;
  }
  MI_TRY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  LapWs w;
  lap_ws(N, H, hb.B, &w, ws);
  st = lap_structure(hb, prim_off, prims, arity, N, H, w, s);
  if (st) return st;
  // the caller's offsets must be the ones the count call produced
  hipLaunchKernelGGL(k_gather_offsets, dim3(ceil_div(hb.B + 1, 256)), dim3(256), 0, s, w.dev_voff,
                     hb.B, w.nnzs, w.edges_s, w.gather);
  std::vector<int64_t> h(2 * (hb.B + 1));
  MI_TRY_HIP(hipMemcpyAsync(h.data(), w.gather, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  st = read_err(w, s);
  if (st) return st;
  for (int b = 0; b <= hb.B; ++b) {
    if (h[b] != nnz_off[b] || h[hb.B + 1 + b] != edge_off[b]) {
      set_error("nnz_off / edge_off do not match the structure (block %d)", b);
      return MI_ERR_ARG;
    }
  }
  hipLaunchKernelGGL(k_fill_csr, dim3(ceil_div(N, 256)), dim3(256), 0, s, w.dev_voff, hb.B, N,
                     weight_mode, coords, user_w, w.slot, w.adj, w.ucnt, w.nnzs, w.edges_s,
                     row_ptr, col, val, edges, edge_w, w.err);
  MI_TRY_HIP(hipGetLastError());
  return read_err(w, s);
}

mi_status mi_laplacian_values(mi_ctx* ctx, const mi_blocks* blk, const int64_t* nnz_off,
                              const int64_t* edge_off, int32_t weight_mode, const float* coords,
                              const float* user_w, const int32_t* row_ptr, const int32_t* col,
                              const int32_t* edges, float* val, float* edge_w, int32_t* err_flag,
                              void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, false);
  if (st) return st;
  MI_CHECK_ARG(nnz_off && edge_off && row_ptr && col && edges && val, "NULL argument");
  MI_CHECK_ARG(weight_mode >= 0 && weight_mode <= 3, "weight_mode %d unknown", weight_mode);
  MI_CHECK_ARG(weight_mode == MI_W_COMBINATORIAL || weight_mode == MI_W_USER || coords,
               "coords required for distance weights");
  MI_CHECK_ARG(weight_mode != MI_W_USER || user_w, "user_w required for MI_W_USER");
  MI_TRY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int B = hb.B;
  const int64_t N = hb.v_off[B];
  // device copies of the three offset tables (stream-ordered allocation)
  int64_t* d = nullptr;
  MI_TRY_HIP(hipMallocAsync((void**)&d, 3 * (B + 1) * sizeof(int64_t), s));
  MI_TRY_HIP(hipMemcpyAsync(d, hb.v_off.data(), (B + 1) * 8, hipMemcpyHostToDevice, s));
  MI_TRY_HIP(hipMemcpyAsync(d + B + 1, nnz_off, (B + 1) * 8, hipMemcpyHostToDevice, s));
  MI_TRY_HIP(hipMemcpyAsync(d + 2 * (B + 1), edge_off, (B + 1) * 8, hipMemcpyHostToDevice, s));
  int32_t* errp = err_flag;
  hipLaunchKernelGGL(k_values, dim3(ceil_div(N, 256)), dim3(256), 0, s, d, B, N, weight_mode,
                     coords, user_w, d + B + 1, d + 2 * (B + 1), row_ptr, col, edges, val, edge_w,
                     errp ? errp : nullptr);
  MI_TRY_HIP(hipGetLastError());
  MI_TRY_HIP(hipFreeAsync(d, s));
  return MI_OK;
}

}  // extern "C"
