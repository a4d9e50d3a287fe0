// Graph Fourier transform of the coordinates onto the tracked subspace and
// back (Section 3: v_bar = U^T v, v = U v_bar; Section 7.1: E = U_c^T v,
// v~ = U_c E), with truncation to the first c_b coefficients.
//
// Both kernels are bound by HBM traffic (one read of U, 4 c_b bytes per
// vertex row); sums run in FP64 and in a fixed order, so results are
// bitwise reproducible.
#include <cstring>
#include <mutex>

#include "common.hpp"
#include "kernels_util.hpp"

namespace mis {

constexpr int PROJ_CHUNKS = 16;  // row ranges per block of the projection sums
constexpr int ENC_TILE = 64;     // rows per workgroup of the reconstruction
constexpr int ENC_KPL = 4;       // columns per lane of the tiled kernels (ld <= 256)

struct EncBlock {
  int64_t v_off, u_off, t_off;
  int32_t n, p, ld, pad;
};

struct EncTile {
  int32_t blk, row0;
};

struct EncPlan {
  std::vector<int64_t> v_off, u_off;
  std::vector<int32_t> p, ld;
  EncBlock* dev = nullptr;
  int64_t* dev_voff = nullptr;
  int64_t* dev_poff = nullptr;  // per-block offset of the projection partials
  EncTile* tiles = nullptr;     // ENC_TILE-row tiles of every block
  int n_tiles = 0;
  int max_ld = 0;
  ~EncPlan() {
    if (dev) (void)hipFree(dev);
    if (dev_voff) (void)hipFree(dev_voff);
    if (dev_poff) (void)hipFree(dev_poff);
    if (tiles) (void)hipFree(tiles);
  }
};

// Doubles of projection partials: PROJ_CHUNKS x ld x 3 per block.
static int64_t proj_part_doubles(const HostBlocks& hb, std::vector<int64_t>* off) {
  int64_t t = 0;
  for (int b = 0; b < hb.B; ++b) {
    if (off) off->push_back(t);
    t += int64_t(PROJ_CHUNKS) * hb.ld[b] * 3;
  }
  return t;
}

static mi_status enc_plan(mi_ctx* ctx, const HostBlocks& hb, EncPlan** out) {
  EncPlan* P = static_cast<EncPlan*>(ctx->enc_plan);
  if (P && P->v_off == hb.v_off && P->u_off == hb.u_off && P->p == hb.p && P->ld == hb.ld) {
    *out = P;
    return MI_OK;
  }
  delete P;
  ctx->enc_plan = nullptr;
  P = new EncPlan();
  P->v_off = hb.v_off;
  P->u_off = hb.u_off;
  P->p = hb.p;
  P->ld = hb.ld;
  std::vector<EncBlock> h(hb.B);
  for (int b = 0; b < hb.B; ++b)
    h[b] = EncBlock{hb.v_off[b], hb.u_off[b], hb.t_off[b], int(hb.v_off[b + 1] - hb.v_off[b]),
                    hb.p[b], hb.ld[b], 0};
  std::vector<int64_t> poff;
  proj_part_doubles(hb, &poff);
  std::vector<EncTile> tiles;
  for (int b = 0; b < hb.B; ++b) {
    P->max_ld = std::max(P->max_ld, hb.ld[b]);
    for (int r0 = 0; r0 < h[b].n; r0 += ENC_TILE) tiles.push_back(EncTile{b, r0});
  }
  P->n_tiles = (int)tiles.size();
  if (hipMalloc(&P->dev, hb.B * sizeof(EncBlock)) != hipSuccess ||
      hipMalloc(&P->dev_voff, (hb.B + 1) * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&P->dev_poff, hb.B * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&P->tiles, std::max<size_t>(tiles.size(), 1) * sizeof(EncTile)) != hipSuccess) {
    delete P;
    set_error("device allocation for the block table failed");
    return MI_ERR_HIP;
  }
  if (!tiles.empty())
    MI_TRY_HIP(hipMemcpy(P->tiles, tiles.data(), tiles.size() * sizeof(EncTile),
                         hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(P->dev, h.data(), hb.B * sizeof(EncBlock), hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(P->dev_voff, hb.v_off.data(), (hb.B + 1) * sizeof(int64_t),
                       hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(P->dev_poff, poff.data(), hb.B * sizeof(int64_t), hipMemcpyHostToDevice));
  ctx->enc_plan = P;
  *out = P;
  return MI_OK;
}

// E[k][:] = sum_i U[i][k] X[i][:] for k < c_b, 0 for c_b <= k < p_b.
// Stage 1: workgroup (b, chunk) sums the rows of one of PROJ_CHUNKS row
// ranges of block b into an FP64 partial (ld x 3); thread t owns the
// coefficients k = t, t + 256, ... (row reads of U coalesced), rows unrolled
// by 4 for memory-level parallelism.  Stage 2 adds the partials in chunk
// order, so the result does not depend on scheduling.
template <typename T>
__global__ void __launch_bounds__(256)
    k_project_part(const EncBlock* __restrict__ blks, const int64_t* __restrict__ poff,
                   const int32_t* __restrict__ cvec, const T* __restrict__ U,
                   const T* __restrict__ X, double* __restrict__ part) {
  constexpr int KPT = 4;  // ld <= 1024
  const EncBlock b = blks[blockIdx.x];
  const int chunk = blockIdx.y;
  const int c = min(max(cvec[blockIdx.x], 0), b.p);
  const int rows_per = (b.n + PROJ_CHUNKS - 1) / PROJ_CHUNKS;
  const int r0 = chunk * rows_per, r1 = min(b.n, r0 + rows_per);
  double acc[KPT][3];
#pragma unroll
  for (int s = 0; s < KPT; ++s) acc[s][0] = acc[s][1] = acc[s][2] = 0.0;
  const T* Ub = U + b.u_off;
  const T* Xb = X + 3 * b.v_off;
#pragma unroll 4
  for (int i = r0; i < r1; ++i) {
    const double x0 = (double)Xb[3 * i], x1 = (double)Xb[3 * i + 1], x2 = (double)Xb[3 * i + 2];
#pragma unroll
    for (int s = 0; s < KPT; ++s) {
      const int k = threadIdx.x + 256 * s;
      if (k < c) {
        const double u = (double)Ub[int64_t(i) * b.ld + k];
        acc[s][0] = fma(u, x0, acc[s][0]);
        acc[s][1] = fma(u, x1, acc[s][1]);
        acc[s][2] = fma(u, x2, acc[s][2]);
      }
    }
  }
  double* pb = part + poff[blockIdx.x] + int64_t(chunk) * b.ld * 3;
#pragma unroll
  for (int s = 0; s < KPT; ++s) {
    const int k = threadIdx.x + 256 * s;
    if (k < b.ld) {
      pb[3 * k] = acc[s][0];
      pb[3 * k + 1] = acc[s][1];
      pb[3 * k + 2] = acc[s][2];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_project_sum(const EncBlock* __restrict__ blks, const int64_t* __restrict__ poff,
                  const int32_t* __restrict__ cvec, const double* __restrict__ part,
                  T* __restrict__ E) {
  const EncBlock b = blks[blockIdx.x];
  const int c = min(max(cvec[blockIdx.x], 0), b.p);
  const double* pb = part + poff[blockIdx.x];
  for (int e = threadIdx.x; e < 3 * b.p; e += 256) {
    double v = 0.0;
    for (int ch = 0; ch < PROJ_CHUNKS; ++ch) v += pb[int64_t(ch) * b.ld * 3 + e];
    E[3 * b.t_off + e] = (e / 3 < c) ? (T)v : (T)0;
  }
}

// The same projection for ld <= 256 with every wavefront busy: the four
// wavefronts of a workgroup take every fourth row of the chunk, lanes the
// columns k = lane + 64 s; the wavefronts' sums meet in LDS and are added in
// wavefront order.
template <typename T>
__global__ void __launch_bounds__(256)
    k_project_part_w(const EncBlock* __restrict__ blks, const int64_t* __restrict__ poff,
                     const int32_t* __restrict__ cvec, const T* __restrict__ U,
                     const T* __restrict__ X, double* __restrict__ part) {
  __shared__ double red[4][64 * ENC_KPL][3];
  const EncBlock b = blks[blockIdx.x];
  const int chunk = blockIdx.y;
  const int c = min(max(cvec[blockIdx.x], 0), b.p);
  const int rows_per = (b.n + PROJ_CHUNKS - 1) / PROJ_CHUNKS;
  const int r0 = chunk * rows_per, r1 = min(b.n, r0 + rows_per);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[ENC_KPL][3];
#pragma unroll
  for (int s = 0; s < ENC_KPL; ++s) acc[s][0] = acc[s][1] = acc[s][2] = 0.0;
  const T* Ub = U + b.u_off;
  const T* Xb = X + 3 * b.v_off;
  // four rows of the wavefront per batch, every load unconditional (a row
  // past the chunk reads the first row with weight 0, a column past c reads
  // column 0 with weight 0), so that a batch's loads are in flight together
  for (int i0 = r0 + wv; i0 < r1; i0 += 16) {
    double x[4][3];
    T ur[4][ENC_KPL];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int i = i0 + 4 * h;
      const bool in = i < r1;
      const int ii = in ? i : r0;
#pragma unroll
      for (int q = 0; q < 3; ++q) x[h][q] = in ? (double)Xb[3 * ii + q] : 0.0;
#pragma unroll
      for (int s = 0; s < ENC_KPL; ++s) {
        const int k = lane + 64 * s;
        ur[h][s] = Ub[int64_t(ii) * b.ld + (k < c ? k : 0)];
      }
    }
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int s = 0; s < ENC_KPL; ++s) {
        const double u = lane + 64 * s < c ? (double)ur[h][s] : 0.0;
        acc[s][0] = fma(u, x[h][0], acc[s][0]);
        acc[s][1] = fma(u, x[h][1], acc[s][1]);
        acc[s][2] = fma(u, x[h][2], acc[s][2]);
      }
  }
#pragma unroll
  for (int s = 0; s < ENC_KPL; ++s) {
    const int k = lane + 64 * s;
    red[wv][k][0] = acc[s][0];
    red[wv][k][1] = acc[s][1];
    red[wv][k][2] = acc[s][2];
  }
  __syncthreads();
  double* pb = part + poff[blockIdx.x] + int64_t(chunk) * b.ld * 3;
  const int k = threadIdx.x;
  if (k < b.ld)
#pragma unroll
    for (int q = 0; q < 3; ++q) pb[3 * k + q] = ((red[0][k][q] + red[1][k][q]) + red[2][k][q]) + red[3][k][q];
}

// Reconstruction over 64-row tiles of one block (no block search per row):
// each lane keeps the coefficients of its columns k = lane + 64 s in
// registers for the tile's rows; the four wavefronts take every fourth row,
// a wave reduction per row.  ld <= 64 KPL.
template <typename T, int KPL>
__global__ void __launch_bounds__(256)
    k_reconstruct_t(const EncBlock* __restrict__ blks, const EncTile* __restrict__ tiles,
                    const int32_t* __restrict__ cvec, const T* __restrict__ U,
                    const T* __restrict__ E, T* __restrict__ Xr) {
  const EncTile t = tiles[blockIdx.x];
  const EncBlock b = blks[t.blk];
  const int c = min(max(cvec[t.blk], 0), b.p);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // coefficients of this lane's columns (unconditional loads, 0 past c)
  double e[KPL][3];
#pragma unroll
  for (int s = 0; s < KPL; ++s) {
    const int k = lane + 64 * s;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double v = (double)E[3 * (b.t_off + (k < c ? k : 0)) + q];
      e[s][q] = k < c ? v : 0.0;
    }
  }
  const int r1 = min(b.n, t.row0 + ENC_TILE);
  const T* Ub = U + b.u_off;
  // four rows of the wavefront per batch, loads unconditional (a row past
  // the tile reads the tile's first row and is not stored)
  for (int i0 = t.row0 + wv; i0 < r1; i0 += 16) {
    T ur[4][KPL];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int i = i0 + 4 * h < r1 ? i0 + 4 * h : t.row0;
#pragma unroll
      for (int s = 0; s < KPL; ++s) {
        const int k = lane + 64 * s;
        ur[h][s] = Ub[int64_t(i) * b.ld + (k < c ? k : 0)];  // e is 0 past c
      }
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int s = 0; s < KPL; ++s) {
        const double u = (double)ur[h][s];
        s0 = fma(u, e[s][0], s0);
        s1 = fma(u, e[s][1], s1);
        s2 = fma(u, e[s][2], s2);
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      const int i = i0 + 4 * h;
      if (lane == 0 && i < r1) {
        T* o = Xr + 3 * (b.v_off + i);
        o[0] = (T)s0;
        o[1] = (T)s1;
        o[2] = (T)s2;
      }
    }
  }
}

// Xr[i][:] = sum_{k < c_b} U[i][k] E[k][:]; one wavefront per vertex row
// (lanes stride the row, FP64 wave reduction).
template <typename T>
__global__ void __launch_bounds__(256)
    k_reconstruct(const EncBlock* __restrict__ blks, const int64_t* __restrict__ voff, int B,
                  int64_t N, const int32_t* __restrict__ cvec, const T* __restrict__ U,
                  const T* __restrict__ E, T* __restrict__ Xr) {
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  const int bi = find_block(voff, B, row);
  const EncBlock b = blks[bi];
  const int c = min(max(cvec[bi], 0), b.p);
  const int64_t i = row - b.v_off;
  const T* u = U + b.u_off + i * b.ld;
  const T* e = E + 3 * b.t_off;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = lane; k < c; k += 64) {
    const double uk = (double)u[k];
    s0 += uk * (double)e[3 * k];
    s1 += uk * (double)e[3 * k + 1];
    s2 += uk * (double)e[3 * k + 2];
  }
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
    s2 += __shfl_xor(s2, o, 64);
  }
  if (lane == 0) {
    Xr[3 * row] = (T)s0;
    Xr[3 * row + 1] = (T)s1;
    Xr[3 * row + 2] = (T)s2;
  }
}

}  // namespace mis

using namespace mis;

// ------------------------------------------------------------------ allocation-free projection
// mi_project_noalloc keeps what mi_project puts in the context's plan (the
// block table) and in the caller's workspace (the FP64 partial sums) in this
// fixed array instead.  Host code never passes the array's name to a kernel
// (in host code it is only a stand-in for the symbol): every use goes
// through the device address looked up for the current device.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;  // 16 MiB per device
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on device dev, looked up once per device with
// that device current (each device holds its own copy of the array).
mi_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    set_error("device %d outside the %d devices the fixed scratch tracks", dev,
              NOALLOC_MAX_DEVICES);
    return MI_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    MI_TRY_HIP(hipSetDevice(dev));
    void* ptr = nullptr;
    MI_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      set_error("hipGetSymbolAddress returned a null address for the fixed scratch");
      return MI_ERR_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MI_OK;
}

// A host table reaches device memory through kernel arguments, STAGE_BYTES at
// a time: the runtime copies the arguments, so nothing is allocated and the
// host copy need not outlive the call.
constexpr int STAGE_BYTES = 2048;
struct StageChunk {
  unsigned char b[STAGE_BYTES];
};

__global__ void __launch_bounds__(256) k_stage(StageChunk ch, int n, unsigned char* __restrict__ dst) {
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = ch.b[i];
}

}  // namespace

extern "C" {

mi_status mi_encdec_workspace_size(mi_ctx* ctx, const mi_blocks* blk, int32_t precision,
                                   size_t* ws_bytes) {
  clear_error();
  MI_CHECK_ARG(ws_bytes != nullptr, "ws_bytes is NULL");
  (void)ctx;
  MI_CHECK_ARG(precision == MI_FP32 || precision == MI_FP64, "precision %d unsupported", precision);
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  *ws_bytes = size_t(proj_part_doubles(hb, nullptr)) * sizeof(double);
  return MI_OK;
}

mi_status mi_project(mi_ctx* ctx, const mi_blocks* blk, int32_t precision, const int32_t* c,
                     const void* U, const void* X, void* E, void* ws, size_t ws_bytes,
                     void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && c && U && X && E, "NULL argument");
  MI_CHECK_ARG(precision == MI_FP32 || precision == MI_FP64, "precision %d unsupported", precision);
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  const size_t need = size_t(proj_part_doubles(hb, nullptr)) * sizeof(double);
  if (!ws || ws_bytes < need) {
    set_error("workspace %zu bytes < %zu required", ws_bytes, need);
    return MI_ERR_WORKSPACE;
  }
  for (int b = 0; b < hb.B; ++b)
    MI_CHECK_ARG(hb.ld[b] <= 1024, "block %d: ld %d > 1024", b, hb.ld[b]);
  MI_TRY_HIP(hipSetDevice(ctx->device));
  EncPlan* P = nullptr;
  st = enc_plan(ctx, hb, &P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  double* part = static_cast<double*>(ws);
  KClose kc_(ctx->timer);
  KScope k_(ctx->timer, MI_K_PROJECT, s);
  const bool tiled = P->max_ld <= 64 * ENC_KPL;
  if (precision == MI_FP64) {
    if (tiled)
      hipLaunchKernelGGL(k_project_part_w<double>, dim3(hb.B, PROJ_CHUNKS), dim3(256), 0, s,
                         P->dev, P->dev_poff, c, (const double*)U, (const double*)X, part);
    else
      hipLaunchKernelGGL(k_project_part<double>, dim3(hb.B, PROJ_CHUNKS), dim3(256), 0, s, P->dev,
                         P->dev_poff, c, (const double*)U, (const double*)X, part);
    hipLaunchKernelGGL(k_project_sum<double>, dim3(hb.B), dim3(256), 0, s, P->dev, P->dev_poff, c,
                       part, (double*)E);
  } else {
    if (tiled)
      hipLaunchKernelGGL(k_project_part_w<float>, dim3(hb.B, PROJ_CHUNKS), dim3(256), 0, s,
                         P->dev, P->dev_poff, c, (const float*)U, (const float*)X, part);
    else
      hipLaunchKernelGGL(k_project_part<float>, dim3(hb.B, PROJ_CHUNKS), dim3(256), 0, s, P->dev,
                         P->dev_poff, c, (const float*)U, (const float*)X, part);
    hipLaunchKernelGGL(k_project_sum<float>, dim3(hb.B), dim3(256), 0, s, P->dev, P->dev_poff, c,
                       part, (float*)E);
  }
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

mi_status mi_reconstruct(mi_ctx* ctx, const mi_blocks* blk, int32_t precision, const int32_t* c,
                         const void* U, const void* E, void* Xr, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && c && U && E && Xr, "NULL argument");
  MI_CHECK_ARG(precision == MI_FP32 || precision == MI_FP64, "precision %d unsupported", precision);
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  MI_TRY_HIP(hipSetDevice(ctx->device));
  EncPlan* P = nullptr;
  st = enc_plan(ctx, hb, &P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = hb.v_off[hb.B];
  const int grid = ceil_div(N, 4);
  KClose kc_(ctx->timer);
  KScope k_(ctx->timer, MI_K_RECONSTRUCT, s);
  // the tiled kernel keeps 4 (ld <= 256) or 5 (ld <= 320) columns per lane
  const bool tiled = P->max_ld <= 64 * (ENC_KPL + 1);
  const bool k4 = P->max_ld <= 64 * ENC_KPL;
  if (tiled && P->n_tiles > 0) {
    if (precision == MI_FP64) {
      if (k4)
        hipLaunchKernelGGL((k_reconstruct_t<double, ENC_KPL>), dim3(P->n_tiles), dim3(256), 0, s,
                           P->dev, P->tiles, c, (const double*)U, (const double*)E, (double*)Xr);
      else
        hipLaunchKernelGGL((k_reconstruct_t<double, ENC_KPL + 1>), dim3(P->n_tiles), dim3(256), 0,
                           s, P->dev, P->tiles, c, (const double*)U, (const double*)E,
                           (double*)Xr);
    } else {
      if (k4)
        hipLaunchKernelGGL((k_reconstruct_t<float, ENC_KPL>), dim3(P->n_tiles), dim3(256), 0, s,
                           P->dev, P->tiles, c, (const float*)U, (const float*)E, (float*)Xr);
      else
        hipLaunchKernelGGL((k_reconstruct_t<float, ENC_KPL + 1>), dim3(P->n_tiles), dim3(256), 0,
                           s, P->dev, P->tiles, c, (const float*)U, (const float*)E, (float*)Xr);
    }
  } else if (!tiled) {
    if (precision == MI_FP64)
      hipLaunchKernelGGL(k_reconstruct<double>, dim3(grid), dim3(256), 0, s, P->dev, P->dev_voff,
                         hb.B, N, c, (const double*)U, (const double*)E, (double*)Xr);
    else
      hipLaunchKernelGGL(k_reconstruct<float>, dim3(grid), dim3(256), 0, s, P->dev, P->dev_voff,
                         hb.B, N, c, (const float*)U, (const float*)E, (float*)Xr);
  }
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

mi_status mi_project_noalloc(mi_ctx* ctx, const mi_blocks* blk, int32_t precision,
                             const int32_t* c, const void* U, const void* X, void* E,
                             void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && c && U && X && E, "NULL argument");
  MI_CHECK_ARG(precision == MI_FP32 || precision == MI_FP64, "precision %d unsupported", precision);
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  for (int b = 0; b < hb.B; ++b)
    MI_CHECK_ARG(hb.ld[b] <= 1024, "block %d: ld %d > 1024", b, hb.ld[b]);
  // scratch layout: block table | partial offsets | FP64 partials
  std::vector<int64_t> poff;
  const int64_t nparts = proj_part_doubles(hb, &poff);
  const size_t tab_bytes = size_t(hb.B) * sizeof(EncBlock);
  const size_t poff_at = align_up(tab_bytes);
  const size_t part_at = align_up(poff_at + size_t(hb.B) * sizeof(int64_t));
  const size_t need = part_at + size_t(nparts) * sizeof(double);
  if (need > NOALLOC_SCRATCH_BYTES) {
    set_error("the projection needs %zu bytes of scratch; the fixed scratch holds %zu "
              "(use mi_project with a workspace)", need, NOALLOC_SCRATCH_BYTES);
    return MI_ERR_WORKSPACE;
  }
  MI_TRY_HIP(hipSetDevice(ctx->device));
  void* base = nullptr;
  st = scratch_address(ctx->device, &base);
  if (st) return st;
  std::vector<unsigned char> host(part_at, 0);
  int max_ld = 0;
  for (int b = 0; b < hb.B; ++b) {
    const EncBlock e{hb.v_off[b], hb.u_off[b], hb.t_off[b], int(hb.v_off[b + 1] - hb.v_off[b]),
                     hb.p[b], hb.ld[b], 0};
    std::memcpy(host.data() + size_t(b) * sizeof(EncBlock), &e, sizeof(EncBlock));
    max_ld = std::max(max_ld, hb.ld[b]);
  }
  if (hb.B > 0) std::memcpy(host.data() + poff_at, poff.data(), size_t(hb.B) * sizeof(int64_t));
  hipStream_t s = (hipStream_t)stream;
  unsigned char* dbase = static_cast<unsigned char*>(base);
  for (size_t o = 0; o < host.size(); o += STAGE_BYTES) {
    StageChunk ch;
    const int n = int(std::min<size_t>(STAGE_BYTES, host.size() - o));
    std::memcpy(ch.b, host.data() + o, size_t(n));
    hipLaunchKernelGGL(k_stage, dim3(1), dim3(256), 0, s, ch, n, dbase + o);
  }
  const EncBlock* dev = reinterpret_cast<const EncBlock*>(dbase);
  const int64_t* dpoff = reinterpret_cast<const int64_t*>(dbase + poff_at);
  double* part = reinterpret_cast<double*>(dbase + part_at);
  const bool tiled = max_ld <= 64 * ENC_KPL;
  if (hb.B > 0) {
    if (precision == MI_FP64) {
      if (tiled)
        hipLaunchKernelGGL(k_project_part_w<double>, dim3(hb.B, PROJ_CHUNKS), dim3(256), 0, s,
                           dev, dpoff, c, (const double*)U, (const double*)X, part);
      else
        hipLaunchKernelGGL(k_project_part<double>, dim3(hb.B, PROJ_CHUNKS), dim3(256), 0, s, dev,
                           dpoff, c, (const double*)U, (const double*)X, part);
      hipLaunchKernelGGL(k_project_sum<double>, dim3(hb.B), dim3(256), 0, s, dev, dpoff, c, part,
                         (double*)E);
    } else {
      if (tiled)
        hipLaunchKernelGGL(k_project_part_w<float>, dim3(hb.B, PROJ_CHUNKS), dim3(256), 0, s,
                           dev, dpoff, c, (const float*)U, (const float*)X, part);
      else
        hipLaunchKernelGGL(k_project_part<float>, dim3(hb.B, PROJ_CHUNKS), dim3(256), 0, s, dev,
                           dpoff, c, (const float*)U, (const float*)X, part);
      hipLaunchKernelGGL(k_project_sum<float>, dim3(hb.B), dim3(256), 0, s, dev, dpoff, c, part,
                         (float*)E);
    }
  }
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

void mis_destroy_enc_plan(mi_ctx* ctx) {
  delete static_cast<EncPlan*>(ctx->enc_plan);
  ctx->enc_plan = nullptr;
}

}  // extern "C"
