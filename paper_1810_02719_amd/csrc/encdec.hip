// Graph Fourier transform of the coordinates onto the tracked subspace and
// back (Section 3: v_bar = U^T v, v = U v_bar; Section 7.1: E = U_c^T v,
// v~ = U_c E), with truncation to the first c_b coefficients.
//
// Both kernels are bound by HBM traffic (one read of U, 4 c_b bytes per
// vertex row); sums run in FP64 and in a fixed order, so results are
// bitwise reproducible.
#include <cstring>

#include "common.hpp"
#include "kernels_util.hpp"

namespace mis {

struct EncBlock {
  int64_t v_off, u_off, t_off;
  int32_t n, p, ld, pad;
};

struct EncPlan {
  std::vector<int64_t> v_off, u_off;
  std::vector<int32_t> p, ld;
  EncBlock* dev = nullptr;
  int64_t* dev_voff = nullptr;
  ~EncPlan() {
    if (dev) (void)hipFree(dev);
    if (dev_voff) (void)hipFree(dev_voff);
  }
};

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
  if (hipMalloc(&P->dev, hb.B * sizeof(EncBlock)) != hipSuccess ||
      hipMalloc(&P->dev_voff, (hb.B + 1) * sizeof(int64_t)) != hipSuccess) {
    delete P;
    set_error("device allocation for the block table failed");
    return MI_ERR_HIP;
  }
  MI_TRY_HIP(hipMemcpy(P->dev, h.data(), hb.B * sizeof(EncBlock), hipMemcpyHostToDevice));
  MI_TRY_HIP(hipMemcpy(P->dev_voff, hb.v_off.data(), (hb.B + 1) * sizeof(int64_t),
                       hipMemcpyHostToDevice));
  ctx->enc_plan = P;
  *out = P;
  return MI_OK;
}

// E[k][:] = sum_i U[i][k] X[i][:] for k < c_b, 0 for c_b <= k < p_b.
// One workgroup per block; thread t owns coefficients k = t, t + 256, ...
// (row reads of U are coalesced across the workgroup).
template <typename T>
__global__ void __launch_bounds__(256)
    k_project(const EncBlock* __restrict__ blks, const int32_t* __restrict__ cvec,
              const T* __restrict__ U, const T* __restrict__ X, T* __restrict__ E) {
  constexpr int KPT = 4;  // ld <= 1024
  const EncBlock b = blks[blockIdx.x];
  const int c = min(max(cvec[blockIdx.x], 0), b.p);
  double acc[KPT][3];
#pragma unroll
  for (int s = 0; s < KPT; ++s) acc[s][0] = acc[s][1] = acc[s][2] = 0.0;
  const T* Ub = U + b.u_off;
  const T* Xb = X + 3 * b.v_off;
  for (int i = 0; i < b.n; ++i) {
    const double x0 = (double)Xb[3 * i], x1 = (double)Xb[3 * i + 1], x2 = (double)Xb[3 * i + 2];
#pragma unroll
    for (int s = 0; s < KPT; ++s) {
      const int k = threadIdx.x + 256 * s;
      if (k < c) {
        const double u = (double)Ub[int64_t(i) * b.ld + k];
        acc[s][0] += u * x0;
        acc[s][1] += u * x1;
        acc[s][2] += u * x2;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < KPT; ++s) {
    const int k = threadIdx.x + 256 * s;
    if (k < b.p) {
      T* e = E + 3 * (b.t_off + k);
      const bool keep = k < c;
      e[0] = keep ? (T)acc[s][0] : (T)0;
      e[1] = keep ? (T)acc[s][1] : (T)0;
      e[2] = keep ? (T)acc[s][2] : (T)0;
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
  *ws_bytes = 0;
  return MI_OK;
}

mi_status mi_project(mi_ctx* ctx, const mi_blocks* blk, int32_t precision, const int32_t* c,
                     const void* U, const void* X, void* E, void* ws, size_t ws_bytes,
                     void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && c && U && X && E, "NULL argument");
  MI_CHECK_ARG(precision == MI_FP32 || precision == MI_FP64, "precision %d unsupported", precision);
  (void)ws;
  (void)ws_bytes;
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);
  if (st) return st;
  MI_TRY_HIP(hipSetDevice(ctx->device));
  EncPlan* P = nullptr;
  st = enc_plan(ctx, hb, &P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  KScope k_(ctx->timer, MI_K_PROJECT, s);
  if (precision == MI_FP64)
    hipLaunchKernelGGL(k_project<double>, dim3(hb.B), dim3(256), 0, s, P->dev, c,
                       (const double*)U, (const double*)X, (double*)E);
  else
    hipLaunchKernelGGL(k_project<float>, dim3(hb.B), dim3(256), 0, s, P->dev, c, (const float*)U,
                       (const float*)X, (float*)E);
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
  KScope k_(ctx->timer, MI_K_RECONSTRUCT, s);
  if (precision == MI_FP64)
    hipLaunchKernelGGL(k_reconstruct<double>, dim3(grid), dim3(256), 0, s, P->dev, P->dev_voff, hb.B,
                       N, c, (const double*)U, (const double*)E, (double*)Xr);
  else
    hipLaunchKernelGGL(k_reconstruct<float>, dim3(grid), dim3(256), 0, s, P->dev, P->dev_voff, hb.B,
                       N, c, (const float*)U, (const float*)E, (float*)Xr);
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

void mis_destroy_enc_plan(mi_ctx* ctx) {
  delete static_cast<EncPlan*>(ctx->enc_plan);
  ctx->enc_plan = nullptr;
}

}  // extern "C"
