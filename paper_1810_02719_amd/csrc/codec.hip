// Uniform quantisation of the feature vectors (Section 8: the coefficients
// E = U_c^T v of every block are quantised with q_c bits, 12 in the paper's
// experiments).  One workgroup per block: the range of each coordinate axis
// over the block's first c_b coefficients (min / max, exact in any order),
// then one code per coefficient.  Every floating-point operation is rounded
// on its own (no contraction), so codes and dequantised values are
// reproducible bit for bit.
#include <cmath>
#include <memory>

#include "common.hpp"
#include "kernels_util.hpp"

namespace mis {

constexpr int QUANT_THREADS = 256;

__global__ void __launch_bounds__(QUANT_THREADS)
    k_quantize(const int64_t* __restrict__ t_off, const int32_t* __restrict__ p,
               const int32_t* __restrict__ c, int qbits, const float* __restrict__ E,
               uint16_t* __restrict__ codes, float* __restrict__ params, float* __restrict__ Eq) {
  __shared__ float red[2][3][QUANT_THREADS / 64];
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t t0 = t_off[b];
  const int pb = p[b], cb = min(max(c[b], 0), pb);
  float lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
  }
  for (int j = tid; j < cb; j += QUANT_THREADS)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float e = E[3 * (t0 + j) + k];
      lo[k] = fminf(lo[k], e);
      hi[k] = fmaxf(hi[k], e);
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    for (int o = 32; o > 0; o >>= 1) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], o, 64));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o, 64));
    }
    if (lane == 0) {
      red[0][k][wv] = lo[k];
      red[1][k][wv] = hi[k];
    }
  }
  __syncthreads();
  const float levels = float((1u << qbits) - 1u);
  float base[3], step[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float l = red[0][k][0], h = red[1][k][0];
    for (int w = 1; w < QUANT_THREADS / 64; ++w) {
      l = fminf(l, red[0][k][w]);
      h = fmaxf(h, red[1][k][w]);
    }
    if (cb == 0) l = h = 0.0f;
    base[k] = l;
    step[k] = __fdiv_rn(__fsub_rn(h, l), levels);
  }
  if (tid == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      params[6 * int64_t(b) + 2 * k] = base[k];
      params[6 * int64_t(b) + 2 * k + 1] = step[k];
    }
  for (int j = tid; j < pb; j += QUANT_THREADS)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int64_t i = 3 * (t0 + j) + k;
      float q = 0.0f;
      if (j < cb && step[k] > 0.0f) {
        q = rintf(__fdiv_rn(__fsub_rn(E[i], base[k]), step[k]));  // ties to even
        q = fminf(fmaxf(q, 0.0f), levels);
      }
      codes[i] = uint16_t(q);
      // lo + code * step rounded twice: the opaque copy of the product keeps
      // the compiler from fusing it into a multiply-add
      float prod = q * step[k];
      asm volatile("" : "+v"(prod));
      if (Eq) Eq[i] = j < cb ? base[k] + prod : 0.0f;
    }
}

struct CodecPlan {
  std::vector<int64_t> t_off;
  std::vector<int32_t> p;
  int64_t* dev_toff = nullptr;
  int32_t* dev_p = nullptr;
  ~CodecPlan() {
    if (dev_toff) (void)hipFree(dev_toff);
    if (dev_p) (void)hipFree(dev_p);
  }
};

}  // namespace mis

using namespace mis;

extern "C" {

void mis_destroy_codec_plan(mi_ctx* ctx) {
  delete static_cast<CodecPlan*>(ctx->codec_plan);
  ctx->codec_plan = nullptr;
}

mi_status mi_quantize(mi_ctx* ctx, const mi_blocks* blk, const int32_t* c, int32_t qbits,
                      const float* E, uint16_t* codes, float* params, float* Eq, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && c && E && codes && params, "NULL argument");
  MI_CHECK_ARG(qbits >= 1 && qbits <= 16, "qbits %d outside [1, 16]", qbits);
  HostBlocks hb;
  mi_status st = load_blocks(blk, &hb, true);  // p and t_off
  if (st) return st;
  MI_TRY_HIP(hipSetDevice(ctx->device));
  CodecPlan* P = static_cast<CodecPlan*>(ctx->codec_plan);
  if (!P || P->t_off != hb.t_off || P->p != hb.p) {
    delete P;
    ctx->codec_plan = nullptr;
    std::unique_ptr<CodecPlan> np(new CodecPlan());
    np->t_off = hb.t_off;
    np->p = hb.p;
    MI_TRY_HIP(hipMalloc(&np->dev_toff, (hb.B + 1) * sizeof(int64_t)));
    MI_TRY_HIP(hipMalloc(&np->dev_p, std::max(hb.B, 1) * sizeof(int32_t)));
    MI_TRY_HIP(hipMemcpy(np->dev_toff, hb.t_off.data(), (hb.B + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice));
    if (hb.B > 0)
      MI_TRY_HIP(hipMemcpy(np->dev_p, hb.p.data(), hb.B * sizeof(int32_t), hipMemcpyHostToDevice));
    P = np.release();
    ctx->codec_plan = P;
  }
  if (hb.B == 0) return MI_OK;
  hipStream_t s = (hipStream_t)stream;
  KClose kc_(ctx->timer);
  KScope k_(ctx->timer, MI_K_QUANTIZE, s);
  hipLaunchKernelGGL(k_quantize, dim3(hb.B), dim3(QUANT_THREADS), 0, s, P->dev_toff, P->dev_p, c,
                     qbits, E, codes, params, Eq);
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

}  // extern "C"
