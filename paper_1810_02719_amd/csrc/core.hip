// Context, error reporting, block-table validation and a device-wide
// exclusive scan used by the Laplacian builder.
#include "common.hpp"
#include "dense.hpp"
#include "kernels_util.hpp"

namespace mis {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

void clear_error() { g_err.clear(); }

mi_status load_blocks(const mi_blocks* blk, HostBlocks* hb, bool need_slab) {
  MI_CHECK_ARG(blk != nullptr, "block table is NULL");
  MI_CHECK_ARG(blk->n_blocks >= 1, "n_blocks must be >= 1 (got %d)", blk->n_blocks);
  MI_CHECK_ARG(blk->v_off != nullptr, "v_off is NULL");
  const int B = blk->n_blocks;
  hb->B = B;
  hb->v_off.assign(blk->v_off, blk->v_off + B + 1);
  MI_CHECK_ARG(hb->v_off[0] == 0, "v_off[0] must be 0");
  for (int b = 0; b < B; ++b) {
    int64_t n = hb->v_off[b + 1] - hb->v_off[b];
    MI_CHECK_ARG(n >= 1 && n < (int64_t(1) << 31), "block %d has %lld vertices", b, (long long)n);
  }
  hb->pred.assign(B, -1);
  if (blk->pred) {
    for (int b = 0; b < B; ++b) {
      hb->pred[b] = blk->pred[b];
      MI_CHECK_ARG(blk->pred[b] >= -1 && blk->pred[b] < B && blk->pred[b] != b,
                   "pred[%d] = %d invalid", b, blk->pred[b]);
    }
  }
  if (!need_slab) return MI_OK;
  MI_CHECK_ARG(blk->p && blk->ld && blk->u_off, "p, ld and u_off are required");
  hb->p.assign(blk->p, blk->p + B);
  hb->ld.assign(blk->ld, blk->ld + B);
  hb->u_off.assign(blk->u_off, blk->u_off + B + 1);
  hb->t_off.assign(B + 1, 0);
  hb->m_off.assign(B + 1, 0);
  MI_CHECK_ARG(hb->u_off[0] == 0, "u_off[0] must be 0");
  for (int b = 0; b < B; ++b) {
    int64_t n = hb->v_off[b + 1] - hb->v_off[b];
    if (hb->p[b] < 1 || hb->p[b] > n) {
      set_error("block %d: p = %d outside [1, n = %lld]", b, hb->p[b], (long long)n);
      return MI_ERR_CAPACITY;
    }
    if (hb->ld[b] < hb->p[b] || hb->ld[b] % 32 != 0 || hb->ld[b] > 1024) {
      set_error("block %d: ld = %d must be a multiple of 32 in [p, 1024]", b, hb->ld[b]);
      return MI_ERR_CAPACITY;
    }
    MI_CHECK_ARG(hb->u_off[b + 1] - hb->u_off[b] == n * hb->ld[b],
                 "block %d: u_off step %lld != n*ld = %lld", b,
                 (long long)(hb->u_off[b + 1] - hb->u_off[b]), (long long)(n * hb->ld[b]));
    hb->t_off[b + 1] = hb->t_off[b] + hb->p[b];
    hb->m_off[b + 1] = hb->m_off[b] + int64_t(hb->ld[b]) * hb->ld[b];
  }
  hb->c = hb->p;
  if (blk->c) {
    for (int b = 0; b < B; ++b) {
      if (blk->c[b] < 1 || blk->c[b] > hb->p[b]) {
        set_error("block %d: c = %d outside [1, p = %d]", b, blk->c[b], hb->p[b]);
        return MI_ERR_CAPACITY;
      }
      hb->c[b] = blk->c[b];
    }
  }
  return MI_OK;
}

// ---------------------------------------------------------------- scan

// Exclusive scan of int32 counts into int64 offsets, out[N] = total.
// Pass 1: each workgroup scans SCAN_TILE elements and emits its total.
__global__ void __launch_bounds__(256) k_scan_tiles(const int32_t* __restrict__ in,
                                                    int64_t* __restrict__ out,
                                                    int64_t* __restrict__ sums, int64_t N) {
  __shared__ int64_t sh[256];
  const int64_t base = int64_t(blockIdx.x) * SCAN_TILE;
  const int t = threadIdx.x;
  int64_t loc[SCAN_PER_THREAD];
  int64_t acc = 0;
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    int64_t i = base + int64_t(t) * SCAN_PER_THREAD + k;
    int64_t v = (i < N) ? in[i] : 0;
    loc[k] = acc;
    acc += v;
  }
  sh[t] = acc;
  __syncthreads();
  // Hillis-Steele over the 256 thread totals
  for (int s = 1; s < 256; s <<= 1) {
    int64_t add = (t >= s) ? sh[t - s] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t excl = sh[t] - acc;
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    int64_t i = base + int64_t(t) * SCAN_PER_THREAD + k;
    if (i < N) out[i] = loc[k] + excl;
  }
  if (t == 255) sums[blockIdx.x] = sh[255];
}

// Pass 2: one workgroup turns the tile totals into exclusive tile offsets.
__global__ void __launch_bounds__(256) k_scan_sums(int64_t* __restrict__ sums, int64_t ntiles,
                                                   int64_t* __restrict__ total) {
  __shared__ int64_t sh[256];
  const int t = threadIdx.x;
  int64_t carry = 0;
  for (int64_t base = 0; base < ntiles; base += 256) {
    int64_t i = base + t;
    int64_t v = (i < ntiles) ? sums[i] : 0;
    sh[t] = v;
    __syncthreads();
    for (int s = 1; s < 256; s <<= 1) {
      int64_t add = (t >= s) ? sh[t - s] : 0;
      __syncthreads();
      sh[t] += add;
      __syncthreads();
    }
    if (i < ntiles) sums[i] = carry + sh[t] - v;
    int64_t tot = sh[255];
    __syncthreads();
    carry += tot;
  }
  if (t == 0) *total = carry;
}

// Pass 3: add the tile offsets.
__global__ void __launch_bounds__(256) k_scan_add(int64_t* __restrict__ out,
                                                  const int64_t* __restrict__ sums,
                                                  const int64_t* __restrict__ total, int64_t N) {
  const int64_t base = int64_t(blockIdx.x) * SCAN_TILE;
  const int64_t add = sums[blockIdx.x];
  for (int k = threadIdx.x; k < SCAN_TILE; k += 256) {
    int64_t i = base + k;
    if (i < N) out[i] += add;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[N] = *total;
}

size_t scan_scratch_bytes(int64_t N) { return (size_t(ceil_div(N, SCAN_TILE)) + 2) * sizeof(int64_t); }

void exclusive_scan(const int32_t* in, int64_t* out, int64_t N, int64_t* scratch, hipStream_t s) {
  int64_t ntiles = ceil_div(N, SCAN_TILE);
  if (ntiles == 0) ntiles = 1;
  int64_t* sums = scratch;
  int64_t* total = scratch + ntiles;
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, in, out, sums, N);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, ntiles, total);
  hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(256), 0, s, out, sums, total, N);
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int g = (int)std::min<int64_t>(ceil_div(n, 256), 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3(g), dim3(256), 0, s, p, v, n);
}

__global__ void k_fill_f64(double* p, double v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

void fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int g = (int)std::min<int64_t>(ceil_div(n, 256), 4096);
  hipLaunchKernelGGL(k_fill_f64, dim3(g), dim3(256), 0, s, p, v, n);
}

mi_status KTimer::collect() {
  close();
  for (const Rec& r : pending) {
    float t = 0.f;
    MI_TRY_HIP(hipEventSynchronize(r.b));
    MI_TRY_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.k] += t;
    n[r.k] += r.cnt;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
  return MI_OK;
}

KTimer::~KTimer() {
  close();
  for (const Rec& r : pending) {
    (void)hipEventSynchronize(r.b);
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

}  // namespace mis

extern "C" {

const char* mi_last_error(void) { return mis::g_err.c_str(); }

const char* mi_version(void) { return "mispectral 0.1 (gfx950)"; }

mi_status mi_ctx_create(mi_ctx** out, int32_t device) {
  mis::clear_error();
  MI_CHECK_ARG(out != nullptr, "out is NULL");
  int count = 0;
  MI_TRY_HIP(hipGetDeviceCount(&count));
  MI_CHECK_ARG(device >= 0 && device < count, "device %d not present (%d devices)", device, count);
  MI_TRY_HIP(hipSetDevice(device));
  mi_ctx* c = new mi_ctx();
  c->device = device;
  *out = c;
  return MI_OK;
}

void mis_destroy_oi_plan(mi_ctx* ctx);
void mis_destroy_enc_plan(mi_ctx* ctx);
void mis_destroy_cc_plan(mi_ctx* ctx);
void mis_destroy_res_plan(mi_ctx* ctx);
void mis_destroy_adj_plan(mi_ctx* ctx);
void mis_destroy_merge_plan(mi_ctx* ctx);
void mis_destroy_codec_plan(mi_ctx* ctx);
void mis_destroy_quality_plan(mi_ctx* ctx);

mi_status mi_ctx_destroy(mi_ctx* ctx) {
  mis::clear_error();
  if (!ctx) return MI_OK;
  mis_destroy_oi_plan(ctx);
  mis_destroy_enc_plan(ctx);
  mis_destroy_cc_plan(ctx);
  mis_destroy_res_plan(ctx);
  mis_destroy_adj_plan(ctx);
  mis_destroy_merge_plan(ctx);
  mis_destroy_codec_plan(ctx);
  mis_destroy_quality_plan(ctx);
  delete ctx->timer;
  delete ctx;
  return MI_OK;
}

static const char* const k_class_names[MI_K_COUNT] = {
    "spmm",        "gram",       "gram_small", "gram_reduce",  "chol",      "rowmul",
    "rowmul_small", "rq_max",    "jacobi_init", "jacobi_sweep", "apply_rot", "rr_finish",
    "perm_cast",   "setup",      "project",    "reconstruct",  "eig_reduce", "eig_values",
    "eig_vectors", "eig_back",   "merge",      "quantize",
    "quality",     "doi",        "cg",         "cheb_pass"};

const char* mi_kernel_class_name(int32_t k) {
  return (k >= 0 && k < MI_K_COUNT) ? k_class_names[k] : nullptr;
}

mi_status mi_ctx_set_timing(mi_ctx* ctx, int32_t on) {
  mis::clear_error();
  MI_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  MI_TRY_HIP(hipSetDevice(ctx->device));
  delete ctx->timer;
  ctx->timer = on ? new mis::KTimer() : nullptr;
  return MI_OK;
}

mi_status mi_oi_force_spmm(mi_ctx* ctx, int32_t variant) {
  mis::clear_error();
  MI_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  MI_CHECK_ARG(variant >= -1 && variant < mis::SPMM_NVAR, "SpMM variant %d unknown", variant);
  ctx->spmm_force = variant;
  return MI_OK;
}

mi_status mi_ctx_kernel_times(mi_ctx* ctx, double* total_ms, int64_t* launches) {
  mis::clear_error();
  MI_CHECK_ARG(ctx != nullptr && total_ms != nullptr && launches != nullptr, "NULL argument");
  MI_CHECK_ARG(ctx->timer != nullptr, "timing is off");
  MI_TRY_HIP(hipSetDevice(ctx->device));
  mi_status st = ctx->timer->collect();
  if (st) return st;
  for (int k = 0; k < MI_K_COUNT; ++k) {
    total_ms[k] = ctx->timer->ms[k];
    launches[k] = ctx->timer->n[k];
  }
  return MI_OK;
}

}  // extern "C"
