// Internal helpers shared by the library's translation units: status and
// error reporting, the device-side block descriptor, launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mispectral.h"

namespace mis {

// Thread-local message of the last error (mi_last_error).
void set_error(const char* fmt, ...);
void clear_error();

// Entry of a call that enqueues GPU work: clears the thread's message and any
// stale HIP error left by earlier, unrelated calls.
inline void begin_call() {
  clear_error();
  (void)hipGetLastError();
}

#define MI_TRY_HIP(expr)                                                              \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) {                                                           \
      ::mis::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                       __LINE__);                                                     \
      return MI_ERR_HIP;                                                              \
    }                                                                                 \
  } while (0)

#define MI_CHECK_ARG(cond, ...)      \
  do {                               \
    if (!(cond)) {                   \
      ::mis::set_error(__VA_ARGS__); \
      return MI_ERR_ARG;             \
    }                                \
  } while (0)

// Device view of one block.
struct BlockDev {
  int64_t v_off;   // first vertex row
  int64_t u_off;   // first element of the slab
  int64_t nnz_off; // first CSR entry
  int64_t t_off;   // offset of per-block p-vectors (ritz values): sum of p
  int64_t m_off;   // offset of per-block ld x ld matrices: sum of ld*ld
  int32_t n;       // vertices
  int32_t p;       // tracked width
  int32_t ld;      // slab row stride
  int32_t id;      // block index in the caller's table
};

// Host-side validated copy of an mi_blocks table.
struct HostBlocks {
  int32_t B = 0;
  std::vector<int64_t> v_off, u_off;
  std::vector<int32_t> p, ld, pred;
  std::vector<int32_t> c;             // kept pairs of the tolerance test (p when not given)
  std::vector<int64_t> t_off, m_off;  // derived
};

mi_status load_blocks(const mi_blocks* blk, HostBlocks* hb, bool need_slab);

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Round-robin (circle method) pairing used by the parallel Jacobi sweeps:
// in round r of a sweep over q (even) indices, slot k pairs the indices at
// positions k and q-1-k of the arrangement where position 0 is fixed and the
// others rotate by r.
__host__ __device__ inline int rr_index(int pos, int r, int q) {
  if (pos == 0) return 0;
  return 1 + ((pos - 1 + r) % (q - 1));
}

// Event timer of the kernel classes (mi_ctx_set_timing): consecutive
// launches of one class on one stream form a group bracketed by two events
// on that stream (a pair per launch would add the event overhead, about
// 2 us, to every launch); the elapsed times and launch counts are summed per
// class when they are read.  Every timed entry point closes its last group
// before it returns.
struct KTimer {
  struct Rec {
    int k, cnt;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double ms[MI_K_COUNT] = {};
  int64_t n[MI_K_COUNT] = {};
  int open_k = -1, open_n = 0;
  hipEvent_t open_a = nullptr;
  hipStream_t open_s = nullptr;
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  void begin(int k, hipStream_t s) {
    if (open_a && k == open_k && s == open_s) {
      ++open_n;
      return;
    }
    close();
    open_k = k;
    open_s = s;
    open_n = 1;
    open_a = take();
    if (open_a) (void)hipEventRecord(open_a, s);
  }
  void close() {
    if (!open_a) return;
    hipEvent_t b = take();
    if (b) {
      (void)hipEventRecord(b, open_s);
      pending.push_back(Rec{open_k, open_n, open_a, b});
    } else {
      pool.push_back(open_a);
    }
    open_a = nullptr;
  }
  mi_status collect();
  ~KTimer();
};

// Marks the launches made during its lifetime as class k (no-op when timing
// is off).
struct KScope {
  KScope(KTimer* t, int k, hipStream_t s) {
    if (t) t->begin(k, s);
  }
};

// Closes the timer's open group when the entry point returns.
struct KClose {
  KTimer* t;
  explicit KClose(KTimer* t_) : t(t_) {}
  ~KClose() {
    if (t) t->close();
  }
};

}  // namespace mis

// Context (opaque in the C ABI).
struct mi_ctx {
  int device = 0;
  // cached plan + captured graph for mi_oi_track (see oi.hip)
  void* oi_plan = nullptr;
  void* doi_plan = nullptr;  // tracking plan of the dynamic walk (oi.hip)
  void* enc_plan = nullptr;
  void* cc_plan = nullptr;
  void* res_plan = nullptr;  // residual tile tables (see resid.hip)
  void* adj_oi = nullptr;    // tracking plan of the recorded forward (adjoint.hip)
  void* adj_plan = nullptr;  // adjoint tables (adjoint.hip)
  void* merge_plan = nullptr;  // occurrence table of overlapped submeshes (merge.hip)
  void* codec_plan = nullptr;  // block offsets of the quantiser (codec.hip)
  void* quality_plan = nullptr;  // partial sums of the quality report (quality.hip)
  mis::KTimer* timer = nullptr;  // non-null while timing is on
  int spmm_force = -1;  // SpMM variant forced on later tracking plans (-1: autotune/default)
};
