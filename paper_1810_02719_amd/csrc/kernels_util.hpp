// Small device/host utilities shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

namespace mis {

constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_TILE = 256 * SCAN_PER_THREAD;

size_t scan_scratch_bytes(int64_t N);
void exclusive_scan(const int32_t* in, int64_t* out, int64_t N, int64_t* scratch, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_f64(double* p, double v, int64_t n, hipStream_t s);

// Largest b with off[b] <= x (off ascending, off[0] = 0, x < off[B]).
__device__ inline int find_block(const int64_t* __restrict__ off, int B, int64_t x) {
  int lo = 0, hi = B;  // invariant: off[lo] <= x < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

// 16-byte vector of a slab element type (one load or store per lane).
template <typename T>
struct VecOf;
template <>
struct VecOf<float> {
  typedef f4v type;
  static constexpr int W = 4;
};
template <>
struct VecOf<double> {
  typedef d2v type;
  static constexpr int W = 2;
};
struct bf16;
template <>
struct VecOf<bf16> {
  typedef uint4 type;  // eight BF16 values
  static constexpr int W = 8;
};

// Slab element of the reduced-precision option: bfloat16 storage (the upper
// half of an FP32 word), arithmetic in FP32.  Rounding to nearest, ties to
// even (NaN kept quiet).
struct bf16 {
  uint16_t u;
};
__host__ __device__ inline float bf16_to_f32(bf16 x) {
  const uint32_t w = uint32_t(x.u) << 16;
  float f;
  __builtin_memcpy(&f, &w, 4);
  return f;
}
__host__ __device__ inline bf16 f32_to_bf16(float f) {
  uint32_t w;
  __builtin_memcpy(&w, &f, 4);
  if ((w & 0x7F800000u) == 0x7F800000u && (w & 0x007FFFFFu)) return bf16{uint16_t((w >> 16) | 0x40u)};
  w += 0x7FFFu + ((w >> 16) & 1u);
  return bf16{uint16_t(w >> 16)};
}

// Arithmetic type of a slab element type and the conversions to and from it.
template <typename T>
struct Acc {
  typedef T type;
  __host__ __device__ static T load(T x) { return x; }
  __host__ __device__ static T store(T x) { return x; }
};
template <>
struct Acc<bf16> {
  typedef float type;
  __host__ __device__ static float load(bf16 x) { return bf16_to_f32(x); }
  __host__ __device__ static bf16 store(float x) { return f32_to_bf16(x); }
};

// Sum over the 64 lanes of a wavefront (every lane gets the total).
__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-provided workspace.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = used;
    used = align_up(used + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

}  // namespace mis
