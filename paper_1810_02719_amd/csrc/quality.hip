// Reconstruction quality of a whole mesh (Section 8): the NMSVE of Eq. 16,
//   ( ||v - v~||_2 + ||GL(v) - GL(v~)||_2 ) / (2n),
//   GL(v)_i = v_i - sum_j d_ij^-1 v_j / sum_j d_ij^-1   (j over the neighbours of i),
// with the edge lengths d_ij of the original mesh for both operands (GL is
// then one linear operator, applied here to the difference v - v~), and
// theta, the angle between the normal of every face of the original mesh
// and of the same face of the reconstruction, averaged over the faces.
//
// One pass over vertices and faces in a fixed grid (one thread per vertex
// and per face, grid-stride), FP64 partial sums per workgroup, then one
// workgroup adds the partials in a fixed order: the result is bitwise
// reproducible.  The work is a gather over the mesh (about 40 bytes per
// vertex and 12 per face from HBM, neighbour coordinates from cache), far
// below a microsecond of HBM time at the meshes of interest: launch latency
// bounds it.
#include <algorithm>
#include <cmath>
#include <memory>

#include "common.hpp"
#include "kernels_util.hpp"

namespace mis {

constexpr int QUAL_THREADS = 256;
constexpr int QUAL_MAX_WG = 1024;
constexpr int QUAL_SUMS = 6;  // |e|^2, |GL e|^2, angle (rad), faces used, zero edges, bad indices

struct QualityPlan {
  double* part = nullptr;  // [QUAL_MAX_WG][QUAL_SUMS]
  ~QualityPlan() {
    if (part) (void)hipFree(part);
  }
};

__device__ inline double3 load3(const float* p, int64_t i) {
  return make_double3(double(p[3 * i]), double(p[3 * i + 1]), double(p[3 * i + 2]));
}
__device__ inline double3 sub3(double3 a, double3 b) {
  return make_double3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ inline double dot3(double3 a, double3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
// each product rounded on its own (the opaque copies keep the compiler from
// fusing one into a multiply-add), so the cross product of two equal
// vectors is exactly zero
__device__ inline double rn_mul(double x, double y) {
  double p = x * y;
  asm volatile("" : "+v"(p));
  return p;
}
__device__ inline double3 cross3(double3 a, double3 b) {
  return make_double3(rn_mul(a.y, b.z) - rn_mul(a.z, b.y), rn_mul(a.z, b.x) - rn_mul(a.x, b.z),
                      rn_mul(a.x, b.y) - rn_mul(a.y, b.x));
}

__global__ void __launch_bounds__(QUAL_THREADS)
    k_quality_part(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                   int64_t nnz, int64_t nf, const int32_t* __restrict__ faces,
                   const float* __restrict__ X, const float* __restrict__ Xr,
                   double* __restrict__ part) {
  __shared__ double red[QUAL_SUMS][QUAL_THREADS / 64];
  double acc[QUAL_SUMS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t stride = int64_t(gridDim.x) * QUAL_THREADS;
  for (int64_t i = int64_t(blockIdx.x) * QUAL_THREADS + threadIdx.x; i < n; i += stride) {
    const double3 xi = load3(X, i);
    const double3 e = sub3(xi, load3(Xr, i));
    acc[0] += dot3(e, e);
    // the row's entries, clamped to the column array; the diagonal (the
    // Laplacian's own entry) is not a neighbour
    const int64_t k0 = max<int64_t>(row_ptr[i], 0), k1 = min<int64_t>(row_ptr[i + 1], nnz);
    double sw = 0.0;
    double3 s = make_double3(0.0, 0.0, 0.0);
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t j = col[k];
      if (j == i) continue;
      if (j < 0 || j >= n) {
        acc[5] += 1.0;
        continue;
      }
      const double3 xj = load3(X, j);
      const double3 dx = sub3(xi, xj);
      const double d = sqrt(dot3(dx, dx));
      if (d == 0.0) {
        acc[4] += 1.0;
        continue;
      }
      const double w = 1.0 / d;
      const double3 ej = sub3(xj, load3(Xr, j));
      sw += w;
      s.x += w * ej.x;
      s.y += w * ej.y;
      s.z += w * ej.z;
    }
    double3 g = e;
    if (sw > 0.0) g = make_double3(e.x - s.x / sw, e.y - s.y / sw, e.z - s.z / sw);
    acc[1] += dot3(g, g);
  }
  for (int64_t f = int64_t(blockIdx.x) * QUAL_THREADS + threadIdx.x; f < nf; f += stride) {
    const int64_t a = faces[3 * f], b = faces[3 * f + 1], c = faces[3 * f + 2];
    if (a < 0 || a >= n || b < 0 || b >= n || c < 0 || c >= n) {
      acc[5] += 1.0;
      continue;
    }
    const double3 xa = load3(X, a), ra = load3(Xr, a);
    const double3 no = cross3(sub3(load3(X, b), xa), sub3(load3(X, c), xa));
    const double3 nr = cross3(sub3(load3(Xr, b), ra), sub3(load3(Xr, c), ra));
    if (dot3(no, no) == 0.0 || dot3(nr, nr) == 0.0) continue;  // no direction: left out
    const double3 cr = cross3(no, nr);
    acc[2] += atan2(sqrt(dot3(cr, cr)), dot3(no, nr));  // well conditioned at 0 and pi
    acc[3] += 1.0;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < QUAL_SUMS; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) red[q][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x < QUAL_SUMS) {
    double t = 0.0;
    for (int w = 0; w < QUAL_THREADS / 64; ++w) t += red[threadIdx.x][w];
    part[int64_t(blockIdx.x) * QUAL_SUMS + threadIdx.x] = t;
  }
}

// out: NMSVE, 10 log10 NMSVE, ||v - v~||, ||GL(v) - GL(v~)||, theta in
// degrees, faces averaged, zero-length edges, out-of-range indices
__global__ void __launch_bounds__(QUAL_THREADS)
    k_quality_final(int nwg, int64_t n, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[QUAL_SUMS][QUAL_THREADS / 64];
  double acc[QUAL_SUMS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int w = threadIdx.x; w < nwg; w += QUAL_THREADS)
#pragma unroll
    for (int q = 0; q < QUAL_SUMS; ++q) acc[q] += part[int64_t(w) * QUAL_SUMS + q];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < QUAL_SUMS; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) red[q][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[QUAL_SUMS];
    for (int q = 0; q < QUAL_SUMS; ++q) {
      s[q] = 0.0;
      for (int w = 0; w < QUAL_THREADS / 64; ++w) s[q] += red[q][w];
    }
    const bool bad = s[4] > 0.0 || s[5] > 0.0;
    const double l2 = sqrt(s[0]), gl = bad ? NAN : sqrt(s[1]);
    const double nm = n > 0 ? (l2 + gl) / (2.0 * double(n)) : 0.0;
    out[0] = bad ? NAN : nm;
    out[1] = bad ? NAN : 10.0 * log10(nm);
    out[2] = l2;
    out[3] = gl;
    out[4] = bad ? NAN : (s[3] > 0.0 ? s[2] / s[3] * (180.0 / M_PI) : 0.0);
    out[5] = s[3];
    out[6] = s[4];
    out[7] = s[5];
  }
}

}  // namespace mis

using namespace mis;

extern "C" {

void mis_destroy_quality_plan(mi_ctx* ctx) {
  delete static_cast<QualityPlan*>(ctx->quality_plan);
  ctx->quality_plan = nullptr;
}

mi_status mi_mesh_quality(mi_ctx* ctx, int64_t n_vertices, const int32_t* row_ptr,
                          const int32_t* col, int64_t nnz, int64_t n_faces, const int32_t* faces,
                          const float* X, const float* Xr, double* out, void* stream) {
  begin_call();
  MI_CHECK_ARG(ctx && out, "NULL argument");
  MI_CHECK_ARG(n_vertices >= 0 && n_vertices < (int64_t(1) << 31), "n_vertices %lld out of range",
               (long long)n_vertices);
  MI_CHECK_ARG(nnz >= 0 && n_faces >= 0, "negative nnz or n_faces");
  MI_CHECK_ARG(n_vertices == 0 || (row_ptr && X && Xr), "row_ptr, X and Xr are required");
  MI_CHECK_ARG(nnz == 0 || col, "col is required when nnz > 0");
  MI_CHECK_ARG(n_faces == 0 || faces, "faces is required when n_faces > 0");
  MI_TRY_HIP(hipSetDevice(ctx->device));
  QualityPlan* P = static_cast<QualityPlan*>(ctx->quality_plan);
  if (!P) {
    std::unique_ptr<QualityPlan> np(new QualityPlan());
    MI_TRY_HIP(hipMalloc(&np->part, size_t(QUAL_MAX_WG) * QUAL_SUMS * sizeof(double)));
    P = np.release();
    ctx->quality_plan = P;
  }
  const int64_t work = std::max<int64_t>(std::max<int64_t>(n_vertices, n_faces), 1);
  const int nwg = int(std::min<int64_t>(ceil_div(work, QUAL_THREADS), QUAL_MAX_WG));
  hipStream_t s = (hipStream_t)stream;
  KClose kc_(ctx->timer);
  KScope k_(ctx->timer, MI_K_QUALITY, s);
  hipLaunchKernelGGL(k_quality_part, dim3(nwg), dim3(QUAL_THREADS), 0, s, n_vertices, row_ptr, col,
                     nnz, n_faces, faces, X, Xr, P->part);
  MI_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_quality_final, dim3(1), dim3(QUAL_THREADS), 0, s, nwg, n_vertices,
                     (const double*)P->part, out);
  MI_TRY_HIP(hipGetLastError());
  return MI_OK;
}

}  // extern "C"
