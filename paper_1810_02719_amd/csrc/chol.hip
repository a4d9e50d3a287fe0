// Cholesky factor and its inverse for the Cholesky-QR step (Section 4,
// Alg. 1, Onorm), blocked for FP64 MFMA, one workgroup per block.
//
// The scaled Gram G^ = D G D (D = diag(G)^-1/2) is factored as G^ = R^T R by
// right-looking block elimination over 16-wide panels K.  The same block
// row operations, applied to the identity, accumulate M = R^-T:
//
//   panel K:    R_KK = chol(G^_KK), M_KK = R_KK^-T        (one wavefront)
//               R_K,J = R_KK^-T G^_K,J        for J > K   (MFMA)
//               M_K  <- R_KK^-T M_K                       (MFMA)
//   trailing:   G^_I,J -= R_K,I^T R_K,J       for K < I <= J
//               M_I    -= R_K,I^T M_K         for I > K
//
// Both trailing updates are products of the same 16-row panel buffer (R row
// panel next to the updated M row panel), so they share one MFMA routine.
// Rinv = D M^T.
//
// Storage: 16 x 16 tiles in the FP64 MFMA accumulator layout, one slot per
// unordered tile pair (a <= b).  The slot holds G^(a, b) until panel a has
// consumed it, then M(b, a): the Gram tile dies in the same step in which
// that M tile is born, so G^ and M together fit in one triangle's worth of
// storage.  Up to ld = 192 every slot is a register tile.  Wider blocks (up
// to ld = 320) keep the slots of the first tile rows in global scratch
// (each lane stores and reloads only its own four values, so no other
// wavefront touches them) and the rest in registers: a slot (a, b) is
// rewritten once per panel K < b, so the slots with the largest b, the ones
// rewritten most often, are the register ones.
#include "small.hpp"

namespace mis {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

// The unit-diagonal Gram is factored with a small diagonal shift: a nearly
// rank-deficient basis then yields bounded (not exploding) columns of Rinv,
// at an orthonormality cost of about shift / lambda_min.  A pivot within ten
// shifts of zero (a column dependent on the previous ones to ~1e-6) flags
// MI_BLOCK_SHIFTED; one below the floor (rounding, or an indefinite input)
// is also raised to the floor.
constexpr double CHOL_SHIFT = 2e-13;
constexpr double CHOL_FLAG = 10.0 * CHOL_SHIFT;
constexpr double CHOL_PIV_TOL = 1e-13;  // pivot floor

// Orders one wavefront's LDS writes before its lanes read each other's
// values (the compiler may otherwise move a read above another lane's write).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1 / sqrt(x) for x > 0: hardware estimate and one Newton step.
__device__ __forceinline__ double inv_sqrt(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  return r * fma(-0.5 * x * r, r, 1.5);
}

// Value of v in lane src (any lane of the wavefront), as a double.
__device__ __forceinline__ double lane_get(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ d4v mfma64(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// acc + sign * sum_{t<16} P[t][16 r + m] Q[t][16 c + n] on one 16 x 16 tile.
__device__ __forceinline__ d4v tile_tn(d4v acc, const double* P, int ldp, int r,
                                       const double* Q, int ldq, int c, double sign, int lane) {
  const int mi = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 16; kk += 4) {
    const double a = sign * P[(kk + kq) * ldp + 16 * r + mi];
    const double b = Q[(kk + kq) * ldq + 16 * c + mi];
    acc = mfma64(a, b, acc);
  }
  return acc;
}

// One wavefront factors the diagonal tile G^_KK = R^T R held in its
// accumulator registers (element (mq + 4 q, mi) in g[q]) by the same row
// operations as the panels, applied to the identity: returns M_KK = R^-T in
// the same layout and writes R^-1 = M^T to Di.  Row k of the working matrix
// and of M is read straight from the lanes that hold it (lane (k mod 4) 16 +
// column); entries below the diagonal of the working matrix collect values
// that are never read.
__device__ d4v diag_factor(d4v g, double* Di, int ldd, int lane, int* fl) {
  const int mi = lane & 15, mq = lane >> 4;
  d4v mm;
#pragma unroll
  for (int q = 0; q < 4; ++q) mm[q] = (mq + 4 * q == mi) ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int kq = k >> 2, src = 16 * (k & 3);
    double piv = lane_get(g[kq], src + k);
    const double gkj = lane_get(g[kq], src + mi);   // working row k, column mi
    const double mkj0 = lane_get(mm[kq], src + mi);  // M row k, column mi
    double gki[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) gki[q] = lane_get(g[kq], src + mq + 4 * q);
    if (!(piv > CHOL_FLAG)) {
      *fl |= isfinite(piv) ? MI_BLOCK_SHIFTED : MI_BLOCK_NONFINITE;
      if (!(piv > CHOL_PIV_TOL)) piv = CHOL_PIV_TOL;
    }
    const double inv = inv_sqrt(piv);
    const double rkj = gkj * inv;   // R[k][j]
    const double mkj = mkj0 * inv;  // new M[k][j]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = mq + 4 * q;
      if (i == k) {
        mm[q] = mkj;
      } else if (i > k) {
        const double rki = gki[q] * inv;
        g[q] = fma(-rki, rkj, g[q]);
        mm[q] = fma(-rki, mkj, mm[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) Di[mi * ldd + mq + 4 * q] = mm[q];
  return mm;
}

}  // namespace

// NT = 16-tiles per dimension of the widest block of the launch
// (ld <= 16 NT <= 320); SG = slots per wavefront kept in global scratch
// (Wk, ld x ld per block, 16 SG x 256 doubles used).
template <int NT, int SG>
__global__ void __launch_bounds__(1024)
    k_chol_mfma(const SmallDesc* __restrict__ sds, const double* __restrict__ G,
                double* __restrict__ Wk, double* __restrict__ Rinv, float* __restrict__ S32,
                int32_t* __restrict__ status) {
  constexpr int NPAIR = NT * (NT + 1) / 2;    // tile pairs (a <= b)
  constexpr int SLOTS = (NPAIR + 15) / 16;    // per wavefront
  static_assert(SG >= 0 && SG <= SLOTS, "global slots");
  constexpr int LDB = 16 * NT + 4;            // panel buffer row stride (doubles)
  constexpr int LDD = 17;
  // bufA doubles as the 16 per-wavefront tile transposes of the stores
  constexpr int LDA_SZ = 16 * LDB > 16 * 16 * 17 ? 16 * LDB : 16 * 16 * 17;
  __shared__ double bufA[LDA_SZ];             // old panel: G^ row K | M row K
  __shared__ double bufB[16 * LDB];           // new panel: R row K  | M row K
  __shared__ double Dg[16 * LDD];             // R_KK^-1
  __shared__ double dsc[16 * NT];
  __shared__ int flag;

  const SmallDesc d = sds[blockIdx.x];
  const int p = d.p, ld = d.ld;
  const int nk = (p + 15) >> 4;  // panels of this block (<= NT)
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: slot logic is scalar
  const int mi = lane & 15, mq = lane >> 4;  // tile element (mq + 4 q, mi)
  const double* Gb = G + d.m_off;

  if (tid == 0) flag = 0;
  for (int i = tid; i < 16 * NT; i += 1024) {
    double v = 1.0;
    if (i < p) {
      const double g = Gb[int64_t(i) * ld + i];
      if (!isfinite(g)) atomicOr(&flag, MI_BLOCK_NONFINITE);
      else if (!(g > 0.0)) atomicOr(&flag, MI_BLOCK_NOT_PD);
      v = (g > 0.0 && isfinite(g)) ? 1.0 / sqrt(g) : 0.0;
    }
    dsc[i] = v;
  }
  __syncthreads();

  // slot s of this wavefront: pair t = wave + 16 s in column-major upper
  // order, a <= b; slots s < SG at gsl(s), the others in reg[s].  With
  // global slots, pairs with b >= nk (past the block's own panels) are never
  // touched: they would only produce zero padding, and skipping them keeps
  // the global slots of a narrow block inside its own ld x ld scratch
  // (256 t + 255 < ld^2 for t < nk (nk + 1) / 2).
  int ta[SLOTS], tb[SLOTS];
  d4v reg[SLOTS];
  d4v* gbase = reinterpret_cast<d4v*>(Wk + d.m_off) + 64 * wave + lane;
  auto gsl = [&](int s) { return gbase + 1024 * s; };
#pragma clang loop unroll(full)
  for (int s = 0; s < SLOTS; ++s) {
    const int t = wave + 16 * s;
    int b = 0;  // column of pair t: the number of x in [1, NT) with x (x + 1) / 2 <= t
#pragma unroll
    for (int x = 1; x < NT; ++x) b += (x * (x + 1) / 2 <= t) ? 1 : 0;
    const int a = t - b * (b + 1) / 2;
    ta[s] = t < NPAIR ? a : -1;
    tb[s] = t < NPAIR ? b : -1;
    d4v v4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * a + mq + 4 * q, j = 16 * b + mi;
      double v = 0.0;
      if (t < NPAIR) {
        if (i < p && j < p) v = (i == j) ? 1.0 + CHOL_SHIFT : Gb[int64_t(i) * ld + j] * dsc[i] * dsc[j];
        else if (i == j) v = 1.0;  // identity padding
      }
      v4[q] = v;
    }
    if (s < SG) {
      if (t < NPAIR && b < nk) *gsl(s) = v4;
      __builtin_amdgcn_sched_barrier(0);
    } else {
      reg[s] = v4;
    }
  }

  for (int K = 0; K < nk; ++K) {
    // launder the slot indices so that the compiler recomputes the per-slot
    // LDS addresses each step instead of keeping dozens of them live
#pragma clang loop unroll(full)
    for (int s = 0; s < SLOTS; ++s) asm volatile("" : "+s"(ta[s]), "+s"(tb[s]));
    // the same for the global slot addresses (one base, offsets per use)
    if (SG > 0) asm volatile("" : "+v"(gbase));
    // 1: publish the Gram row panel and the old M row panel; the wavefront
    // that owns the diagonal tile factors it (M_KK = R_KK^-T into its slot
    // and the new M panel, R_KK^-1 into Dg)
#pragma clang loop unroll(full)
    for (int s = 0; s < SLOTS; ++s) {
      const int a = ta[s], b = tb[s];
      if ((SG == 0 || b < nk) && (a == K || (b == K && a >= 0))) {
        d4v cur = s < SG ? *gsl(s) : reg[s];
        if (a == K && b == K) {
          int fl = 0;
          cur = diag_factor(cur, Dg, LDD, lane, &fl);
          if (lane == 0 && fl) atomicOr(&flag, fl);
          if (s < SG) *gsl(s) = cur;
          else reg[s] = cur;
        } else {
          const int c = a == K ? b : a;
#pragma unroll
          for (int q = 0; q < 4; ++q) bufA[(mq + 4 * q) * LDB + 16 * c + mi] = cur[q];
        }
      }
      if (s < SG) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // 3: R row panel and new M row panel (both: R_KK^-T times the old panel)
#pragma clang loop unroll(full)
    for (int s = 0; s < SLOTS; ++s) {
      const int a = ta[s], b = tb[s];
      if (a == K && b > K && (SG == 0 || b < nk)) {
        d4v acc = {0.0, 0.0, 0.0, 0.0};
        acc = tile_tn(acc, Dg, LDD, 0, bufA, LDB, b, 1.0, lane);
#pragma unroll
        for (int q = 0; q < 4; ++q) bufB[(mq + 4 * q) * LDB + 16 * b + mi] = acc[q];
        // the slot now holds M(b, a) = 0
        if (s < SG) *gsl(s) = d4v{0.0, 0.0, 0.0, 0.0};
        else reg[s] = d4v{0.0, 0.0, 0.0, 0.0};
      } else if (a == K && b == K) {
        // M_KK (already in the slot) joins the new M panel; written only now
        // because other wavefronts read bufB in the previous step 4
        const d4v cur = s < SG ? *gsl(s) : reg[s];
#pragma unroll
        for (int q = 0; q < 4; ++q) bufB[(mq + 4 * q) * LDB + 16 * K + mi] = cur[q];
      } else if (b == K && a >= 0) {
        d4v acc = {0.0, 0.0, 0.0, 0.0};
        acc = tile_tn(acc, Dg, LDD, 0, bufA, LDB, a, 1.0, lane);
        if (s < SG) *gsl(s) = acc;
        else reg[s] = acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) bufB[(mq + 4 * q) * LDB + 16 * a + mi] = acc[q];
      }
      if (s < SG) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // 4: trailing updates of G^ (a, b > K) and of M (row b > K, column a <= K)
#pragma clang loop unroll(full)
    for (int s = 0; s < SLOTS; ++s) {
      const int a = ta[s], b = tb[s];
      if ((SG == 0 || b < nk) && (a > K || (b > K && a >= 0))) {
        d4v cur = s < SG ? *gsl(s) : reg[s];
        if (a > K) cur = tile_tn(cur, bufB, LDB, a, bufB, LDB, b, -1.0, lane);
        else cur = tile_tn(cur, bufB, LDB, b, bufB, LDB, a, -1.0, lane);
        if (s < SG) *gsl(s) = cur;
        else reg[s] = cur;
      }
      __builtin_amdgcn_sched_barrier(0);  // one tile's operands live at a time
    }
    // the next step 1 writes bufA and Dg only; the barrier after it orders
    // these bufB reads before the next step 3
  }
  __syncthreads();  // bufA is reused as the transpose buffers below

  // Rinv[r][c] = dsc[r] M[c][r] for r <= c < p; zero elsewhere.  Slot (a, b)
  // holds M(b, a) and writes the two transposed tiles (a, b) and (b, a); the
  // first goes through a per-wavefront LDS transpose so that consecutive
  // lanes store consecutive columns.
  double* Rb = Rinv + d.m_off;
  float* Sb = S32 ? S32 + d.m_off : nullptr;
  double* tw = bufA + wave * (16 * 17);
#pragma clang loop unroll(full)
  for (int s = 0; s < SLOTS; ++s) {
    const int a = ta[s], b = tb[s];
    if (a < 0) continue;
    // tiles past the block's panels only hold padding: their outputs are 0
    const d4v cur = (SG > 0 && b >= nk) ? d4v{0.0, 0.0, 0.0, 0.0} : s < SG ? *gsl(s) : reg[s];
    // tw[x][y] = M(b, a)[y][x]
#pragma unroll
    for (int q = 0; q < 4; ++q) tw[mi * 17 + mq + 4 * q] = cur[q];
    wave_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = mq + 4 * q;
      // M(b, a)[mi][rr] = M[16 b + mi][16 a + rr] -> Rinv[16 a + rr][16 b + mi]
      const int r = 16 * a + rr, c = 16 * b + mi;
      if (r < ld && c < ld) {
        const double v = (r <= c && c < p) ? dsc[r] * tw[rr * 17 + mi] : 0.0;
        Rb[int64_t(r) * ld + c] = v;
        if (Sb) Sb[int64_t(r) * ld + c] = (float)v;
      }
    }
    wave_sync();  // the reads above before the next slot's writes
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = mq + 4 * q;
      if (a != b) {  // the tile below the diagonal
        const int r2 = 16 * b + m, c2 = 16 * a + mi;
        if (r2 < ld && c2 < ld) {
          Rb[int64_t(r2) * ld + c2] = 0.0;
          if (Sb) Sb[int64_t(r2) * ld + c2] = 0.0f;
        }
      }
    }
  }
  if (tid == 0 && flag) atomicOr(&status[d.blk], flag);
}

bool launch_chol_mfma(const SmallDesc* sd, int nb, const double* G, double* Wk, double* Rinv,
                      float* S32, int32_t* status, int max_ld, hipStream_t s) {
  // at most 5 register slots per wavefront (3 above ld = 192, where the global
  // slots need registers of their own; more spill at 128 VGPRs); the rest in Wk
#define MI_CHOL_CASE(N)                                                                         \
  case N: {                                                                                     \
    constexpr int NT = 2 * N, SL = (NT * (NT + 1) / 2 + 15) / 16;                              \
    constexpr int RS = NT <= 12 ? 5 : NT <= 16 ? 3 : 2, SG = SL > RS ? SL - RS : 0;             \
    hipLaunchKernelGGL((k_chol_mfma<NT, SG>), dim3(nb), dim3(1024), 0, s, sd, G, Wk, Rinv, S32, \
                       status);                                                                 \
    return true;                                                                                \
  }
  switch ((max_ld + 31) / 32) {
    MI_CHOL_CASE(1)
    MI_CHOL_CASE(2)
    MI_CHOL_CASE(3)
    MI_CHOL_CASE(4)
    MI_CHOL_CASE(5)
    MI_CHOL_CASE(6)
    MI_CHOL_CASE(7)
    MI_CHOL_CASE(8)
    MI_CHOL_CASE(9)
    MI_CHOL_CASE(10)
#undef MI_CHOL_CASE
    default:
      return false;
  }
}

}  // namespace mis
