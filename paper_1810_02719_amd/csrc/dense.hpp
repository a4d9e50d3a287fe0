// Tall-skinny kernels shared by the tracking and the encoder: CSR SpMM with
// the three-term update of the Chebyshev recurrence, Gram products A^T B
// with FP64 MFMA and a deterministic split-K reduction, and row-block
// products A S on MFMA.
#pragma once

#include "common.hpp"
#include "kernels_util.hpp"

namespace mis {

// A set of per-block matrices: block k of the set is a rows x ld row-major
// matrix at element offset off (ld = row stride; only the first `cols`
// columns are meaningful, the rest are zero padding).
struct MatDesc {
  int64_t off;
  int32_t rows;
  int32_t ld;
  int32_t cols;
  int32_t blk;  // index into per-block parameter arrays (coefficients, flags)
};

// SpMM / Chebyshev tiles: rows [row0, row0 + SPMM_ROWS) of block `set`.
struct SpmmTile {
  int32_t set;
  int32_t row0;
};
constexpr int SPMM_ROWS = 16;

// CSR location of a block: row_ptr at rp_off, col/val at nnz_off.
struct CsrDesc {
  int64_t rp_off;
  int64_t nnz_off;
};

// Gram tiles: a 64 x 64 output super-tile (I0, J0) of block `set`, summed
// over the rows [r0, r1).  Output goes to part + tile_index * 64 * 64 (and a
// second plane for the dual product).
struct GramTile {
  int32_t set;
  int32_t I0, J0;
  int32_t r0, r1;
};
constexpr int GRAM_TILE = 64;

// Reduce jobs: block `set`, super-tile (I0, J0), partial tiles first,
// first + stride, ..., count of them, in chunk order.
struct GramReduce {
  int32_t set;
  int32_t I0, J0;
  int32_t first, count, stride;
};

// Row-product tiles: rows [row0, row0 + 64) x output columns [n0, n0 + NCH).
struct RowTile {
  int32_t set;
  int32_t row0;
  int32_t n0;
};
constexpr int ROW_TILE = 64;

// Variants of the wavefront-per-row SpMM (the autotuner picks one per wave):
// one row per wavefront gathering 8 neighbour rows at a time, the same with
// 4 at a time (fewer registers, more wavefronts per CU), two rows per
// wavefront, one row per wavefront in workgroups of 4 wavefronts, or 2 or 4
// rows per wavefront one after the other with all their indices loaded
// first (2 also in workgroups of 4 wavefronts); and one row per wavefront
// gathering only the off-diagonal entries, the product in difference form
// (sum_j L_rj (Y_j - Y_r) plus the row sum times Y_r), in workgroups of 8,
// 16 or 4 wavefronts over consecutive rows, with the previous iterate and
// the output streamed non-temporally (8 also with ordinary loads and
// stores); and the same product with half a wavefront per row (two rows
// per wavefront, twice the elements per lane), in workgroups of 8 or 4
// wavefronts.  Variants 0-6 give bit-identical results, and so do 7-12
// among themselves.
constexpr int SPMM_VAR_ROW = 0;
constexpr int SPMM_VAR_ROW_G4 = 1;
constexpr int SPMM_VAR_ROW2 = 2;
constexpr int SPMM_VAR_ROW_W4 = 3;
constexpr int SPMM_VAR_ROWS2 = 4;
constexpr int SPMM_VAR_ROWS4 = 5;
constexpr int SPMM_VAR_ROWS2_W4 = 6;
constexpr int SPMM_VAR_X8_NT = 7;
constexpr int SPMM_VAR_X16_NT = 8;
constexpr int SPMM_VAR_X8 = 9;
constexpr int SPMM_VAR_X4_NT = 10;
constexpr int SPMM_VAR_XH8_NT = 11;
constexpr int SPMM_VAR_XH4_NT = 12;
constexpr int SPMM_NVAR = 13;
int spmm_default_var(int epl);

template <typename T>
void launch_spmm(const SpmmTile* tiles, int ntiles, const MatDesc* sets, const CsrDesc* csr,
                 const int32_t* row_ptr, const int32_t* col, const float* val, const T* Yin,
                 const T* Yprev, T* Yout, const double* coef, int coef_stride, int step,
                 hipStream_t s, int epl = 0, int var = -1);
// Elements per lane of the wavefront-per-row SpMM when every block of a
// launch has the same ld, a multiple of 64 up to 320; 0 otherwise.
int spmm_epl(const std::vector<MatDesc>& sets);

// A whole Chebyshev filter pass (m steps) of a wave in one persistent
// launch: `grid` workgroups claim blocks (sets[order[i]], i = 0, 1, ...) from
// the queue head *queue (reset to 0 on the stream first) and run the m steps
// on each with workgroup barriers between them; step k writes o[k mod 3].
// Rows as SPMM variants 7-12 (bit-identical).  Waves of one width only
// (epl = spmm_epl of the wave, > 0).
constexpr int PASS_WAVES = 8;  // wavefronts per workgroup
template <typename T>
void launch_cheb_pass(const MatDesc* sets, const CsrDesc* csr, const int32_t* order, int nsets,
                      const int32_t* row_ptr, const int32_t* col, const float* val, const T* X,
                      T* o0, T* o1, T* o2, const double* coef, int coef_stride, int m,
                      int32_t* queue, int grid, int epl, hipStream_t s);
// Workgroups of that launch: the resident ones (occupancy times CUs), at most
// one per block; 0 when epl has no kernel.
template <typename T>
int cheb_pass_grid(int epl, int nsets);

template <typename T>
void launch_gram(const GramTile* tiles, int ntiles, const MatDesc* sets, const T* A, const T* B,
                 const T* W, double* part, hipStream_t s);

void launch_gram_reduce(const GramReduce* jobs, int njobs, const MatDesc* outsets,
                        const double* part, bool dual, double* G, double* H, hipStream_t s);
// The same products written straight into G (and H for the dual product)
// when no super-tile is split over row chunks (every reduce job has one
// partial: gram_unsplit), with no partials and no reduction.  FP32 and
// FP64 slabs.
template <typename T>
void launch_gram_direct(const GramTile* tiles, int ntiles, const MatDesc* sets,
                        const MatDesc* outsets, const T* A, const T* B, const T* W, double* G,
                        double* H, hipStream_t s);
bool gram_unsplit(const std::vector<GramReduce>& jobs);

// a_lo[blk] <- max_{j < p} q_j^T L q_j of each block's orthonormalised basis
// X (the tall sets) from W = L X; part: scratch in each block's p x p
// matrix slot (osets: 8 ld doubles per block, ld >= 8).
template <typename T>
void launch_rq(const MatDesc* sets, const MatDesc* osets, int nb, const T* X, const T* W,
               double* part, double* a_lo, hipStream_t s);

// Out = A S row tile by row tile; A may be a BF16 slab with S and the MFMA in
// FP32 (TA = bf16, T = float).  upper: S is upper triangular (zero below
// the diagonal, as R^-1 of a Cholesky-QR), so each output-column chunk reads
// only the rows of S down to its last column.
template <typename TA, typename T, typename TO>
void launch_rowmul(const RowTile* tiles, int ntiles, const MatDesc* asets, const TA* A,
                   const MatDesc* ssets, const T* S, const MatDesc* osets, TO* Out, int nch,
                   hipStream_t s, bool upper = false);

// Tile tables (host).  Gram: 64 x 64 super-tiles of the upper triangle,
// split over row chunks when `split` (about 2048 workgroups in total);
// rows: 64-row x nch-column tiles; SpMM: SPMM_ROWS-row tiles.
constexpr int GRAM_TARGET = 384;  // default workgroups of a split Gram launch
int gram_chunks(int nsets, int npairs, int rows, int target = GRAM_TARGET);
void gram_tables(const std::vector<MatDesc>& sets, bool split, std::vector<GramTile>* tiles,
                 std::vector<GramReduce>* red, int target = GRAM_TARGET);
void row_tables(const std::vector<MatDesc>& sets, int nch, std::vector<RowTile>* tiles);
void spmm_tables(const std::vector<MatDesc>& sets, std::vector<SpmmTile>* tiles);

}  // namespace mis
