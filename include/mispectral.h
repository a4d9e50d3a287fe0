/*
 * mispectral — block-based spectral processing of triangle meshes on MI355X.
 *
 * C ABI of the GPU library.  A mesh is split into submeshes ("blocks"); for
 * every block the library builds the graph Laplacian, tracks the eigenspace
 * of its c lowest eigenvalues by orthogonal iteration warm-started from a
 * predecessor block, projects the xyz coordinates onto it (graph Fourier
 * transform), truncates and reconstructs.  Method: Arvanitis, Lalos,
 * Moustakas, "Block-Based Spectral Processing of Static and Dynamic 3D Meshes
 * using Orthogonal Iterations" (arXiv 1810.02719); sections, equations and
 * algorithms below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns mi_status: 0 on success, a negative MI_ERR_* code
 *    otherwise; mi_last_error() gives a message for the calling thread.
 *    Argument errors are detected on the host before anything is enqueued.
 *  - Memory: the caller owns every buffer.  Pointers documented "device"
 *    must point to device memory of the context's GPU; "host" pointers to
 *    host memory read during the call only.  The library keeps no pointer
 *    after a call returns, except inside an mi_ctx (see mi_oi_track).
 *  - Streams: `stream` is a hipStream_t (NULL = default stream).  Calls only
 *    enqueue work on it unless documented as synchronous.
 *  - The *_workspace_size queries are host arithmetic only (ctx may be NULL);
 *    they validate the block table and parameters like the calls they size.
 *  - Block layout: blocks are concatenated.  Block b owns the vertex rows
 *    v_off[b] .. v_off[b+1]-1 of every per-vertex array (vertex ids inside a
 *    block are block-local, 0 .. n_b-1).  The tracked subspace of block b is
 *    a row-major n_b x ld_b slab (vertex-major: the p_b coefficients of a
 *    vertex are contiguous) starting at element u_off[b]; columns
 *    p_b .. ld_b-1 are padding and hold zeros on output.
 *  - CSR of the block Laplacians: row_ptr holds n_b+1 block-local offsets
 *    per block, at position v_off[b] + b; col / val of block b start at
 *    nnz_off[b]; column ids are block-local, ascending, the diagonal is
 *    always stored.
 */
#ifndef MISPECTRAL_H
#define MISPECTRAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mi_status;

#define MI_OK 0
#define MI_ERR_ARG (-1)        /* invalid argument (checked on the host)            */
#define MI_ERR_INDEX (-2)      /* a primitive references a vertex outside its block */
#define MI_ERR_DEGENERATE (-3) /* zero-length edge under a distance weight          */
#define MI_ERR_NOT_PD (-4)     /* a Gram matrix was not positive definite           */
#define MI_ERR_NOCONV (-5)     /* an eigen-solve did not converge                   */
#define MI_ERR_HIP (-6)        /* a HIP runtime call failed                         */
#define MI_ERR_WORKSPACE (-7)  /* workspace smaller than the size query returned    */
#define MI_ERR_CAPACITY (-8)   /* c > p_b, p_b > n_b or ld_b too small             */

/* Off-diagonal weights C_ij of the Laplacian L = D - C (Section 3). */
#define MI_W_COMBINATORIAL 0 /* C = adjacency, D_ii = |N(i)|                       */
#define MI_W_INV_SQ_DIST 1   /* C_ij = 1/||v_i - v_j||^2 (Eq. 2), D_ii = sum_j C_ij */
#define MI_W_USER 2          /* C_ij = user weight per canonical edge              */
#define MI_W_INV_DIST 3      /* C_ij = 1/||v_i - v_j|| (the GL operator of Eq. 16)  */

/* Arithmetic of the tall-skinny products (SpMM, Gram operands, rotations). */
#define MI_FP32 0
#define MI_FP64 1
#define MI_BF16_IN 2   /* mi_oi_track only: the working slabs of the filter and the
                          Cholesky-QR (the inputs of the SpMM and Gram products) in
                          bfloat16, rounded to nearest even, with FP32 accumulation
                          inside a product and FP64 across a Gram's row chunks; FP64
                          Cholesky and Rayleigh-Ritz solves; the row products in FP32;
                          V0 and V are FP32 (float).  Chebyshev filter, fixed
                          iteration counts, every block of a wave with the same ld
                          (a multiple of 64 up to 320); not for the dynamic walk or
                          the adjoint (MI_ERR_ARG). */

/* Start subspace of a block in mi_oi_track. */
#define MI_WARM_GIVEN 0 /* V0 holds a start for every block                          */
#define MI_WARM_PRED 1  /* blocks with pred >= 0 start from their predecessor's result */
#define MI_RANDOM 2     /* blocks without a predecessor (all blocks when pred is NULL)
                           start from seeded pseudo-random numbers (mi_oi_params.seed),
                           the others from their predecessor as under MI_WARM_PRED;
                           V0 is not read.  Entry (i, j) of block b's start is
                           2 u - 1 with u = (z >> 11) 2^-53, z = SplitMix64 of the
                           counter seed + 0x9E3779B97F4A7C15 (1 + b 2^40 + i 2^12 + j)
                           (Steele, Lea and Flood 2014; b < 2^24, i < 2^28, j < 2^12),
                           for j < p_b; the start is orthonormalised by a Cholesky-QR
                           before its first filter pass */

/* Per-block status codes written to `status` by mi_oi_track (device). */
#define MI_BLOCK_OK 0
#define MI_BLOCK_SHIFTED 1   /* a Cholesky factorisation needed a diagonal shift   */
#define MI_BLOCK_NOT_PD 2    /* a Cholesky factorisation failed even when shifted */
#define MI_BLOCK_NOCONV 4    /* Jacobi sweeps exhausted before convergence         */
#define MI_BLOCK_NONFINITE 8 /* NaN / Inf met in a small matrix                    */
#define MI_BLOCK_UNCONVERGED 16 /* tolerance mode: the kept pairs did not meet tol
                                   within the iteration limit                     */

typedef struct mi_ctx mi_ctx;

/* Block table (all host memory). */
typedef struct {
  int32_t n_blocks;
  const int64_t* v_off; /* [n_blocks+1] first vertex row of each block                 */
  const int32_t* p;     /* [n_blocks]   tracked subspace width p_b (1 <= p_b <= n_b)   */
  const int32_t* ld;    /* [n_blocks]   row stride of the slab, multiple of 32, >= p_b */
  const int64_t* u_off; /* [n_blocks+1] slab offsets, u_off[b+1]-u_off[b] = n_b*ld_b    */
  const int32_t* pred;  /* [n_blocks] warm-start predecessor (-1 none), or NULL        */
  const int32_t* c;     /* [n_blocks] kept pairs c_b (1 <= c_b <= p_b): the Ritz pairs
                           the tolerance test of mi_oi_track covers; NULL = p_b.
                           Other calls ignore it                                    */
} mi_blocks;

/* Parameters of the eigenspace tracking (mi_oi_track). */
typedef struct {
  int32_t precision; /* MI_FP32, MI_FP64 or MI_BF16_IN                                */
  int32_t warm;      /* MI_WARM_GIVEN, MI_WARM_PRED or MI_RANDOM                      */
  int32_t T;         /* outer iterations of blocks that have a predecessor            */
  int32_t m;         /* Chebyshev degree of one filter pass, same blocks              */
  int32_t passes;    /* filter passes per iteration, same blocks (>= 1)               */
  int32_t T0;        /* the same three for blocks without a predecessor (and for      */
  int32_t m0;        /* every block under MI_WARM_GIVEN)                              */
  int32_t passes0;
  int32_t adapt;     /* 1: lower filter bound a <- largest Ritz value after each
                        Rayleigh-Ritz step; 0: keep the initial a                      */
  int32_t max_sweeps;/* cap on Jacobi sweeps per Rayleigh-Ritz step (e.g. 12)         */
  int32_t a_mode;    /* initial a of blocks that do not start from a predecessor:      */
                     /*   MI_A_WEYL: a_value * b * p_b / n_b                            */
                     /*   MI_A_ABS:  a_value                                            */
                     /*   MI_A_RITZ: largest entry of the block's `ritz` on input      */
                     /* (a block starting from predecessor P takes the largest Ritz    */
                     /*  value of P scaled by n_P / n_b)                               */
  int32_t rr_every;  /* 1: Rayleigh-Ritz on every iteration; 0: only on the last one
                        (the others end with a Cholesky-QR and take a from the
                        largest Rayleigh quotient of its basis)                    */
  int32_t eig;       /* eigen-solver of the Rayleigh-Ritz matrix: MI_EIG_TRIDIAG
                        (Householder tridiagonalisation, Sturm multisection and
                        inverse iteration; used when every ld_b <= 320, else the
                        Jacobi sweeps) or MI_EIG_JACOBI (parallel cyclic Jacobi) */
  int32_t autotune;  /* 1: when the plan is made (first call, or after the block
                        table, parameters or buffers change), time candidate launch
                        shapes of the Gram (split-K), the row product (output
                        width) and the SpMM (variant) per wave on the plan's own
                        tables and keep the fastest; 0: fixed heuristics.
                        The results agree to rounding (the Gram split changes the
                        summation order).  mi_oi_tuning reports the choice. */
  double a_value;
  double b_abs;      /* > 0: upper filter bound b for every block; else Gershgorin     */
  double jacobi_tol; /* off-diagonal threshold relative to ||A||_F on the last
                        iteration (e.g. 1e-14); earlier ones use max(tol, 1e-8)      */
  int32_t op;        /* operator of a filter pass: MI_OP_CHEB (the Chebyshev filter
                        above) or MI_OP_RZ: R^z = (L + delta I)^-z, Section 4's
                        operator, applied as z linear solves, each by cg_iters
                        iterations of column-wise conjugate gradients (FP64
                        scalars and column sums, reproducible) from a zero
                        start; each filter pass applies R^z, m only numbers
                        the coefficient slots then (m >= 1), and the
                        adjoint (mi_encdec_adjoint) rejects it            */
  int32_t z;         /* power of R (MI_OP_RZ), 1..16                               */
  int32_t cg_iters;  /* conjugate-gradient iterations per solve (MI_OP_RZ)         */
  int32_t persistent; /* 1: every filter pass (MI_OP_CHEB) of a wave whose blocks share
                        one ld (a multiple of 64 up to 320) runs as one persistent
                        launch: workgroups claim whole blocks from a device queue,
                        largest first, and run the pass's m Chebyshev steps on each
                        with workgroup barriers between steps.  The rows are those
                        of SPMM variants 7-12 (bit-identical to them); the tuned
                        SpMM variant still serves the Rayleigh-Ritz product.
                        Other waves, and 0, launch each step over the whole wave */
  double delta;      /* shift of R (MI_OP_RZ), > 0                                  */
  double tol;        /* 0: fixed iteration counts (T, T0).  > 0: tolerance mode
                        (Section 4 leaves the number of iterations to the user):
                        every iteration ends with the Rayleigh-Ritz step and a
                        Cholesky-QR, then the residuals r_j = ||L v_j - theta_j v_j||
                        of the Ritz pairs; a block whose kept pairs j < c_b satisfy
                        max_j r_j <= tol |theta_{p_b - 1}| is converged, and its
                        basis, Ritz values and residuals of that iteration are the
                        output (later iterations do not change them).  T and T0
                        cap the iterations; a block still unconverged there
                        returns its last iterate with MI_BLOCK_UNCONVERGED.  The
                        launch sequence stays fixed (converged blocks keep being
                        iterated in the batch, their output is frozen)          */
  uint64_t seed;     /* seed of the MI_RANDOM start                                 */
} mi_oi_params;

#define MI_OP_CHEB 0
#define MI_OP_RZ 1

#define MI_A_WEYL 0
#define MI_A_ABS 1
#define MI_A_RITZ 2

#define MI_EIG_TRIDIAG 0
#define MI_EIG_JACOBI 1

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device` (owns the launch plans, captured
 * graphs and a device copy of block tables).  Synchronous. */
mi_status mi_ctx_create(mi_ctx** out, int32_t device);
mi_status mi_ctx_destroy(mi_ctx* ctx);
/* Message of the last error on the calling thread ("" if none). */
const char* mi_last_error(void);
/* Library version string. */
const char* mi_version(void);

/* Kernel classes of the per-kernel event timer. */
enum {
  MI_K_SPMM = 0,       /* Chebyshev step / W = L Y over the vertex slab */
  MI_K_GRAM,           /* Y^T Y (and Y^T W) partial products over the slab */
  MI_K_GRAM_SMALL,     /* products of p x p FP64 matrices (Rayleigh-Ritz) */
  MI_K_GRAM_REDUCE,    /* fixed-order reduction of the Gram partials */
  MI_K_CHOL,           /* Cholesky factor and triangular inverse of the Gram */
  MI_K_ROWMUL,         /* slab times p x p matrix (basis update) */
  MI_K_ROWMUL_SMALL,   /* p x p times p x p */
  MI_K_RQ_MAX,         /* largest Rayleigh quotient (filter bound) */
  MI_K_JACOBI_INIT,    /* pack the Rayleigh-Ritz matrix */
  MI_K_JACOBI_SWEEP,   /* one parallel cyclic Jacobi sweep */
  MI_K_APPLY_ROT,      /* accumulate one sweep's rotations */
  MI_K_RR_FINISH,      /* Ritz values, order, filter bound */
  MI_K_PERM_CAST,      /* reorder / cast the Ritz rotation */
  MI_K_SETUP,          /* bounds, coefficients, warm-start copies, fills */
  MI_K_PROJECT,        /* E = U^T X */
  MI_K_RECONSTRUCT,    /* Xr = U E */
  MI_K_EIG_REDUCE,     /* Householder tridiagonalisation of the Rayleigh-Ritz matrix */
  MI_K_EIG_VALUES,     /* its eigenvalues by Sturm multisection */
  MI_K_EIG_VECTORS,    /* eigenvectors of the tridiagonal matrix */
  MI_K_EIG_BACK,       /* back-transformation by the reflectors */
  MI_K_MERGE,          /* degree-weighted merge of overlapped submeshes */
  MI_K_QUANTIZE,       /* uniform quantisation of the feature vectors */
  MI_K_QUALITY,        /* whole-mesh NMSVE and face-normal angle */
  MI_K_DOI,            /* decisions of the dynamic walk (Alg. 2) */
  MI_K_CG,             /* conjugate-gradient updates of R^z */
  MI_K_CHEB_PASS,      /* a whole filter pass in one persistent launch (persistent = 1) */
  MI_K_COUNT
};
/* Name of a kernel class ("spmm", ...), NULL when out of range. */
const char* mi_kernel_class_name(int32_t k);
/* Per-kernel timing, for measurement.  With on != 0 the context's later
 * mi_oi_track, mi_project, mi_reconstruct and mi_merge_overlapped calls
 * launch eagerly (no graph
 * replay) and bracket every kernel launch with a pair of HIP events on the
 * caller's stream; totals restart from zero.  on = 0 stops timing and frees
 * the events.  Synchronous. */
mi_status mi_ctx_set_timing(mi_ctx* ctx, int32_t on);
/* Launch-shape override, for measurement and for checking the variants
 * against each other: tracking plans made after the call (the plan is
 * rebuilt when the variant differs) run the wavefront-per-row SpMM as
 * `variant` (the codes of mi_oi_tuning, 0..12) in every wave that uses it,
 * whatever the autotuner would pick; -1 restores the autotuner or the
 * default.  MI_ERR_ARG for other values.  Host only. */
mi_status mi_oi_force_spmm(mi_ctx* ctx, int32_t variant);
/* Sums of the event-timed kernel durations (ms) and launch counts per class
 * since timing was switched on: total_ms and launches hold MI_K_COUNT
 * entries (host arrays).  Waits for the recorded events.  MI_ERR_ARG when
 * timing is off. */
mi_status mi_ctx_kernel_times(mi_ctx* ctx, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------- Laplacian
 * Section 3, Eq. 1-2: edge set E derived from the faces, L = D - C.  The
 * block's graph is the subgraph induced by its vertices: every edge of a
 * primitive whose two corners are in the block (corner id -1 marks a corner
 * outside the block; its edges are dropped).  Self loops are dropped and
 * duplicate edges merged.  Weighted modes use D_ii = sum_j C_ij so that L is
 * a true Laplacian (rows sum to zero).
 *
 * prims    device int32 [prim_off[B]][arity], arity 3 (faces) or 2 (edges),
 *          block-local corner ids in [-1, n_b).
 * prim_off host int64 [B+1], first primitive of each block.
 * Canonical edges of a block: (i, j), i < j, sorted lexicographically. */

/* Workspace bytes for the two calls below. */
mi_status mi_laplacian_workspace_size(const mi_blocks* blk, const int64_t* prim_off,
                                      int32_t arity, size_t* ws_bytes);

/* Counts the CSR entries and canonical edges of every block.  Writes host
 * nnz_off[B+1] and edge_off[B+1] (offsets into col/val and edges).
 * Synchronous (waits for the stream).  MI_ERR_INDEX if a corner id is out of
 * range. */
mi_status mi_build_laplacian_count(mi_ctx* ctx, const mi_blocks* blk, const int64_t* prim_off,
                                   const int32_t* prims, int32_t arity, int64_t* nnz_off,
                                   int64_t* edge_off, void* ws, size_t ws_bytes, void* stream);

/* Builds the CSR (row_ptr int32 [v_off[B]+B], col int32 / val float
 * [nnz_off[B]]) and the canonical edges (edges int32 [edge_off[B]][2] block-
 * local, edge_w float [edge_off[B]] = C_ij).  coords: device float [v_off[B]][3]
 * (read for the distance modes, may be NULL otherwise); user_w: device float
 * per canonical edge for MI_W_USER (else NULL).  Structure is bit-exact;
 * weights are computed in FP64 and rounded once.  Synchronous; returns
 * MI_ERR_INDEX / MI_ERR_DEGENERATE for bad input. */
mi_status mi_build_laplacian(mi_ctx* ctx, const mi_blocks* blk, const int64_t* prim_off,
                             const int32_t* prims, int32_t arity, const int64_t* nnz_off,
                             const int64_t* edge_off, int32_t weight_mode, const float* coords,
                             const float* user_w, int32_t* row_ptr, int32_t* col, float* val,
                             int32_t* edges, float* edge_w, void* ws, size_t ws_bytes,
                             void* stream);

/* Recomputes only the values (val, edge_w) on an existing structure (row_ptr,
 * col, edges from mi_build_laplacian), e.g. for a new frame of a mesh with
 * fixed connectivity (Section 7.3).  Enqueue only; a zero-length edge sets
 * *err_flag (device int32, may be NULL) to MI_ERR_DEGENERATE. */
mi_status mi_laplacian_values(mi_ctx* ctx, const mi_blocks* blk, const int64_t* nnz_off,
                              const int64_t* edge_off, int32_t weight_mode, const float* coords,
                              const float* user_w, const int32_t* row_ptr, const int32_t* col,
                              const int32_t* edges, float* val, float* edge_w, int32_t* err_flag,
                              void* stream);

/* ---------------------------------------------------------------- tracking
 * Section 4, Algorithm 1: U(t) = Onorm(R^z U(t-1)) started from the
 * previous block's subspace.  Here the operator is a polynomial filter of L
 * (Chebyshev polynomial of degree m, damping [a, b] and amplifying the low
 * end of the spectrum; applied `passes` times per iteration by CSR SpMMs,
 * with a span-preserving Cholesky-QR between passes), Onorm is Cholesky-QR
 * with an FP64 Cholesky of an FP64-accumulated Gram matrix, and every
 * iteration ends with a Rayleigh-Ritz step (FP64 Jacobi eigen-solve of the
 * p x p projected matrix) that orders the basis by Ritz value, so the first
 * c columns are the tracked U_c.  A final Cholesky-QR pass re-orthonormalises
 * the output without changing the span of any leading column set.
 *
 * Blocks are processed in waves: a block runs once its predecessor has
 * finished (Section 4: the first block from its own start, the others in
 * topological order); all blocks of a wave run in the same launches.
 *
 * val       device float [nnz] Laplacian values (FP32; promoted exactly in FP64 mode)
 * V0        device [u_off[B]] start slabs (double for MI_FP64, else float);
 *           MI_WARM_GIVEN: all blocks; MI_WARM_PRED: blocks without predecessor;
 *           MI_RANDOM: not read (may be NULL).
 * V         device [u_off[B]] output slabs, same type (may alias V0).
 * ritz      device double [sum p_b] Ritz values per block, ascending
 *           (block b at sum_{b'<b} p_b').
 * resid     device double [sum p_b] residual norms ||L v_j - theta_j v_j||_2 of
 *           the returned pairs (same layout as ritz), or NULL (then not
 *           computed; required in tolerance mode).
 * iters     device int32 [B] iterations whose result is returned: the first
 *           iteration meeting tol in tolerance mode (the cap when none did),
 *           else the fixed count; or NULL.
 * status    device int32 [B] MI_BLOCK_* flags (valid after the stream syncs).
 * Workspace from mi_oi_workspace_size.  Enqueue only.  The launch sequence
 * is captured into a HIP graph per context and replayed while the block
 * table, parameters and pointers stay the same. */
mi_status mi_oi_workspace_size(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                               size_t* ws_bytes);
/* Launch shapes of the context's current tracking plan, four int32 per wave
 * (Gram split-K target in workgroups, row-product output width, SpMM elements
 * per lane or 0 for the generic kernel, SpMM variant: 0 one row per
 * wavefront gathering 8 neighbour rows at a time, 1 the same gathering 4,
 * 2 two rows per wavefront, 3 one row per wavefront in 4-wavefront
 * workgroups, 4 and 5 two and four rows per wavefront one after the other
 * with their indices loaded first, 6 the same with two rows in
 * 4-wavefront workgroups; 7 to 10 one row per wavefront gathering only the
 * off-diagonal entries, in the difference form sum_j L_rj (Y_j - Y_r) plus
 * the row sum times Y_r (more accurate for the smooth iterates of a
 * Laplacian),
 * over consecutive rows in workgroups of 8 (7, 9), 16 (8) or 4 (10)
 * wavefronts, the previous iterate and the output streamed non-temporally
 * except in 9; 11 and 12 the same with half a wavefront per row (two rows
 * per wavefront, twice the elements per lane; rows of up to 256 columns,
 * wider ones as 7) in workgroups of 8 and 4 wavefronts; 7 to 12 give the
 * same bits; -1 the default, 7) for up to `cap` waves;
 * *n_waves gets the plan's wave count.  Variants 0 to 6 give bit-identical
 * results, and so do 7 to 12 among themselves.  Host only. */
mi_status mi_oi_tuning(mi_ctx* ctx, int32_t* out, int32_t cap, int32_t* n_waves);

mi_status mi_oi_track(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                      const int32_t* row_ptr, const int32_t* col, const float* val,
                      const int64_t* nnz_off, const void* V0, void* V, double* ritz,
                      double* resid, int32_t* iters, int32_t* status, void* ws,
                      size_t ws_bytes, void* stream);

/* Same computation without the persistent graph and with one block per
 * launch sequence: the "plain per-block GPU OI" reference the batched path
 * is measured against.  Same arguments and results. */
mi_status mi_oi_track_per_block(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                                const int32_t* row_ptr, const int32_t* col, const float* val,
                                const int64_t* nnz_off, const void* V0, void* V, double* ritz,
                                double* resid, int32_t* iters, int32_t* status, void* ws,
                                size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- dynamic OI
 * Section 5, Algorithm 2 (dynamic OI), with the branches as the text states
 * them: every iteration U(t) = Onorm(F(L) U(t-1)), with F the tracking
 * path's filter (`passes` Chebyshev passes of degree m on [a, b], as in
 * mi_oi_track; no Rayleigh-Ritz step), then the Eq. 6 residual
 *   e = sum over x, y, z of (v_j - U U^T v_j)      (v_j: the block's coordinates)
 * decides: ||e|| > eps_h and c < min(c_max, p_b): append e/||e|| as column c
 * (Eq. 7; the next Onorm orthonormalises it), c <- c + 1; ||e|| < eps_l and
 * c > 1: drop column c - 1, c <- c - 1; otherwise stop.  A block stops at
 * the latest after t_max iterations, with the last decision applied.
 * Blocks run in waves as in mi_oi_track; under MI_WARM_PRED a block starts
 * from its predecessor's final basis (index-aligned rows, re-orthonormalised)
 * and final c, blocks without predecessor from V0 and their c on input.
 * The active columns are the first c of the slab; the others are zero.
 * X       device float [v_off[B]][3] block coordinates (Eq. 6's v).
 * V0      start slabs as for mi_oi_track; must not alias V.
 * V       device slabs out: the final bases (columns >= c_b zero).
 * c       device int32 [B]: start sizes in (blocks without predecessor),
 *         final sizes out.
 * traj    device double [B][t_max][2]: (c, ||e||) before every decision,
 *         (-1, -1) after the block stopped.
 * iters   device int32 [B]: iterations run.
 * status  device int32 [B] MI_BLOCK_* flags (MI_BLOCK_NOT_PD is cleared:
 *         the zero columns read as rank deficiency).
 * prm     as for mi_oi_track except that T, rr_every, eig, max_sweeps and
 *         jacobi_tol are unused and a_mode MI_A_RITZ is rejected; with
 *         adapt = 1, a follows the largest Rayleigh quotient of the basis.
 * Every ld_b <= 1024.  Workspace from mi_doi_workspace_size (the tracking
 * workspace plus one slab and B flags).  Runs eagerly on the stream (no
 * graph) and synchronises it after every iteration to read the stop flags:
 * a wave ends as soon as all its blocks have stopped.  Returns when the
 * walk is complete. */
typedef struct {
  double eps_l, eps_h; /* band of ||e||_2, 0 <= eps_l <= eps_h                     */
  int32_t c_max;       /* upper limit of c (with p_b)                             */
  int32_t t_max;       /* iteration limit per block                               */
} mi_doi_params;

mi_status mi_doi_workspace_size(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                                const mi_doi_params* dp, size_t* ws_bytes);
mi_status mi_doi_track(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                       const mi_doi_params* dp, const int32_t* row_ptr, const int32_t* col,
                       const float* val, const int64_t* nnz_off, const float* X, const void* V0,
                       void* V, int32_t* c, double* traj, int32_t* iters, int32_t* status,
                       void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- Ritz residuals
 * Section 4 (how many iterations the orthogonal iteration needs): the
 * accuracy of a tracked pair (theta_j, v_j) is measured by its residual
 * norm r_j = || L v_j - theta_j v_j ||_2, which bounds the distance of
 * theta_j to the spectrum of L; a caller iterates until every kept pair
 * meets its tolerance.  For every block b and column j < p_b:
 *   resid[t_off_b + j] = || L_b V_b[:, j] - ritz[t_off_b + j] V_b[:, j] ||_2
 * with L_b the CSR block Laplacian (layout as for mi_oi_track), V the slab
 * (element type float for MI_FP32, double for MI_FP64), ritz and resid
 * device double [sum p_b].  Products and sums are FP64; the column sums are
 * reduced in a fixed order (tile partials in the workspace, then one pass
 * per block), so results are reproducible.  Workspace (device, no alignment
 * beyond 8 bytes) from mi_residual_workspace_size; MI_ERR_WORKSPACE if
 * smaller.  Enqueue only. */
mi_status mi_residual_workspace_size(mi_ctx* ctx, const mi_blocks* blk, size_t* ws_bytes);
mi_status mi_ritz_residuals(mi_ctx* ctx, const mi_blocks* blk, int32_t precision,
                            const int32_t* row_ptr, const int32_t* col, const float* val,
                            const int64_t* nnz_off, const void* V, const double* ritz,
                            double* resid, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- adjoint of encode / decode
 * Gradient of loss = <Gbar, X~> for X~_b = U_c U_c^T X_b (Section 3 GFT and
 * inverse GFT, Section 7.1 truncation to c_b), where U_c holds the first c_b
 * Ritz vectors that mi_oi_track computes with `prm` (Section 4, Alg. 1:
 * T0 iterations of passes0 Chebyshev passes of degree m0 for the blocks
 * started from V0 or the seeded start, T of passes of degree m for blocks
 * warm-started from their predecessor under MI_WARM_PRED; Cholesky-QR
 * between passes, Rayleigh-Ritz at the end).  The paper does not
 * differentiate its method; the derivative is that of the unrolled
 * iteration, with respect to the coordinates X and to the edge weights w of
 * L = sum_e w_e (e_a - e_b)(e_a - e_b)^T (Eq. 1-2).  The gradient is stopped
 * at every block's start basis (V0, the seeded start, or the predecessor's
 * result) and at the filter interval of every iteration (the Gershgorin or
 * given b, the initial a of a_mode, and with adapt = 1 the Rayleigh-quotient
 * updates of a): these are recorded in the forward and held constant.
 * The call replays the tracking with checkpoints (every pass input, the
 * Cholesky-QR factors, the coefficients of every iteration and the
 * Rayleigh-Ritz rotation) in its workspace, then runs the reverse sweep
 * wave by wave, every wave's blocks batched in each launch.
 * Requires tol = 0, op = MI_OP_CHEB, rr_every = 0, eig = MI_EIG_TRIDIAG,
 * precision MI_FP32 or MI_FP64, T0 >= 1 (and T >= 1 when blocks are
 * warm-started) and every ld_b <= 192 (else MI_ERR_ARG).
 * mode      weight mode the CSR values were built with: for MI_W_INV_SQ_DIST
 *           and MI_W_INV_DIST the weights depend on X and Xbar includes that
 *           path; MI_W_COMBINATORIAL / MI_W_USER weights are independent of X.
 * row_ptr, col, val, nnz_off   the block Laplacians (layout as mi_oi_track);
 * edges     device int32 [sum |E_b|][2] canonical edges (a < b, block-local)
 *           at edge_off[b] (host int64 [B+1]), as mi_build_laplacian emits.
 * V0        device start slab (precision's element type), as for mi_oi_track
 *           (may be NULL under MI_RANDOM).
 * X, Gbar   device [v_off[B]][3] coordinates and d loss/d X~ (element type).
 * c         device int32 [B], 1 <= c_b <= p_b.
 * Xbar      device double [v_off[B]][3]: d loss/d X.
 * wbar      device double [sum |E_b|]: d loss/d w_e per canonical edge (for
 *           distance weights: the gradient at the weights before the chain
 *           rule into X, which Xbar already includes).
 * Workspace from mi_adjoint_workspace_size (holds about
 * (max(T0*passes0, T*passes) + max(m0, m) + 10) slabs).  Enqueue only;
 * eager launches. */
mi_status mi_adjoint_workspace_size(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                                    const int64_t* nnz_off, size_t* ws_bytes);
mi_status mi_encdec_adjoint(mi_ctx* ctx, const mi_blocks* blk, const mi_oi_params* prm,
                            int32_t mode, const int32_t* row_ptr, const int32_t* col,
                            const float* val, const int64_t* nnz_off, const int32_t* edges,
                            const int64_t* edge_off, const void* V0, const void* X,
                            const int32_t* c, const void* Gbar, double* Xbar, double* wbar,
                            void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- encode / decode
 * Section 3 (GFT v_bar = U^T v, inverse GFT v = U v_bar) and Section 7.1
 * (E[i] = U_c^T v[i], v~[i] = U_c E[i]).  c: device int32 [B], 1 <= c_b <= p_b.
 * X, Xr: device [v_off[B]][3]; E: device [sum p_b][3] (rows k >= c_b are
 * written as zero: the truncation).  Element type float (MI_FP32) or double
 * (MI_FP64) for X, E, Xr and U.  Workspace from mi_encdec_workspace_size. */
mi_status mi_encdec_workspace_size(mi_ctx* ctx, const mi_blocks* blk, int32_t precision,
                                   size_t* ws_bytes);
mi_status mi_project(mi_ctx* ctx, const mi_blocks* blk, int32_t precision, const int32_t* c,
                     const void* U, const void* X, void* E, void* ws, size_t ws_bytes,
                     void* stream);
mi_status mi_reconstruct(mi_ctx* ctx, const mi_blocks* blk, int32_t precision, const int32_t* c,
                         const void* U, const void* E, void* Xr, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * projection of mi_project, same arguments, layouts and result (the same
 * kernels, bit for bit), with no workspace argument and no allocation of
 * any kind.  Its block table and FP64 partial sums live in a fixed 16 MiB
 * array in device memory that the library holds on every device it runs on
 * until the process ends; the table is staged into it through kernel
 * arguments.  Needs 48 B per block plus 16 x ld_b x 3 x 8 B of partials
 * per block (about 170 blocks at ld = 256, 220 at ld = 192); a larger
 * block table returns MI_ERR_WORKSPACE before anything is enqueued.  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (different streams, or host threads) race and must not be issued;
 * calls on one stream are ordered.  Nothing in the array must start at zero
 * (every partial is written before it is read).  Enqueue only. */
mi_status mi_project_noalloc(mi_ctx* ctx, const mi_blocks* blk, int32_t precision,
                             const int32_t* c, const void* U, const void* X, void* E,
                             void* stream);

/* ---------------------------------------------------------------- merge of overlapped submeshes
 * Section 6.1, Alg. 3: the submeshes overlap (each part extended with the
 * neighbours of its boundary vertices to n_d vertices), so a mesh vertex can
 * have several reconstructions.  Its merged position is their average, each
 * weighted by the vertex's degree in that submesh: the number of its
 * neighbours there, i.e. the entries of its Laplacian row minus the
 * diagonal.  Sums run in FP64 over the submeshes in ascending block order,
 * so the result is bitwise reproducible.  A vertex whose weights are all
 * zero (isolated in every submesh that holds it) gets the plain mean of its
 * reconstructions; a vertex in no submesh gets 0.
 * gid        host int32 [v_off[B]]: the mesh vertex of every block row (row i
 *            of block b at v_off[b] + i), in [0, n_vertices).
 * n_vertices mesh vertex count, < 2^31.
 * row_ptr    device int32: the blocks' Laplacian row pointers as
 *            mi_build_laplacian writes them (n_b + 1 entries per block, block
 *            b starting at v_off[b] + b).
 * Xr         device float [v_off[B]][3]: reconstructed block coordinates
 *            (the output of mi_reconstruct).
 * Xout       device float [n_vertices][3]: merged mesh coordinates.
 * The occurrence table is built on the host from gid on the first call for
 * a given (v_off, gid, n_vertices) and cached in the context (synchronous
 * upload); later calls only enqueue the kernel.  MI_ERR_INDEX when a gid
 * entry is out of range. */
mi_status mi_merge_overlapped(mi_ctx* ctx, const mi_blocks* blk, const int32_t* gid,
                              int64_t n_vertices, const int32_t* row_ptr, const float* Xr,
                              float* Xout, void* stream);

/* ---------------------------------------------------------------- quantisation
 * Section 8 (compression): the feature vectors E are quantised uniformly
 * with qbits bits (12 in the paper's experiments).  For each block and
 * coordinate axis the first c_b coefficients are mapped onto 2^qbits levels
 * spanning their range [lo, hi]: step = (hi - lo) / (2^qbits - 1),
 * code = rint((e - lo) / step) (ties to even, clamped to the levels; every
 * code 0 when step is 0), dequantised e' = lo + code * step.  All in FP32,
 * each operation rounded on its own, so the result is reproducible bit for
 * bit.  The rate is 3 * qbits * sum_b c_b bits for the whole mesh (plus the
 * per-block ranges).
 * c       device int32 [B], 0 <= c_b <= p_b.
 * E       device float [sum p_b][3] (from mi_project; rows >= c_b are ignored).
 * codes   device uint16 [sum p_b][3]; rows >= c_b are written as 0.
 * params  device float [B][3][2]: (lo, step) of every block and axis.
 * Eq      device float [sum p_b][3] or NULL: the dequantised coefficients
 *         (rows >= c_b zero), ready for mi_reconstruct.
 * qbits in [1, 16].  Enqueue only. */
mi_status mi_quantize(mi_ctx* ctx, const mi_blocks* blk, const int32_t* c, int32_t qbits,
                      const float* E, uint16_t* codes, float* params, float* Eq, void* stream);

/* ---------------------------------------------------------------- quality report
 * Section 8: the reconstruction quality of a whole mesh.
 *   NMSVE = ( ||v - v~||_2 + ||GL(v) - GL(v~)||_2 ) / (2n)          (Eq. 16)
 *   GL(v)_i = v_i - sum_j d_ij^-1 v_j / sum_j d_ij^-1, j over the neighbours of i,
 * over the 3n-vectors of coordinates, with the edge lengths d_ij of the
 * ORIGINAL mesh X for both operands (GL is one linear operator; a vertex
 * without neighbours keeps GL(v)_i = v_i).  theta = the angle between the
 * normal (x_b - x_a) x (x_c - x_a) of every face in X and in Xr, averaged
 * over the faces whose normal is nonzero on both sides, in degrees.  All
 * sums in FP64 over a fixed grid, bitwise reproducible.
 * row_ptr  device int32 [n_vertices + 1], col device int32 [nnz]: the
 *          neighbour lists of the mesh vertices (entries with col == row,
 *          such as a Laplacian's diagonal, are skipped), e.g. the Laplacian
 *          mi_build_laplacian writes for one block holding the whole mesh.
 * faces    device int32 [n_faces][3], mesh vertex ids.
 * X, Xr    device float [n_vertices][3]: original and reconstructed mesh.
 * out      device double [8], written by the stream: NMSVE, 10 log10 NMSVE,
 *          ||v - v~||_2, ||GL(v) - GL(v~)||_2, theta (degrees; 0 when no
 *          face counts), faces averaged, zero-length edges, out-of-range
 *          indices.  A zero-length edge or an index outside [0, n_vertices)
 *          (counted in out[6] / out[7] and skipped, never dereferenced)
 *          makes the NMSVE entries and theta NaN.
 * The first call on a context allocates its partial-sum buffer (48 KiB);
 * later calls only enqueue two kernels. */
mi_status mi_mesh_quality(mi_ctx* ctx, int64_t n_vertices, const int32_t* row_ptr,
                          const int32_t* col, int64_t nnz, int64_t n_faces, const int32_t* faces,
                          const float* X, const float* Xr, double* out, void* stream);

/* ---------------------------------------------------------------- choice of c
 * Section 5 (smallest subspace meeting a reconstruction-quality target) with
 * the NMSVE of Eq. 16 as the quality measure: for every c in 1..c_max the
 * library evaluates NMSVE(c) = (||X - U_c U_c^T X|| + ||GL X - GL U_c U_c^T X||)/(2n)
 * from prefix sums of the projected coefficients and a quadratic form on the
 * Gram of GL U (GL with the 1/d weights of the original mesh: the CSR
 * gl_row_ptr/gl_col/gl_val of an MI_W_INV_DIST Laplacian).  c_b is the
 * smallest c meeting `target` (c_max if none), moved up to the first c with
 * a relative Ritz gap (theta_{c+1}-theta_c)/theta_{c+1} >= g_min.
 * c_max: device int32 [B] per-block cap (<= p_b).  c_out: device int32 [B];
 * metric_out: device double [sum p_b] NMSVE(c) for c = 1..p_b (entries past
 * c_max_b undefined).  FP32 only.  Enqueue only. */
mi_status mi_choose_c_workspace_size(mi_ctx* ctx, const mi_blocks* blk, size_t* ws_bytes);
mi_status mi_choose_c(mi_ctx* ctx, const mi_blocks* blk, const int32_t* c_max, double target,
                      double g_min, const float* U, const double* ritz, const float* X,
                      const int32_t* gl_row_ptr, const int32_t* gl_col, const float* gl_val,
                      const int64_t* nnz_off, int32_t* c_out, double* metric_out, void* ws,
                      size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MISPECTRAL_H */
