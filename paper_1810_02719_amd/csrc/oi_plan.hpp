// Plans of the eigenspace tracking (oi.hip), shared with the adjoint
// (adjoint.hip), which replays the same forward with checkpoints.
#pragma once

#include <vector>

#include "dense.hpp"
#include "small.hpp"

namespace mis {

struct BlkInfo {
  int64_t t_off;
  int32_t n, p, pred, c;  // c: kept pairs of the tolerance test
};

struct WaveTables {
  int nb = 0;
  int T = 0, m = 0, passes = 0;
  bool from_pred = false;
  int max_ld = 0, max_q = 0, max_p = 0;
  int nch = 64, nchs = 64;
  int epl = 0;  // elements per lane of the row-per-wavefront SpMM (0: generic kernel)
  int spmm_var = -1;  // SpMM variant (SPMM_VAR_*; -1: the default for epl)
  int gram_target = GRAM_TARGET;  // workgroups of the split Gram launch
  bool gram_direct = false;        // no super-tile split: the Gram writes G itself
  int lane = 0;  // stream lane: the waves of one lane form one dependency chain
  bool persistent = false;  // filter passes as one persistent launch each
  int pgrid = 0;            // its workgroups
  std::vector<MatDesc> tall_host;  // host copy of `tall` (for retuning)
  // device tables
  MatDesc *tall = nullptr, *ptall = nullptr, *small = nullptr;
  CsrDesc* csr = nullptr;
  SmallDesc* sd = nullptr;
  SpmmTile* spmm = nullptr;
  int n_spmm = 0;
  GramTile* gt = nullptr;
  int n_gt = 0;
  GramReduce* gr = nullptr;
  int n_gr = 0;
  GramTile* gts = nullptr;
  int n_gts = 0;
  GramReduce* grs = nullptr;
  int n_grs = 0;
  RowTile* rt = nullptr;
  int n_rt = 0;
  RowTile* rts = nullptr;
  int n_rts = 0;
  int32_t* porder = nullptr;  // persistent pass: indices into `tall`, largest block first
};

struct WsLayout {
  size_t slab[4], G, H, Rinv, T1, A, Z, S64, S32, Wk, pk, log, perm, tri, part, a_lo, b_hi, coef,
      conv;
  size_t cg_part;    // R^z: three tile-partial buffers [tiles][cg_ldp] (0 without R^z)
  size_t rpart;      // residual norms: per-tile column partials [tiles][cg_ldp]
  // tolerance mode only (zero-size otherwise): the working basis, Ritz values
  // and residuals of the current iteration, and per-block flags (frozen,
  // frozen in this iteration)
  size_t slab_w, ritz_w, resid_w, frozen, fnow;
  int cg_ldp = 0;    // largest ld (row stride of the partials)
  int64_t cg_tiles = 0;  // 16-row tiles of all blocks
  size_t part_lane;  // Gram partial doubles of one stream lane
  size_t queue;      // persistent passes: one int32 queue head per stream lane
  size_t total;
  int coef_stride;
};

// Launch shape of one wave (the autotuner's choices).
struct WaveTune {
  int gram_target;  // split-K target of the Gram
  int nch;          // output-column width of the row product
  int epl;          // row-per-wavefront SpMM elements per lane (0: generic)
  int spmm_var;     // SpMM variant (SPMM_VAR_*, -1: the default for epl)
};

struct OiPlan {
  // key
  HostBlocks hb;
  std::vector<int64_t> nnz_off;
  mi_oi_params prm;
  std::vector<const void*> ptrs;
  size_t ws_bytes = 0;
  bool per_block = false;
  int spmm_force = -1;  // SpMM variant forced on every wave that uses the per-row kernels
  // content
  std::vector<WaveTables> waves;
  WsLayout L;
  void* arena = nullptr;
  BlkInfo* info = nullptr;
  int64_t* v_off = nullptr;  // first vertex row of every block [B + 1]
  int64_t* tile_base = nullptr;  // first 16-row tile of every block [B + 1]
  MatDesc* all_tall = nullptr;
  CsrDesc* all_csr = nullptr;
  int lds_max = 65536;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  // independent trees of the block forest run on separate stream lanes
  // inside the captured graph
  int n_lanes = 1;
  std::vector<hipStream_t> lane_s;
  std::vector<hipEvent_t> lane_ev;
  hipEvent_t fork_ev = nullptr;
  ~OiPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipStream_t x : lane_s) (void)hipStreamDestroy(x);
    for (hipEvent_t e : lane_ev) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (arena) (void)hipFree(arena);
  }
};

// Checkpoints of one recorded forward (single wave, MI_WARM_GIVEN, no
// adaptation of the filter interval): everything the reverse sweep needs.
// Checkpoints of the forward for the adjoint.  Pass j of a wave is the j-th
// filter pass of that wave's blocks (T passes-long per wave); every wave
// writes only its own blocks' rows and matrices, so the slots are shared.
struct OiRecord {
  void** X = nullptr;       // [npass] input basis of every filter pass (slab)
  void** S = nullptr;       // [npass-1] operand of the Cholesky-QR row product
                            // after pass j (ld x ld, slab element type)
  void* Y = nullptr;        // output of the last pass (slab)
  double* Rrr = nullptr;    // Rinv of the Rayleigh-Ritz step (FP64 ld x ld)
  double* Z = nullptr;      // Ritz vectors of A (FP64 ld x ld, ascending)
  double* coef = nullptr;   // filter coefficients [iteration][B][coef_stride]
  int npass = 0;            // passes of the longest wave
  int n_iter = 0;           // iterations of the longest wave
};

// The dynamic walk of Alg. 2 (mi_doi_track): the iteration count and the
// band of the Eq. 6 residual, the caller's buffers, and the workspace
// beyond the plan's own layout (frozen bases, stop flags).
struct DoiArgs {
  const float* X = nullptr;  // block coordinates [v_off[B]][3]
  int32_t* c = nullptr;      // [B] start size in, final size out
  double* traj = nullptr;    // [B][t_max][2]: (c, ||e||) before each decision
  int32_t* iters = nullptr;  // [B] iterations run
  double eps_l = 0, eps_h = 0;
  int c_max = 0, t_max = 0;
  size_t off_vf = 0, off_done = 0;  // workspace offsets
  int32_t* host_done = nullptr;     // pinned copy of the stop flags [B] (early exit)
};

struct Args {
  const int32_t* row_ptr;
  const int32_t* col;
  const float* val;
  const void* V0;
  void* V;
  double* ritz;
  int32_t* status;
  char* ws;
  KTimer* tm;
  const OiRecord* rec;  // checkpoints to write (eager runs only), or null
  bool fork;            // run the plan's lanes on its lane streams (graph capture)
  const DoiArgs* doi = nullptr;  // the walk of Alg. 2 instead of fixed iterations
  double* resid = nullptr;       // residual norms of the returned pairs, or null
  int32_t* iters = nullptr;      // iterations of the returned result per block, or null
};

// Runs the tracking eagerly on `s` with the plan held in *slot (created or
// rebuilt as needed; ws must hold the plan's workspace), recording into
// *rec when it is non-null.
mi_status oi_run_plan(mi_ctx* ctx, void** slot, const HostBlocks& hb,
                      const std::vector<int64_t>& nnz, const mi_oi_params& prm,
                      const int32_t* row_ptr, const int32_t* col, const float* val,
                      const void* V0, void* V, double* ritz, int32_t* status, void* ws,
                      size_t ws_bytes, const OiRecord* rec, hipStream_t s, OiPlan** plan_out);
// Workspace bytes of the plan for (hb, prm).
size_t oi_ws_bytes(const HostBlocks& hb, const mi_oi_params& prm);
mi_status oi_check_params(const mi_oi_params* prm);

}  // namespace mis
