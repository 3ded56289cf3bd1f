// Internal declarations shared by the translation units of the library: the
// plan object behind the opaque dnls_plan handle, error reporting, and the
// entry points of the bundle-adjustment (Schur) path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dnls.h"

namespace dnls {

extern thread_local std::string g_err;

inline dnls_status fail(dnls_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::dnls::fail(DNLS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Poll limit of the waits between co-resident workgroups (DNLS_FLAG_PAIR):
// the environment variable DNLS_PAIR_SPIN (a positive count) overrides the
// default, which lets tests drive the give-up path without a real fault.
inline int pair_spin_limit() {
  const char* e = std::getenv("DNLS_PAIR_SPIN");
  const long v = e ? std::strtol(e, nullptr, 10) : 0;
  return v > 0 && v < (1L << 30) ? (int)v : (1 << 24);
}

// one pose graph of the dense path
struct GraphDesc {
  int pose0, npose, edge0, nedge, prior0, nprior, n, npad;
  long long fac_off;   // doubles: L ((npad + 16) x npad) then the 64x64 panel inverses
  long long h_off;     // doubles: assembled H ((npad + 16) x npad) in the solve workspace
  long long dlm_winv_off;   // doubles: panel inverses of the DLM backward system
  int od0, nod;        // off-diagonal Hessian blocks of the graph
};

// one bundle-adjustment problem of the Schur path
struct BADesc {
  int cam0, ncam, pt0, npt, obs0, nobs, prior0, nprior, n, npad;
  long long fac_off;   // doubles: Schur factor ((npad + 16) x npad) then panel inverses
  int blk0, nblk;      // camera-pair blocks of the Schur complement (lower, all)
  int lin_blk0, nlin_blk;   // linearisation thread blocks of this problem
};

// one pose graph of the block-sparse path
struct SpDesc {
  int pose0, npose, edge0, nedge, prior0, nprior, n;
  int P;               // tile rows = tile columns
  int ntile;           // non-zero tiles of the factor
  int tix_off;         // tile-id table [P x P] offset
  int col_off;         // column pointer offset (P + 1 entries)
  int row_off;         // row pointer offset (P + 1 entries)
  int od0, nod;        // off-diagonal Hessian blocks
  int nvec;            // vector length (P x tile size)
  long long vec_off;   // doubles: 4 vectors of nvec in the workspace
  long long pool_off;  // doubles: tile pool
  long long winv_off;  // doubles: inverses of the diagonal tiles
  int lvl_off, nlvl;   // BLOCK schedule: elimination-tree levels ([lvl_off, lvl_off + nlvl] pointers)
  // bundle adjustment on this solver: points [pt0, pt0 + npt), observations,
  // camera-point Hessian blocks [cp0, cp0 + ncp); unit diagonal on the
  // padding scalars [pad0, pad1) between the points and the cameras
  int pt0, npt, obs0, nobs, cp0, ncp, pad0, pad1;
};

}  // namespace dnls

struct dnls_plan_s {
  int B = 0, group = 3, d = 6, sz = 12;
  dnls_options opt{};
  int V = 0, E = 0, P = 0;
  int npad_max = 0;
  std::vector<dnls::GraphDesc> gd;
  size_t ws_bytes = 0, fac_bytes = 0, bwd_bytes = 0;
  double flops_alg = 0.0, flops_exec = 0.0;   // one numeric factorisation over the batch
  size_t ws32_off = 0, ycost_off = 0, h_off = 0, bak_off = 0, dlmw_off = 0, hvp_off = 0;
  long long traj_off = 0;   // doubles into the factor cache: kept iterates (DNLS_FLAG_KEEP_ITERATES)
  // DNLS_FLAG_PAIR: whether the pair kernel fits, its counters and launch epoch
  bool pair_ok = false;
  int ba_nway = 1;            // SCHUR: workgroups per problem in the factorisation
  int pair_spin = 1 << 24;    // polls of a wait between the workgroups of a graph (about a second)
  unsigned long long* d_pair = nullptr;
  unsigned long long pair_epoch = 0;   // byte offsets inside the solve workspace
  // device tables of the dense path
  dnls::GraphDesc* d_gd = nullptr;
  int* d_order = nullptr;
  int* d_edge_ij = nullptr;
  int* d_prior_var = nullptr;
  int* d_inc_off = nullptr;
  int* d_inc_slot = nullptr;
  int4* d_od_blk = nullptr;
  int* d_od_slot = nullptr;
  // bundle adjustment (solver SCHUR)
  int Vp = 0, O = 0;
  double intr[4] = {0, 0, 0, 0};
  double huber = 0.0;
  std::vector<dnls::BADesc> bd;
  int nlin_blocks = 0;
  dnls::BADesc* d_bd = nullptr;
  int* d_lin_prob = nullptr;      // problem of each linearisation thread block
  int* d_obs_cam = nullptr;
  int* d_obs_pt = nullptr;
  int* d_cam_obs_off = nullptr;   // per camera: observations, then priors
  int* d_cam_obs = nullptr;
  int* d_pt_obs_off = nullptr;
  int* d_pt_obs = nullptr;
  int4* d_sblk = nullptr;         // (row cam, col cam, start, count) per Schur block
  int2* d_spair = nullptr;        // (obs a, obs b) contributions
  size_t ba_off[17] = {0};        // byte offsets of the BA workspace regions
  size_t ba_fac_off[4] = {0};     // byte offsets of the BA backward cache inside the factor
  // block-sparse path (solver SPARSE)
  std::vector<dnls::SpDesc> sd;
  dnls::SpDesc* d_sd = nullptr;
  int* d_pos = nullptr;
  int* d_tix = nullptr;
  int* d_colptr = nullptr;
  int* d_rowidx = nullptr;
  int* d_rowptr = nullptr;
  int* d_rowcol = nullptr;
  int2* d_sn = nullptr;           // supernode (first, last tile column) of every tile column
  std::vector<int> sp_ntrsm;
  std::vector<int> sp_nrow;       // per tile row: widest row (off-diagonal tiles) over the batch
  std::vector<long long> sp_npair;
  int sp_maxP = 0;
  bool sp_solve_wg = false;       // triangular solves: one workgroup per graph (vector in LDS)
  bool sp_persistent = false;     // the whole solve in one persistent launch (graph work queue)
  int sp_ts = 48;                 // tile size of the factor: 48 (MFMA tiles) or d (pose blocks, BLOCK)
  bool sp_ba = false;             // bundle adjustment on the block-sparse solver (points eliminated first)
  int* d_soff_cam = nullptr;      // its scalar offset of every camera and point in the elimination order
  int* d_soff_pt = nullptr;
  int4* d_cp_blk = nullptr;       // (camera, point, first, count) per camera-point block
  int* d_cp_obs = nullptr;
  int* d_lvlptr = nullptr;        // BLOCK: columns of each level ([lvl_off + L] .. [+1] into d_lvlcol)
  int* d_lvlcol = nullptr;
  int* d_lvlbptr = nullptr;       // BLOCK: factor blocks of each level's columns (into d_lvlblk)
  int4* d_lvlblk = nullptr;       //   (tile id, update pairs [first, end) in d_cpair, 2 J + diagonal)
  int2* d_cpair = nullptr;        // BLOCK: (L_IK, L_JK) tile ids of the left-looking updates
  int* d_rowid = nullptr;         // BLOCK: tile id of every row-structure entry
  int sp_grid = 0;                // its workgroups: min(B, resident slots)
  int* d_sp_order = nullptr;      // its queue order: graphs by decreasing factor work
  unsigned* d_sp_queue = nullptr; // its two queue counters (self-resetting)
  bool sp_factor_wg = false;      // factorisation: one workgroup per graph
  size_t sp_off[18] = {0};
  std::vector<void*> allocs;
  // captured launch sequence of dnls_solve (DNLS_FLAG_GRAPH)
  std::mutex graph_mu;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<const void*> graph_key;   // argument pointers the graph was captured with
};

namespace dnls {

template <class T>
dnls_status upload(dnls_plan p, T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return DNLS_OK;
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(dst), v.size() * sizeof(T)));
  p->allocs.push_back(*dst);
  HIP_TRY(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return DNLS_OK;
}

dnls_status ba_plan_create(dnls_plan p, const dnls_problem* pr, const dnls_options* op);
dnls_status ba_solve(dnls_plan p, const dnls_solve_args* s, hipStream_t st);
dnls_status ba_backward(dnls_plan p, const dnls_backward_args* s, hipStream_t st);
dnls_status sp_plan_create(dnls_plan p, const dnls_problem* pr);
dnls_status sp_plan_create_ba(dnls_plan p, const dnls_problem* pr);
dnls_status sp_solve(dnls_plan p, const dnls_solve_args* s, hipStream_t st);
dnls_status sp_backward(dnls_plan p, const dnls_backward_args* s, hipStream_t st);

}  // namespace dnls
