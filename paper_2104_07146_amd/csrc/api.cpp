// C ABI of the H-MLE library: problem lifecycle, state machine, device
// memory, plan upload and the drivers of the assembly, factorisation and
// solve sweeps. Every numerical step runs in the HIP kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hmle.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "fit_support.hpp"

using namespace hmle;

namespace {

thread_local std::string g_last_error;

struct HipError {
  std::string msg;
  hmle_status code;
};

#define HIP_TRY(expr)                                                                                 \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      throw HipError{std::string(#expr) + ": " + hipGetErrorString(e_),                               \
                     e_ == hipErrorOutOfMemory ? HMLE_E_NOMEM : HMLE_E_HIP};                          \
  } while (0)

// Raise the first failed kernel launch since the last check, by name.
void check_launches() {
  const char* what = nullptr;
  const hipError_t e = take_launch_error(&what);
  if (e != hipSuccess)
    throw HipError{std::string("launch of ") + (what ? what : "a kernel") + ": " + hipGetErrorString(e),
                   e == hipErrorOutOfMemory ? HMLE_E_NOMEM : HMLE_E_HIP};
}

// Device memory of a problem: from the caller's allocator when one was given
// (alloc/free callbacks with the problem's stream), else hipMalloc/hipFree;
// every block is kept until the problem is destroyed.
struct DevPool {
  hmle_allocator al{};
  bool custom = false;
  hipStream_t stream = nullptr;
  std::vector<void*> owned;
  void* get(size_t bytes) {
    void* p = nullptr;
    if (custom) {
      p = al.alloc(bytes, stream, al.user);
      if (!p) throw HipError{"the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes",
                             HMLE_E_NOMEM};
    } else {
      HIP_TRY(hipMalloc(&p, bytes));
    }
    owned.push_back(p);
    return p;
  }
  // a temporary block, freed by the caller with temp_free (not kept)
  void* temp_alloc(size_t bytes) {
    void* p = nullptr;
    if (custom) return al.alloc(bytes, stream, al.user);
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
  }
  void temp_free(void* p) {
    if (custom) al.free(p, stream, al.user);
    else (void)hipFree(p);
  }
  void release_all() {
    for (void* p : owned) {
      if (custom) al.free(p, stream, al.user);
      else (void)hipFree(p);
    }
    owned.clear();
  }
};

template <typename T>
T* dev_alloc(size_t count, DevPool& owned) {
  if (count == 0) count = 1;
  return static_cast<T*>(owned.get(count * sizeof(T)));
}

template <typename T>
T* dev_upload(const std::vector<T>& v, hipStream_t st, DevPool& owned) {
  T* p = dev_alloc<T>(v.size(), owned);
  if (!v.empty()) HIP_TRY(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return p;
}

}  // namespace

namespace hmle {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace hmle

struct hmle_problem_s {
  std::string err;
  hipStream_t stream = nullptr;
  int32_t n = 0, dim = 0;
  hmle_opts opts{};
  ClusterTree tree;
  BlockTree bt;
  Plan plan;
  DevPool owned;
  // device structure
  int32_t* d_perm = nullptr;
  double* d_coords = nullptr;
  BlockDesc* d_blocks = nullptr;
  PairDesc* d_pairs = nullptr;
  int64_t* d_pair_beg = nullptr;
  int32_t *d_leaf_lo = nullptr, *d_leaf_hi = nullptr, *d_leaf_diag = nullptr;
  int64_t *d_leaf_inv_off = nullptr, *d_diag_off = nullptr;
  int32_t* d_active = nullptr;
  ChunkDesc *d_dchunks = nullptr, *d_r1chunks = nullptr, *d_r2chunks = nullptr;
  TargetDesc* d_dtargets = nullptr;
  RTargetDesc* d_rtargets = nullptr;
  RPairDesc *d_rpairs1 = nullptr, *d_rpairs2 = nullptr;
  GItem *d_g1 = nullptr, *d_g2 = nullptr;
  GFin *d_gf1 = nullptr, *d_gf2 = nullptr;
  void* d_gseg = nullptr;
  RowTile *d_t1 = nullptr, *d_t2 = nullptr;
  TileChunk *d_tc1 = nullptr, *d_tc2 = nullptr;
  TileSeg *d_sg1 = nullptr, *d_sg2 = nullptr;
  void* d_spart = nullptr;
  void *d_dpart = nullptr, *d_rpart = nullptr, *d_gbuf = nullptr, *d_gram = nullptr;
  double *d_gpart = nullptr, *d_qbuf = nullptr;
  int32_t* d_qint = nullptr;
  PairDesc* d_grams = nullptr;
  InnerDesc* d_inner = nullptr;
  InnerDesc* d_tsolve = nullptr;
  InnerDesc* d_fsolve = nullptr;
  int32_t *d_rowp_beg = nullptr, *d_rowp = nullptr;
  int32_t *d_colp_beg = nullptr, *d_colp = nullptr;
  double* d_mvh = nullptr;                     // H-matrix-vector product: two short vectors per low-rank block
  double* d_h = nullptr;
  // device numerical storage
  void *d_L = nullptr, *d_A = nullptr, *d_S = nullptr;
  double *d_D = nullptr, *d_inv = nullptr;
  int32_t *d_rank = nullptr, *d_arank = nullptr, *d_rank1 = nullptr, *d_status = nullptr;
  double* d_status_val = nullptr;
  // batch: per-problem parameters, leaf ranges, step leaf lists and status
  int32_t n_probs = 1;
  MaternParams* d_mp = nullptr;
  MaternParams* h_mp = nullptr;              // pinned host staging of the parameters
  int32_t *d_prob_leaf0 = nullptr, *d_step_leaf = nullptr, *d_pstatus = nullptr;
  double* d_pstatus_val = nullptr;
  std::vector<hmle_theta> thetas;
  std::vector<int64_t> lr_count;             // per problem: number of low-rank blocks
  // assembly reuse (single problems): the dense near field of the last full
  // assembly, its theta, and the variance the cross-approximation factors hold now
  void* d_Lsave = nullptr;
  double* d_Dsave = nullptr;
  int64_t l_dense = 0;                       // factor-pool elements of the off-diagonal dense blocks
  bool saved = false;
  hmle_theta theta_saved{};
  double sigma2_aca = 0.0;
  int64_t reuse_last = 0, reuse_total = 0;
  std::vector<int32_t> pfail;                // per problem: failing leaf + 1 of the last factorisation
  std::vector<double> pfail_val;
  // captured evaluation of a batch (assembly, factorisation, solve, reduction)
  hipStream_t gstream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t fgraph = nullptr;             // the factorisation alone (hmle_factor), captured once
  hipGraphExec_t fgraph_exec = nullptr;
  hipEvent_t ev_in = nullptr;
  double* d_zin = nullptr;
  double *d_v = nullptr, *d_partial = nullptr, *d_out = nullptr;
  double *d_w = nullptr, *d_bpart = nullptr;   // prediction: C~^{-1} z1 and backward-solve parts
  double *d_vmulti = nullptr;                  // kriging variance: two n x 32 blocks of right-hand sides
  double* d_zrep = nullptr;                    // candidate fit: copies of the data, one per problem of the batch
  double* d_mlw = nullptr;                     // prediction-error measures: n x 32 cross covariances + 2 n
  int32_t* d_flag = nullptr;
  // state
  int state = 0;   // 1 built, 2 assembled, 3 factored
  hmle_theta theta{};
  MaternParams mp{};
  hipEvent_t ev[2]{};
  hipStream_t side = nullptr;   // second stream of the factorisation (default priority)
  hipEvent_t ev_main = nullptr, ev_side = nullptr;
  double t_ms[3]{0, 0, 0};
  int64_t counters[3]{0, 0, 0};
  // live timing of the dense-target update kernel (k_dpairs) in the factorisation
  bool profile = false;
  std::vector<hipEvent_t> pev;
  double prof[9] = {};   // dense pairs: ms, launches, flops; sketch passes; diagonal leaves: the same

  bool mixed() const { return opts.precision == HMLE_MIXED; }
  template <typename TS>
  DevCtx<TS> ctx() const {
    DevCtx<TS> c{};
    c.blocks = d_blocks; c.pairs = d_pairs; c.pair_beg = d_pair_beg;
    c.leaf_lo = d_leaf_lo; c.leaf_hi = d_leaf_hi; c.leaf_diag = d_leaf_diag; c.leaf_inv_off = d_leaf_inv_off;
    c.coords = d_coords;
    c.L = static_cast<TS*>(d_L); c.D = d_D; c.A = static_cast<TS*>(d_A); c.S = static_cast<TS*>(d_S);
    c.gram = static_cast<TS*>(d_gram);
    c.inv = d_inv; c.rank = d_rank; c.arank = d_arank; c.rank1 = d_rank1; c.status = d_status;
    c.pstatus = d_pstatus; c.pstatus_val = d_pstatus_val; c.mp = d_mp; c.prob_leaf0 = d_prob_leaf0;
    c.n = n; c.dim = dim; c.R = plan.rank_width; c.Ra = plan.aca_width;
    c.sum_kc = opts.sum_kc;
    return c;
  }
  ~hmle_problem_s() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (gstream) (void)hipStreamSynchronize(gstream);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (fgraph_exec) (void)hipGraphExecDestroy(fgraph_exec);
    if (fgraph) (void)hipGraphDestroy(fgraph);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (h_mp) (void)hipHostFree(h_mp);
    owned.release_all();
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : pev) (void)hipEventDestroy(e);
    if (ev_main) (void)hipEventDestroy(ev_main);
    if (ev_side) (void)hipEventDestroy(ev_side);
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
  }
};

namespace {

// HMLE_PLAIN_LAUNCHES=1 in the environment: the factorisation and the batched
// evaluation launch their kernels one by one instead of capturing them into a
// HIP graph and replaying it (same kernels, same order, same results; meant
// for tools that trace individual launches).
bool plain_launches() {
  const char* e = std::getenv("HMLE_PLAIN_LAUNCHES");
  return e && e[0] == '1';
}

hmle_status fail(hmle_problem p, hmle_status code, const std::string& msg) {
  if (p) p->err = msg;
  g_last_error = msg;
  return code;
}

template <typename F>
hmle_status guarded(hmle_problem p, F&& f) {
  (void)take_launch_error(nullptr);   // a failure of an earlier call is not this call's
  try {
    const hmle_status s = f();
    if (s == HMLE_OK) check_launches();
    return s;
  } catch (const HipError& e) {
    return fail(p, e.code, e.msg);
  } catch (const DeviceAllocFailure& e) {
    return fail(p, HMLE_E_NOMEM, e.what());
  } catch (const std::bad_alloc&) {
    return fail(p, HMLE_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(p, HMLE_E_HIP, e.what());
  }
}

// Covariance constants of problem q at theta, with the absolute floor of its
// truncation accuracy: the assembly's cross approximation and the
// factorisation's truncations each leave a symmetric error whose low-rank
// blocks (N of them, each mirrored) have Frobenius norms <= delta, so its
// spectral norm is <= sqrt(2 N) delta; delta = spd_margin * tau^2 / sqrt(2 N)
// keeps each error below spd_margin * tau^2 <= the smallest eigenvalue share
// of the nugget, and C~ and the factor positive definite (for spd_margin <=
// 1/2). No floor without a nugget or with spd_margin = 0.
MaternParams problem_params(hmle_problem p, int32_t q, const hmle_theta& t) {
  MaternParams mp = matern_params(t);
  const double nlr = (double)p->lr_count[q];
  mp.abs_tol = (p->opts.spd_margin > 0.0 && t.tau2 > 0.0 && nlr > 0.0)
                   ? p->opts.spd_margin * t.tau2 / std::sqrt(2.0 * nlr)
                   : 0.0;
  return mp;
}

bool valid_theta(const hmle_theta* t, std::string& why) {
  if (!t) { why = "theta is NULL"; return false; }
  if (!std::isfinite(t->sigma2) || !std::isfinite(t->range) || !std::isfinite(t->nu) || !std::isfinite(t->tau2)) {
    why = "theta has a non-finite component"; return false;
  }
  if (t->sigma2 <= 0) { why = "sigma2 must be > 0"; return false; }
  if (t->range <= 0) { why = "range must be > 0"; return false; }
  if (t->nu < 0.05 || t->nu > 8.0) { why = "nu must lie in [0.05, 8]"; return false; }
  if (t->tau2 < 0) { why = "tau2 must be >= 0"; return false; }
  return true;
}

template <typename TS>
void run_assemble(hmle_problem p, hipStream_t st) {
  launch_assemble<TS>(p->ctx<TS>(), p->plan.n_dense, p->plan.n_lowrank, p->opts.aca_tol, st);
}

// Steps s = 0 .. n_steps-1 of the factorisation (leaf column s of every problem).
template <typename TS>
void run_factor(hmle_problem p, hipStream_t st, bool timed) {
  const Plan& pl = p->plan;
  const DevCtx<TS> c = p->ctx<TS>();
  for (int32_t j = 0; j < pl.n_steps; ++j) {
    StepLists sl{};
    sl.dchunks = p->d_dchunks + pl.dchunk_beg[j];
    sl.n_dchunks = pl.dchunk_beg[j + 1] - pl.dchunk_beg[j];
    sl.dtargets = p->d_dtargets + pl.dtarget_beg[j];
    sl.n_dtargets = pl.dtarget_beg[j + 1] - pl.dtarget_beg[j];
    sl.rtargets = p->d_rtargets + pl.rtarget_beg[j];
    sl.n_rtargets = pl.rtarget_beg[j + 1] - pl.rtarget_beg[j];
    sl.r1chunks = p->d_r1chunks + pl.r1chunk_beg[j];
    sl.n_r1chunks = pl.r1chunk_beg[j + 1] - pl.r1chunk_beg[j];
    sl.r2chunks = p->d_r2chunks + pl.r2chunk_beg[j];
    sl.n_r2chunks = pl.r2chunk_beg[j + 1] - pl.r2chunk_beg[j];
    sl.rpairs1 = p->d_rpairs1;
    sl.rpairs2 = p->d_rpairs2;
    sl.g1 = p->d_g1 + pl.g1_beg[j];
    sl.n_g1 = pl.g1_beg[j + 1] - pl.g1_beg[j];
    sl.g2 = p->d_g2 + pl.g2_beg[j];
    sl.gf1 = p->d_gf1 + pl.gf1_beg[j];
    sl.n_gf1 = pl.gf1_beg[j + 1] - pl.gf1_beg[j];
    sl.gf2 = p->d_gf2 + pl.gf2_beg[j];
    sl.n_gf2 = pl.gf2_beg[j + 1] - pl.gf2_beg[j];
    sl.gseg = p->d_gseg;
    sl.n_g2 = pl.g2_beg[j + 1] - pl.g2_beg[j];
    sl.tiles1 = p->d_t1 + pl.t1_beg[j];
    sl.n_t1 = pl.t1_beg[j + 1] - pl.t1_beg[j];
    sl.tiles2 = p->d_t2 + pl.t2_beg[j];
    sl.n_t2 = pl.t2_beg[j + 1] - pl.t2_beg[j];
    sl.tc1 = p->d_tc1 + pl.tc1_beg[j];
    sl.tc2 = p->d_tc2 + pl.tc2_beg[j];
    sl.sg1 = p->d_sg1 + pl.sg1_beg[j];
    sl.n_sg1 = pl.sg1_beg[j + 1] - pl.sg1_beg[j];
    sl.sg2 = p->d_sg2 + pl.sg2_beg[j];
    sl.n_sg2 = pl.sg2_beg[j + 1] - pl.sg2_beg[j];
    sl.spart = p->d_spart;
    sl.dpart = p->d_dpart;
    sl.rpart = p->d_rpart;
    sl.gbuf = p->d_gbuf;
    sl.gpart = p->d_gpart;
    sl.qbuf = p->d_qbuf;
    sl.qint = p->d_qint;
    sl.grams = p->d_grams + pl.gram_beg[j];
    sl.n_grams = pl.gram_beg[j + 1] - pl.gram_beg[j];
    sl.active = p->d_active + pl.active_beg[j];
    sl.n_active = pl.active_beg[j + 1] - pl.active_beg[j];
    sl.inner = p->d_inner + pl.inner_beg[j];
    sl.n_inner = pl.inner_beg[j + 1] - pl.inner_beg[j];
    sl.tsolve = p->d_tsolve + pl.tsolve_beg[j];
    sl.n_tsolve = pl.tsolve_beg[j + 1] - pl.tsolve_beg[j];
    sl.leaves = p->d_step_leaf + pl.step_leaf_beg[j];
    sl.n_leaves = pl.step_leaf_beg[j + 1] - pl.step_leaf_beg[j];
    // the low-rank targets of this step run on the side stream once the previous step is done
    HIP_TRY(hipEventRecord(p->ev_main, st));
    HIP_TRY(hipStreamWaitEvent(p->side, p->ev_main, 0));
    launch_step_lowrank<TS>(c, sl, p->opts.aca_tol, p->side, timed ? &p->pev[8 * j + 2] : nullptr);
    HIP_TRY(hipEventRecord(p->ev_side, p->side));
    if (timed) HIP_TRY(hipEventRecord(p->pev[8 * j], st));
    launch_dense_pairs<TS>(c, sl, st);
    if (timed) HIP_TRY(hipEventRecord(p->pev[8 * j + 1], st));
    launch_dense_reduce<TS>(c, sl, st);
    if (timed) HIP_TRY(hipEventRecord(p->pev[8 * j + 6], st));
    launch_step_diag<TS>(c, sl, st);
    if (timed) HIP_TRY(hipEventRecord(p->pev[8 * j + 7], st));
    HIP_TRY(hipStreamWaitEvent(st, p->ev_side, 0));
    launch_step_cols<TS>(c, j, sl, st);
  }
}

template <typename TS>
void run_solve(hmle_problem p, hipStream_t st) {
  const Plan& pl = p->plan;
  const DevCtx<TS> c = p->ctx<TS>();
  for (int32_t j = 0; j < pl.n_steps; ++j)
    launch_solve_step<TS>(c, j, p->d_step_leaf + pl.step_leaf_beg[j], pl.step_leaf_beg[j + 1] - pl.step_leaf_beg[j],
                          p->d_fsolve + pl.fsolve_beg[j], pl.fsolve_beg[j + 1] - pl.fsolve_beg[j], p->d_v, st);
}

// Everything from assembly to the per-problem sums, on one stream (the body
// of a captured batch evaluation); z_internal: the data already in d_zin.
template <typename TS>
void run_eval(hmle_problem p, hipStream_t st) {
  launch_zero_i32(p->d_status, 4, st);
  launch_zero_i32(p->d_pstatus, p->n_probs, st);
  run_assemble<TS>(p, st);
  run_factor<TS>(p, st, false);
  launch_gather(p->d_zin, p->d_perm, p->n, p->d_v, st);
  run_solve<TS>(p, st);
  launch_reduce(p->d_D, p->d_diag_off, p->d_leaf_lo, p->d_leaf_hi, p->plan.n_leaves, p->d_prob_leaf0, p->n_probs,
                p->d_v + p->n, p->d_partial, p->d_out, st);
}

}  // namespace

extern "C" {

void hmle_default_opts(hmle_opts* o) {
  if (!o) return;
  o->leaf_size = 64;
  o->eta = 2.0;
  o->aca_tol = 1e-6;
  o->max_rank = 32;
  o->precision = HMLE_FP64;
  o->pair_chunk = 1;
  o->sketch_group = 8;
  o->spd_margin = -1.0;
  o->seg_entries = 8;
  o->gseg_rows = 512;
  o->sum_kc = 16;
}

void hmle_default_fit_opts(hmle_fit_opts* o) {
  if (!o) return;
  o->max_iter = 400;
  o->tol = 1e-4;
  o->step = 1.0;
  o->use_backoff = 1;
  o->report_every = 0;
  o->profile_variance = 0;
}

}  // extern "C"

namespace {

hmle_status check_opts(const hmle_opts& o) {
  if (o.leaf_size < 1 || o.leaf_size > 128) return fail(nullptr, HMLE_E_INVALID, "leaf_size must be in [1, 128]");
  if (!(o.eta > 0) || !std::isfinite(o.eta)) return fail(nullptr, HMLE_E_INVALID, "eta must be > 0");
  if (!(o.aca_tol > 0 && o.aca_tol < 1)) return fail(nullptr, HMLE_E_INVALID, "aca_tol must be in (0, 1)");
  if (o.max_rank < 4 || o.max_rank > 64) return fail(nullptr, HMLE_E_INVALID, "max_rank must be in [4, 64]");
  if (o.precision != HMLE_FP64 && o.precision != HMLE_MIXED) return fail(nullptr, HMLE_E_INVALID, "bad precision");
  if (o.pair_chunk < 0 || o.pair_chunk > 16) return fail(nullptr, HMLE_E_INVALID, "pair_chunk must be in [0, 16]");
  if (o.sketch_group < 0 || o.sketch_group > 16) return fail(nullptr, HMLE_E_INVALID, "sketch_group must be in [0, 16]");
  if (!(o.spd_margin <= 1.0))
    return fail(nullptr, HMLE_E_INVALID, "spd_margin must be <= 1 (negative: automatic)");
  if (o.seg_entries < 0 || o.seg_entries > 32) return fail(nullptr, HMLE_E_INVALID, "seg_entries must be in [0, 32]");
  if (o.gseg_rows != 0 && (o.gseg_rows < 64 || o.gseg_rows > 4096))
    return fail(nullptr, HMLE_E_INVALID, "gseg_rows must be 0 or in [64, 4096]");
  if (o.sum_kc != 0 && o.sum_kc != 16 && o.sum_kc != 32)
    return fail(nullptr, HMLE_E_INVALID, "sum_kc must be 0, 16 or 32");
  return HMLE_OK;
}

// Zero schedule options mean the defaults.
hmle_opts with_defaults(hmle_opts o) {
  if (o.pair_chunk == 0) o.pair_chunk = 1;
  if (o.sketch_group == 0) o.sketch_group = 8;
  if (o.seg_entries == 0) o.seg_entries = 8;
  if (o.gseg_rows == 0) o.gseg_rows = 512;
  if (o.sum_kc == 0) o.sum_kc = 16;
  // automatic floor: on in FP64; off in the mixed mode, where the float32 storage of the
  // large blocks alone perturbs C by about 6e-8 ||C||_2, more than the nugget at large n
  if (o.spd_margin < 0.0) o.spd_margin = o.precision == HMLE_MIXED ? 0.0 : 0.5;
  return o;
}

// Trees, plan and device storage of a batch of problems whose points are
// concatenated in pts (device, row-major) at the offsets offs (count + 1).
hmle_status build_problem(const double* pts, const std::vector<int64_t>& offs, int32_t dim, const hmle_opts& o,
                          const hmle_allocator* alloc, void* hip_stream, hmle_problem* out) {
  const int64_t n = offs.back();
  auto* p = new hmle_problem_s();
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->owned.stream = p->stream;
  if (alloc) {
    p->owned.al = *alloc;
    p->owned.custom = true;
  }
  p->n = (int32_t)n;
  p->dim = dim;
  p->opts = o;
  p->n_probs = (int32_t)offs.size() - 1;
  hmle_status st = guarded(p, [&]() -> hmle_status {
    std::vector<double> hpts((size_t)n * dim);
    HIP_TRY(hipMemcpyAsync(hpts.data(), pts, hpts.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    for (double v : hpts)
      if (!std::isfinite(v)) return fail(p, HMLE_E_INVALID, "non-finite coordinate");
    if (p->n_probs == 1) {
      // one problem: both trees on the GPU, from the caller's device points
      TreeAlloc ta{[](size_t b, void* ctx) { return static_cast<DevPool*>(ctx)->temp_alloc(b); },
                   [](void* q, void* ctx) { static_cast<DevPool*>(ctx)->temp_free(q); }, &p->owned};
      build_trees_gpu(pts, (int32_t)n, dim, o.leaf_size, o.eta, p->stream, ta, p->tree, p->bt);
    } else {
      build_forest(hpts.data(), offs, dim, o.leaf_size, o.eta, p->tree, p->bt);
    }
    build_plan(p->tree, p->bt, offs, o.max_rank, o.max_rank, o.pair_chunk, o.sketch_group, p->plan, o.seg_entries,
               o.gseg_rows);
    Plan& pl = p->plan;
    const size_t ts = o.precision == HMLE_MIXED ? sizeof(float) : sizeof(double);
    auto& own = p->owned;
    p->d_perm = dev_upload(p->tree.perm, p->stream, own);
    p->d_coords = dev_alloc<double>((size_t)n * dim, own);
    launch_gather_coords(pts, p->d_perm, p->n, dim, p->d_coords, p->stream);
    p->d_blocks = dev_upload(pl.blocks, p->stream, own);
    p->d_pairs = dev_upload(pl.pairs, p->stream, own);
    p->d_pair_beg = dev_upload(pl.pair_beg, p->stream, own);
    p->d_leaf_lo = dev_upload(pl.leaf_lo, p->stream, own);
    p->d_leaf_hi = dev_upload(pl.leaf_hi, p->stream, own);
    p->d_leaf_diag = dev_upload(pl.leaf_diag, p->stream, own);
    p->d_leaf_inv_off = dev_upload(pl.leaf_inv_off, p->stream, own);
    p->d_prob_leaf0 = dev_upload(pl.prob_leaf0, p->stream, own);
    p->d_step_leaf = dev_upload(pl.step_leaf, p->stream, own);
    std::vector<int64_t> diag_off(pl.n_leaves);
    for (int32_t j = 0; j < pl.n_leaves; ++j) diag_off[j] = pl.blocks[pl.leaf_diag[j]].loff;
    p->d_diag_off = dev_upload(diag_off, p->stream, own);
    p->d_active = dev_upload(pl.active, p->stream, own);
    p->d_dchunks = dev_upload(pl.dchunks, p->stream, own);
    p->d_r1chunks = dev_upload(pl.r1chunks, p->stream, own);
    p->d_r2chunks = dev_upload(pl.r2chunks, p->stream, own);
    p->d_dtargets = dev_upload(pl.dtargets, p->stream, own);
    p->d_rtargets = dev_upload(pl.rtargets, p->stream, own);
    p->d_rpairs1 = dev_upload(pl.rpairs1, p->stream, own);
    p->d_rpairs2 = dev_upload(pl.rpairs2, p->stream, own);
    p->d_g1 = dev_upload(pl.g1items, p->stream, own);
    p->d_g2 = dev_upload(pl.g2items, p->stream, own);
    p->d_gf1 = dev_upload(pl.gf1, p->stream, own);
    p->d_gf2 = dev_upload(pl.gf2, p->stream, own);
    p->d_gseg = dev_alloc<char>((size_t)(std::max(1, pl.max_gparts) * 4096) * ts, own);
    p->d_grams = dev_upload(pl.grams, p->stream, own);
    p->d_gram = dev_alloc<char>((size_t)(std::max<int64_t>(1, pl.n_grams) * pl.rank_width * pl.rank_width) * ts, own);
    p->d_t1 = dev_upload(pl.tiles1, p->stream, own);
    p->d_t2 = dev_upload(pl.tiles2, p->stream, own);
    p->d_tc1 = dev_upload(pl.tc1, p->stream, own);
    p->d_tc2 = dev_upload(pl.tc2, p->stream, own);
    p->d_sg1 = dev_upload(pl.sg1, p->stream, own);
    p->d_sg2 = dev_upload(pl.sg2, p->stream, own);
    p->d_spart = dev_alloc<char>((size_t)std::max(1, pl.max_segs) * 128 * 64 * ts, own);
    p->d_gbuf = dev_alloc<char>((size_t)(std::max(1, pl.max_gslots) * 4096) * ts, own);
    p->d_gpart = dev_alloc<double>((size_t)std::max(1, pl.max_tiles) * pl.rank_width * pl.rank_width, own);
    p->d_qbuf = dev_alloc<double>((size_t)std::max(1, pl.max_rtargets) * 2 * 64 * 64, own);
    p->d_qint = dev_alloc<int32_t>((size_t)std::max(1, pl.max_rtargets) * 4, own);
    p->d_dpart = dev_alloc<char>((size_t)(pl.dpart_size + 64) * ts, own);
    p->d_rpart = dev_alloc<char>((size_t)(pl.rpart_size + 64) * ts, own);
    p->d_inner = dev_upload(pl.inner, p->stream, own);
    p->d_tsolve = dev_upload(pl.tsolve, p->stream, own);
    p->d_fsolve = dev_upload(pl.fsolve, p->stream, own);
    p->d_rowp_beg = dev_upload(pl.rowp_beg, p->stream, own);
    p->d_rowp = dev_upload(pl.rowp, p->stream, own);
    p->d_colp_beg = dev_upload(pl.colp_beg, p->stream, own);
    p->d_colp = dev_upload(pl.colp, p->stream, own);
    p->d_h = dev_alloc<double>((size_t)std::max(1, pl.n_lowrank) * pl.rank_width, own);
    p->d_L = dev_alloc<char>((size_t)pl.l_size * ts, own);
    p->d_A = dev_alloc<char>((size_t)pl.a_size * ts, own);
    p->d_S = dev_alloc<char>((size_t)pl.s_size * ts, own);
    p->d_D = dev_alloc<double>((size_t)pl.d_size, own);
    p->d_inv = dev_alloc<double>((size_t)pl.inv_size, own);
    p->d_rank = dev_alloc<int32_t>(pl.blocks.size(), own);
    p->d_arank = dev_alloc<int32_t>(pl.blocks.size(), own);
    p->d_rank1 = dev_alloc<int32_t>(pl.blocks.size(), own);
    HIP_TRY(hipMemsetAsync(p->d_rank1, 0, pl.blocks.size() * sizeof(int32_t), p->stream));
    HIP_TRY(hipMemsetAsync(p->d_rank, 0, pl.blocks.size() * sizeof(int32_t), p->stream));
    HIP_TRY(hipMemsetAsync(p->d_arank, 0, pl.blocks.size() * sizeof(int32_t), p->stream));
    p->d_status = dev_alloc<int32_t>(4, own);
    p->d_status_val = dev_alloc<double>(2, own);
    p->d_pstatus = dev_alloc<int32_t>(p->n_probs, own);
    p->d_pstatus_val = dev_alloc<double>(p->n_probs, own);
    p->d_mp = dev_alloc<MaternParams>(p->n_probs, own);
    HIP_TRY(hipHostMalloc((void**)&p->h_mp, p->n_probs * sizeof(MaternParams), hipHostMallocDefault));
    p->d_v = dev_alloc<double>(2 * (size_t)n, own);
    p->d_zin = dev_alloc<double>((size_t)n, own);
    p->d_partial = dev_alloc<double>(2 * (size_t)pl.n_leaves, own);
    p->d_out = dev_alloc<double>(2 * (size_t)p->n_probs, own);
    p->d_flag = dev_alloc<int32_t>(1, own);
    p->thetas.assign(p->n_probs, hmle_theta{});
    p->lr_count.assign(p->n_probs, 0);
    p->l_dense = pl.n_lowrank > 0 ? pl.blocks[pl.n_dense].loff : pl.l_size;
    for (int32_t bi = pl.n_dense; bi < (int32_t)pl.blocks.size(); ++bi) p->lr_count[pl.blocks[bi].prob]++;
    p->pfail.assign(p->n_probs, 0);
    p->pfail_val.assign(p->n_probs, 0.0);
    if (o.precision == HMLE_MIXED) launch_gen_omega<float>(p->ctx<float>(), pl.n_dense, pl.n_lowrank, p->stream);
    else launch_gen_omega<double>(p->ctx<double>(), pl.n_dense, pl.n_lowrank, p->stream);
    check_launches();
    for (auto& e : p->ev) HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventCreateWithFlags(&p->ev_main, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&p->ev_side, hipEventDisableTiming));
    HIP_TRY(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->state = 1;
    return HMLE_OK;
  });
  if (st != HMLE_OK) {
    g_last_error = p->err;
    delete p;
    return st;
  }
  *out = p;
  return HMLE_OK;
}

}  // namespace

extern "C" {

hmle_status hmle_build_tree(const double* pts, int64_t n, int32_t dim, const hmle_opts* opts, void* hip_stream,
                            hmle_problem* out) {
  if (!out) return fail(nullptr, HMLE_E_INVALID, "out is NULL");
  *out = nullptr;
  hmle_opts o;
  hmle_default_opts(&o);
  if (opts) o = *opts;
  if (!pts) return fail(nullptr, HMLE_E_INVALID, "pts is NULL");
  if (n < 1 || n > (int64_t)1 << 30) return fail(nullptr, HMLE_E_INVALID, "n must be in [1, 2^30]");
  if (dim != 2 && dim != 3) return fail(nullptr, HMLE_E_INVALID, "dim must be 2 or 3");
  const hmle_status os = check_opts(o);
  if (os != HMLE_OK) return os;
  return build_problem(pts, {0, n}, dim, with_defaults(o), nullptr, hip_stream, out);
}

hmle_status hmle_build_tree_alloc(const double* pts, int64_t n, int32_t dim, const hmle_opts* opts,
                                  const hmle_allocator* alloc, void* hip_stream, hmle_problem* out) {
  if (!out) return fail(nullptr, HMLE_E_INVALID, "out is NULL");
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(nullptr, HMLE_E_INVALID, "allocator without alloc or free");
  hmle_opts o;
  hmle_default_opts(&o);
  if (opts) o = *opts;
  if (!pts) return fail(nullptr, HMLE_E_INVALID, "pts is NULL");
  if (n < 1 || n > (int64_t)1 << 30) return fail(nullptr, HMLE_E_INVALID, "n must be in [1, 2^30]");
  if (dim != 2 && dim != 3) return fail(nullptr, HMLE_E_INVALID, "dim must be 2 or 3");
  const hmle_status os = check_opts(o);
  if (os != HMLE_OK) return os;
  return build_problem(pts, {0, n}, dim, with_defaults(o), alloc, hip_stream, out);
}

hmle_status hmle_build_batch(const double* pts, const int64_t* offsets, int32_t count, int32_t dim,
                             const hmle_opts* opts, void* hip_stream, hmle_problem* out) {
  if (!out) return fail(nullptr, HMLE_E_INVALID, "out is NULL");
  *out = nullptr;
  hmle_opts o;
  hmle_default_opts(&o);
  if (opts) o = *opts;
  if (!pts || !offsets) return fail(nullptr, HMLE_E_INVALID, "pts and offsets must not be NULL");
  if (count < 1 || count > (1 << 20)) return fail(nullptr, HMLE_E_INVALID, "count must be in [1, 2^20]");
  if (dim != 2 && dim != 3) return fail(nullptr, HMLE_E_INVALID, "dim must be 2 or 3");
  if (offsets[0] != 0) return fail(nullptr, HMLE_E_INVALID, "offsets[0] must be 0");
  for (int32_t q = 0; q < count; ++q)
    if (offsets[q + 1] <= offsets[q]) return fail(nullptr, HMLE_E_INVALID, "every problem needs at least one point");
  if (offsets[count] > (int64_t)1 << 30) return fail(nullptr, HMLE_E_INVALID, "total points must be <= 2^30");
  const hmle_status os = check_opts(o);
  if (os != HMLE_OK) return os;
  return build_problem(pts, std::vector<int64_t>(offsets, offsets + count + 1), dim, with_defaults(o), nullptr,
                       hip_stream, out);
}

hmle_status hmle_build_batch_alloc(const double* pts, const int64_t* offsets, int32_t count, int32_t dim,
                                   const hmle_opts* opts, const hmle_allocator* alloc, void* hip_stream,
                                   hmle_problem* out) {
  if (!out) return fail(nullptr, HMLE_E_INVALID, "out is NULL");
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(nullptr, HMLE_E_INVALID, "allocator without alloc or free");
  hmle_opts o;
  hmle_default_opts(&o);
  if (opts) o = *opts;
  if (!pts || !offsets) return fail(nullptr, HMLE_E_INVALID, "pts and offsets must not be NULL");
  if (count < 1 || count > (1 << 20)) return fail(nullptr, HMLE_E_INVALID, "count must be in [1, 2^20]");
  if (dim != 2 && dim != 3) return fail(nullptr, HMLE_E_INVALID, "dim must be 2 or 3");
  if (offsets[0] != 0) return fail(nullptr, HMLE_E_INVALID, "offsets[0] must be 0");
  for (int32_t q = 0; q < count; ++q)
    if (offsets[q + 1] <= offsets[q]) return fail(nullptr, HMLE_E_INVALID, "every problem needs at least one point");
  if (offsets[count] > (int64_t)1 << 30) return fail(nullptr, HMLE_E_INVALID, "total points must be <= 2^30");
  const hmle_status os = check_opts(o);
  if (os != HMLE_OK) return os;
  return build_problem(pts, std::vector<int64_t>(offsets, offsets + count + 1), dim, with_defaults(o), alloc,
                       hip_stream, out);
}

hmle_status hmle_structure_batch_host(const double* pts, const int64_t* offsets, int32_t count, int32_t dim,
                                     const hmle_opts* opts, hmle_problem* out) {
  if (!out) return fail(nullptr, HMLE_E_INVALID, "out is NULL");
  *out = nullptr;
  hmle_opts o;
  hmle_default_opts(&o);
  if (opts) o = *opts;
  if (!pts || !offsets || count < 1 || (dim != 2 && dim != 3) || offsets[0] != 0)
    return fail(nullptr, HMLE_E_INVALID, "bad arguments");
  for (int32_t q = 0; q < count; ++q)
    if (offsets[q + 1] <= offsets[q]) return fail(nullptr, HMLE_E_INVALID, "every problem needs at least one point");
  const int64_t n = offsets[count];
  if (n > (int64_t)1 << 30) return fail(nullptr, HMLE_E_INVALID, "total points must be <= 2^30");
  const hmle_status os = check_opts(o);
  if (os != HMLE_OK) return os;
  o = with_defaults(o);
  for (int64_t i = 0; i < n * dim; ++i)
    if (!std::isfinite(pts[i])) return fail(nullptr, HMLE_E_INVALID, "non-finite coordinate");
  auto* p = new hmle_problem_s();
  p->n = (int32_t)n;
  p->dim = dim;
  p->opts = o;
  p->n_probs = count;
  hmle_status st = guarded(p, [&]() -> hmle_status {
    const std::vector<int64_t> offs(offsets, offsets + count + 1);
    build_forest(pts, offs, dim, o.leaf_size, o.eta, p->tree, p->bt);
    build_plan(p->tree, p->bt, offs, o.max_rank, o.max_rank, o.pair_chunk, o.sketch_group, p->plan, o.seg_entries,
               o.gseg_rows);
    return HMLE_OK;
  });
  if (st != HMLE_OK) {
    g_last_error = p->err;
    delete p;
    return st;
  }
  *out = p;
  return HMLE_OK;
}

hmle_status hmle_structure_host(const double* pts, int64_t n, int32_t dim, const hmle_opts* opts, hmle_problem* out) {
  if (!out) return fail(nullptr, HMLE_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > (int64_t)1 << 30) return fail(nullptr, HMLE_E_INVALID, "bad arguments");
  const int64_t offs[2] = {0, n};
  return hmle_structure_batch_host(pts, offs, 1, dim, opts, out);
}

hmle_status hmle_plan_stats(hmle_problem p, int64_t s[16]) {
  if (!p || !s) return fail(p, HMLE_E_INVALID, "NULL argument");
  const Plan& pl = p->plan;
  s[0] = (int64_t)pl.pairs.size();
  s[1] = (int64_t)pl.inner.size();
  s[2] = pl.dense_entries;
  s[3] = pl.lr_dims;
  s[4] = pl.n_leaves;
  s[5] = pl.rank_width;
  s[6] = (int64_t)pl.active.size();
  int64_t lr_pairs = 0;
  for (int32_t bi = pl.n_dense; bi < (int32_t)pl.blocks.size(); ++bi) lr_pairs += pl.pair_beg[bi + 1] - pl.pair_beg[bi];
  s[7] = lr_pairs;
  s[8] = pl.n_grams;
  int64_t rr = 0;
  for (const PairDesc& pr : pl.pairs) rr += pr.gram >= 0;
  s[9] = rr;
  s[10] = pl.n_steps;
  s[11] = pl.n_probs;
  // pairs into low-rank targets by kind of (x, y): dense-dense, dense-lowrank, lowrank-dense, lowrank-lowrank
  for (int q = 12; q < 16; ++q) s[q] = 0;
  for (int32_t bi = pl.n_dense; bi < (int32_t)pl.blocks.size(); ++bi)
    for (int64_t q = pl.pair_beg[bi]; q < pl.pair_beg[bi + 1]; ++q) {
      const PairDesc& pr = pl.pairs[q];
      const int xl = pl.blocks[pr.x].kind == BK_LOWRANK, yl = pl.blocks[pr.y].kind == BK_LOWRANK;
      s[12 + 2 * xl + yl] += 1;
    }
  return HMLE_OK;
}

}  // extern "C"

namespace {

hmle_status assemble_thetas(hmle_problem p, const hmle_theta* thetas, bool broadcast) {
  if (p->state < 1) return fail(p, HMLE_E_STATE, "build_tree first");
  std::string why;
  for (int32_t q = 0; q < (broadcast ? 1 : p->n_probs); ++q)
    if (!valid_theta(thetas + q, why)) return fail(p, HMLE_E_INVALID, why + " (problem " + std::to_string(q) + ")");
  return guarded(p, [&]() -> hmle_status {
    HIP_TRY(hipStreamSynchronize(p->stream));   // the staging buffer may still feed a previous copy
    for (int32_t q = 0; q < p->n_probs; ++q) {
      p->thetas[q] = thetas[broadcast ? 0 : q];
      p->h_mp[q] = problem_params(p, q, p->thetas[q]);
    }
    p->theta = p->thetas[0];
    p->mp = p->h_mp[0];
    HIP_TRY(hipEventRecord(p->ev[0], p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_mp, p->h_mp, p->n_probs * sizeof(MaternParams), hipMemcpyHostToDevice, p->stream));
    const Plan& pl = p->plan;
    const size_t ts = p->mixed() ? sizeof(float) : sizeof(double);
    const hmle_theta& t1 = p->theta;
    const hmle_theta& t0 = p->theta_saved;
    // reuse: same range and smoothness; with the definiteness floor on, the saved
    // ranks meet the new floor only if the nugget did not shrink relative to the variance
    const bool floor_ok = p->opts.spd_margin == 0.0 ||
                          (t0.tau2 > 0.0 && t1.tau2 * t0.sigma2 >= t0.tau2 * t1.sigma2);
    const bool reuse = p->n_probs == 1 && p->saved && t1.range == t0.range && t1.nu == t0.nu && floor_ok;
    if (reuse) {
      const double sc = t1.sigma2 / t0.sigma2, f = t1.sigma2 / p->sigma2_aca;
      if (p->mixed())
        launch_rescale<float>(p->ctx<float>(), pl.n_dense, pl.n_lowrank, pl.n_leaves,
                              static_cast<const float*>(p->d_Lsave), p->l_dense, p->d_Dsave, sc, t0.tau2, t1.tau2, f,
                              p->stream);
      else
        launch_rescale<double>(p->ctx<double>(), pl.n_dense, pl.n_lowrank, pl.n_leaves,
                               static_cast<const double*>(p->d_Lsave), p->l_dense, p->d_Dsave, sc, t0.tau2, t1.tau2,
                               f, p->stream);
      p->sigma2_aca = t1.sigma2;
      p->reuse_last = 1;
      p->reuse_total++;
    } else {
      if (p->mixed()) run_assemble<float>(p, p->stream);
      else run_assemble<double>(p, p->stream);
      p->reuse_last = 0;
      if (p->n_probs == 1) {
        // keep the dense near field of this full assembly for later sigma^2 / tau^2 changes
        if (!p->d_Dsave) {
          p->d_Lsave = dev_alloc<char>((size_t)std::max<int64_t>(1, p->l_dense) * ts, p->owned);
          p->d_Dsave = dev_alloc<double>((size_t)pl.d_size, p->owned);
        }
        if (p->l_dense > 0)
          HIP_TRY(hipMemcpyAsync(p->d_Lsave, p->d_L, (size_t)p->l_dense * ts, hipMemcpyDeviceToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->d_Dsave, p->d_D, (size_t)pl.d_size * sizeof(double), hipMemcpyDeviceToDevice,
                               p->stream));
        p->saved = true;
        p->theta_saved = t1;
        p->sigma2_aca = t1.sigma2;
      }
    }
    check_launches();
    HIP_TRY(hipEventRecord(p->ev[1], p->stream));
    HIP_TRY(hipEventSynchronize(p->ev[1]));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
    p->t_ms[0] = ms;
    p->state = 2;
    return HMLE_OK;
  });
}

// Per-problem outcome of the last factorisation; ranks and cap counters.
void read_factor_status(hmle_problem p) {
  int32_t status[4];
  HIP_TRY(hipMemcpy(status, p->d_status, sizeof(status), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(p->pfail.data(), p->d_pstatus, p->n_probs * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(p->pfail_val.data(), p->d_pstatus_val, p->n_probs * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<int32_t> rk(p->plan.blocks.size());
  HIP_TRY(hipMemcpy(rk.data(), p->d_rank, rk.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  int64_t sum = 0, mx = 0;
  for (int32_t bi = p->plan.n_dense; bi < (int32_t)rk.size(); ++bi) { sum += rk[bi]; mx = std::max<int64_t>(mx, rk[bi]); }
  p->counters[0] = sum; p->counters[1] = mx; p->counters[2] = status[1] + status[2];
  if (p->profile) {
    const Plan& pl = p->plan;
    std::vector<int32_t> rk1(pl.blocks.size());
    HIP_TRY(hipMemcpy(rk1.data(), p->d_rank1, rk1.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int32_t j = 0; j < pl.n_steps; ++j) {
      float t = 0;
      if (pl.dchunk_beg[j + 1] > pl.dchunk_beg[j]) {
        HIP_TRY(hipEventElapsedTime(&t, p->pev[8 * j], p->pev[8 * j + 1]));
        p->prof[0] += t;
        p->prof[1] += 1.0;
      }
      if (pl.r1chunk_beg[j + 1] > pl.r1chunk_beg[j]) {
        HIP_TRY(hipEventElapsedTime(&t, p->pev[8 * j + 2], p->pev[8 * j + 3]));
        p->prof[3] += t;
        p->prof[4] += 1.0;
      }
      if (pl.r2chunk_beg[j + 1] > pl.r2chunk_beg[j]) {
        HIP_TRY(hipEventElapsedTime(&t, p->pev[8 * j + 4], p->pev[8 * j + 5]));
        p->prof[3] += t;
        p->prof[4] += 1.0;
      }
      if (pl.step_leaf_beg[j + 1] > pl.step_leaf_beg[j]) {
        HIP_TRY(hipEventElapsedTime(&t, p->pev[8 * j + 6], p->pev[8 * j + 7]));
        p->prof[6] += t;
        p->prof[7] += 1.0;
        // the Cholesky's m^3/3 per diagonal leaf (the inverse formed beside it is
        // the library's choice, not work of the method, and is not counted)
        for (int32_t q = pl.step_leaf_beg[j]; q < pl.step_leaf_beg[j + 1]; ++q) {
          const double m = pl.leaf_hi[pl.step_leaf[q]] - pl.leaf_lo[pl.step_leaf[q]];
          p->prof[8] += m * m * m / 3.0;
        }
      }
    }
    auto lr = [&](int32_t b) { return pl.blocks[b].kind == BK_LOWRANK; };
    // algorithmic flops of the dense-target pair products with the ranks of this factorisation
    double fl = 0.0;
    for (const ChunkDesc& ch : pl.dchunks)
      for (int32_t q = ch.pair_lo; q < ch.pair_hi; ++q) {
        const PairDesc& pr = pl.pairs[q];
        const double nr = pr.rx1 - pr.rx0, nc = pr.ry1 - pr.ry0, nw = pr.w1 - pr.w0;
        const bool xl = lr(pr.x), yl = lr(pr.y);
        const double kx = xl ? rk[pr.x] : 0, ky = yl ? rk[pr.y] : 0;
        if (!xl && !yl) fl += 2 * nr * nc * nw;
        else if (xl && !yl) fl += 2 * kx * nc * nw + 2 * nr * nc * kx;
        else if (!xl && yl) fl += 2 * nr * ky * nw + 2 * nr * nc * ky;
        else fl += 2 * kx * ky * nw + 2 * kx * nc * ky + 2 * nr * nc * kx;
      }
    p->prof[2] += fl;
    // sketch passes: per pair, output block q and input block p of the pass,
    // X = the test matrix (pass 1, width min(R, m, k)) or the range basis
    // (pass 2, width rank1): low-rank q, p: H += (W_q^T W_p) (U_p^T X);
    // low-rank q, dense p: H += W_q^T (L_p^T X); dense q: rows += L_q (W_p G_p | L_p^T X)
    double fs = 0.0;
    for (int pass = 1; pass <= 2; ++pass) {
      const std::vector<ChunkDesc>& chs = pass == 1 ? pl.r1chunks : pl.r2chunks;
      const std::vector<RPairDesc>& rps = pass == 1 ? pl.rpairs1 : pl.rpairs2;
      for (const ChunkDesc& ch : chs) {
        const BlockDesc& b = pl.blocks[ch.b];
        const double ncol = pass == 1 ? std::min<int64_t>(pl.rank_width, std::min(b.r1 - b.r0, b.c1 - b.c0)) : rk1[ch.b];
        for (int32_t q = ch.pair_lo; q < ch.pair_hi; ++q) {
          const RPairDesc& r = rps[q];
          const int32_t qb = pass == 1 ? r.x : r.y, pb = pass == 1 ? r.y : r.x;
          const double nq = pass == 1 ? r.rx1 - r.rx0 : r.ry1 - r.ry0, np = pass == 1 ? r.ry1 - r.ry0 : r.rx1 - r.rx0;
          const double nw = r.w1 - r.w0;
          if (lr(qb) && lr(pb)) fs += 2.0 * rk[qb] * rk[pb] * ncol;
          else if (lr(qb)) fs += 2.0 * nw * np * ncol + 2.0 * rk[qb] * nw * ncol;
          else if (lr(pb)) fs += 2.0 * nw * rk[pb] * ncol + 2.0 * nq * nw * ncol;
          else fs += 2.0 * nw * np * ncol + 2.0 * nq * nw * ncol;
        }
      }
    }
    p->prof[5] += fs;
  }
}

std::string not_spd_message(hmle_problem p, int32_t q) {
  const int32_t leaf = p->pfail[q] - 1;
  char buf[200];
  std::snprintf(buf, sizeof buf, "not positive definite: problem %d, leaf %d (points %d..%d), pivot %.6g", q,
                leaf - p->plan.prob_leaf0[q], p->plan.leaf_lo[leaf] - (int32_t)p->plan.prob_off[q],
                p->plan.leaf_hi[leaf] - (int32_t)p->plan.prob_off[q], p->pfail_val[q]);
  return buf;
}

// Per-problem logL from the device sums out = [logdet_p, quad_p]; NaN rows for failed problems.
void finish_loglik(hmle_problem p, const double* r, double* out, hmle_status* per) {
  for (int32_t q = 0; q < p->n_probs; ++q) {
    const double np = (double)(p->plan.prob_off[q + 1] - p->plan.prob_off[q]);
    if (p->pfail[q] != 0) {
      out[3 * q] = out[3 * q + 1] = out[3 * q + 2] = std::nan("");
      if (per) per[q] = HMLE_E_NOT_SPD;
      continue;
    }
    const double logdet = r[2 * q], quad = r[2 * q + 1];
    out[3 * q] = -0.5 * np * std::log(2.0 * M_PI) - 0.5 * logdet - 0.5 * quad;
    out[3 * q + 1] = logdet;
    out[3 * q + 2] = quad;
    if (per) per[q] = HMLE_OK;
  }
}

}  // namespace

extern "C" {

hmle_status hmle_assemble(hmle_problem p, const hmle_theta* theta) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  return assemble_thetas(p, theta, true);
}

hmle_status hmle_assemble_batch(hmle_problem p, const hmle_theta* thetas) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (!thetas) return fail(p, HMLE_E_INVALID, "thetas is NULL");
  return assemble_thetas(p, thetas, false);
}

hmle_status hmle_factor(hmle_problem p) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (p->state != 2) return fail(p, HMLE_E_STATE, p->state == 3 ? "already factored; assemble again" : "assemble first");
  return guarded(p, [&]() -> hmle_status {
    if (p->profile || plain_launches()) {
      // timed kernels (or plain launches requested): launches with events around them
      launch_zero_i32(p->d_status, 4, p->stream);
      launch_zero_i32(p->d_pstatus, p->n_probs, p->stream);
      HIP_TRY(hipEventRecord(p->ev[0], p->stream));
      if (p->mixed()) run_factor<float>(p, p->stream, p->profile);
      else run_factor<double>(p, p->stream, p->profile);
      check_launches();
      HIP_TRY(hipEventRecord(p->ev[1], p->stream));
    } else {
      // the launch sequence is fixed per problem (theta enters through device
      // buffers): captured once on the internal stream, replayed after that,
      // ordered after the caller's stream and before its next work
      if (!p->gstream) HIP_TRY(hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking));
      if (!p->ev_in) HIP_TRY(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
      if (!p->fgraph_exec) {
        HIP_TRY(hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal));
        try {
          launch_zero_i32(p->d_status, 4, p->gstream);
          launch_zero_i32(p->d_pstatus, p->n_probs, p->gstream);
          if (p->mixed()) run_factor<float>(p, p->gstream, false);
          else run_factor<double>(p, p->gstream, false);
        } catch (...) {
          hipGraph_t g = nullptr;   // end the capture so that the streams stay usable
          (void)hipStreamEndCapture(p->gstream, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        HIP_TRY(hipStreamEndCapture(p->gstream, &p->fgraph));
        check_launches();
        HIP_TRY(hipGraphInstantiate(&p->fgraph_exec, p->fgraph, nullptr, nullptr, 0));
      }
      HIP_TRY(hipEventRecord(p->ev_in, p->stream));
      HIP_TRY(hipStreamWaitEvent(p->gstream, p->ev_in, 0));
      HIP_TRY(hipEventRecord(p->ev[0], p->gstream));
      HIP_TRY(hipGraphLaunch(p->fgraph_exec, p->gstream));
      HIP_TRY(hipEventRecord(p->ev[1], p->gstream));
      HIP_TRY(hipStreamWaitEvent(p->stream, p->ev[1], 0));
    }
    HIP_TRY(hipEventSynchronize(p->ev[1]));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
    p->t_ms[1] = ms;
    read_factor_status(p);
    p->state = 3;
    if (p->n_probs == 1 && p->pfail[0] != 0) {
      p->state = 1;   // the assembled matrix is consumed; a new assemble is required
      return fail(p, HMLE_E_NOT_SPD, not_spd_message(p, 0));
    }
    return HMLE_OK;
  });
}

hmle_status hmle_factor_status(hmle_problem p, hmle_status* per_problem) {
  if (!p || !per_problem) return fail(p, HMLE_E_INVALID, "NULL argument");
  if (p->state != 3) return fail(p, HMLE_E_STATE, "factor first");
  for (int32_t q = 0; q < p->n_probs; ++q) per_problem[q] = p->pfail[q] ? HMLE_E_NOT_SPD : HMLE_OK;
  return HMLE_OK;
}

}  // extern "C"

namespace {

hmle_status loglik_any(hmle_problem p, const double* z, double* out, hmle_status* per) {
  return guarded(p, [&]() -> hmle_status {
    HIP_TRY(hipEventRecord(p->ev[0], p->stream));
    launch_gather(z, p->d_perm, p->n, p->d_v, p->stream);
    if (p->mixed()) run_solve<float>(p, p->stream);
    else run_solve<double>(p, p->stream);
    launch_reduce(p->d_D, p->d_diag_off, p->d_leaf_lo, p->d_leaf_hi, p->plan.n_leaves, p->d_prob_leaf0, p->n_probs,
                  p->d_v + p->n, p->d_partial, p->d_out, p->stream);
    check_launches();
    std::vector<double> r(2 * (size_t)p->n_probs);
    HIP_TRY(hipMemcpyAsync(r.data(), p->d_out, r.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipEventRecord(p->ev[1], p->stream));
    HIP_TRY(hipEventSynchronize(p->ev[1]));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
    p->t_ms[2] = ms;
    finish_loglik(p, r.data(), out, per);
    return HMLE_OK;
  });
}

}  // namespace

namespace hmle {

hmle_status candidate_layout(hmle_problem p, int32_t* count, int64_t* n1) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (p->state < 1) return fail(p, HMLE_E_STATE, "build first");
  return guarded(p, [&]() -> hmle_status {
    const std::vector<int64_t>& off = p->plan.prob_off;
    const int32_t q = p->n_probs;
    const int64_t m = off[1] - off[0];
    for (int32_t k = 1; k < q; ++k)
      if (off[k + 1] - off[k] != m) return fail(p, HMLE_E_INVALID, "candidate batch: problems differ in size");
    const std::vector<int32_t>& perm = p->tree.perm;
    for (int32_t k = 1; k < q; ++k)
      for (int64_t i = 0; i < m; ++i)
        if (perm[off[k] + i] - off[k] != perm[i] - off[0])
          return fail(p, HMLE_E_INVALID, "candidate batch: problems differ in their ordering");
    std::vector<double> xy((size_t)p->n * p->dim);
    HIP_TRY(hipMemcpy(xy.data(), p->d_coords, xy.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int32_t d = 0; d < p->dim; ++d)
      for (int32_t k = 1; k < q; ++k)
        for (int64_t i = 0; i < m; ++i)
          if (xy[(size_t)d * p->n + off[k] + i] != xy[(size_t)d * p->n + i])
            return fail(p, HMLE_E_INVALID, "candidate batch: problems are not copies of one point set");
    *count = q;
    *n1 = m;
    return HMLE_OK;
  });
}

hmle_status candidate_data(hmle_problem p, const double* z, int32_t count, int64_t n1, double** out) {
  return guarded(p, [&]() -> hmle_status {
    if ((int64_t)count * n1 != p->n) return fail(p, HMLE_E_INVALID, "candidate batch: wrong layout");
    if (!p->d_zrep) p->d_zrep = dev_alloc<double>((size_t)p->n, p->owned);
    for (int32_t k = 0; k < count; ++k)
      HIP_TRY(hipMemcpyAsync(p->d_zrep + (size_t)k * n1, z, n1 * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    *out = p->d_zrep;
    return HMLE_OK;
  });
}

hmle_status fit_fingerprint(hmle_problem p, const double* z, uint32_t* out) {
  if (p->state < 1) return fail(p, HMLE_E_STATE, "a structure-only problem cannot be fitted");
  return guarded(p, [&]() -> hmle_status {
    std::vector<double> h((size_t)p->n);
    HIP_TRY(hipMemcpyAsync(h.data(), z, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    uint32_t x = 2166136261u;
    auto mix = [&](const void* d, size_t len) {
      const unsigned char* b = static_cast<const unsigned char*>(d);
      for (size_t i = 0; i < len; ++i) x = (x ^ b[i]) * 16777619u;
    };
    mix(h.data(), h.size() * sizeof(double));
    const hmle_opts& o = p->opts;
    mix(&o.leaf_size, sizeof o.leaf_size);
    mix(&o.eta, sizeof o.eta);
    mix(&o.aca_tol, sizeof o.aca_tol);
    mix(&o.max_rank, sizeof o.max_rank);
    mix(&o.precision, sizeof o.precision);
    mix(&o.spd_margin, sizeof o.spd_margin);
    *out = x;
    return HMLE_OK;
  });
}

}  // namespace hmle

extern "C" {

hmle_status hmle_loglik(hmle_problem p, const double* z, double out[3]) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (!z || !out) return fail(p, HMLE_E_INVALID, "z and out must not be NULL");
  if (p->n_probs != 1) return fail(p, HMLE_E_INVALID, "a batch of problems: use hmle_loglik_batch");
  if (p->state != 3) return fail(p, HMLE_E_STATE, "factor first");
  return loglik_any(p, z, out, nullptr);
}

hmle_status hmle_loglik_batch(hmle_problem p, const double* z, double* out, hmle_status* per_problem) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (!z || !out || !per_problem) return fail(p, HMLE_E_INVALID, "z, out and per_problem must not be NULL");
  if (p->state != 3) return fail(p, HMLE_E_STATE, "factor first");
  return loglik_any(p, z, out, per_problem);
}

hmle_status hmle_eval_batch(hmle_problem p, const hmle_theta* thetas, const double* z, double* out,
                            hmle_status* per_problem) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (!thetas || !z || !out || !per_problem) return fail(p, HMLE_E_INVALID, "NULL argument");
  if (p->state < 1) return fail(p, HMLE_E_STATE, "build first");
  std::string why;
  for (int32_t q = 0; q < p->n_probs; ++q)
    if (!valid_theta(thetas + q, why)) return fail(p, HMLE_E_INVALID, why + " (problem " + std::to_string(q) + ")");
  return guarded(p, [&]() -> hmle_status {
    if (!p->gstream) HIP_TRY(hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking));
    // the caller's stream has produced z; the parameters' staging buffer is free after this sync
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipStreamSynchronize(p->gstream));
    for (int32_t q = 0; q < p->n_probs; ++q) {
      p->thetas[q] = thetas[q];
      p->h_mp[q] = problem_params(p, q, thetas[q]);
    }
    p->theta = p->thetas[0];
    p->mp = p->h_mp[0];
    p->saved = false;   // the captured evaluation reassembles: the cross-approximation factors change
    const bool plain = plain_launches();
    if (!p->graph_exec && !plain) {
      HIP_TRY(hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal));
      try {
        if (p->mixed()) run_eval<float>(p, p->gstream);
        else run_eval<double>(p, p->gstream);
      } catch (...) {
        hipGraph_t g = nullptr;   // end the capture so that the streams stay usable
        (void)hipStreamEndCapture(p->gstream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIP_TRY(hipStreamEndCapture(p->gstream, &p->graph));
      check_launches();
      HIP_TRY(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
    }
    HIP_TRY(hipEventRecord(p->ev[0], p->gstream));
    HIP_TRY(hipMemcpyAsync(p->d_mp, p->h_mp, p->n_probs * sizeof(MaternParams), hipMemcpyHostToDevice, p->gstream));
    HIP_TRY(hipMemcpyAsync(p->d_zin, z, (size_t)p->n * sizeof(double), hipMemcpyDeviceToDevice, p->gstream));
    if (plain) {
      if (p->mixed()) run_eval<float>(p, p->gstream);
      else run_eval<double>(p, p->gstream);
      check_launches();
    } else {
      HIP_TRY(hipGraphLaunch(p->graph_exec, p->gstream));
    }
    std::vector<double> r(2 * (size_t)p->n_probs);
    HIP_TRY(hipMemcpyAsync(r.data(), p->d_out, r.size() * sizeof(double), hipMemcpyDeviceToHost, p->gstream));
    HIP_TRY(hipEventRecord(p->ev[1], p->gstream));
    HIP_TRY(hipEventSynchronize(p->ev[1]));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
    p->t_ms[0] = 0.0;
    p->t_ms[1] = ms;
    p->t_ms[2] = 0.0;
    const bool prof = p->profile;
    p->profile = false;
    read_factor_status(p);
    p->profile = prof;
    p->state = 3;
    finish_loglik(p, r.data(), out, per_problem);
    return HMLE_OK;
  });
}

hmle_status hmle_predict(hmle_problem p, const double* z1, const double* pts2, int64_t m, double* z2) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (!z1 || m < 0 || (m > 0 && (!pts2 || !z2))) return fail(p, HMLE_E_INVALID, "bad z1, pts2, m or z2");
  if (p->state != 3) return fail(p, HMLE_E_STATE, "factor first");
  if (p->n_probs != 1) return fail(p, HMLE_E_INVALID, "prediction takes a single problem, not a batch");
  return guarded(p, [&]() -> hmle_status {
    const Plan& pl = p->plan;
    // forward substitution of P z1 (as for the log-likelihood): v = L~^{-1} P z1 in d_v + n
    launch_gather(z1, p->d_perm, p->n, p->d_v, p->stream);
    if (p->mixed()) run_solve<float>(p, p->stream);
    else run_solve<double>(p, p->stream);
    int32_t max_items = 1;
    for (int32_t j = 0; j < pl.n_steps; ++j) max_items = std::max(max_items, pl.fsolve_beg[j + 1] - pl.fsolve_beg[j]);
    if (!p->d_w) p->d_w = dev_alloc<double>((size_t)p->n, p->owned);
    if (!p->d_bpart) {
      p->d_bpart = dev_alloc<double>((size_t)max_items * 128, p->owned);
    }
    // backward substitution w = L~^{-T} v, leaves in reverse order
    for (int32_t j = pl.n_steps - 1; j >= 0; --j) {
      const int32_t* leaves = p->d_step_leaf + pl.step_leaf_beg[j];
      const int32_t nl = pl.step_leaf_beg[j + 1] - pl.step_leaf_beg[j];
      const InnerDesc* items = p->d_fsolve + pl.fsolve_beg[j];
      const int32_t ni = pl.fsolve_beg[j + 1] - pl.fsolve_beg[j];
      if (p->mixed()) launch_bsolve_step<float>(p->ctx<float>(), j, leaves, nl, items, ni, p->d_bpart, p->d_v + p->n,
                                                p->d_w, p->stream);
      else launch_bsolve_step<double>(p->ctx<double>(), j, leaves, nl, items, ni, p->d_bpart, p->d_v + p->n, p->d_w,
                                      p->stream);
    }
    launch_predict(p->d_coords, p->d_w, p->n, pts2, m, p->dim, p->mp, z2, p->stream);
    check_launches();
    HIP_TRY(hipStreamSynchronize(p->stream));
    return HMLE_OK;
  });
}

hmle_status hmle_predict_var(hmle_problem p, const double* pts2, int64_t m, double* var) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (m < 0 || (m > 0 && (!pts2 || !var))) return fail(p, HMLE_E_INVALID, "bad pts2, m or var");
  if (p->state != 3) return fail(p, HMLE_E_STATE, "factor first");
  if (p->n_probs != 1) return fail(p, HMLE_E_INVALID, "prediction takes a single problem, not a batch");
  return guarded(p, [&]() -> hmle_status {
    const Plan& pl = p->plan;
    if (!p->d_vmulti) p->d_vmulti = dev_alloc<double>(2 * (size_t)p->n * 32, p->owned);
    double* V = p->d_vmulti;
    double* Vout = p->d_vmulti + (size_t)p->n * 32;
    for (int64_t k0 = 0; k0 < m; k0 += 32) {
      const int32_t kk = (int32_t)std::min<int64_t>(32, m - k0);
      if (p->mixed())
        launch_predict_var<float>(p->ctx<float>(), pl.n_steps, p->d_step_leaf, pl.step_leaf_beg.data(), p->d_fsolve,
                                  pl.fsolve_beg.data(), pts2 + k0 * p->dim, kk, p->mp, p->theta.sigma2, V, Vout,
                                  var + k0, p->stream);
      else
        launch_predict_var<double>(p->ctx<double>(), pl.n_steps, p->d_step_leaf, pl.step_leaf_beg.data(), p->d_fsolve,
                                   pl.fsolve_beg.data(), pts2 + k0 * p->dim, kk, p->mp, p->theta.sigma2, V, Vout,
                                   var + k0, p->stream);
      check_launches();
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    return HMLE_OK;
  });
}

hmle_status hmle_mloe_mmom(hmle_problem pa, hmle_problem pt, const double* pts2, int64_t m, int32_t noisy,
                           double* e_ta, double* e_tt, double* e_aa, double out[2]) {
  if (!pa || !pt) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (m < 1 || !pts2 || !out) return fail(pa, HMLE_E_INVALID, "need m >= 1 new points, pts2 and out");
  if (pa->state != 3 || pt->state != 3) return fail(pa, HMLE_E_STATE, "both problems must be factored");
  if (pa->n_probs != 1 || pt->n_probs != 1) return fail(pa, HMLE_E_INVALID, "single problems only, not batches");
  if (pa->n != pt->n || pa->dim != pt->dim || pa->tree.perm != pt->tree.perm || pa->opts.leaf_size != pt->opts.leaf_size)
    return fail(pa, HMLE_E_INVALID, "the two problems must be built on the same points with the same leaf size");
  if (pa->stream != pt->stream) return fail(pa, HMLE_E_INVALID, "the two problems must share one stream");
  return guarded(pa, [&]() -> hmle_status {
    const int64_t n = pa->n;
    hipStream_t st = pa->stream;
    if (pa != pt) {   // the same coordinates in the same internal order
      std::vector<double> ca((size_t)n * pa->dim), cb((size_t)n * pa->dim);
      HIP_TRY(hipMemcpy(ca.data(), pa->d_coords, ca.size() * sizeof(double), hipMemcpyDeviceToHost));
      HIP_TRY(hipMemcpy(cb.data(), pt->d_coords, cb.size() * sizeof(double), hipMemcpyDeviceToHost));
      if (ca != cb) return fail(pa, HMLE_E_INVALID, "the two problems must be built on the same points");
    }
    // workspace (the estimated model's problem): cross covariances of both models, their
    // forward substitutions, one weight vector, one product, the short vectors of the
    // transposed product, and the three error arrays when the caller passes none
    if (!pa->d_vmulti) pa->d_vmulti = dev_alloc<double>(2 * (size_t)n * 32, pa->owned);
    if (!pa->d_mlw) pa->d_mlw = dev_alloc<double>((size_t)n * 32 + 2 * (size_t)n, pa->owned);
    int32_t max_items = 1;
    for (int32_t j = 0; j < pa->plan.n_steps; ++j)
      max_items = std::max(max_items, pa->plan.fsolve_beg[j + 1] - pa->plan.fsolve_beg[j]);
    if (!pa->d_bpart) pa->d_bpart = dev_alloc<double>((size_t)max_items * 128, pa->owned);
    if (!pt->d_mvh) pt->d_mvh = dev_alloc<double>((size_t)std::max(1, pt->plan.n_lowrank) * 2 * pt->plan.aca_width,
                                                  pt->owned);
    auto arr = [&](double* given) -> double* { return given ? given : dev_alloc<double>((size_t)m, pa->owned); };
    double* Eta = arr(e_ta);
    double* Ett = arr(e_tt);
    double* Eaa = arr(e_aa);
    double* V = pa->d_vmulti;                      // n x 32: right-hand sides, then their running values
    double* Vout = pa->d_vmulti + (size_t)n * 32;  // n x 32: L_a^{-1} c_a
    double* Ct = pa->d_mlw;                        // n x 32: the true model's cross covariances
    double* w = pa->d_mlw + (size_t)n * 32;        // kriging weights of one point
    double* y = w + n;                             // L_t^T w
    const Plan& pl = pa->plan;
    const Plan& plt = pt->plan;
    const double var_t = pt->theta.sigma2 + (noisy ? pt->theta.tau2 : 0.0);
    for (int64_t k0 = 0; k0 < m; k0 += 32) {
      const int32_t kk = (int32_t)std::min<int64_t>(32, m - k0);
      const double* p2 = pts2 + k0 * pa->dim;
      // E_t and E_a of the true and the estimated model's own predictions: kriging
      // variances (plus the nugget of a noisy target); the estimated model's call
      // leaves L_a^{-1} c_a in Vout
      double* Vt = Ct;   // the true model's forward substitutions use Ct and the V pair as scratch
      if (pt->mixed())
        launch_predict_var<float>(pt->ctx<float>(), plt.n_steps, pt->d_step_leaf, plt.step_leaf_beg.data(), pt->d_fsolve,
                                  plt.fsolve_beg.data(), p2, kk, pt->mp, pt->theta.sigma2, Vt, Vout, Ett + k0, st);
      else
        launch_predict_var<double>(pt->ctx<double>(), plt.n_steps, pt->d_step_leaf, plt.step_leaf_beg.data(),
                                   pt->d_fsolve, plt.fsolve_beg.data(), p2, kk, pt->mp, pt->theta.sigma2, Vt, Vout,
                                   Ett + k0, st);
      if (pa->mixed())
        launch_predict_var<float>(pa->ctx<float>(), pl.n_steps, pa->d_step_leaf, pl.step_leaf_beg.data(), pa->d_fsolve,
                                  pl.fsolve_beg.data(), p2, kk, pa->mp, pa->theta.sigma2, V, Vout, Eaa + k0, st);
      else
        launch_predict_var<double>(pa->ctx<double>(), pl.n_steps, pa->d_step_leaf, pl.step_leaf_beg.data(),
                                   pa->d_fsolve, pl.fsolve_beg.data(), p2, kk, pa->mp, pa->theta.sigma2, V, Vout,
                                   Eaa + k0, st);
      if (noisy) {
        launch_add_scalar(Ett + k0, kk, pt->theta.tau2, st);
        launch_add_scalar(Eaa + k0, kk, pa->theta.tau2, st);
      }
      launch_cross_cols(pa->d_coords, pa->n, p2, kk, pa->dim, pt->mp, Ct, st);
      for (int32_t k = 0; k < kk; ++k) {
        // w = L_a^{-T} (L_a^{-1} c_a): the backward substitution, leaves in reverse order
        for (int32_t j = pl.n_steps - 1; j >= 0; --j) {
          const int32_t* leaves = pa->d_step_leaf + pl.step_leaf_beg[j];
          const int32_t nl = pl.step_leaf_beg[j + 1] - pl.step_leaf_beg[j];
          const InnerDesc* items = pa->d_fsolve + pl.fsolve_beg[j];
          const int32_t ni = pl.fsolve_beg[j + 1] - pl.fsolve_beg[j];
          if (pa->mixed())
            launch_bsolve_step<float>(pa->ctx<float>(), j, leaves, nl, items, ni, pa->d_bpart, Vout + (size_t)k * n, w,
                                      st);
          else
            launch_bsolve_step<double>(pa->ctx<double>(), j, leaves, nl, items, ni, pa->d_bpart, Vout + (size_t)k * n,
                                       w, st);
        }
        // y = L_t^T w, so that w^T C~_t w = |y|^2
        if (pt->mixed())
          launch_factor_t_product<float>(pt->ctx<float>(), plt.n_dense, plt.n_lowrank, plt.n_leaves, pt->d_colp_beg,
                                         pt->d_colp, w, pt->d_mvh, y, st);
        else
          launch_factor_t_product<double>(pt->ctx<double>(), plt.n_dense, plt.n_lowrank, plt.n_leaves, pt->d_colp_beg,
                                          pt->d_colp, w, pt->d_mvh, y, st);
        launch_eta_point(w, Ct + (size_t)k * n, y, n, var_t, Eta + k0 + k, st);
      }
      check_launches();
    }
    double* dout = pa->d_out;   // two doubles (single problem)
    launch_mloe_final(Eta, Ett, Eaa, m, dout, st);
    check_launches();
    HIP_TRY(hipMemcpyAsync(out, dout, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return HMLE_OK;
  });
}

hmle_status hmle_sample(hmle_problem p, const double* w, double* z) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (!w || !z) return fail(p, HMLE_E_INVALID, "w and z must not be NULL");
  if (p->state != 3) return fail(p, HMLE_E_STATE, "factor first");
  return guarded(p, [&]() -> hmle_status {
    const Plan& pl = p->plan;
    if (p->mixed())
      launch_sample<float>(p->ctx<float>(), pl.n_dense, pl.n_lowrank, pl.n_leaves, p->d_rowp_beg, p->d_rowp, w, p->d_h,
                           p->d_v, p->stream);
    else
      launch_sample<double>(p->ctx<double>(), pl.n_dense, pl.n_lowrank, pl.n_leaves, p->d_rowp_beg, p->d_rowp, w,
                            p->d_h, p->d_v, p->stream);
    launch_scatter(p->d_v, p->d_perm, p->n, z, p->stream);
    check_launches();
    HIP_TRY(hipStreamSynchronize(p->stream));
    return HMLE_OK;
  });
}

hmle_status hmle_matvec(hmle_problem p, const double* x, double* y) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (!x || !y) return fail(p, HMLE_E_INVALID, "x and y must not be NULL");
  if (p->state != 2) return fail(p, HMLE_E_STATE, p->state == 3 ? "the factorisation consumed the assembled matrix; "
                                                                   "assemble again" : "assemble first");
  return guarded(p, [&]() -> hmle_status {
    const Plan& pl = p->plan;
    if (!p->d_mvh) p->d_mvh = dev_alloc<double>((size_t)std::max(1, pl.n_lowrank) * 2 * pl.aca_width, p->owned);
    launch_gather(x, p->d_perm, p->n, p->d_v, p->stream);
    if (p->mixed())
      launch_matvec<float>(p->ctx<float>(), pl.n_dense, pl.n_lowrank, pl.n_leaves, p->d_rowp_beg, p->d_rowp,
                           p->d_colp_beg, p->d_colp, p->d_v, p->d_mvh, p->d_v + p->n, p->stream);
    else
      launch_matvec<double>(p->ctx<double>(), pl.n_dense, pl.n_lowrank, pl.n_leaves, p->d_rowp_beg, p->d_rowp,
                            p->d_colp_beg, p->d_colp, p->d_v, p->d_mvh, p->d_v + p->n, p->stream);
    launch_scatter(p->d_v + p->n, p->d_perm, p->n, y, p->stream);
    check_launches();
    HIP_TRY(hipStreamSynchronize(p->stream));
    return HMLE_OK;
  });
}

hmle_status hmle_matern(const double* h, int64_t count, const hmle_theta* theta, hmle_precision precision,
                        void* hip_stream, double* out) {
  std::string why;
  if (!valid_theta(theta, why)) return fail(nullptr, HMLE_E_INVALID, why);
  if (count < 0 || (count > 0 && (!h || !out))) return fail(nullptr, HMLE_E_INVALID, "bad buffers");
  return guarded(nullptr, [&]() -> hmle_status {
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    launch_matern(h, count, matern_params(*theta), precision == HMLE_MIXED ? 1 : 0, out, st);
    check_launches();
    HIP_TRY(hipStreamSynchronize(st));
    return HMLE_OK;
  });
}

hmle_status hmle_sizes(hmle_problem p, int64_t sizes[6]) {
  if (!p || !sizes) return fail(p, HMLE_E_INVALID, "NULL argument");
  sizes[0] = p->n; sizes[1] = p->dim; sizes[2] = p->tree.n_nodes();
  sizes[3] = p->plan.n_dense; sizes[4] = p->plan.n_lowrank; sizes[5] = p->plan.n_leaves;
  return HMLE_OK;
}

hmle_status hmle_export_tree(hmle_problem p, int64_t* perm, int64_t* nodes, double* bmin, double* bmax) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  const ClusterTree& t = p->tree;
  if (perm) for (int32_t i = 0; i < t.n; ++i) perm[i] = t.perm[i];
  if (nodes)
    for (int32_t i = 0; i < t.n_nodes(); ++i) {
      nodes[4 * i] = t.lo[i]; nodes[4 * i + 1] = t.hi[i];
      nodes[4 * i + 2] = t.child0[i]; nodes[4 * i + 3] = t.child1[i];
    }
  if (bmin) std::memcpy(bmin, t.bmin.data(), t.bmin.size() * sizeof(double));
  if (bmax) std::memcpy(bmax, t.bmax.data(), t.bmax.size() * sizeof(double));
  return HMLE_OK;
}

hmle_status hmle_export_blocks(hmle_problem p, int64_t* dense, int64_t* lowrank) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (dense)
    for (size_t i = 0; i < p->bt.dense_t.size(); ++i) { dense[2 * i] = p->bt.dense_t[i]; dense[2 * i + 1] = p->bt.dense_s[i]; }
  if (lowrank)
    for (size_t i = 0; i < p->bt.lr_t.size(); ++i) { lowrank[2 * i] = p->bt.lr_t[i]; lowrank[2 * i + 1] = p->bt.lr_s[i]; }
  return HMLE_OK;
}

hmle_status hmle_export_block(hmle_problem p, int32_t kind, int64_t which, double* data, int64_t cap, int32_t* rank) {
  if (!p || !data || !rank) return fail(p, HMLE_E_INVALID, "NULL argument");
  if (p->state < 2) return fail(p, HMLE_E_STATE, "nothing assembled");
  const Plan& pl = p->plan;
  int64_t bi = kind == 0 ? which : pl.n_dense + which;
  if (which < 0 || (kind == 0 && which >= pl.n_dense) || (kind == 1 && which >= pl.n_lowrank) || (kind != 0 && kind != 1))
    return fail(p, HMLE_E_INVALID, "block index out of range");
  return guarded(p, [&]() -> hmle_status {
    HIP_TRY(hipStreamSynchronize(p->stream));
    const BlockDesc& b = pl.blocks[bi];
    const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
    const bool mixed = p->mixed();
    const size_t ts = mixed ? sizeof(float) : sizeof(double);
    auto fetch = [&](const void* base, int64_t off, int64_t count, std::vector<double>& dst) {
      dst.resize(count);
      if (mixed) {
        std::vector<float> f(count);
        HIP_TRY(hipMemcpy(f.data(), static_cast<const char*>(base) + off * ts, count * ts, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < count; ++i) dst[i] = f[i];
      } else {
        HIP_TRY(hipMemcpy(dst.data(), static_cast<const char*>(base) + off * ts, count * ts, hipMemcpyDeviceToHost));
      }
    };
    if (b.kind == BK_DIAG) {
      if (cap < m * k) return fail(p, HMLE_E_INVALID, "cap too small");
      HIP_TRY(hipMemcpy(data, p->d_D + b.loff, m * k * sizeof(double), hipMemcpyDeviceToHost));
      *rank = -1;
    } else if (b.kind == BK_DENSE) {
      if (cap < m * k) return fail(p, HMLE_E_INVALID, "cap too small");
      std::vector<double> w;
      fetch(p->d_L, b.loff, m * k, w);     // transposed storage: entry (i,j) at j + i*k
      for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < k; ++j) data[i + j * m] = w[j + i * k];
      *rank = -1;
    } else {
      int32_t r = 0;
      const bool factored = p->state == 3;
      HIP_TRY(hipMemcpy(&r, (factored ? p->d_rank : p->d_arank) + bi, sizeof(int32_t), hipMemcpyDeviceToHost));
      if (cap < (m + k) * r) return fail(p, HMLE_E_INVALID, "cap too small");
      const int64_t width = factored ? pl.rank_width : pl.aca_width;
      const void* base = factored ? p->d_L : p->d_A;
      const int64_t off = factored ? b.loff : b.aoff;
      std::vector<double> u, w;
      fetch(base, off, m * width, u);
      fetch(base, off + m * width, k * width, w);
      for (int64_t l = 0; l < r; ++l) {
        for (int64_t i = 0; i < m; ++i) data[i + l * m] = u[i + l * m];
        for (int64_t j = 0; j < k; ++j) data[m * r + j + l * k] = w[j + l * k];
      }
      *rank = r;
    }
    return HMLE_OK;
  });
}

hmle_status hmle_profile(hmle_problem p, int32_t enable, double out[9]) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (p->state < 1) return fail(p, HMLE_E_STATE, "build_tree first");
  return guarded(p, [&]() -> hmle_status {
    if (out)
      for (int i = 0; i < 9; ++i) out[i] = p->prof[i];
    if (enable >= 0) {
      p->profile = enable != 0;
      for (double& v : p->prof) v = 0.0;
      if (p->profile && p->pev.empty()) {
        p->pev.resize(8 * (size_t)p->plan.n_steps);
        for (auto& e : p->pev) HIP_TRY(hipEventCreate(&e));
      }
    }
    return HMLE_OK;
  });
}

hmle_status hmle_assembly_info(hmle_problem p, int64_t info[2]) {
  if (!p || !info) return fail(p, HMLE_E_INVALID, "NULL argument");
  info[0] = p->reuse_last;
  info[1] = p->reuse_total;
  return HMLE_OK;
}

hmle_status hmle_stats(hmle_problem p, double t[3], int64_t c[3]) {
  if (!p) return fail(nullptr, HMLE_E_INVALID, "problem is NULL");
  if (t) for (int i = 0; i < 3; ++i) t[i] = p->t_ms[i];
  if (c) for (int i = 0; i < 3; ++i) c[i] = p->counters[i];
  return HMLE_OK;
}

hmle_status hmle_autotune(const double* pts, int64_t n, int32_t dim, const hmle_opts* opts, const hmle_theta* theta,
                          void* hip_stream, hmle_opts* best, hmle_tune_entry* tried, int32_t max_tried,
                          int32_t* n_tried) {
  if (!best) return fail(nullptr, HMLE_E_INVALID, "best is NULL");
  if (max_tried < 0) return fail(nullptr, HMLE_E_INVALID, "max_tried must be >= 0");
  hmle_opts o;
  hmle_default_opts(&o);
  if (opts) o = *opts;
  const hmle_status os = check_opts(o);
  if (os != HMLE_OK) return os;
  std::string why;
  if (!valid_theta(theta, why)) return fail(nullptr, HMLE_E_INVALID, why);
  if (n_tried) *n_tried = 0;
  // a warm factorisation with the candidate options (the second of two: the replayed one)
  std::vector<std::pair<hmle_opts, double>> seen;
  auto same = [](const hmle_opts& a, const hmle_opts& b) {
    return a.pair_chunk == b.pair_chunk && a.sketch_group == b.sketch_group && a.seg_entries == b.seg_entries &&
           a.gseg_rows == b.gseg_rows && a.sum_kc == b.sum_kc;
  };
  auto measure = [&](const hmle_opts& c, double& ms) -> hmle_status {
    for (const auto& e : seen)
      if (same(e.first, c)) { ms = e.second; return HMLE_OK; }
    hmle_problem p = nullptr;
    hmle_status st = hmle_build_tree(pts, n, dim, &c, hip_stream, &p);
    if (st != HMLE_OK) return st;
    for (int rep = 0; rep < 2; ++rep) {
      st = hmle_assemble(p, theta);
      if (st == HMLE_OK) st = hmle_factor(p);
      if (st != HMLE_OK) break;
    }
    ms = p->t_ms[1];
    hmle_destroy(p);
    if (st != HMLE_OK && st != HMLE_E_NOT_SPD) return st;
    seen.push_back({c, ms});
    if (tried && (int32_t)seen.size() <= max_tried) tried[seen.size() - 1] = {c, ms};
    if (n_tried) *n_tried = (int32_t)seen.size();
    return HMLE_OK;
  };
  hmle_opts cur = with_defaults(o);
  double cur_ms = 0.0;
  hmle_status st = measure(cur, cur_ms);
  if (st != HMLE_OK) return st;
  const std::vector<int32_t> chunks = {1, 2, 4}, groups = {2, 4, 8, 16}, segs = {2, 4, 8, 16},
                             gsegs = {128, 256, 512, 1024}, kcs = {16, 32};
  for (int sweep = 0; sweep < 2; ++sweep)
    for (int knob = 0; knob < 5; ++knob) {
      const std::vector<int32_t>& vals = knob == 0 ? chunks : knob == 1 ? groups : knob == 2 ? segs : knob == 3 ? gsegs : kcs;
      for (int32_t v : vals) {
        hmle_opts c = cur;
        int32_t& f = knob == 0 ? c.pair_chunk : knob == 1 ? c.sketch_group : knob == 2 ? c.seg_entries
                   : knob == 3 ? c.gseg_rows : c.sum_kc;
        f = v;
        double ms = 0.0;
        st = measure(c, ms);
        if (st != HMLE_OK) return st;
        if (ms < cur_ms) { cur_ms = ms; cur = c; }
      }
    }
  *best = cur;
  return HMLE_OK;
}

const char* hmle_last_error(hmle_problem p) { return p ? p->err.c_str() : g_last_error.c_str(); }

void hmle_destroy(hmle_problem p) { delete p; }

}  // extern "C"
