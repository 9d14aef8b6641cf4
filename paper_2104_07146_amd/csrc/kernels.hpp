// Launch interface between the host runtime and the HIP kernels.
#pragma once
#include "common.hpp"

namespace hmle {

// Device view of one problem, passed by value to every kernel.
// TS: storage/arithmetic type of off-diagonal and low-rank blocks
// (double in the FP64 mode, float in the mixed mode).
template <typename TS>
struct DevCtx {
  const BlockDesc* blocks;
  const PairDesc* pairs;
  const int64_t* pair_beg;
  const int32_t* leaf_lo;
  const int32_t* leaf_hi;
  const int32_t* leaf_diag;
  const int64_t* leaf_inv_off;
  const double* coords;     // dim x n, internal order (structure of arrays)
  TS* L;                    // off-diagonal factor pool
  double* D;                // diagonal leaves
  TS* A;                    // cross-approximation factors
  TS* S;                    // sketch scratch
  double* inv;              // inverted diagonal leaves
  int32_t* rank;            // per block: current rank of low-rank blocks
  int32_t* rank1;           // per low-rank block: width of its range basis after the first sketch pass
  int32_t* arank;           // per block: cross-approximation rank
  int32_t* status;          // [1] rank-cap hits, [2] cross-approximation cap hits
  int32_t* pstatus;         // per problem: first failing leaf + 1 (0: positive definite so far)
  double* pstatus_val;      // per problem: the failing pivot
  const MaternParams* mp;   // per problem: covariance parameters
  const int32_t* prob_leaf0;   // per problem: index of its first leaf (leaf of problem p at step s: prob_leaf0[p] + s)
  TS* gram;                 // cached W_x^T W_y of low-rank pairs (R x R per slot)
  int32_t n, dim, R, Ra;
  int32_t sum_kc;           // inner-dimension columns per staged chunk of the sketch-sum tiles (16 or 32)
};

struct StepLists {
  const ChunkDesc* dchunks; int32_t n_dchunks;
  const TargetDesc* dtargets; int32_t n_dtargets;
  const RTargetDesc* rtargets; int32_t n_rtargets;
  const ChunkDesc* r1chunks; int32_t n_r1chunks;
  const ChunkDesc* r2chunks; int32_t n_r2chunks;
  const RPairDesc* rpairs1;   // pair arrays of the two passes (chunks index them)
  const RPairDesc* rpairs2;
  const GItem* g1; int32_t n_g1;
  const GItem* g2; int32_t n_g2;
  const GFin* gf1; int32_t n_gf1;      // sums of segmented input-side products
  const GFin* gf2; int32_t n_gf2;
  void* gseg;                          // their segment partials (TS, 64 x 64 each)
  const RowTile* tiles1; int32_t n_t1;
  const RowTile* tiles2; int32_t n_t2;
  const TileChunk* tc1;   // tile-chunk lists of the two passes
  const TileChunk* tc2;
  const TileSeg* sg1; int32_t n_sg1;   // segments of the tiles' chunk lists
  const TileSeg* sg2; int32_t n_sg2;
  void* spart;                         // partial tiles of the segments (TS, 128 x 64 each)
  void* dpart;   // partial sums of the dense-target chunks (TS)
  void* rpart;   // partial sums of the low-rank-target chunks (TS)
  void* gbuf;    // input-side products of the sketch passes (TS, 64 x 64 per slot)
  double* gpart; // Gram partials of the sketch tiles (R x R float64 per tile of the step)
  double* qbuf;  // per low-rank target of the step: two 64 x 64 float64 factors of its QR
  int* qint;     // per low-rank target of the step: 4 ints (ranks, column count)
  const int32_t* active; int32_t n_active;
  const InnerDesc* inner; int32_t n_inner;
  const InnerDesc* tsolve; int32_t n_tsolve;   // column solves per 32-column slice
  const PairDesc* grams; int32_t n_grams;   // Gram matrices that become computable after this step
  const int32_t* leaves; int32_t n_leaves;  // diagonal leaves of this step (one per problem still running)
};

template <typename TS> void launch_assemble(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, double eps,
                                            hipStream_t st);
// One factorisation step (leaf column j) in four parts: dense-target updates,
// low-rank-target updates (independent of the former, may run on a second
// stream), the diagonal leaf, and the column solves / inner updates / Gram
// matrices (after both update parts).
template <typename TS> void launch_step_dense(const DevCtx<TS>& c, const StepLists& sl, hipStream_t st);
// ev (may be NULL): four events recorded around the two sketch-pass launches (k_rpass)
template <typename TS> void launch_step_lowrank(const DevCtx<TS>& c, const StepLists& sl, double eps, hipStream_t st,
                                                hipEvent_t* ev = nullptr);
template <typename TS> void launch_step_diag(const DevCtx<TS>& c, const StepLists& sl, hipStream_t st);
template <typename TS> void launch_step_cols(const DevCtx<TS>& c, int32_t s, const StepLists& sl, hipStream_t st);
template <typename TS> void launch_dense_pairs(const DevCtx<TS>& c, const StepLists& sl, hipStream_t st);
template <typename TS> void launch_dense_reduce(const DevCtx<TS>& c, const StepLists& sl, hipStream_t st);
template <typename TS> void launch_gen_omega(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, hipStream_t st);
// items: (block, rows [r0, c0)) of the blocks in the step's columns
template <typename TS> void launch_solve_step(const DevCtx<TS>& c, int32_t s, const int32_t* leaves, int32_t n_leaves,
                                              const InnerDesc* items, int32_t n_items, double* v, hipStream_t st);
// y = L w (internal order): h = W_b^T w[sigma_b] for low-rank blocks, then one
// workgroup per leaf row gathers its diagonal, dense and low-rank terms.
template <typename TS> void launch_sample(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, int32_t n_leaves,
                                          const int32_t* rowp_beg, const int32_t* rowp, const double* w, double* h,
                                          double* y, hipStream_t st);
// y = C~ x of the assembled matrix (internal order) before the factorisation:
// h = (W0^T x[cols], U0^T x[rows]) per low-rank block (n_lowrank * 2 * Ra
// doubles), then one workgroup per leaf gathers its diagonal block, its row
// panel and, mirrored, its column panel (colp: off-diagonal blocks whose
// columns hold the leaf, CSR over leaves).
template <typename TS> void launch_matvec(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, int32_t n_leaves,
                                          const int32_t* rowp_beg, const int32_t* rowp, const int32_t* colp_beg,
                                          const int32_t* colp, const double* x, double* h, double* y, hipStream_t st);

// Assembly reuse when theta changes only in sigma^2 and tau^2: dense
// off-diagonal entries (the first l_dense elements of the factor pool) = s *
// Lsave; diagonal leaves = s (Dsave - t0 I) + t1 I; cross-approximation
// factors U0 *= f.
template <typename TS> void launch_rescale(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, int32_t n_leaves,
                                           const TS* Lsave, int64_t l_dense, const double* Dsave, double s, double t0,
                                           double t1, double f, hipStream_t st);

// y = L~^T x with the factor (internal order; g: n_lowrank * R doubles).
template <typename TS> void launch_factor_t_product(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank,
                                                    int32_t n_leaves, const int32_t* colp_beg, const int32_t* colp,
                                                    const double* x, double* g, double* y, hipStream_t st);
// B (n x 32, column-major): Matern cross covariances of kk <= 32 new points p2
// (row-major, dim) to the internal-order points (no nugget), zero columns after kk.
void launch_cross_cols(const double* coords, int32_t n, const double* p2, int32_t kk, int32_t dim,
                       const MaternParams& mp, double* B, hipStream_t st);
// out = |y|^2 - 2 w . ct + var (one new point's expected squared error).
void launch_eta_point(const double* w, const double* ct, const double* y, int64_t n, double var, double* out,
                      hipStream_t st);
// out[0] = mean(e_ta / e_tt - 1), out[1] = mean(e_aa / e_ta - 1) over m points.
void launch_mloe_final(const double* e_ta, const double* e_tt, const double* e_aa, int64_t m, double* out,
                       hipStream_t st);
void launch_add_scalar(double* x, int64_t count, double v, hipStream_t st);

void launch_matern(const double* h, int64_t count, const MaternParams& mp, int precision, double* out, hipStream_t st);
void launch_gather_coords(const double* pts, const int32_t* perm, int32_t n, int32_t dim, double* coords, hipStream_t st);
void launch_gather(const double* z, const int32_t* perm, int32_t n, double* v, hipStream_t st);
// Backward substitution step s of a single problem: w[leaf] from v[leaf] and
// the final w of the rows below (part: n_items x TILE doubles of scratch).
template <typename TS> void launch_bsolve_step(const DevCtx<TS>& c, int32_t s, const int32_t* leaves, int32_t n_leaves,
                                               const InnerDesc* items, int32_t n_items, double* part, const double* v,
                                               double* w, hipStream_t st);
// Kriging variance at kk <= 32 points p2 of a single problem: step_leaf and
// step_leaf_beg, fsolve and fsolve_beg as in the plan (device lists, host
// CSR offsets); V, Vout: n x 32 doubles of scratch; var: kk doubles.
template <typename TS>
void launch_predict_var(const DevCtx<TS>& c, int32_t n_steps, const int32_t* step_leaf, const int32_t* step_leaf_beg,
                        const InnerDesc* fsolve, const int32_t* fsolve_beg, const double* p2, int32_t kk,
                        const MaternParams& mp, double sigma2, double* V, double* Vout, double* var, hipStream_t st);
// Kriging mean at m points p2 (row-major m x dim) from w = C~^{-1} z1.
void launch_predict(const double* c1, const double* w, int32_t n1, const double* p2, int64_t m, int32_t dim,
                    const MaternParams& mp, double* z2, hipStream_t st);
void launch_scatter(const double* v, const int32_t* perm, int32_t n, double* z, hipStream_t st);
void launch_check_finite(const double* x, int64_t count, int32_t* flag, hipStream_t st);
// per problem p: out[2p] = sum over its leaves of 2 sum log L_ii, out[2p+1] = v^T v over its points
void launch_reduce(const double* D, const int64_t* diag_off, const int32_t* leaf_lo, const int32_t* leaf_hi,
                   int32_t n_leaves, const int32_t* prob_leaf0, int32_t n_probs, const double* v, double* partial,
                   double* out, hipStream_t st);
// x[0:count) = 0 with a kernel (safe inside captured graphs)
void launch_zero_i32(int32_t* x, int32_t count, hipStream_t st);

}  // namespace hmle
