// Host-side, theta-independent structure of one problem: cluster tree, block
// tree (Section 2's recursive partition, under the rules stated in tree.cpp)
// and the schedule of the left-looking H-Cholesky.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.hpp"

namespace hmle {

struct ClusterTree {
  int32_t n = 0, dim = 0;
  std::vector<int32_t> perm;               // perm[k] = caller index of internal point k
  std::vector<int32_t> lo, hi, child0, child1, level, parent;
  std::vector<double> bmin, bmax;          // n_nodes * dim
  int32_t n_nodes() const { return (int32_t)lo.size(); }
  bool is_leaf(int32_t t) const { return child0[t] < 0; }
};

struct BlockTree {
  std::vector<int32_t> dense_t, dense_s;   // sorted by (col lo, row lo)
  std::vector<int32_t> lr_t, lr_s;
};

// Schedule of the factorisation. A plan covers a batch of independent
// problems (a forest: problem p owns points [prob_off[p], prob_off[p+1]) of the
// internal order and leaves [prob_leaf0[p], prob_leaf0[p+1])); a single problem
// is a batch of one. Step s processes the s-th leaf column j of every problem
// that has one, so the batch takes as many steps as its largest problem has
// leaves. At step s, for each problem's leaf j:
//   1. external updates of every block whose column range starts at leaf j
//      (dense targets: ext_dense; low-rank targets: ext_lr), each a list of
//      PairDesc (CSR by target in pair_beg);
//   2. Cholesky of the diagonal leaf j;
//   3. the column solve W_b[leaf j rows] <- L_jj^{-1} W_b[leaf j rows] for every
//      off-diagonal block b whose column range contains leaf j (active);
//   4. inner updates W_b[rows of x] -= L_x[:, leaf j] W_b[leaf j rows] for the
//      active b not ending at leaf j and active x inside b's column range.
struct Plan {
  std::vector<BlockDesc> blocks;           // dense first (diag + off-diag), then low-rank
  int32_t n_dense = 0, n_lowrank = 0, n_leaves = 0;
  int32_t n_probs = 1, n_steps = 0;
  std::vector<int64_t> prob_off;           // per problem: first point (internal order), n_probs + 1 entries
  std::vector<int32_t> prob_leaf0;         // per problem: first leaf, n_probs + 1 entries
  std::vector<int32_t> step_leaf_beg, step_leaf;   // leaves of each step (CSR over steps)
  std::vector<int32_t> leaf_lo, leaf_hi, leaf_diag;   // per leaf
  std::vector<int64_t> leaf_inv_off;                  // offset of L_jj^{-1} (m*m doubles)
  // pairs of every block (CSR over block index)
  std::vector<int64_t> pair_beg;
  std::vector<PairDesc> pairs;
  // per-step lists (CSR over steps)
  std::vector<int32_t> ext_dense_beg, ext_dense;
  std::vector<int32_t> ext_lr_beg, ext_lr;
  // pair chunks per step (CSR over steps), dense and low-rank targets, and the
  // per-step target lists pointing into them
  std::vector<int32_t> dchunk_beg, dtarget_beg;
  std::vector<ChunkDesc> dchunks;
  std::vector<TargetDesc> dtargets;
  // low-rank targets: per step, pass-1 / pass-2 pair orders, chunks and
  // input-side products (CSR over steps)
  std::vector<RPairDesc> rpairs1, rpairs2;
  std::vector<int32_t> r1chunk_beg, r2chunk_beg, rtarget_beg, g1_beg, g2_beg;
  std::vector<ChunkDesc> r1chunks, r2chunks;
  std::vector<RTargetDesc> rtargets;
  std::vector<GItem> g1items, g2items;
  std::vector<int32_t> gf1_beg, gf2_beg;     // segmented input-side products (CSR over steps)
  std::vector<GFin> gf1, gf2;
  int32_t max_gparts = 0;                    // segment partials in any one step (either pass)
  std::vector<int32_t> t1_beg, t2_beg;
  std::vector<RowTile> tiles1, tiles2;
  std::vector<int32_t> tc1_beg, tc2_beg;   // per tile: the chunks touching its rows (CSR over steps)
  std::vector<TileChunk> tc1, tc2;
  std::vector<int32_t> sg1_beg, sg2_beg;     // segments of the tiles' entry lists (CSR over steps)
  std::vector<TileSeg> sg1, sg2;
  int32_t max_segs = 0;                      // segments in any one step (either pass)
  int32_t max_gslots = 0;
  int32_t max_tiles = 0;      // row tiles of the low-rank targets in any one step (either pass)
  int32_t max_rtargets = 0;   // low-rank targets in any one step
  int64_t dpart_size = 0;   // partial buffer elements needed by any one step (dense)
  int64_t rpart_size = 0;   // (low-rank: max(m, k) * R per chunk)
  int32_t pair_chunk = 4;
  int32_t seg_entries = 8;   // chunk entries per segment of a sketch-sum tile
  int32_t gseg_rows = 512;   // rows per segment of an input-side product
  // Gram matrices W_x[w]^T W_y[w] of the distinct low-rank/low-rank pairs,
  // computed once at the step after which both blocks are final (CSR over steps)
  std::vector<int32_t> gram_beg;
  std::vector<PairDesc> grams;      // x, y, w0, w1 used; rx0 = slot
  int64_t n_grams = 0;
  std::vector<int32_t> active_beg, active;
  std::vector<int32_t> inner_beg;
  std::vector<InnerDesc> inner;
  std::vector<int32_t> fsolve_beg;   // forward-solve items of a step: (block, rows [r0, c0)) (CSR over steps)
  std::vector<InnerDesc> fsolve;
  std::vector<int32_t> tsolve_beg;   // column solves of a step, per 32-column slice (CSR over steps)
  std::vector<InnerDesc> tsolve;
  // row panels: off-diagonal blocks whose rows contain leaf i (CSR over leaves)
  std::vector<int32_t> rowp_beg, rowp;
  // column panels: off-diagonal blocks whose columns contain leaf i (CSR over leaves)
  std::vector<int32_t> colp_beg, colp;
  // storage sizes (elements)
  int64_t l_size = 0;       // factor pool (off-diagonal blocks)
  int64_t d_size = 0;       // diagonal leaves (always float64)
  int64_t a_size = 0;       // cross-approximation factors
  int64_t s_size = 0;       // sketch scratch
  int64_t inv_size = 0;     // inverted diagonal leaves
  int32_t rank_width = 0;   // R: low-rank storage width / sketch width
  int32_t aca_width = 0;    // Ra: cross-approximation rank cap
  int32_t max_leaf = 0;
  int64_t max_dense_dim = 0;
  // algorithmic counters
  int64_t dense_entries = 0;     // entries of all dense blocks (diag full squares)
  int64_t lr_dims = 0;           // sum over low-rank blocks of (m + k)
};

void build_cluster_tree(const double* pts, int32_t n, int32_t dim, int32_t leaf_size, ClusterTree& tr);
void build_block_tree(const ClusterTree& tr, double eta, BlockTree& bt);
bool admissible(const ClusterTree& tr, int32_t t, int32_t s, double eta);
// Trees of a batch: each problem's cluster tree (over its own points, offsets
// offs[p] .. offs[p+1] of the caller's concatenated array) and block tree,
// merged with node and point offsets; the trees of different problems share
// no blocks.
void build_forest(const double* pts, const std::vector<int64_t>& offs, int32_t dim, int32_t leaf_size, double eta,
                  ClusterTree& tr, BlockTree& bt);
// A device allocation of the GPU construction failed.
struct DeviceAllocFailure : std::runtime_error {
  using std::runtime_error::runtime_error;
};
// Temporary device memory for the GPU construction: alloc(bytes, ctx) returns
// a device pointer or NULL; free(ptr, ctx) releases it.
struct TreeAlloc {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
};
// The same two trees of one problem built on the GPU (tree_gpu.hip), from
// device points (n x dim, row-major), with results identical to
// build_cluster_tree + build_block_tree. Throws std::runtime_error on a HIP
// error and DeviceAllocFailure when alloc fails.
void build_trees_gpu(const double* d_pts, int32_t n, int32_t dim, int32_t leaf_size, double eta, hipStream_t st,
                     const TreeAlloc& alloc, ClusterTree& tr, BlockTree& bt);
void build_plan(const ClusterTree& tr, const BlockTree& bt, const std::vector<int64_t>& prob_off, int32_t rank_width,
                int32_t aca_width, int32_t pair_chunk, int32_t sketch_group, Plan& pl, int32_t seg_entries = 8,
                int32_t gseg_rows = 512);

}  // namespace hmle
