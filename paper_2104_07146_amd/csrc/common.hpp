// Shared definitions of the HIP H-MLE library (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "../../include/hmle.h"

namespace hmle {

// Kernel launches. Every launch skips an empty grid (a grid dimension of 0 is
// not a valid launch), and the first launch error of the calling thread is
// kept with the kernel's name until take_launch_error() collects it, so a
// failing launch is named even when errors are only checked after a whole
// sweep (including launches recorded into a graph capture).
inline thread_local hipError_t t_launch_err = hipSuccess;
inline thread_local const char* t_launch_what = nullptr;
inline void after_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess && t_launch_err == hipSuccess) {
    t_launch_err = e;
    t_launch_what = what;
  }
}
inline hipError_t take_launch_error(const char** what) {
  const hipError_t e = t_launch_err;
  if (what) *what = t_launch_what;
  t_launch_err = hipSuccess;
  t_launch_what = nullptr;
  return e;
}
// The first launch error kept since the last collection, else the runtime's
// last error.
inline hipError_t launch_status(const char** what = nullptr) {
  hipError_t e = take_launch_error(what);
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}
#define HMLE_LAUNCH(kernel, grid, block, shmem, stream, ...)                                       \
  do {                                                                                            \
    const dim3 g_ = (grid);                                                                       \
    if (g_.x > 0 && g_.y > 0 && g_.z > 0) {                                                       \
      hipLaunchKernelGGL(kernel, g_, block, shmem, stream, __VA_ARGS__);                          \
      ::hmle::after_launch(#kernel);                                                              \
    }                                                                                             \
  } while (0)

// Block kinds of the H-matrix partition (Section 2: dense and low-rank sub-blocks).
enum BlockKind : int32_t { BK_DIAG = 0, BK_DENSE = 1, BK_LOWRANK = 2 };

// One block of the lower triangle, rows [r0,r1) x columns [c0,c1) of the
// internal (cluster-tree) order.
//
// Storage of the factor L (and of the assembled matrix before factorisation):
//   BK_DIAG    m x m column-major at loff of the float64 diagonal pool (full
//              square; the factor keeps the lower triangle, upper part zeroed).
//   BK_DENSE   the transpose: W = L_b^T, k x m column-major at loff
//              (entry (i, j) of the block at loff + j + i*k).
//   BK_LOWRANK U (m x R) at loff, W (k x R) at loff + m*R, block = U W^T with
//              the current rank in rank[b] (R = sketch width).
// So every off-diagonal block is L_b = U_b W_b^T with U = identity for dense
// blocks; the column solves of the factorisation act on W only.
struct BlockDesc {
  int32_t r0, r1, c0, c1;
  int32_t kind;
  int32_t t, s;          // row / column cluster node
  int32_t leaf;          // diag: leaf index; else -1
  int32_t prob;          // problem of a batch (0 for a single problem)
  int32_t sid;           // index of the block in its own problem's block list (seeds its test matrix)
  int64_t loff;          // factor storage (doubles or floats, see precision)
  int64_t aoff;          // low-rank: cross-approximation factors U0 (m x Ra), W0 (k x Ra)
  int64_t soff;          // low-rank: sketch scratch Y (m x R), B^T (k x R), Omega (k x R)
};

// One term of the external update of a target block b:
//   S_b[rx, ry] -= L_x[rx, w] L_y[ry, w]^T, rows rx = [rx0,rx1), ry = [ry0,ry1),
//   shared column range w = [w0,w1) (global indices).
struct PairDesc {
  int32_t x, y, rx0, rx1, ry0, ry1, w0, w1;
  int32_t gram;    // slot of the cached W_x[w]^T W_y[w] when both blocks are low-rank, else -1
  int32_t pad;
};

// A chunk of consecutive pairs of one target, reduced into its own partial
// buffer at poff (elements) so that several workgroups share a target's
// update; the partial buffers of a target are summed in chunk order.
struct ChunkDesc {
  int32_t b;          // target block
  int32_t pair_lo;    // first pair (index into the pair array)
  int32_t pair_hi;    // one past the last pair
  int32_t slot;       // chunk index within the target (0-based)
  int64_t poff;       // partial buffer offset
};

// A pair of a low-rank target's update in one of the two sketch passes; the
// pairs of a chunk share their output block. gslot: slot of the precomputed
// product U_p^T X of the input-side block p (-1 when p is dense).
struct RPairDesc {
  int32_t x, y, rx0, rx1, ry0, ry1, w0, w1;
  int32_t gslot, gram;
};

// Precomputed input-side product of a sketch pass: G = U_blk[r0:r1]^T X
// (X = the target's test matrix in pass 1, its range basis in pass 2); blk = -1
// is the base term: W0^T Omega (pass 1) or U0^T Q (pass 2) of the target's
// cross approximation, over its rows [r0, r1) relative to the block. Long row
// ranges are cut into segments: part >= 0 writes segment partial `part`
// instead of the slot, and a GFin sums the partials into the slot.
struct GItem {
  int32_t b, blk, r0, r1;
  int32_t slot, part;
};

// Sum of the segment partials [lo, hi) of one input-side product into its
// slot, in segment order; b, blk as in its GItem (they fix the valid extent).
struct GFin {
  int32_t b, blk, slot, lo, hi, pad;
};

// Low-rank target of a step: pass-1 and pass-2 chunk ranges.
struct RTargetDesc {
  int32_t b;
  int32_t c1lo, c1hi, c2lo, c2hi;
  int32_t gb1, gb2;     // slots of the base products W0^T Omega (pass 1) and U0^T Q (pass 2)
  int32_t t1lo, t1hi;   // its row tiles in the step's pass-1 tile list (m rows)
  int32_t t2lo, t2hi;   // and in the pass-2 list (k rows)
  int32_t pad;
};

// A 128-row tile of a low-rank target's sketch (index t into the step's
// target list), summed from the chunk partials by its own workgroup; the
// chunks whose output rows meet the tile are entries [cb, ce) of the step's
// tile-chunk list.
struct RowTile {
  int32_t t, r0;
  int32_t cb, ce;
  int32_t sb, se;     // its segments [sb, se) in the step's segment list
};

// A segment of a tile's chunk entries [eb, ee) (with the base term when
// first): one workgroup forms the partial tile of these terms.
struct TileSeg {
  int32_t tile;       // index in the step's tile list
  int32_t eb, ee;
  int32_t first;
};

// One entry of a tile's chunk list: the chunk's output block, its rows
// (global) and the offset of its compact output in the step's partial buffer.
struct TileChunk {
  int32_t qb;
  int32_t rq0, rq1;
  int32_t lr;         // 1: low-rank output block (compact -H), 0: dense (touched rows)
  int64_t poff;
};

// Per target of a step: its chunks [chunk_lo, chunk_hi) of the step's chunk list.
struct TargetDesc {
  int32_t b;
  int32_t chunk_lo, chunk_hi;
  int32_t pad;
};

// Internal column update at one leaf step, rows [r0, r0 + 128) of x and the
// 32 columns of W_b from c0: W_b[rows of x] -= L_x[:, leaf] W_b[leaf rows]
// (x = -1: the column solve of those columns of b).
struct InnerDesc {
  int32_t b, x, r0, c0;
};

struct MaternParams {
  double sigma2;
  double inv_ell;
  double nu;
  double pref;     // sigma2 * 2^(1-nu) / Gamma(nu)
  double mu;       // nu - m, |mu| <= 1/2
  double tau2;
  double abs_tol;  // absolute floor of the per-block truncation accuracy (0: relative accuracy only)
  int32_t m;       // number of upward recurrence steps
  int32_t kind;    // 0: nu = 1/2, 1: nu = 3/2, 2: nu = 5/2, 3: general
};

// The constants above for one theta (host).
inline MaternParams matern_params(const hmle_theta& t) {
  MaternParams mp{};
  mp.sigma2 = t.sigma2;
  mp.inv_ell = 1.0 / t.range;
  mp.nu = t.nu;
  mp.tau2 = t.tau2;
  mp.pref = t.sigma2 * std::exp((1.0 - t.nu) * std::log(2.0) - std::lgamma(t.nu));
  mp.m = (int32_t)std::floor(t.nu + 0.5);
  mp.mu = t.nu - mp.m;
  mp.kind = (t.nu == 0.5) ? 0 : (t.nu == 1.5) ? 1 : (t.nu == 2.5) ? 2 : 3;
  return mp;
}

}  // namespace hmle
