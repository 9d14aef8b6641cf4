// Cluster tree, block tree and factorisation schedule (host, built once per
// point set; nothing here depends on theta).
//
// Section 2 describes the H-matrix as a recursive partition of the matrix
// into sub-blocks and leaves the partitioning rules to the literature. The
// rules used:
//   Cluster tree: a cluster with more than leaf_size points is split along
//   the longest side of its bounding box (lowest axis on ties); its points are
//   ordered by (coordinate, caller index) and the first half (rounded down)
//   forms the first child. Nodes are numbered level by level.
//   Admissibility: min(diam t, diam s) <= eta * dist(t, s) on bounding boxes,
//   compared squared; a diagonal pair is never admissible.
//   Block tree (lower triangle): (t,t) -> dense if t is a leaf, else
//   (t1,t1), (t2,t1), (t2,t2); (t,s) -> low-rank if admissible, dense if t or
//   s is a leaf, else the four child pairs.
// This file is compiled without floating-point contraction so that every
// bounding-box sum is the plain sequence of products and additions.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <unordered_map>

#include "plan.hpp"

namespace hmle {

void build_cluster_tree(const double* pts, int32_t n, int32_t dim, int32_t leaf_size, ClusterTree& tr) {
  tr = ClusterTree();
  tr.n = n;
  tr.dim = dim;
  tr.perm.resize(n);
  std::iota(tr.perm.begin(), tr.perm.end(), 0);
  std::vector<std::pair<int32_t, int32_t>> frontier{{0, n}}, next;
  std::vector<int32_t> parents{-1}, next_par;
  int32_t lev = 0;
  while (!frontier.empty()) {
    next.clear();
    next_par.clear();
    const int32_t base = tr.n_nodes() + (int32_t)frontier.size();
    for (size_t f = 0; f < frontier.size(); ++f) {
      const int32_t a = frontier[f].first, b = frontier[f].second;
      const int32_t id = tr.n_nodes();
      tr.lo.push_back(a);
      tr.hi.push_back(b);
      tr.level.push_back(lev);
      tr.parent.push_back(parents[f]);
      double mn[3], mx[3];
      for (int k = 0; k < dim; ++k) { mn[k] = INFINITY; mx[k] = -INFINITY; }
      for (int32_t i = a; i < b; ++i) {
        const double* p = pts + (int64_t)tr.perm[i] * dim;
        for (int k = 0; k < dim; ++k) { mn[k] = std::min(mn[k], p[k]); mx[k] = std::max(mx[k], p[k]); }
      }
      for (int k = 0; k < dim; ++k) { tr.bmin.push_back(mn[k]); tr.bmax.push_back(mx[k]); }
      const int32_t m = b - a;
      if (m > leaf_size) {
        int axis = 0;
        double best = mx[0] - mn[0];
        for (int k = 1; k < dim; ++k) {
          const double e = mx[k] - mn[k];
          if (e > best) { best = e; axis = k; }
        }
        std::sort(tr.perm.begin() + a, tr.perm.begin() + b, [&](int32_t u, int32_t v) {
          const double cu = pts[(int64_t)u * dim + axis], cv = pts[(int64_t)v * dim + axis];
          return cu < cv || (cu == cv && u < v);
        });
        const int32_t half = m / 2;
        const int32_t c = base + (int32_t)next.size();
        tr.child0.push_back(c);
        tr.child1.push_back(c + 1);
        next.push_back({a, a + half});
        next.push_back({a + half, b});
        next_par.push_back(id);
        next_par.push_back(id);
      } else {
        tr.child0.push_back(-1);
        tr.child1.push_back(-1);
      }
    }
    frontier.swap(next);
    parents.swap(next_par);
    ++lev;
  }
}

static double diam2(const ClusterTree& tr, int32_t t) {
  double acc = 0.0;
  for (int k = 0; k < tr.dim; ++k) {
    const double e = tr.bmax[(int64_t)t * tr.dim + k] - tr.bmin[(int64_t)t * tr.dim + k];
    acc = acc + e * e;
  }
  return acc;
}

static double dist2(const ClusterTree& tr, int32_t t, int32_t s) {
  double acc = 0.0;
  for (int k = 0; k < tr.dim; ++k) {
    const double g = std::max(std::max(0.0, tr.bmin[(int64_t)s * tr.dim + k] - tr.bmax[(int64_t)t * tr.dim + k]),
                              tr.bmin[(int64_t)t * tr.dim + k] - tr.bmax[(int64_t)s * tr.dim + k]);
    acc = acc + g * g;
  }
  return acc;
}

bool admissible(const ClusterTree& tr, int32_t t, int32_t s, double eta) {
  if (t == s) return false;
  return std::min(diam2(tr, t), diam2(tr, s)) <= (eta * eta) * dist2(tr, t, s);
}

void build_block_tree(const ClusterTree& tr, double eta, BlockTree& bt) {
  bt = BlockTree();
  std::vector<std::pair<int32_t, int32_t>> stack{{0, 0}}, dense, lr;
  while (!stack.empty()) {
    auto [t, s] = stack.back();
    stack.pop_back();
    if (t == s) {
      if (tr.is_leaf(t)) {
        dense.push_back({t, t});
      } else {
        const int32_t c1 = tr.child0[t], c2 = tr.child1[t];
        stack.push_back({c1, c1});
        stack.push_back({c2, c1});
        stack.push_back({c2, c2});
      }
    } else if (admissible(tr, t, s, eta)) {
      lr.push_back({t, s});
    } else if (tr.is_leaf(t) || tr.is_leaf(s)) {
      dense.push_back({t, s});
    } else {
      for (int32_t a : {tr.child0[t], tr.child1[t]})
        for (int32_t b : {tr.child0[s], tr.child1[s]}) stack.push_back({a, b});
    }
  }
  auto canon = [&](std::vector<std::pair<int32_t, int32_t>>& v, std::vector<int32_t>& ot, std::vector<int32_t>& os) {
    std::sort(v.begin(), v.end(), [&](const auto& p, const auto& q) {
      if (tr.lo[p.second] != tr.lo[q.second]) return tr.lo[p.second] < tr.lo[q.second];
      return tr.lo[p.first] < tr.lo[q.first];
    });
    for (auto& p : v) { ot.push_back(p.first); os.push_back(p.second); }
  };
  canon(dense, bt.dense_t, bt.dense_s);
  canon(lr, bt.lr_t, bt.lr_s);
}

void build_forest(const double* pts, const std::vector<int64_t>& offs, int32_t dim, int32_t leaf_size, double eta,
                  ClusterTree& tr, BlockTree& bt) {
  tr = ClusterTree();
  bt = BlockTree();
  const int32_t P = (int32_t)offs.size() - 1;
  tr.n = (int32_t)offs[P];
  tr.dim = dim;
  ClusterTree t1;
  BlockTree b1;
  for (int32_t p = 0; p < P; ++p) {
    const int32_t po = (int32_t)offs[p], np = (int32_t)(offs[p + 1] - offs[p]);
    build_cluster_tree(pts + (int64_t)po * dim, np, dim, leaf_size, t1);
    build_block_tree(t1, eta, b1);
    const int32_t no = tr.n_nodes();
    for (int32_t v : t1.perm) tr.perm.push_back(v + po);
    for (int32_t u = 0; u < t1.n_nodes(); ++u) {
      tr.lo.push_back(t1.lo[u] + po);
      tr.hi.push_back(t1.hi[u] + po);
      tr.child0.push_back(t1.child0[u] < 0 ? -1 : t1.child0[u] + no);
      tr.child1.push_back(t1.child1[u] < 0 ? -1 : t1.child1[u] + no);
      tr.parent.push_back(t1.parent[u] < 0 ? -1 : t1.parent[u] + no);
      tr.level.push_back(t1.level[u]);
    }
    tr.bmin.insert(tr.bmin.end(), t1.bmin.begin(), t1.bmin.end());
    tr.bmax.insert(tr.bmax.end(), t1.bmax.begin(), t1.bmax.end());
    // block lists stay sorted by (col lo, row lo): problem p's ranges follow p-1's
    for (int32_t v : b1.dense_t) bt.dense_t.push_back(v + no);
    for (int32_t v : b1.dense_s) bt.dense_s.push_back(v + no);
    for (int32_t v : b1.lr_t) bt.lr_t.push_back(v + no);
    for (int32_t v : b1.lr_s) bt.lr_s.push_back(v + no);
  }
}

// ---------------------------------------------------------------------------
// Schedule of the left-looking H-Cholesky.
//
// For a block b = (tau, sigma) of the factor, with P the columns left of sigma,
//   L_b = (C_b - L[tau, P] L[sigma, P]^T) L_{sigma sigma}^{-T}.
// The update L[tau,P] L[sigma,P]^T is the sum over pairs (x, y) of factor
// blocks left of sigma whose rows meet tau (x) and sigma (y) and whose column
// clusters meet; clusters are nested or disjoint, so the shared columns are the
// smaller of the two clusters. The solve with L_{sigma sigma} runs leaf by leaf
// across sigma as the sweep reaches each leaf column.
void build_plan(const ClusterTree& tr, const BlockTree& bt, const std::vector<int64_t>& prob_off, int32_t R,
                int32_t Ra, int32_t pair_chunk, int32_t sketch_group, Plan& pl, int32_t seg_entries,
                int32_t gseg_rows) {
  pl = Plan();
  pl.pair_chunk = pair_chunk;
  pl.rank_width = R;
  pl.aca_width = Ra;
  pl.n_probs = (int32_t)prob_off.size() - 1;
  pl.prob_off = prob_off;
  auto prob_of_row = [&](int32_t r) {
    return (int32_t)(std::upper_bound(prob_off.begin(), prob_off.end(), (int64_t)r) - prob_off.begin()) - 1;
  };
  const int32_t nn = tr.n_nodes();
  // leaves in order
  std::vector<int32_t> leaves;
  for (int32_t t = 0; t < nn; ++t)
    if (tr.is_leaf(t)) leaves.push_back(t);
  std::sort(leaves.begin(), leaves.end(), [&](int32_t a, int32_t b) { return tr.lo[a] < tr.lo[b]; });
  const int32_t B = (int32_t)leaves.size();
  pl.n_leaves = B;
  std::vector<int32_t> leaf_index(nn, -1);
  for (int32_t j = 0; j < B; ++j) {
    leaf_index[leaves[j]] = j;
    pl.leaf_lo.push_back(tr.lo[leaves[j]]);
    pl.leaf_hi.push_back(tr.hi[leaves[j]]);
    pl.max_leaf = std::max(pl.max_leaf, tr.hi[leaves[j]] - tr.lo[leaves[j]]);
  }
  // first leaf index covering a global row -> map lo position to leaf index
  std::vector<int32_t> leaf_of_row(tr.n);
  for (int32_t j = 0; j < B; ++j)
    for (int32_t i = pl.leaf_lo[j]; i < pl.leaf_hi[j]; ++i) leaf_of_row[i] = j;
  // leaves of each problem, and the step of each leaf (its index within its problem)
  pl.prob_leaf0.assign(pl.n_probs + 1, 0);
  for (int32_t j = 0; j < B; ++j) pl.prob_leaf0[prob_of_row(pl.leaf_lo[j]) + 1]++;
  for (int32_t p = 0; p < pl.n_probs; ++p) pl.prob_leaf0[p + 1] += pl.prob_leaf0[p];
  std::vector<int32_t> step_of(B);
  for (int32_t j = 0; j < B; ++j) {
    step_of[j] = j - pl.prob_leaf0[prob_of_row(pl.leaf_lo[j])];
    pl.n_steps = std::max(pl.n_steps, step_of[j] + 1);
  }
  {
    std::vector<std::vector<int32_t>> at(pl.n_steps);
    for (int32_t j = 0; j < B; ++j) at[step_of[j]].push_back(j);
    pl.step_leaf_beg.push_back(0);
    for (auto& v : at) {
      pl.step_leaf.insert(pl.step_leaf.end(), v.begin(), v.end());
      pl.step_leaf_beg.push_back((int32_t)pl.step_leaf.size());
    }
  }
  const int32_t S = pl.n_steps;
  auto step_of_row = [&](int32_t r) { return step_of[leaf_of_row[r]]; };

  // blocks: dense (diag + off-diag) in block-tree order, then low-rank
  // sid: the index the block has in its own problem's list (dense, then low-rank)
  std::vector<int32_t> n_dense_of(pl.n_probs, 0), seen_d(pl.n_probs, 0), seen_l(pl.n_probs, 0);
  for (int32_t t : bt.dense_t) n_dense_of[prob_of_row(tr.lo[t])]++;
  auto add_block = [&](int32_t t, int32_t s, int32_t kind) {
    BlockDesc b{};
    b.t = t; b.s = s;
    b.r0 = tr.lo[t]; b.r1 = tr.hi[t]; b.c0 = tr.lo[s]; b.c1 = tr.hi[s];
    b.kind = kind;
    b.leaf = (kind == BK_DIAG) ? leaf_index[t] : -1;
    b.prob = prob_of_row(b.r0);
    b.sid = kind == BK_LOWRANK ? n_dense_of[b.prob] + seen_l[b.prob]++ : seen_d[b.prob]++;
    pl.blocks.push_back(b);
  };
  for (size_t i = 0; i < bt.dense_t.size(); ++i)
    add_block(bt.dense_t[i], bt.dense_s[i], bt.dense_t[i] == bt.dense_s[i] ? BK_DIAG : BK_DENSE);
  pl.n_dense = (int32_t)bt.dense_t.size();
  for (size_t i = 0; i < bt.lr_t.size(); ++i) add_block(bt.lr_t[i], bt.lr_s[i], BK_LOWRANK);
  pl.n_lowrank = (int32_t)bt.lr_t.size();
  const int32_t nb = (int32_t)pl.blocks.size();

  // storage offsets
  pl.leaf_diag.assign(B, -1);
  pl.leaf_inv_off.assign(B, 0);
  for (int32_t bi = 0; bi < nb; ++bi) {
    BlockDesc& b = pl.blocks[bi];
    const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
    if (b.kind == BK_DIAG) {
      b.loff = pl.d_size;
      pl.d_size += m * k;
      pl.dense_entries += m * k;
    } else if (b.kind == BK_LOWRANK) {
      b.loff = pl.l_size;
      pl.l_size += (m + k) * R;
      b.aoff = pl.a_size;
      pl.a_size += (m + k) * Ra;
      b.soff = pl.s_size;
      pl.s_size += (m + 2 * k) * R;
      pl.lr_dims += m + k;
    } else {
      b.loff = pl.l_size;
      pl.l_size += m * k;
      pl.dense_entries += m * k;
      pl.max_dense_dim = std::max<int64_t>(pl.max_dense_dim, std::max(m, k));
    }
    if (b.kind == BK_DIAG) {
      pl.leaf_diag[b.leaf] = bi;
      pl.leaf_inv_off[b.leaf] = pl.inv_size;
      pl.inv_size += m * m;
    }
  }
  // round pools up so that every view may be read as float2/double2 safely
  pl.l_size += 64; pl.d_size += 64; pl.a_size += 64; pl.s_size += 64; pl.inv_size += 64;

  // rows index: blocks grouped by row node
  std::vector<std::vector<int32_t>> rowlist(nn);
  for (int32_t bi = 0; bi < nb; ++bi) rowlist[pl.blocks[bi].t].push_back(bi);

  // candidates: blocks whose rows meet cluster c and whose columns end at or before cend
  auto candidates = [&](int32_t c, int32_t cend, std::vector<int32_t>& out) {
    out.clear();
    for (int32_t a = c; a >= 0; a = tr.parent[a])
      for (int32_t bi : rowlist[a])
        if (pl.blocks[bi].c1 <= cend) out.push_back(bi);
    // descendants of c
    std::vector<int32_t> st;
    if (!tr.is_leaf(c)) { st.push_back(tr.child0[c]); st.push_back(tr.child1[c]); }
    while (!st.empty()) {
      const int32_t u = st.back();
      st.pop_back();
      for (int32_t bi : rowlist[u])
        if (pl.blocks[bi].c1 <= cend) out.push_back(bi);
      if (!tr.is_leaf(u)) { st.push_back(tr.child0[u]); st.push_back(tr.child1[u]); }
    }
  };

  pl.pair_beg.assign(nb + 1, 0);
  std::vector<int32_t> A, Bc;
  std::vector<int32_t> stamp(nn, -1);
  std::vector<std::vector<int32_t>> groups(nn);
  std::vector<int32_t> touched;
  std::vector<std::pair<int32_t, int32_t>> glist;   // (col lo, node) of groups present
  for (int32_t bi = 0; bi < nb; ++bi) {
    const BlockDesc& b = pl.blocks[bi];
    pl.pair_beg[bi] = (int64_t)pl.pairs.size();
    if (b.c0 == pl.prob_off[b.prob]) continue;   // first column of its problem: nothing to the left
    candidates(b.t, b.c0, A);
    candidates(b.s, b.c0, Bc);
    // group y candidates by column node
    touched.clear();
    glist.clear();
    for (int32_t yi : Bc) {
      const int32_t g = pl.blocks[yi].s;
      if (stamp[g] != bi) { stamp[g] = bi; groups[g].clear(); touched.push_back(g); glist.push_back({tr.lo[g], g}); }
      groups[g].push_back(yi);
    }
    std::sort(glist.begin(), glist.end());
    for (int32_t xi : A) {
      const BlockDesc& x = pl.blocks[xi];
      const int32_t sx = x.s;
      auto emit = [&](int32_t g) {
        for (int32_t yi : groups[g]) {
          const BlockDesc& y = pl.blocks[yi];
          PairDesc p;
          p.x = xi; p.y = yi;
          p.gram = -1; p.pad = 0;
          p.rx0 = std::max(x.r0, b.r0); p.rx1 = std::min(x.r1, b.r1);
          p.ry0 = std::max(y.r0, b.c0); p.ry1 = std::min(y.r1, b.c1);
          p.w0 = std::max(x.c0, y.c0); p.w1 = std::min(x.c1, y.c1);
          pl.pairs.push_back(p);
        }
      };
      // strict ancestors of sx
      for (int32_t a = tr.parent[sx]; a >= 0; a = tr.parent[a])
        if (stamp[a] == bi) emit(a);
      // sx itself and its descendants: group nodes with lo in [lo(sx), hi(sx)) nested in sx
      auto it = std::lower_bound(glist.begin(), glist.end(), std::make_pair(tr.lo[sx], -1));
      for (; it != glist.end() && it->first < tr.hi[sx]; ++it) {
        const int32_t g = it->second;
        if (tr.hi[g] <= tr.hi[sx] && (g == sx || tr.level[g] > tr.level[sx])) emit(g);
      }
    }
  }
  pl.pair_beg[nb] = (int64_t)pl.pairs.size();

  // distinct low-rank x low-rank pairs: one cached Gram matrix each, computed at
  // the step after which both blocks are final (their last leaf column)
  {
    std::vector<int32_t> fin(nb);
    for (int32_t bi = 0; bi < nb; ++bi) fin[bi] = step_of_row(pl.blocks[bi].c1 - 1);
    std::unordered_map<int64_t, int32_t> slot_of;
    std::vector<std::vector<PairDesc>> at(S);
    for (PairDesc& pr : pl.pairs) {
      if (pl.blocks[pr.x].kind != BK_LOWRANK || pl.blocks[pr.y].kind != BK_LOWRANK) continue;
      const int64_t key = (int64_t)pr.x * nb + pr.y;
      auto it = slot_of.find(key);
      if (it == slot_of.end()) {
        const int32_t slot = (int32_t)slot_of.size();
        it = slot_of.emplace(key, slot).first;
        PairDesc g = pr;
        g.rx0 = slot;
        at[std::max(fin[pr.x], fin[pr.y])].push_back(g);
      }
      pr.gram = it->second;
    }
    pl.n_grams = (int64_t)slot_of.size();
    pl.gram_beg.push_back(0);
    for (int32_t j = 0; j < S; ++j) {
      for (const PairDesc& g : at[j]) pl.grams.push_back(g);
      pl.gram_beg.push_back((int32_t)pl.grams.size());
    }
  }

  // per-step lists
  std::vector<std::vector<int32_t>> start_at(S);
  for (int32_t bi = 0; bi < nb; ++bi) start_at[step_of_row(pl.blocks[bi].c0)].push_back(bi);
  std::vector<std::vector<int32_t>> active_at(S);
  for (int32_t bi = 0; bi < nb; ++bi) {
    const BlockDesc& b = pl.blocks[bi];
    if (b.kind == BK_DIAG) continue;
    for (int32_t j = step_of_row(b.c0); j <= step_of_row(b.c1 - 1); ++j) active_at[j].push_back(bi);
  }
  pl.dchunk_beg.push_back(0);
  pl.dtarget_beg.push_back(0);
  pl.r1chunk_beg.push_back(0);
  pl.r2chunk_beg.push_back(0);
  pl.rtarget_beg.push_back(0);
  pl.g1_beg.push_back(0);
  pl.g2_beg.push_back(0);
  pl.gf1_beg.push_back(0);
  pl.gf2_beg.push_back(0);
  pl.t1_beg.push_back(0);
  pl.t2_beg.push_back(0);
  pl.tc1_beg.push_back(0);
  pl.tc2_beg.push_back(0);
  pl.sg1_beg.push_back(0);
  pl.sg2_beg.push_back(0);
  pl.seg_entries = seg_entries;
  pl.gseg_rows = gseg_rows;
  const int32_t kSeg = seg_entries;   // chunk entries per segment of a sketch-sum tile
  const int32_t kGSeg = gseg_rows;    // rows per segment of an input-side product
  const int32_t max_group = sketch_group;    // work budget of a chunk of a low-rank target pass
  for (int32_t j = 0; j < S; ++j) {
    int64_t dpart = 0, rpart1 = 0, rpart2 = 0;
    int32_t gs1 = 0, gs2 = 0;
    for (int32_t bi : start_at[j]) {
      const BlockDesc& b = pl.blocks[bi];
      const int64_t p0 = pl.pair_beg[bi], p1 = pl.pair_beg[bi + 1];
      const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
      if (b.kind != BK_LOWRANK) {
        TargetDesc td{bi, (int32_t)(pl.dchunks.size() - pl.dchunk_beg.back()), 0, 0};
        int32_t slot = 0;
        for (int64_t q = p0; q < p1; q += pl.pair_chunk) {
          ChunkDesc cd;
          cd.b = bi;
          cd.pair_lo = (int32_t)q;
          cd.pair_hi = (int32_t)std::min<int64_t>(p1, q + pl.pair_chunk);
          cd.slot = slot++;
          cd.poff = dpart;
          dpart += m * k;
          pl.dchunks.push_back(cd);
        }
        td.chunk_hi = (int32_t)(pl.dchunks.size() - pl.dchunk_beg.back());
        pl.dtargets.push_back(td);
        continue;
      }
      RTargetDesc rt{};
      rt.b = bi;
      const int32_t tix = (int32_t)(pl.rtargets.size() - pl.rtarget_beg.back());
      rt.t1lo = (int32_t)(pl.tiles1.size() - pl.t1_beg.back());
      for (int64_t r0 = 0; r0 < m; r0 += 128) pl.tiles1.push_back({tix, (int32_t)r0, 0, 0, 0, 0});
      rt.t1hi = (int32_t)(pl.tiles1.size() - pl.t1_beg.back());
      rt.t2lo = (int32_t)(pl.tiles2.size() - pl.t2_beg.back());
      for (int64_t r0 = 0; r0 < k; r0 += 128) pl.tiles2.push_back({tix, (int32_t)r0, 0, 0, 0, 0});
      rt.t2hi = (int32_t)(pl.tiles2.size() - pl.t2_beg.back());
      rt.gb1 = gs1++;
      pl.g1items.push_back({bi, -1, 0, (int32_t)k, rt.gb1, -1});
      rt.gb2 = gs2++;
      pl.g2items.push_back({bi, -1, 0, (int32_t)m, rt.gb2, -1});
      // pass 1: output side x, input side y; pass 2: output y, input x
      for (int pass = 1; pass <= 2; ++pass) {
        std::vector<RPairDesc> v;
        for (int64_t q = p0; q < p1; ++q) {
          const PairDesc& pr = pl.pairs[q];
          RPairDesc r{pr.x, pr.y, pr.rx0, pr.rx1, pr.ry0, pr.ry1, pr.w0, pr.w1, -1, pr.gram};
          v.push_back(r);
        }
        auto outb = [&](const RPairDesc& r) { return pass == 1 ? r.x : r.y; };
        auto inb = [&](const RPairDesc& r) { return pass == 1 ? r.y : r.x; };
        // cost of a pair in a chunk: 1 for low-rank x low-rank (a small product of cached
        // factors), max_group for a pair with a dense block (it gets a workgroup of its own)
        auto cost = [&](const RPairDesc& r) {
          return (pl.blocks[r.x].kind == BK_LOWRANK && pl.blocks[r.y].kind == BK_LOWRANK) ? 1 : max_group;
        };
        std::stable_sort(v.begin(), v.end(), [&](const RPairDesc& a, const RPairDesc& c) {
          return outb(a) < outb(c) || (outb(a) == outb(c) && cost(a) < cost(c));
        });
        // a pair with a dense block is cut into pieces of at most 64 shared
        // columns and (dense output block) 128 output rows: the terms are sums
        // over the shared columns, and output rows are independent
        {
          std::vector<RPairDesc> cut;
          for (const RPairDesc& r : v) {
            if (cost(r) == 1) { cut.push_back(r); continue; }
            const bool qlr = pl.blocks[outb(r)].kind == BK_LOWRANK;
            const int32_t o0 = pass == 1 ? r.rx0 : r.ry0, o1 = pass == 1 ? r.rx1 : r.ry1;
            for (int32_t a = o0; a < o1; a += qlr ? (o1 - o0) : 128)
              for (int32_t w = r.w0; w < r.w1; w += 64) {
                RPairDesc q = r;
                q.w0 = w;
                q.w1 = std::min(r.w1, w + 64);
                if (!qlr) {
                  (pass == 1 ? q.rx0 : q.ry0) = a;
                  (pass == 1 ? q.rx1 : q.ry1) = std::min(o1, a + 128);
                }
                cut.push_back(q);
              }
          }
          v.swap(cut);
        }
        // input-side products: one slot per distinct low-rank input block
        std::vector<std::pair<int32_t, int32_t>> seen;   // (block, slot)
        for (RPairDesc& r : v) {
          const int32_t ib = inb(r);
          if (pl.blocks[ib].kind != BK_LOWRANK) continue;
          int32_t slot = -1;
          for (auto& s : seen)
            if (s.first == ib) { slot = s.second; break; }
          if (slot < 0) {
            slot = pass == 1 ? gs1++ : gs2++;
            seen.push_back({ib, slot});
            GItem g{bi, ib, pass == 1 ? r.ry0 : r.rx0, pass == 1 ? r.ry1 : r.rx1, slot, -1};
            (pass == 1 ? pl.g1items : pl.g2items).push_back(g);
          }
          r.gslot = slot;
        }
        std::vector<RPairDesc>& dst = pass == 1 ? pl.rpairs1 : pl.rpairs2;
        std::vector<ChunkDesc>& ch = pass == 1 ? pl.r1chunks : pl.r2chunks;
        const int32_t cbase = pass == 1 ? pl.r1chunk_beg.back() : pl.r2chunk_beg.back();
        const int32_t clo = (int32_t)ch.size() - cbase;
        int64_t& rp = pass == 1 ? rpart1 : rpart2;
        // chunks touching each 128-row tile of this pass, in chunk order
        const int32_t obase = pass == 1 ? b.r0 : b.c0;
        const int32_t ntile = (int32_t)(((pass == 1 ? m : k) + 127) / 128);
        std::vector<std::vector<TileChunk>> per_tile(ntile);
        size_t i = 0;
        int32_t slot = 0;
        while (i < v.size()) {
          size_t e = i + 1;
          int32_t load = cost(v[i]);
          while (e < v.size() && outb(v[e]) == outb(v[i]) && load + cost(v[e]) <= max_group) load += cost(v[e++]);
          ChunkDesc cd;
          cd.b = bi;
          cd.pair_lo = (int32_t)dst.size();
          for (size_t q = i; q < e; ++q) dst.push_back(v[q]);
          cd.pair_hi = (int32_t)dst.size();
          cd.slot = slot++;
          cd.poff = rp;
          // output of a chunk: -H (rank x ncol) for a low-rank output block, the
          // negated touched rows (|rows| x ncol) for a dense one
          const int32_t qb = outb(v[i]);
          const int64_t nq = pass == 1 ? v[i].rx1 - v[i].rx0 : v[i].ry1 - v[i].ry0;
          rp += (pl.blocks[qb].kind == BK_LOWRANK ? (int64_t)R : nq) * R;
          const int32_t q0 = (pass == 1 ? v[i].rx0 : v[i].ry0) - obase, q1 = (pass == 1 ? v[i].rx1 : v[i].ry1) - obase;
          const TileChunk tce{qb, q0 + obase, q1 + obase, pl.blocks[qb].kind == BK_LOWRANK ? 1 : 0, cd.poff};
          for (int32_t tt = q0 / 128; tt <= (q1 - 1) / 128; ++tt) per_tile[tt].push_back(tce);
          ch.push_back(cd);
          i = e;
        }
        {
          std::vector<RowTile>& tl = pass == 1 ? pl.tiles1 : pl.tiles2;
          std::vector<TileChunk>& tc = pass == 1 ? pl.tc1 : pl.tc2;
          const int32_t tbase = (pass == 1 ? pl.t1_beg.back() : pl.t2_beg.back()) + (pass == 1 ? rt.t1lo : rt.t2lo);
          const int32_t tcbase = pass == 1 ? pl.tc1_beg.back() : pl.tc2_beg.back();
          std::vector<TileSeg>& sg = pass == 1 ? pl.sg1 : pl.sg2;
          const int32_t sgbase = pass == 1 ? pl.sg1_beg.back() : pl.sg2_beg.back();
          const int32_t tlbase = pass == 1 ? pl.t1_beg.back() : pl.t2_beg.back();
          for (int32_t tt = 0; tt < ntile; ++tt) {
            RowTile& T = tl[tbase + tt];
            T.cb = (int32_t)tc.size() - tcbase;
            tc.insert(tc.end(), per_tile[tt].begin(), per_tile[tt].end());
            T.ce = (int32_t)tc.size() - tcbase;
            // segments of at most kSeg entries; the first also takes the base term
            T.sb = (int32_t)sg.size() - sgbase;
            int32_t e = T.cb;
            do {
              const int32_t ee = std::min(T.ce, e + kSeg);
              sg.push_back({tbase + tt - tlbase, e, ee, e == T.cb ? 1 : 0});
              e = ee;
            } while (e < T.ce);
            T.se = (int32_t)sg.size() - sgbase;
          }
        }
        if (pass == 1) { rt.c1lo = clo; rt.c1hi = (int32_t)ch.size() - cbase; }
        else { rt.c2lo = clo; rt.c2hi = (int32_t)ch.size() - cbase; }
      }
      pl.rtargets.push_back(rt);
    }
    pl.dchunk_beg.push_back((int32_t)pl.dchunks.size());
    pl.dtarget_beg.push_back((int32_t)pl.dtargets.size());
    pl.r1chunk_beg.push_back((int32_t)pl.r1chunks.size());
    pl.r2chunk_beg.push_back((int32_t)pl.r2chunks.size());
    pl.rtarget_beg.push_back((int32_t)pl.rtargets.size());
    // input-side products over more than kGSeg rows: one workgroup per segment
    // of kGSeg rows writes a partial, a GFin sums them in segment order
    for (int pass = 1; pass <= 2; ++pass) {
      std::vector<GItem>& items = pass == 1 ? pl.g1items : pl.g2items;
      std::vector<GFin>& fins = pass == 1 ? pl.gf1 : pl.gf2;
      const size_t beg = (size_t)(pass == 1 ? pl.g1_beg.back() : pl.g2_beg.back());
      std::vector<GItem> out;
      int32_t np = 0;
      for (size_t i = beg; i < items.size(); ++i) {
        const GItem g = items[i];
        if (g.r1 - g.r0 <= kGSeg) { out.push_back(g); continue; }
        GFin f{g.b, g.blk, g.slot, np, 0, 0};
        for (int32_t s = g.r0; s < g.r1; s += kGSeg) {
          GItem q = g;
          q.r0 = s;
          q.r1 = std::min(g.r1, s + kGSeg);
          q.part = np++;
          out.push_back(q);
        }
        f.hi = np;
        fins.push_back(f);
      }
      items.resize(beg);
      items.insert(items.end(), out.begin(), out.end());
      (pass == 1 ? pl.gf1_beg : pl.gf2_beg).push_back((int32_t)fins.size());
      pl.max_gparts = std::max(pl.max_gparts, np);
    }
    pl.g1_beg.push_back((int32_t)pl.g1items.size());
    pl.g2_beg.push_back((int32_t)pl.g2items.size());
    pl.t1_beg.push_back((int32_t)pl.tiles1.size());
    pl.t2_beg.push_back((int32_t)pl.tiles2.size());
    pl.tc1_beg.push_back((int32_t)pl.tc1.size());
    pl.tc2_beg.push_back((int32_t)pl.tc2.size());
    pl.sg1_beg.push_back((int32_t)pl.sg1.size());
    pl.sg2_beg.push_back((int32_t)pl.sg2.size());
    pl.max_segs = std::max(pl.max_segs, std::max(pl.sg1_beg.back() - pl.sg1_beg[pl.sg1_beg.size() - 2],
                                                 pl.sg2_beg.back() - pl.sg2_beg[pl.sg2_beg.size() - 2]));
    pl.max_tiles = std::max(pl.max_tiles, std::max(pl.t1_beg.back() - pl.t1_beg[pl.t1_beg.size() - 2],
                                                   pl.t2_beg.back() - pl.t2_beg[pl.t2_beg.size() - 2]));
    pl.max_rtargets = std::max(pl.max_rtargets, pl.rtarget_beg.back() - pl.rtarget_beg[pl.rtarget_beg.size() - 2]);
    pl.dpart_size = std::max(pl.dpart_size, dpart);
    pl.rpart_size = std::max(pl.rpart_size, std::max(rpart1, rpart2));
    pl.max_gslots = std::max(pl.max_gslots, std::max(gs1, gs2));
  }
  pl.ext_dense_beg.push_back(0);
  pl.ext_lr_beg.push_back(0);
  pl.active_beg.push_back(0);
  pl.inner_beg.push_back(0);
  pl.tsolve_beg.push_back(0);
  pl.fsolve_beg.push_back(0);
  // columns of W_b a step works on: all rows of a dense b, the storage width of a low-rank b
  auto wcols = [&](const BlockDesc& b) { return b.kind == BK_LOWRANK ? R : b.r1 - b.r0; };
  for (int32_t j = 0; j < S; ++j) {
    for (int32_t bi : start_at[j]) {
      if (pl.blocks[bi].kind == BK_LOWRANK) pl.ext_lr.push_back(bi);
      else pl.ext_dense.push_back(bi);
    }
    pl.ext_dense_beg.push_back((int32_t)pl.ext_dense.size());
    pl.ext_lr_beg.push_back((int32_t)pl.ext_lr.size());
    for (int32_t bi : active_at[j]) pl.active.push_back(bi);
    pl.active_beg.push_back((int32_t)pl.active.size());
    for (int32_t bi : active_at[j])
      for (int32_t c0 = 0; c0 < wcols(pl.blocks[bi]); c0 += 32) pl.tsolve.push_back({bi, -1, 0, c0});
    pl.tsolve_beg.push_back((int32_t)pl.tsolve.size());
    // forward solve: the rows of every block of the column in chunks of 2048
    for (int32_t bi : active_at[j]) {
      const int32_t mb = pl.blocks[bi].r1 - pl.blocks[bi].r0;
      for (int32_t r0 = 0; r0 < mb; r0 += 2048) pl.fsolve.push_back({bi, -1, r0, std::min(mb, r0 + 2048)});
    }
    pl.fsolve_beg.push_back((int32_t)pl.fsolve.size());
    for (int32_t bi : active_at[j]) {
      const BlockDesc& b = pl.blocks[bi];
      if (b.c1 <= pl.leaf_hi[pl.prob_leaf0[b.prob] + j]) continue;   // ends at this step's leaf
      for (int32_t xi : active_at[j]) {
        const BlockDesc& x = pl.blocks[xi];
        if (x.r0 >= b.c0 && x.r1 <= b.c1)
          for (int32_t r0 = 0; r0 < x.r1 - x.r0; r0 += 128)
            for (int32_t c0 = 0; c0 < wcols(b); c0 += 32) pl.inner.push_back({bi, xi, r0, c0});
      }
    }
    pl.inner_beg.push_back((int32_t)pl.inner.size());
  }
  std::vector<std::vector<int32_t>> rows_at(B);
  for (int32_t bi = 0; bi < nb; ++bi) {
    const BlockDesc& b = pl.blocks[bi];
    if (b.kind == BK_DIAG) continue;
    for (int32_t j = leaf_of_row[b.r0]; j <= leaf_of_row[b.r1 - 1]; ++j) rows_at[j].push_back(bi);
  }
  pl.rowp_beg.push_back(0);
  for (int32_t j = 0; j < B; ++j) {
    for (int32_t bi : rows_at[j]) pl.rowp.push_back(bi);
    pl.rowp_beg.push_back((int32_t)pl.rowp.size());
  }
  std::vector<std::vector<int32_t>> cols_at(B);
  for (int32_t bi = 0; bi < nb; ++bi) {
    const BlockDesc& b = pl.blocks[bi];
    if (b.kind == BK_DIAG) continue;
    for (int32_t j = leaf_of_row[b.c0]; j <= leaf_of_row[b.c1 - 1]; ++j) cols_at[j].push_back(bi);
  }
  pl.colp_beg.push_back(0);
  for (int32_t j = 0; j < B; ++j) {
    for (int32_t bi : cols_at[j]) pl.colp.push_back(bi);
    pl.colp_beg.push_back((int32_t)pl.colp.size());
  }
}

}  // namespace hmle
