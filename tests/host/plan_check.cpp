// Host-only check of the H-Cholesky schedule (cluster tree, block tree and
// plan of plan.hpp), built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_host_plan.py. Every invariant below follows from the
// left-looking block Cholesky of Section 2 on a partition of the lower
// triangle; none depends on the GPU kernels:
//   * the leaves split each problem's points in order, and each leaf is taken
//     at the step equal to its index within its problem;
//   * the blocks tile the lower triangle of each problem exactly once;
//   * for every entry (i, j) of a block whose columns start at c0, the external
//     update pairs covering (i, j) have disjoint column ranges that together
//     are [problem start, c0), and each pair reads only inside its two blocks;
//   * every block is listed once for its external update, at the step of its
//     first column; a cached Gram product is formed at a step before the one
//     that consumes it;
//   * dense targets' chunks split their pair lists in order into
//     non-overlapping partial buffers;
//   * at each step, the column solves cover every active block's stored
//     columns once, and the inner updates cover every row of an active block's
//     column range after the step's leaf once per 32-column slice.
//   * low-rank targets (the randomized sketch of their update, two passes):
//     each pass's pieces cover every entry's columns to the left exactly once,
//     a chunk's pieces share one output block and fit the work budget, chunk
//     outputs do not overlap, each cached input-side product (whole or as
//     segments summed in order) has one row range per input block, and every
//     128-row tile lists exactly the chunks that write its rows, in order, in
//     segments of at most 8.
// Then, for a few configurations, the schedule is executed in exact dense
// arithmetic (every block kept dense, every update applied in full, in the
// order of the plan's steps: external updates, the diagonal leaf's Cholesky,
// the column solves, the inner updates) on an exponential covariance matrix,
// and the result must equal a textbook Cholesky factor of the same matrix;
// the forward substitution by the plan's solve lists, and the backward
// substitution by the same lists in reverse, must equal textbook
// substitutions with that factor, and the sampler's product L w by row
// panels the plain product.
// Exit status 0 and a line per configuration on success; the first violated
// invariant is printed and the program exits with status 1.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "../../paper_2104_07146_amd/csrc/plan.hpp"

using namespace hmle;

#define REQUIRE(cond)                                                              \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      std::printf("FAILED %s at %s:%d (%s)\n", #cond, __FILE__, __LINE__, label); \
      std::exit(1);                                                                \
    }                                                                              \
  } while (0)

static bool contains(const BlockDesc& b, int64_t i, int64_t j) { return b.r0 <= i && i < b.r1 && b.c0 <= j && j < b.c1; }

static void check_lowrank(const char* label, const Plan& pl, const std::vector<int64_t>& offs, int R, int group,
                          std::mt19937_64& g) {
  const int32_t S = pl.n_steps;
  const auto& bl = pl.blocks;
  auto cost = [&](const RPairDesc& r) { return bl[r.x].kind == BK_LOWRANK && bl[r.y].kind == BK_LOWRANK ? 1 : group; };
  for (int32_t s = 0; s < S; ++s) {
    const int32_t nt = pl.rtarget_beg[s + 1] - pl.rtarget_beg[s];
    REQUIRE(nt == pl.ext_lr_beg[s + 1] - pl.ext_lr_beg[s] && nt <= pl.max_rtargets);
    for (int pass = 1; pass <= 2; ++pass) {
      const auto& rp = pass == 1 ? pl.rpairs1 : pl.rpairs2;
      const auto& chv = pass == 1 ? pl.r1chunks : pl.r2chunks;
      const auto& chb = pass == 1 ? pl.r1chunk_beg : pl.r2chunk_beg;
      const auto& tlv = pass == 1 ? pl.tiles1 : pl.tiles2;
      const auto& tlb = pass == 1 ? pl.t1_beg : pl.t2_beg;
      const auto& tcv = pass == 1 ? pl.tc1 : pl.tc2;
      const auto& tcb = pass == 1 ? pl.tc1_beg : pl.tc2_beg;
      const auto& sgv = pass == 1 ? pl.sg1 : pl.sg2;
      const auto& sgb = pass == 1 ? pl.sg1_beg : pl.sg2_beg;
      const auto& giv = pass == 1 ? pl.g1items : pl.g2items;
      const auto& gib = pass == 1 ? pl.g1_beg : pl.g2_beg;
      const auto& gfv = pass == 1 ? pl.gf1 : pl.gf2;
      const auto& gfb = pass == 1 ? pl.gf1_beg : pl.gf2_beg;
      const ChunkDesc* ch = chv.data() + chb[s];
      const int32_t nch = chb[s + 1] - chb[s];
      const int32_t ntl = tlb[s + 1] - tlb[s], ntc = tcb[s + 1] - tcb[s], nsg = sgb[s + 1] - sgb[s];
      REQUIRE(ntl <= pl.max_tiles && nsg <= pl.max_segs);
      // input-side products of the step: slot -> (target, input block, rows), whole or in segments
      struct Slot { int32_t b = -2, blk = -2, r0 = 0, r1 = 0, whole = 0, parts = 0; };
      std::map<int32_t, Slot> slots;
      std::map<int32_t, std::vector<const GItem*>> seg_items;
      std::set<int32_t> parts_seen;
      for (int32_t q = gib[s]; q < gib[s + 1]; ++q) {
        const GItem& gi = giv[q];
        REQUIRE(gi.slot >= 0 && gi.slot < pl.max_gslots && gi.r0 < gi.r1);
        if (gi.part < 0) {
          Slot& sl = slots[gi.slot];
          REQUIRE(sl.b == -2 && gi.r1 - gi.r0 <= pl.gseg_rows);
          sl = Slot{gi.b, gi.blk, gi.r0, gi.r1, 1, 0};
        } else {
          REQUIRE(gi.part < pl.max_gparts && parts_seen.insert(gi.part).second && gi.r1 - gi.r0 <= pl.gseg_rows);
          seg_items[gi.slot].push_back(&gi);
        }
      }
      for (int32_t q = gfb[s]; q < gfb[s + 1]; ++q) {
        const GFin& f = gfv[q];
        auto& v = seg_items[f.slot];
        REQUIRE(!v.empty() && slots.count(f.slot) == 0 && f.hi - f.lo == (int32_t)v.size());
        for (size_t k = 0; k < v.size(); ++k) {
          REQUIRE(v[k]->part == f.lo + (int32_t)k && v[k]->b == f.b && v[k]->blk == f.blk);
          if (k) REQUIRE(v[k]->r0 == v[k - 1]->r1);
        }
        slots[f.slot] = Slot{f.b, f.blk, v.front()->r0, v.back()->r1, 0, (int32_t)v.size()};
      }
      for (const auto& kv : seg_items) REQUIRE(slots.count(kv.first) && slots[kv.first].parts > 0);
      std::vector<std::pair<int64_t, int64_t>> outs;
      for (int32_t t = 0; t < nt; ++t) {
        const RTargetDesc& rt = pl.rtargets[pl.rtarget_beg[s] + t];
        const int32_t bi = rt.b;
        const BlockDesc& b = bl[bi];
        REQUIRE(pl.ext_lr[pl.ext_lr_beg[s] + t] == bi);
        const int32_t m = b.r1 - b.r0, k = b.c1 - b.c0;
        const int32_t olen = pass == 1 ? m : k, obase = pass == 1 ? b.r0 : b.c0;
        // the base product of the target's cross approximation
        const int32_t gb = pass == 1 ? rt.gb1 : rt.gb2;
        REQUIRE(slots.count(gb) && slots[gb].b == bi && slots[gb].blk == -1 && slots[gb].r0 == 0 &&
                slots[gb].r1 == (pass == 1 ? k : m));
        const int32_t clo = pass == 1 ? rt.c1lo : rt.c2lo, chi = pass == 1 ? rt.c1hi : rt.c2hi;
        REQUIRE(0 <= clo && clo <= chi && chi <= nch);
        std::map<int32_t, std::pair<int32_t, int32_t>> in_rows;   // input block -> rows (one range each)
        std::vector<const RPairDesc*> pieces;
        std::vector<std::vector<const ChunkDesc*>> tile_chunks((olen + 127) / 128);
        int64_t at = clo < chi ? ch[clo].pair_lo : 0;
        for (int32_t c = clo; c < chi; ++c) {
          const ChunkDesc& cd = ch[c];
          REQUIRE(cd.b == bi && cd.slot == c - clo && cd.pair_lo == at && cd.pair_hi > cd.pair_lo);
          at = cd.pair_hi;
          const RPairDesc& r0 = rp[cd.pair_lo];
          const int32_t qb = pass == 1 ? r0.x : r0.y;
          const int32_t q0 = pass == 1 ? r0.rx0 : r0.ry0, q1 = pass == 1 ? r0.rx1 : r0.ry1;
          int32_t load = 0;
          for (int32_t q = cd.pair_lo; q < cd.pair_hi; ++q) {
            const RPairDesc& r = rp[q];
            REQUIRE((pass == 1 ? r.x : r.y) == qb && (pass == 1 ? r.rx0 : r.ry0) == q0 && (pass == 1 ? r.rx1 : r.ry1) == q1);
            load += cost(r);
            pieces.push_back(&r);
            const BlockDesc &x = bl[r.x], &y = bl[r.y];
            REQUIRE(r.rx0 < r.rx1 && r.ry0 < r.ry1 && r.w0 < r.w1 && r.w1 <= b.c0);
            REQUIRE(b.r0 <= r.rx0 && r.rx1 <= b.r1 && b.c0 <= r.ry0 && r.ry1 <= b.c1);
            REQUIRE(x.r0 <= r.rx0 && r.rx1 <= x.r1 && x.c0 <= r.w0 && r.w1 <= x.c1);
            REQUIRE(y.r0 <= r.ry0 && r.ry1 <= y.r1 && y.c0 <= r.w0 && r.w1 <= y.c1);
            if (cost(r) > 1) REQUIRE(r.w1 - r.w0 <= 64 && (bl[qb].kind == BK_LOWRANK || q1 - q0 <= 128));
            const int32_t ib = pass == 1 ? r.y : r.x;
            const int32_t i0 = pass == 1 ? r.ry0 : r.rx0, i1 = pass == 1 ? r.ry1 : r.rx1;
            if (bl[ib].kind == BK_LOWRANK) {
              auto it = in_rows.find(ib);
              if (it == in_rows.end()) in_rows[ib] = {i0, i1};
              else REQUIRE(it->second == std::make_pair(i0, i1));
              REQUIRE(slots.count(r.gslot) && slots[r.gslot].b == bi && slots[r.gslot].blk == ib &&
                      slots[r.gslot].r0 == i0 && slots[r.gslot].r1 == i1);
            } else {
              REQUIRE(r.gslot == -1);
            }
          }
          REQUIRE(cd.pair_hi - cd.pair_lo == 1 || load <= group);
          const int64_t sz = (int64_t)(bl[qb].kind == BK_LOWRANK ? R : q1 - q0) * R;
          REQUIRE(cd.poff >= 0 && cd.poff + sz <= pl.rpart_size);
          outs.push_back({cd.poff, cd.poff + sz});
          for (int32_t tt = (q0 - obase) / 128; tt <= (q1 - 1 - obase) / 128; ++tt) tile_chunks[tt].push_back(&cd);
        }
        // coverage of sampled entries by this pass's pieces
        for (int rep = 0; rep < 3 && b.c0 > offs[b.prob]; ++rep) {
          const int64_t i = b.r0 + (int64_t)(g() % m), j = b.c0 + (int64_t)(g() % k);
          std::vector<std::pair<int32_t, int32_t>> w;
          for (const RPairDesc* r : pieces)
            if (r->rx0 <= i && i < r->rx1 && r->ry0 <= j && j < r->ry1) w.push_back({r->w0, r->w1});
          std::sort(w.begin(), w.end());
          int64_t pos = offs[b.prob];
          for (const auto& iv : w) {
            REQUIRE(iv.first == pos);
            pos = iv.second;
          }
          REQUIRE(pos == b.c0);
        }
        if (b.c0 == offs[b.prob]) REQUIRE(pieces.empty());
        // row tiles of this pass and the chunks they sum
        const int32_t tlo = pass == 1 ? rt.t1lo : rt.t2lo, thi = pass == 1 ? rt.t1hi : rt.t2hi;
        REQUIRE(thi - tlo == (olen + 127) / 128 && 0 <= tlo && thi <= ntl);
        for (int32_t tt = 0; tt < thi - tlo; ++tt) {
          const RowTile& T = tlv[tlb[s] + tlo + tt];
          REQUIRE(T.t == t && T.r0 == 128 * tt && 0 <= T.cb && T.cb <= T.ce && T.ce <= ntc);
          REQUIRE(T.ce - T.cb == (int32_t)tile_chunks[tt].size());
          for (int32_t e = T.cb; e < T.ce; ++e) {
            const TileChunk& tc = tcv[tcb[s] + e];
            const ChunkDesc* cd = tile_chunks[tt][e - T.cb];
            const RPairDesc& r0 = rp[cd->pair_lo];
            const int32_t qb = pass == 1 ? r0.x : r0.y;
            REQUIRE(tc.qb == qb && tc.poff == cd->poff && tc.lr == (bl[qb].kind == BK_LOWRANK ? 1 : 0));
            REQUIRE(tc.rq0 == (pass == 1 ? r0.rx0 : r0.ry0) && tc.rq1 == (pass == 1 ? r0.rx1 : r0.ry1));
          }
          REQUIRE(0 <= T.sb && T.sb < T.se && T.se <= nsg);
          int32_t e = T.cb;
          for (int32_t q = T.sb; q < T.se; ++q) {
            const TileSeg& sg = sgv[sgb[s] + q];
            REQUIRE(sg.tile == tlo + tt && sg.eb == e && (sg.ee > sg.eb || (T.cb == T.ce && sg.ee == sg.eb)) && sg.ee - sg.eb <= pl.seg_entries);
            REQUIRE(sg.first == (q == T.sb ? 1 : 0));
            e = sg.ee;
          }
          REQUIRE(e == T.ce);
        }
      }
      std::sort(outs.begin(), outs.end());
      for (size_t q = 1; q < outs.size(); ++q) REQUIRE(outs[q].first >= outs[q - 1].second);
    }
  }
}

static void check(const char* label, const std::vector<double>& pts, const std::vector<int64_t>& offs, int dim,
                  int leaf, double eta, int R, int chunk, int group, std::mt19937_64& g, int seg = 8, int gseg = 512) {
  ClusterTree tr;
  BlockTree bt;
  Plan pl;
  build_forest(pts.data(), offs, dim, leaf, eta, tr, bt);
  build_plan(tr, bt, offs, R, R, chunk, group, pl, seg, gseg);
  REQUIRE(pl.seg_entries == seg && pl.gseg_rows == gseg);
  const int32_t P = (int32_t)offs.size() - 1, B = pl.n_leaves, S = pl.n_steps;
  const int32_t nb = (int32_t)pl.blocks.size();
  auto prob_of = [&](int64_t r) {
    int32_t p = 0;
    while (offs[p + 1] <= r) ++p;
    return p;
  };
  // leaves and steps
  REQUIRE(pl.prob_off == offs && (int32_t)pl.prob_leaf0.size() == P + 1 && pl.prob_leaf0[P] == B);
  REQUIRE(pl.max_leaf <= leaf);   // the leaf Cholesky holds a whole leaf of at most leaf_size rows
  std::vector<int32_t> step_of(B, -1);
  for (int32_t p = 0; p < P; ++p) {
    int64_t r = offs[p];
    for (int32_t j = pl.prob_leaf0[p]; j < pl.prob_leaf0[p + 1]; ++j) {
      REQUIRE(pl.leaf_lo[j] == r && pl.leaf_hi[j] > pl.leaf_lo[j] && pl.leaf_hi[j] - pl.leaf_lo[j] <= pl.max_leaf);
      r = pl.leaf_hi[j];
      step_of[j] = j - pl.prob_leaf0[p];
    }
    REQUIRE(r == offs[p + 1]);
  }
  REQUIRE((int32_t)pl.step_leaf_beg.size() == S + 1 && pl.step_leaf_beg[S] == B);
  for (int32_t s = 0; s < S; ++s)
    for (int32_t q = pl.step_leaf_beg[s]; q < pl.step_leaf_beg[s + 1]; ++q) REQUIRE(step_of[pl.step_leaf[q]] == s);
  std::vector<int32_t> leaf_of_row(offs[P]);
  for (int32_t j = 0; j < B; ++j)
    for (int32_t i = pl.leaf_lo[j]; i < pl.leaf_hi[j]; ++i) leaf_of_row[i] = j;
  // blocks tile the lower triangle
  std::vector<long double> area(P, 0);
  for (int32_t bi = 0; bi < nb; ++bi) {
    const BlockDesc& b = pl.blocks[bi];
    REQUIRE(b.r0 < b.r1 && b.c0 < b.c1 && b.prob == prob_of(b.r0) && b.r1 <= offs[b.prob + 1] && b.c0 >= offs[b.prob]);
    REQUIRE((bi < pl.n_dense) == (b.kind != BK_LOWRANK));
    if (b.kind == BK_DIAG) {
      REQUIRE(b.r0 == b.c0 && b.r1 == b.c1 && pl.leaf_lo[b.leaf] == b.r0 && pl.leaf_hi[b.leaf] == b.r1);
      REQUIRE(pl.leaf_diag[b.leaf] == bi);
      area[b.prob] += (long double)(b.r1 - b.r0) * (b.r1 - b.r0 + 1) / 2;
    } else {
      REQUIRE(b.r0 >= b.c1);
      area[b.prob] += (long double)(b.r1 - b.r0) * (b.c1 - b.c0);
    }
  }
  for (int32_t p = 0; p < P; ++p) {
    const long double np = (long double)(offs[p + 1] - offs[p]);
    REQUIRE(area[p] == np * (np + 1) / 2);
  }
  for (int t = 0; t < 300; ++t) {
    const int64_t i = (int64_t)(g() % offs[P]);
    const int32_t p = prob_of(i);
    const int64_t j = offs[p] + (int64_t)(g() % (i - offs[p] + 1));
    int hits = 0;
    for (const BlockDesc& b : pl.blocks) hits += contains(b, i, j);
    REQUIRE(hits == 1);
  }
  // external update pairs
  REQUIRE((int32_t)pl.pair_beg.size() == nb + 1 && pl.pair_beg[nb] == (int64_t)pl.pairs.size());
  for (int32_t bi = 0; bi < nb; ++bi) {
    const BlockDesc& b = pl.blocks[bi];
    REQUIRE(pl.pair_beg[bi] <= pl.pair_beg[bi + 1]);
    for (int64_t q = pl.pair_beg[bi]; q < pl.pair_beg[bi + 1]; ++q) {
      const PairDesc& pr = pl.pairs[q];
      REQUIRE(pr.x >= 0 && pr.x < nb && pr.y >= 0 && pr.y < nb);
      const BlockDesc &x = pl.blocks[pr.x], &y = pl.blocks[pr.y];
      REQUIRE(pr.rx0 < pr.rx1 && pr.ry0 < pr.ry1 && pr.w0 < pr.w1 && pr.w1 <= b.c0);
      REQUIRE(b.r0 <= pr.rx0 && pr.rx1 <= b.r1 && b.c0 <= pr.ry0 && pr.ry1 <= b.c1);
      REQUIRE(x.r0 <= pr.rx0 && pr.rx1 <= x.r1 && x.c0 <= pr.w0 && pr.w1 <= x.c1 && x.c1 <= b.c0);
      REQUIRE(y.r0 <= pr.ry0 && pr.ry1 <= y.r1 && y.c0 <= pr.w0 && pr.w1 <= y.c1 && y.c1 <= b.c0);
      const bool both_lr = x.kind == BK_LOWRANK && y.kind == BK_LOWRANK;
      REQUIRE(both_lr ? (pr.gram >= 0 && pr.gram < pl.n_grams) : pr.gram == -1);
    }
    const int64_t samples[3][2] = {{b.r0, b.c0}, {b.r1 - 1, b.c1 - 1},
                                   {b.r0 + (int64_t)(g() % (b.r1 - b.r0)), b.c0 + (int64_t)(g() % (b.c1 - b.c0))}};
    for (const auto& ij : samples) {
      const int64_t i = ij[0], j = ij[1];
      if (b.kind == BK_DIAG && j > i) continue;
      std::vector<std::pair<int32_t, int32_t>> w;
      for (int64_t q = pl.pair_beg[bi]; q < pl.pair_beg[bi + 1]; ++q) {
        const PairDesc& pr = pl.pairs[q];
        if (pr.rx0 <= i && i < pr.rx1 && pr.ry0 <= j && j < pr.ry1) w.push_back({pr.w0, pr.w1});
      }
      std::sort(w.begin(), w.end());
      int64_t at = offs[b.prob];
      for (const auto& iv : w) {
        REQUIRE(iv.first == at);
        at = iv.second;
      }
      REQUIRE(at == b.c0);
    }
  }
  // external update lists, Gram schedule
  std::vector<int32_t> ext_step(nb, -1);
  REQUIRE((int32_t)pl.ext_dense_beg.size() == S + 1 && (int32_t)pl.ext_lr_beg.size() == S + 1);
  for (int32_t s = 0; s < S; ++s) {
    for (int32_t q = pl.ext_dense_beg[s]; q < pl.ext_dense_beg[s + 1]; ++q) {
      const int32_t bi = pl.ext_dense[q];
      REQUIRE(pl.blocks[bi].kind != BK_LOWRANK && ext_step[bi] < 0);
      ext_step[bi] = s;
    }
    for (int32_t q = pl.ext_lr_beg[s]; q < pl.ext_lr_beg[s + 1]; ++q) {
      const int32_t bi = pl.ext_lr[q];
      REQUIRE(pl.blocks[bi].kind == BK_LOWRANK && ext_step[bi] < 0);
      ext_step[bi] = s;
    }
  }
  for (int32_t bi = 0; bi < nb; ++bi) REQUIRE(ext_step[bi] == step_of[leaf_of_row[pl.blocks[bi].c0]]);
  std::vector<int32_t> gram_step(pl.n_grams, -1);
  REQUIRE((int32_t)pl.gram_beg.size() == S + 1 && pl.gram_beg[S] == (int32_t)pl.grams.size());
  for (int32_t s = 0; s < S; ++s)
    for (int32_t q = pl.gram_beg[s]; q < pl.gram_beg[s + 1]; ++q) {
      const PairDesc& gd = pl.grams[q];
      REQUIRE(gd.rx0 >= 0 && gd.rx0 < pl.n_grams && gram_step[gd.rx0] < 0);
      gram_step[gd.rx0] = s;
      REQUIRE(s >= step_of[leaf_of_row[pl.blocks[gd.x].c1 - 1]] && s >= step_of[leaf_of_row[pl.blocks[gd.y].c1 - 1]]);
    }
  for (int32_t bi = 0; bi < nb; ++bi)
    for (int64_t q = pl.pair_beg[bi]; q < pl.pair_beg[bi + 1]; ++q)
      if (pl.pairs[q].gram >= 0) REQUIRE(gram_step[pl.pairs[q].gram] >= 0 && gram_step[pl.pairs[q].gram] < ext_step[bi]);
  // dense targets' chunks
  REQUIRE((int32_t)pl.dtarget_beg.size() == S + 1 && (int32_t)pl.dchunk_beg.size() == S + 1);
  for (int32_t s = 0; s < S; ++s) {
    const ChunkDesc* ch = pl.dchunks.data() + pl.dchunk_beg[s];
    const int32_t nch = pl.dchunk_beg[s + 1] - pl.dchunk_beg[s];
    std::vector<std::pair<int64_t, int64_t>> parts;
    int32_t n_targets = 0;
    for (int32_t q = pl.dtarget_beg[s]; q < pl.dtarget_beg[s + 1]; ++q, ++n_targets) {
      const TargetDesc& td = pl.dtargets[q];
      const BlockDesc& b = pl.blocks[td.b];
      REQUIRE(ext_step[td.b] == s && 0 <= td.chunk_lo && td.chunk_lo <= td.chunk_hi && td.chunk_hi <= nch);
      int64_t at = pl.pair_beg[td.b];
      for (int32_t c = td.chunk_lo; c < td.chunk_hi; ++c) {
        REQUIRE(ch[c].b == td.b && ch[c].slot == c - td.chunk_lo && ch[c].pair_lo == at && ch[c].pair_hi > at);
        REQUIRE(ch[c].pair_hi - ch[c].pair_lo <= pl.pair_chunk);
        at = ch[c].pair_hi;
        const int64_t sz = (int64_t)(b.r1 - b.r0) * (b.c1 - b.c0);
        REQUIRE(ch[c].poff >= 0 && ch[c].poff + sz <= pl.dpart_size);
        parts.push_back({ch[c].poff, ch[c].poff + sz});
      }
      REQUIRE(at == pl.pair_beg[td.b + 1]);
    }
    REQUIRE(n_targets == pl.ext_dense_beg[s + 1] - pl.ext_dense_beg[s]);
    std::sort(parts.begin(), parts.end());
    for (size_t k = 1; k < parts.size(); ++k) REQUIRE(parts[k].first >= parts[k - 1].second);
  }
  // column solves and inner updates
  auto wcols = [&](const BlockDesc& b) { return b.kind == BK_LOWRANK ? R : b.r1 - b.r0; };
  REQUIRE((int32_t)pl.active_beg.size() == S + 1 && (int32_t)pl.tsolve_beg.size() == S + 1);
  REQUIRE((int32_t)pl.inner_beg.size() == S + 1 && (int32_t)pl.fsolve_beg.size() == S + 1);
  for (int32_t s = 0; s < S; ++s) {
    std::set<int32_t> act(pl.active.begin() + pl.active_beg[s], pl.active.begin() + pl.active_beg[s + 1]);
    REQUIRE((int32_t)act.size() == pl.active_beg[s + 1] - pl.active_beg[s]);
    for (int32_t bi = 0; bi < nb; ++bi) {
      const BlockDesc& b = pl.blocks[bi];
      const bool want = b.kind != BK_DIAG && step_of[leaf_of_row[b.c0]] <= s && s <= step_of[leaf_of_row[b.c1 - 1]];
      REQUIRE(want == (act.count(bi) == 1));
    }
    std::map<int32_t, std::vector<int32_t>> tcols;
    for (int32_t q = pl.tsolve_beg[s]; q < pl.tsolve_beg[s + 1]; ++q) {
      const InnerDesc& d = pl.tsolve[q];
      REQUIRE(act.count(d.b) && d.x == -1 && d.c0 % 32 == 0 && d.c0 < wcols(pl.blocks[d.b]));
      tcols[d.b].push_back(d.c0);
    }
    for (int32_t bi : act) {
      std::vector<int32_t> c = tcols[bi];
      std::sort(c.begin(), c.end());
      REQUIRE((int32_t)c.size() == (wcols(pl.blocks[bi]) + 31) / 32);
      for (size_t k = 0; k < c.size(); ++k) REQUIRE(c[k] == 32 * (int32_t)k);
    }
    std::map<int32_t, int64_t> frows;
    for (int32_t q = pl.fsolve_beg[s]; q < pl.fsolve_beg[s + 1]; ++q) {
      const InnerDesc& d = pl.fsolve[q];
      const BlockDesc& b = pl.blocks[d.b];
      REQUIRE(act.count(d.b) && d.r0 == frows[d.b] && d.c0 > d.r0 && d.c0 <= b.r1 - b.r0);
      frows[d.b] = d.c0;
    }
    for (int32_t bi : act) REQUIRE(frows[bi] == pl.blocks[bi].r1 - pl.blocks[bi].r0);
    // inner updates: (block, row, 32-column slice) -> count
    std::map<std::tuple<int32_t, int32_t, int32_t>, int32_t> cover;
    for (int32_t q = pl.inner_beg[s]; q < pl.inner_beg[s + 1]; ++q) {
      const InnerDesc& d = pl.inner[q];
      REQUIRE(act.count(d.b) && act.count(d.x) && d.c0 % 32 == 0 && d.c0 < wcols(pl.blocks[d.b]));
      const BlockDesc &b = pl.blocks[d.b], &x = pl.blocks[d.x];
      REQUIRE(x.r0 >= b.c0 && x.r1 <= b.c1 && d.r0 >= 0 && d.r0 < x.r1 - x.r0 && d.r0 % 128 == 0);
      for (int32_t r = x.r0 + d.r0; r < std::min(x.r1, x.r0 + d.r0 + 128); ++r) cover[{d.b, r, d.c0}]++;
    }
    for (int32_t bi : act) {
      const BlockDesc& b = pl.blocks[bi];
      const int32_t lf = pl.prob_leaf0[b.prob] + s;
      for (int32_t c0 = 0; c0 < wcols(b); c0 += 32)
        for (int32_t r = b.c0; r < b.c1; ++r) {
          const auto it = cover.find({bi, r, c0});
          const int32_t n = it == cover.end() ? 0 : it->second;
          REQUIRE(n == (r >= pl.leaf_hi[lf] ? 1 : 0));
        }
    }
  }
  check_lowrank(label, pl, offs, R, group, g);
  std::printf("ok %s: n=%lld problems=%d leaves=%d steps=%d blocks=%d (low-rank %d) pairs=%zu grams=%lld\n", label,
              (long long)offs[P], P, B, S, nb, pl.n_lowrank, pl.pairs.size(), (long long)pl.n_grams);
}

// Executes the plan's schedule on a dense copy of an exponential covariance
// matrix (internal order) and compares with a plain Cholesky factorisation.
static void execute_exact(const char* label, const std::vector<double>& pts, const std::vector<int64_t>& offs,
                          int dim, int leaf, double eta) {
  ClusterTree tr;
  BlockTree bt;
  Plan pl;
  build_forest(pts.data(), offs, dim, leaf, eta, tr, bt);
  build_plan(tr, bt, offs, 32, 32, 1, 8, pl);
  const int64_t n = offs.back();
  const int32_t P = (int32_t)offs.size() - 1;
  std::vector<int32_t> prob(n);
  for (int32_t p = 0; p < P; ++p)
    for (int64_t i = offs[p]; i < offs[p + 1]; ++i) prob[i] = p;
  // A = exp(-|x_i - x_j| / 0.2) + 0.01 [i == j] within a problem, 0 across problems
  std::vector<double> A((size_t)n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      if (prob[i] != prob[j]) continue;
      double d2 = 0.0;
      for (int k = 0; k < dim; ++k) {
        const double t = pts[(size_t)tr.perm[i] * dim + k] - pts[(size_t)tr.perm[j] * dim + k];
        d2 += t * t;
      }
      A[i * n + j] = A[j * n + i] = std::exp(-std::sqrt(d2) / 0.2) + (i == j ? 0.01 : 0.0);
    }
  // textbook reference: L L^T = A, column by column
  std::vector<double> R(A);
  for (int64_t k = 0; k < n; ++k) {
    double d = R[k * n + k];
    for (int64_t t = 0; t < k; ++t) d -= R[k * n + t] * R[k * n + t];
    REQUIRE(d > 0);
    d = std::sqrt(d);
    R[k * n + k] = d;
    for (int64_t i = k + 1; i < n; ++i) {
      double v = R[i * n + k];
      for (int64_t t = 0; t < k; ++t) v -= R[i * n + t] * R[k * n + t];
      R[i * n + k] = v / d;
    }
  }
  // the schedule, applied to S (starts as A; ends holding L in the lower triangle)
  std::vector<double> S(A);
  auto at = [&](int64_t i, int64_t j) -> double& { return S[i * n + j]; };
  for (int32_t s = 0; s < pl.n_steps; ++s) {
    // 1. external updates of the blocks whose columns start at this step's leaf
    auto external = [&](int32_t bi) {
      for (int64_t q = pl.pair_beg[bi]; q < pl.pair_beg[bi + 1]; ++q) {
        const PairDesc& pr = pl.pairs[q];
        for (int32_t i = pr.rx0; i < pr.rx1; ++i)
          for (int32_t j = pr.ry0; j < pr.ry1; ++j) {
            double v = 0.0;
            for (int32_t w = pr.w0; w < pr.w1; ++w) v += at(i, w) * at(j, w);
            at(i, j) -= v;
          }
      }
    };
    for (int32_t q = pl.ext_dense_beg[s]; q < pl.ext_dense_beg[s + 1]; ++q) external(pl.ext_dense[q]);
    for (int32_t q = pl.ext_lr_beg[s]; q < pl.ext_lr_beg[s + 1]; ++q) external(pl.ext_lr[q]);
    // 2. Cholesky of each diagonal leaf of the step (lower triangle, in place)
    for (int32_t q = pl.step_leaf_beg[s]; q < pl.step_leaf_beg[s + 1]; ++q) {
      const int32_t j = pl.step_leaf[q], lo = pl.leaf_lo[j], hi = pl.leaf_hi[j];
      for (int32_t k = lo; k < hi; ++k) {
        double d = at(k, k);
        for (int32_t t = lo; t < k; ++t) d -= at(k, t) * at(k, t);
        REQUIRE(d > 0);
        at(k, k) = std::sqrt(d);
        for (int32_t i = k + 1; i < hi; ++i) {
          double v = at(i, k);
          for (int32_t t = lo; t < k; ++t) v -= at(i, t) * at(k, t);
          at(i, k) = v / at(k, k);
        }
      }
    }
    auto leaf_of = [&](const BlockDesc& b) { return pl.prob_leaf0[b.prob] + s; };
    // 3. column solves: L_b[:, leaf] <- L_b[:, leaf] L_jj^{-T}
    for (int32_t q = pl.tsolve_beg[s]; q < pl.tsolve_beg[s + 1]; ++q) {
      if (pl.tsolve[q].c0 != 0) continue;   // column slices of the stored factor: one exact solve per block
      const BlockDesc& b = pl.blocks[pl.tsolve[q].b];
      const int32_t j = leaf_of(b), lo = pl.leaf_lo[j], hi = pl.leaf_hi[j];
      for (int32_t i = b.r0; i < b.r1; ++i)
        for (int32_t k = lo; k < hi; ++k) {
          double v = at(i, k);
          for (int32_t t = lo; t < k; ++t) v -= at(i, t) * at(k, t);
          at(i, k) = v / at(k, k);
        }
    }
    // 4. inner updates: L_b[:, rows of x] -= L_b[:, leaf] L_x[rows, leaf]^T
    for (int32_t q = pl.inner_beg[s]; q < pl.inner_beg[s + 1]; ++q) {
      const InnerDesc& d = pl.inner[q];
      if (d.c0 != 0) continue;
      const BlockDesc &b = pl.blocks[d.b], &x = pl.blocks[d.x];
      const int32_t j = leaf_of(b), lo = pl.leaf_lo[j], hi = pl.leaf_hi[j];
      for (int32_t i = b.r0; i < b.r1; ++i)
        for (int32_t r = x.r0 + d.r0; r < std::min(x.r1, x.r0 + d.r0 + 128); ++r) {
          double v = 0.0;
          for (int32_t k = lo; k < hi; ++k) v += at(i, k) * at(r, k);
          at(i, r) -= v;
        }
    }
  }
  double err = 0.0, scale = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      err = std::max(err, std::fabs(S[i * n + j] - R[i * n + j]));
      scale = std::max(scale, std::fabs(R[i * n + j]));
    }
  REQUIRE(err <= 1e-11 * scale);
  // forward substitution by the plan's solve lists: at step s each leaf's
  // values become L_jj^{-1} v[leaf]; each item subtracts L_x[rows, leaf] times
  // them from the rows [r0, c0) of its block x
  std::vector<double> z(n), v(n), out(n, 0.0), ref(n);
  for (int64_t i = 0; i < n; ++i) z[i] = std::sin(0.37 * (double)i + 1.0);
  v = z;
  auto leaf_solve = [&](int32_t j, std::vector<double>& y) {
    const int32_t lo = pl.leaf_lo[j], hi = pl.leaf_hi[j];
    y.assign(hi - lo, 0.0);
    for (int32_t k = lo; k < hi; ++k) {
      double t = v[k];
      for (int32_t a = lo; a < k; ++a) t -= at(k, a) * y[a - lo];
      y[k - lo] = t / at(k, k);
    }
  };
  std::vector<double> y;
  for (int32_t s = 0; s < pl.n_steps; ++s) {
    for (int32_t q = pl.step_leaf_beg[s]; q < pl.step_leaf_beg[s + 1]; ++q) {
      const int32_t j = pl.step_leaf[q];
      leaf_solve(j, y);
      for (int32_t k = pl.leaf_lo[j]; k < pl.leaf_hi[j]; ++k) out[k] = y[k - pl.leaf_lo[j]];
    }
    for (int32_t q = pl.fsolve_beg[s]; q < pl.fsolve_beg[s + 1]; ++q) {
      const InnerDesc& d = pl.fsolve[q];
      const BlockDesc& x = pl.blocks[d.b];
      const int32_t j = pl.prob_leaf0[x.prob] + s, lo = pl.leaf_lo[j], hi = pl.leaf_hi[j];
      leaf_solve(j, y);
      for (int32_t i = x.r0 + d.r0; i < x.r0 + d.c0; ++i) {
        double t = 0.0;
        for (int32_t k = lo; k < hi; ++k) t += at(i, k) * y[k - lo];
        v[i] -= t;
      }
    }
  }
  double serr = 0.0, sscale = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t = z[i];
    for (int64_t k = 0; k < i; ++k) t -= R[i * n + k] * ref[k];
    ref[i] = t / R[i * n + i];
    serr = std::max(serr, std::fabs(out[i] - ref[i]));
    sscale = std::max(sscale, std::fabs(ref[i]));
  }
  REQUIRE(serr <= 1e-10 * sscale);
  // backward substitution L^T w = out by the same lists in reverse step order:
  // w[leaf j] = L_jj^{-T} (out[leaf j] - sum over the step's items of
  // L_x[rows, leaf j]^T w[rows]); the rows of every item lie after leaf j
  std::vector<double> w(n, 0.0), wref(n);
  for (int32_t s = pl.n_steps - 1; s >= 0; --s) {
    for (int32_t q = pl.step_leaf_beg[s]; q < pl.step_leaf_beg[s + 1]; ++q) {
      const int32_t j = pl.step_leaf[q], lo = pl.leaf_lo[j], hi = pl.leaf_hi[j];
      std::vector<double> r(out.begin() + lo, out.begin() + hi);
      for (int32_t it = pl.fsolve_beg[s]; it < pl.fsolve_beg[s + 1]; ++it) {
        const InnerDesc& d = pl.fsolve[it];
        const BlockDesc& x = pl.blocks[d.b];
        if (pl.prob_leaf0[x.prob] + s != j) continue;
        for (int32_t i = x.r0 + d.r0; i < x.r0 + d.c0; ++i) {
          REQUIRE(i >= hi);
          for (int32_t k = lo; k < hi; ++k) r[k - lo] -= at(i, k) * w[i];
        }
      }
      for (int32_t k = hi - 1; k >= lo; --k) {
        double t = r[k - lo];
        for (int32_t a = k + 1; a < hi; ++a) t -= at(a, k) * w[a];
        w[k] = t / at(k, k);
      }
    }
  }
  double berr = 0.0, bscale = 0.0;
  for (int64_t i = n - 1; i >= 0; --i) {
    double t = ref[i];
    for (int64_t k = i + 1; k < n; ++k) t -= R[k * n + i] * wref[k];
    wref[i] = t / R[i * n + i];
    berr = std::max(berr, std::fabs(w[i] - wref[i]));
    bscale = std::max(bscale, std::fabs(wref[i]));
  }
  REQUIRE(berr <= 1e-10 * bscale);
  // the sampler's product y = L w by row panels: y[leaf j] = L_jj w[leaf j]
  // plus, for each off-diagonal block of the leaf's row panel, its rows of the
  // leaf times w over the block's columns
  std::vector<double> yv(n, 0.0);
  REQUIRE((int32_t)pl.rowp_beg.size() == pl.n_leaves + 1);
  for (int32_t j = 0; j < pl.n_leaves; ++j) {
    const int32_t lo = pl.leaf_lo[j], hi = pl.leaf_hi[j];
    for (int32_t r = lo; r < hi; ++r) {
      double acc = 0.0;
      for (int32_t a = lo; a <= r; ++a) acc += at(r, a) * z[a];
      for (int32_t q = pl.rowp_beg[j]; q < pl.rowp_beg[j + 1]; ++q) {
        const BlockDesc& b = pl.blocks[pl.rowp[q]];
        REQUIRE(b.kind != BK_DIAG && b.r0 <= lo && hi <= b.r1);
        for (int32_t c = b.c0; c < b.c1; ++c) acc += at(r, c) * z[c];
      }
      yv[r] = acc;
    }
  }
  double perr = 0.0, pscale = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t = 0.0;
    for (int64_t k = 0; k <= i; ++k) t += R[i * n + k] * z[k];
    perr = std::max(perr, std::fabs(yv[i] - t));
    pscale = std::max(pscale, std::fabs(t));
  }
  REQUIRE(perr <= 1e-12 * pscale);
  std::printf("exact %s: n=%lld steps=%d blocks=%zu, max |L - chol| = %.3g, forward %.3g, backward %.3g, "
              "product %.3g\n", label, (long long)n, pl.n_steps, pl.blocks.size(), err, serr, berr, perr);
}

// Random configurations (fixed seed): 2-D or 3-D, one to four problems of up
// to 3000 points in all, uniform, duplicated (an 8 x 8 lattice), collinear or
// strongly anisotropic points, leaf sizes 1..128 (8..128 above 400 points),
// eta in [0.2, 50], storage width 4..64, chunk and group options 1..16,
// segment entries 1..32 and input-product segment rows 64..4096; every fifth
// one with at most 900 points is also executed exactly.
static void fuzz(int iters) {
  std::mt19937_64 g(424242);
  std::uniform_real_distribution<double> u(0, 1);
  char label[200];
  for (int it = 0; it < iters; ++it) {
    const int dim = 2 + (int)(g() % 2);
    const int probs = 1 + (int)(g() % 4);
    std::vector<int64_t> offs{0};
    for (int p = 0; p < probs; ++p) offs.push_back(offs.back() + 1 + (int64_t)(g() % (3000 / probs)));
    const int64_t n = offs.back();
    std::vector<double> pts(n * dim);
    const int kind = (int)(g() % 4);
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < dim; ++d) {
        double x = u(g);
        if (kind == 1) x = std::floor(x * 8) / 8;
        if (kind == 2 && d > 0) x = pts[i * dim] * 0.3;
        if (kind == 3) x = (d == 0 ? 1e-3 : 1.0) * x;
        pts[i * dim + d] = x;
      }
    const int leaf = n <= 400 ? 1 + (int)(g() % 128) : 8 + (int)(g() % 121);
    const double eta = std::exp(std::log(0.2) + u(g) * std::log(250.0));
    const int R = 4 + (int)(g() % 61);
    const int chunk = 1 + (int)(g() % 16), group = 1 + (int)(g() % 16);
    const int seg = 1 + (int)(g() % 32), gseg = 64 << (int)(g() % 7);
    std::snprintf(label, sizeof label,
                  "random %d: dim=%d problems=%d kind=%d leaf=%d eta=%.3g R=%d chunk=%d group=%d seg=%d gseg=%d", it,
                  dim, probs, kind, leaf, eta, R, chunk, group, seg, gseg);
    check(label, pts, offs, dim, leaf, eta, R, chunk, group, g, seg, gseg);
    if (n <= 900 && it % 5 == 0) execute_exact(label, pts, offs, dim, leaf, eta);
  }
}

int main() {
  std::mt19937_64 g(20210415);
  std::uniform_real_distribution<double> u(0, 1);
  auto uniform = [&](int64_t n, int dim) {
    std::vector<double> p(n * dim);
    for (auto& x : p) x = u(g);
    return p;
  };
  char label[128];
  for (int dim : {2, 3})
    for (int64_t n : {1, 2, 63, 64, 65, 1999, 5000})
      for (int leaf : {32, 64, 128}) {
        std::snprintf(label, sizeof label, "uniform d=%d n=%lld leaf=%d", dim, (long long)n, leaf);
        check(label, uniform(n, dim), {0, n}, dim, leaf, 2.0, 32, 1, 8, g);
      }
  {
    const int64_t n = 3000;
    std::vector<double> p(n * 2);
    for (int64_t i = 0; i < n; ++i) {
      const double t = u(g);
      p[2 * i] = t;
      p[2 * i + 1] = 0.5 * t;
    }
    check("collinear", p, {0, n}, 2, 64, 2.0, 16, 4, 4, g);
  }
  check("all points equal", std::vector<double>(2000, 0.25), {0, 1000}, 2, 64, 2.0, 16, 1, 8, g);
  {
    std::vector<double> p = uniform(1000, 2);
    for (int i = 1000; i < 2000; ++i) p[i] = p[i - 1000];
    check("every point twice", p, {0, 1000}, 2, 64, 2.0, 32, 2, 16, g);
  }
  check("leaf size 1", uniform(300, 2), {0, 300}, 2, 1, 2.0, 8, 1, 8, g);
  check("leaf size 128, 3-D duplicates", std::vector<double>(3 * 700, 0.5), {0, 700}, 3, 128, 2.0, 16, 1, 8, g);
  check("batch of 5 ragged", uniform(4000, 2), {0, 300, 301, 1500, 1564, 4000}, 2, 64, 2.0, 32, 1, 8, g);
  {
    std::vector<int64_t> offs{0};
    for (int p = 0; p < 64; ++p) offs.push_back(offs.back() + 200 + p);
    check("batch of 64", uniform(offs.back(), 2), offs, 2, 64, 2.0, 32, 16, 1, g);
  }
  for (double eta : {0.5, 1.0, 2.0, 4.0}) {
    std::snprintf(label, sizeof label, "uniform n=20000 leaf=128 eta=%g", eta);
    check(label, uniform(20000, 2), {0, 20000}, 2, 128, eta, 32, 1, 8, g);
  }
  execute_exact("uniform d=2 n=1000 leaf=64 eta=2", uniform(1000, 2), {0, 1000}, 2, 64, 2.0);
  execute_exact("uniform d=3 n=800 leaf=32 eta=1", uniform(800, 3), {0, 800}, 3, 32, 1.0);
  execute_exact("batch of 3 leaf=32 eta=2", uniform(1007, 2), {0, 300, 750, 1007}, 2, 32, 2.0);
  execute_exact("uniform d=2 n=600 leaf=16 eta=4", uniform(600, 2), {0, 600}, 2, 16, 4.0);
  execute_exact("leaf size 1", uniform(150, 2), {0, 150}, 2, 1, 2.0);
  execute_exact("eta=0.01 (nearly all dense)", uniform(700, 2), {0, 700}, 2, 32, 0.01);
  execute_exact("eta=50 (nearly all low-rank)", uniform(700, 2), {0, 700}, 2, 32, 50.0);
  fuzz(200);
  return 0;
}
