// Cluster tree and block tree of one problem on the GPU, under the same
// rules as the host construction in tree.cpp (Section 2's recursive
// partition), with identical results:
//   Cluster tree, level by level: a workgroup per node reduces its bounding
//   box; the host reads the boxes, numbers the nodes level by level and
//   picks each split axis (the longest side, the lowest axis on ties); the
//   points of every node being split are then ordered by (coordinate on its
//   axis, caller index) with two stable segmented radix sorts (by caller
//   index, then by the coordinate mapped to an order-preserving integer), and
//   the first half (rounded down) forms the first child.
//   Block tree, level by level: one thread per candidate pair (t, s) decides
//   dense leaf, admissible low-rank leaf or split, with the admissibility sums
//   formed in the host's order without contraction; exclusive scans place the
//   children and the leaves; the leaf lists are finally sorted by (column
//   cluster start, row cluster start), a total order on a partition.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.hpp"
#include "plan.hpp"

namespace hmle {

namespace {

constexpr int TNT = 256;

#define TREE_TRY(expr)                                                                               \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) throw std::runtime_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Temporary device memory of one construction (the problem's allocator).
thread_local const TreeAlloc* t_alloc = nullptr;

// Device buffer freed at scope exit.
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  explicit DBuf(size_t count) : n(count) {
    p = static_cast<T*>(t_alloc->alloc(std::max<size_t>(1, count) * sizeof(T), t_alloc->ctx));
    if (!p)
      throw DeviceAllocFailure("device allocation of " + std::to_string(std::max<size_t>(1, count) * sizeof(T)) +
                               " bytes for the trees failed (the problem's allocator returned NULL)");
  }
  ~DBuf() { if (p) t_alloc->free(p, t_alloc->ctx); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
};

__global__ void __launch_bounds__(TNT) k_iota(int32_t* perm, int32_t n) {
  const int32_t i = blockIdx.x * TNT + threadIdx.x;
  if (i < n) perm[i] = i;
}

// Bounding box of node f: points perm[lo[f] .. hi[f]) of pts (n x dim, row-major).
__global__ void __launch_bounds__(TNT) k_bbox(const double* pts, const int32_t* perm, int32_t dim, const int32_t* lo,
                                              const int32_t* hi, double* box) {
  __shared__ double smn[TNT], smx[TNT];
  const int f = blockIdx.x;
  for (int k = 0; k < dim; ++k) {
    double mn = INFINITY, mx = -INFINITY;
    for (int32_t i = lo[f] + threadIdx.x; i < hi[f]; i += TNT) {
      const double v = pts[(int64_t)perm[i] * dim + k];
      mn = fmin(mn, v);
      mx = fmax(mx, v);
    }
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int o = TNT / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + o]);
        smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + o]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      box[(int64_t)f * 2 * dim + k] = smn[0];
      box[(int64_t)f * 2 * dim + dim + k] = smx[0];
    }
    __syncthreads();
  }
}

// Order-preserving 64-bit key of a finite double (-0 read as +0).
__device__ __forceinline__ uint64_t order_key(double x) {
  if (x == 0.0) x = 0.0;
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Keys of segment g: the coordinate on its split axis of every point in it.
__global__ void __launch_bounds__(TNT) k_keys(const double* pts, const int32_t* perm, int32_t dim, const int32_t* sb,
                                              const int32_t* se, const int32_t* sax, uint64_t* keys) {
  const int g = blockIdx.x;
  for (int32_t i = sb[g] + threadIdx.x; i < se[g]; i += TNT) keys[i] = order_key(pts[(int64_t)perm[i] * dim + sax[g]]);
}

// Admissibility exactly as on the host: sums in axis order, every product and
// sum rounded on its own.
__device__ bool adm(const double* bmin, const double* bmax, int dim, int t, int s, double eta) {
#pragma clang fp contract(off)
  if (t == s) return false;
  double dt = 0.0, ds = 0.0, g2 = 0.0;
  for (int k = 0; k < dim; ++k) {
    const double et = bmax[t * dim + k] - bmin[t * dim + k];
    dt = dt + et * et;
    const double es = bmax[s * dim + k] - bmin[s * dim + k];
    ds = ds + es * es;
    const double a = bmin[s * dim + k] - bmax[t * dim + k], b = bmin[t * dim + k] - bmax[s * dim + k];
    const double m0 = 0.0 < a ? a : 0.0;
    const double g = m0 < b ? b : m0;
    g2 = g2 + g * g;
  }
  const double md = ds < dt ? ds : dt;
  return md <= (eta * eta) * g2;
}

// kind: 0 dense leaf, 1 low-rank leaf, 2 split; nch: children of a split (3 or 4)
__global__ void __launch_bounds__(TNT) k_classify(const int32_t* ct, const int32_t* cs, int32_t nc,
                                                  const int32_t* child0, const double* bmin, const double* bmax,
                                                  int dim, double eta, int32_t* isd, int32_t* isl, int32_t* nch) {
  const int32_t c = blockIdx.x * TNT + threadIdx.x;
  if (c >= nc) return;
  const int t = ct[c], s = cs[c];
  int kind, k = 0;
  if (t == s) {
    if (child0[t] < 0) kind = 0;
    else { kind = 2; k = 3; }
  } else if (adm(bmin, bmax, dim, t, s, eta)) {
    kind = 1;
  } else if (child0[t] < 0 || child0[s] < 0) {
    kind = 0;
  } else {
    kind = 2;
    k = 4;
  }
  isd[c] = kind == 0;
  isl[c] = kind == 1;
  nch[c] = k;
}

__global__ void __launch_bounds__(TNT) k_emit(const int32_t* ct, const int32_t* cs, int32_t nc, const int32_t* child0,
                                              const int32_t* child1, const int32_t* isd, const int32_t* isl,
                                              const int32_t* nch, const int32_t* od, const int32_t* ol,
                                              const int32_t* oc, int32_t* dt, int32_t* ds, int32_t* lt, int32_t* ls,
                                              int32_t* nt, int32_t* ns) {
  const int32_t c = blockIdx.x * TNT + threadIdx.x;
  if (c >= nc) return;
  const int t = ct[c], s = cs[c];
  if (isd[c]) { dt[od[c]] = t; ds[od[c]] = s; }
  if (isl[c]) { lt[ol[c]] = t; ls[ol[c]] = s; }
  if (nch[c] == 3) {
    const int c1 = child0[t], c2 = child1[t], o = oc[c];
    nt[o] = c1; ns[o] = c1;
    nt[o + 1] = c2; ns[o + 1] = c1;
    nt[o + 2] = c2; ns[o + 2] = c2;
  } else if (nch[c] == 4) {
    const int a[2] = {child0[t], child1[t]}, b[2] = {child0[s], child1[s]};
    const int o = oc[c];
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) { nt[o + 2 * u + v] = a[u]; ns[o + 2 * u + v] = b[v]; }
  }
}

__global__ void __launch_bounds__(TNT) k_pair_keys(const int32_t* t, const int32_t* s, int32_t cnt, const int32_t* lo,
                                                   uint64_t* key, int32_t* idx) {
  const int32_t c = blockIdx.x * TNT + threadIdx.x;
  if (c >= cnt) return;
  key[c] = ((uint64_t)(uint32_t)lo[s[c]] << 32) | (uint32_t)lo[t[c]];
  idx[c] = c;
}

unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TNT - 1) / TNT); }

template <typename T>
void upload(T* d, const std::vector<T>& h, hipStream_t st) {
  if (!h.empty()) TREE_TRY(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

template <typename T>
void download(std::vector<T>& h, const T* d, size_t count, hipStream_t st) {
  h.resize(count);
  if (count) TREE_TRY(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, st));
  TREE_TRY(hipStreamSynchronize(st));
}

// Exclusive prefix sum of in[0..n) into out; returns the total.
int64_t exclusive_scan(const int32_t* in, int32_t* out, int32_t n, hipStream_t st) {
  size_t bytes = 0;
  TREE_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, n, st));
  DBuf<char> tmp(bytes);
  TREE_TRY(hipcub::DeviceScan::ExclusiveSum(tmp.p, bytes, in, out, n, st));
  int32_t last_o = 0, last_i = 0;
  TREE_TRY(hipMemcpyAsync(&last_o, out + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TREE_TRY(hipMemcpyAsync(&last_i, in + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TREE_TRY(hipStreamSynchronize(st));
  return (int64_t)last_o + last_i;
}

}  // namespace

void build_trees_gpu(const double* d_pts, int32_t n, int32_t dim, int32_t leaf_size, double eta, hipStream_t st,
                     const TreeAlloc& alloc, ClusterTree& tr, BlockTree& bt) {
  struct Scope {
    const TreeAlloc* prev;
    explicit Scope(const TreeAlloc* a) : prev(t_alloc) { t_alloc = a; }
    ~Scope() { t_alloc = prev; }
  } scope(&alloc);
  tr = ClusterTree();
  bt = BlockTree();
  tr.n = n;
  tr.dim = dim;
  DBuf<int32_t> perm(n), perm2(n);
  DBuf<uint64_t> keys(n), keys2(n);
  hipLaunchKernelGGL(k_iota, dim3(nblk(n)), dim3(TNT), 0, st, perm.p, n);
  TREE_TRY(hipGetLastError());
  // ---- cluster tree, level by level
  std::vector<int32_t> flo{0}, fhi{n}, fpar{-1};
  int32_t lev = 0;
  while (!flo.empty()) {
    const int32_t nf = (int32_t)flo.size();
    DBuf<int32_t> dlo(nf), dhi(nf);
    DBuf<double> dbox((size_t)nf * 2 * dim);
    upload(dlo.p, flo, st);
    upload(dhi.p, fhi, st);
    hipLaunchKernelGGL(k_bbox, dim3(nf), dim3(TNT), 0, st, d_pts, perm.p, dim, dlo.p, dhi.p, dbox.p);
    TREE_TRY(hipGetLastError());
    std::vector<double> box;
    download(box, dbox.p, (size_t)nf * 2 * dim, st);
    const int32_t base = tr.n_nodes() + nf;
    std::vector<int32_t> nlo, nhi, npar, sb, se, sax;
    for (int32_t f = 0; f < nf; ++f) {
      const int32_t a = flo[f], b = fhi[f], id = tr.n_nodes();
      tr.lo.push_back(a);
      tr.hi.push_back(b);
      tr.level.push_back(lev);
      tr.parent.push_back(fpar[f]);
      const double* mn = box.data() + (size_t)f * 2 * dim;
      const double* mx = mn + dim;
      for (int k = 0; k < dim; ++k) { tr.bmin.push_back(mn[k]); tr.bmax.push_back(mx[k]); }
      if (b - a > leaf_size) {
        int axis = 0;
        double best = mx[0] - mn[0];
        for (int k = 1; k < dim; ++k) {
          const double e = mx[k] - mn[k];
          if (e > best) { best = e; axis = k; }
        }
        const int32_t half = (b - a) / 2, c = base + (int32_t)nlo.size();
        tr.child0.push_back(c);
        tr.child1.push_back(c + 1);
        nlo.push_back(a); nhi.push_back(a + half); npar.push_back(id);
        nlo.push_back(a + half); nhi.push_back(b); npar.push_back(id);
        sb.push_back(a); se.push_back(b); sax.push_back(axis);
      } else {
        tr.child0.push_back(-1);
        tr.child1.push_back(-1);
      }
    }
    if (!sb.empty()) {
      const int32_t ns = (int32_t)sb.size();
      DBuf<int32_t> dsb(ns), dse(ns), dsax(ns);
      upload(dsb.p, sb, st);
      upload(dse.p, se, st);
      upload(dsax.p, sax, st);
      // positions outside the segments keep their values in both buffers
      TREE_TRY(hipMemcpyAsync(perm2.p, perm.p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
      size_t bytes = 0;
      TREE_TRY(hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, bytes, perm.p, perm2.p, n, ns, dsb.p, dse.p, 0,
                                                           32, st));
      {
        DBuf<char> tmp(bytes);
        TREE_TRY(hipcub::DeviceSegmentedRadixSort::SortKeys(tmp.p, bytes, perm.p, perm2.p, n, ns, dsb.p, dse.p, 0,
                                                             32, st));
      }
      hipLaunchKernelGGL(k_keys, dim3(ns), dim3(TNT), 0, st, d_pts, perm2.p, dim, dsb.p, dse.p, dsax.p, keys.p);
      TREE_TRY(hipGetLastError());
      TREE_TRY(hipMemcpyAsync(perm.p, perm2.p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
      bytes = 0;
      TREE_TRY(hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, bytes, keys.p, keys2.p, perm2.p, perm.p, n, ns,
                                                            dsb.p, dse.p, 0, 64, st));
      DBuf<char> tmp(bytes);
      TREE_TRY(hipcub::DeviceSegmentedRadixSort::SortPairs(tmp.p, bytes, keys.p, keys2.p, perm2.p, perm.p, n, ns,
                                                            dsb.p, dse.p, 0, 64, st));
      TREE_TRY(hipStreamSynchronize(st));
    }
    flo.swap(nlo);
    fhi.swap(nhi);
    fpar.swap(npar);
    ++lev;
  }
  download(tr.perm, perm.p, (size_t)n, st);
  // ---- block tree, level by level
  const int32_t nn = tr.n_nodes();
  DBuf<int32_t> dlo(nn), dc0(nn), dc1(nn);
  DBuf<double> dbmin((size_t)nn * dim), dbmax((size_t)nn * dim);
  upload(dlo.p, tr.lo, st);
  upload(dc0.p, tr.child0, st);
  upload(dc1.p, tr.child1, st);
  upload(dbmin.p, tr.bmin, st);
  upload(dbmax.p, tr.bmax, st);
  std::vector<int32_t> hd_t, hd_s, hl_t, hl_s;
  std::vector<int32_t> ct0{0}, cs0{0};
  int32_t nc = 1;
  DBuf<int32_t>* ct = new DBuf<int32_t>(1);
  DBuf<int32_t>* cs = new DBuf<int32_t>(1);
  upload(ct->p, ct0, st);
  upload(cs->p, cs0, st);
  // leaf lists on the device, appended level by level
  std::vector<int32_t> all_dt, all_ds, all_lt, all_ls;
  try {
    while (nc > 0) {
      DBuf<int32_t> isd(nc), isl(nc), nch(nc), od(nc), ol(nc), oc(nc);
      hipLaunchKernelGGL(k_classify, dim3(nblk(nc)), dim3(TNT), 0, st, ct->p, cs->p, nc, dc0.p, dbmin.p, dbmax.p, dim,
                         eta, isd.p, isl.p, nch.p);
      TREE_TRY(hipGetLastError());
      const int64_t nd = exclusive_scan(isd.p, od.p, nc, st);
      const int64_t nl = exclusive_scan(isl.p, ol.p, nc, st);
      const int64_t nx = exclusive_scan(nch.p, oc.p, nc, st);
      DBuf<int32_t> dt(nd), ds(nd), lt(nl), ls(nl);
      auto* nt = new DBuf<int32_t>(nx);
      auto* nsb = new DBuf<int32_t>(nx);
      hipLaunchKernelGGL(k_emit, dim3(nblk(nc)), dim3(TNT), 0, st, ct->p, cs->p, nc, dc0.p, dc1.p, isd.p, isl.p, nch.p,
                         od.p, ol.p, oc.p, dt.p, ds.p, lt.p, ls.p, nt->p, nsb->p);
      TREE_TRY(hipGetLastError());
      std::vector<int32_t> tmp;
      download(tmp, dt.p, (size_t)nd, st); all_dt.insert(all_dt.end(), tmp.begin(), tmp.end());
      download(tmp, ds.p, (size_t)nd, st); all_ds.insert(all_ds.end(), tmp.begin(), tmp.end());
      download(tmp, lt.p, (size_t)nl, st); all_lt.insert(all_lt.end(), tmp.begin(), tmp.end());
      download(tmp, ls.p, (size_t)nl, st); all_ls.insert(all_ls.end(), tmp.begin(), tmp.end());
      delete ct;
      delete cs;
      ct = nt;
      cs = nsb;
      nc = (int32_t)nx;
    }
  } catch (...) {
    delete ct;
    delete cs;
    throw;
  }
  delete ct;
  delete cs;
  // canonical order of each leaf list: (column cluster start, row cluster start), sorted on the device
  auto canon = [&](const std::vector<int32_t>& ht, const std::vector<int32_t>& hs, std::vector<int32_t>& ot,
                   std::vector<int32_t>& os) {
    const int32_t cnt = (int32_t)ht.size();
    if (cnt == 0) return;
    DBuf<int32_t> dt(cnt), ds(cnt), idx(cnt), idx2(cnt);
    DBuf<uint64_t> k1(cnt), k2(cnt);
    upload(dt.p, ht, st);
    upload(ds.p, hs, st);
    hipLaunchKernelGGL(k_pair_keys, dim3(nblk(cnt)), dim3(TNT), 0, st, dt.p, ds.p, cnt, dlo.p, k1.p, idx.p);
    TREE_TRY(hipGetLastError());
    size_t bytes = 0;
    TREE_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, k1.p, k2.p, idx.p, idx2.p, cnt, 0, 64, st));
    DBuf<char> tmp(bytes);
    TREE_TRY(hipcub::DeviceRadixSort::SortPairs(tmp.p, bytes, k1.p, k2.p, idx.p, idx2.p, cnt, 0, 64, st));
    std::vector<int32_t> order;
    download(order, idx2.p, (size_t)cnt, st);
    for (int32_t q : order) { ot.push_back(ht[q]); os.push_back(hs[q]); }
  };
  canon(all_dt, all_ds, bt.dense_t, bt.dense_s);
  canon(all_lt, all_ls, bt.lr_t, bt.lr_s);
}

}  // namespace hmle
