// HIP kernels of the H-MLE hot path for gfx950 (wave64, 256-thread workgroups).
//
//   assembly     dense near-field blocks (k_assemble_dense) and adaptive cross
//                approximation of the admissible far-field blocks (k_aca),
//                Section 2: low-rank blocks "on the fly", without dense
//                sub-matrices;
//   factor       left-looking H-Cholesky, one sweep step per leaf column:
//                external update of the blocks that start at this column
//                (dense targets exactly, low-rank targets by a randomized
//                range sketch followed by truncation with column-pivoted QR
//                to the block accuracy eps), Cholesky of the diagonal leaf,
//                column solve and inner updates;
//   solve        forward substitution v = L^{-1} P z, log-determinant
//                2 sum log L_ii and v^T v (Section 2, "Storage and complexity");
//   sample       z = P^T L w by row panels (k_sample_h, k_sample_rows);
//   predict      kriging mean (eq. (4)): backward substitution (k_bsolve_part,
//                k_bsolve_fin) and the exact cross-covariance sum (k_predict);
//                kriging variance: cross-covariance columns, forward
//                substitution of 32 of them at a time and sums of squares
//                (k_cross_cols, k_solve_step_multi, k_var_finish).
//
// Every reduction runs in a fixed order, so results are bit-reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"
#include "matern.hpp"

namespace hmle {

constexpr int NT = 256;
constexpr int TILE = 128;     // maximum leaf size handled by the leaf kernels
constexpr int CH = 16;        // column chunk of the dense update tiles

// ------------------------------------------------------------ reductions ----
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ T block_sum(T v, T* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  T r = sh[0];
  for (int i = 1; i < NT / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// argmax of v (ties: lowest index); indices < 0 are ignored.
template <typename T>
__device__ void block_argmax(T v, int idx, T* shv, int* shi, T& best, int& bidx) {
  for (int o = 32; o > 0; o >>= 1) {
    const T ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(idx, o, 64);
    const bool take = (oi >= 0) && (idx < 0 || ov > v || (ov == v && oi < idx));
    if (take) { v = ov; idx = oi; }
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) { shv[w] = v; shi[w] = idx; }
  __syncthreads();
  best = shv[0];
  bidx = shi[0];
  for (int i = 1; i < NT / 64; ++i) {
    const T ov = shv[i];
    const int oi = shi[i];
    if (oi >= 0 && (bidx < 0 || ov > best || (ov == best && oi < bidx))) { best = ov; bidx = oi; }
  }
  __syncthreads();
}

// out (P x Q, column-major in LDS) = A^T B with A: K x P (ld lda), B: K x Q
// (ld ldb), K possibly long; the reduction is split over thread slices and
// summed in slice order.
template <typename TA, typename TB, typename TO>
__device__ void wg_gemm_tn(int K, int P, int Q, const TA* A, int64_t lda, const TB* B, int64_t ldb, TO* out,
                           TO* red) {
  const int E = P * Q;
  if (E <= 0) return;
  if (E * 2 > NT) {
    for (int e = threadIdx.x; e < E; e += NT) {
      const int p = e % P, q = e / P;
      const TA* a = A + (int64_t)p * lda;
      const TB* b = B + (int64_t)q * ldb;
      TO s = TO(0);
#pragma unroll 8
      for (int kk = 0; kk < K; ++kk) s += TO(a[kk]) * TO(b[kk]);
      out[e] = s;
    }
    __syncthreads();
    return;
  }
  const int S = NT / E;
  const int t = threadIdx.x;
  TO s = TO(0);
  if (t < E * S) {
    const int e = t % E, sl = t / E;
    const int p = e % P, q = e / P;
    const TA* a = A + (int64_t)p * lda;
    const TB* b = B + (int64_t)q * ldb;
    // one running sum per thread in k order, unrolled so that several loads are in flight
#pragma unroll 8
    for (int kk = sl; kk < K; kk += S) s += TO(a[kk]) * TO(b[kk]);
  }
  red[t] = s;
  __syncthreads();
  if (t < E) {
    TO r = TO(0);
    for (int sl = 0; sl < S; ++sl) r += red[t + sl * E];
    out[t] = r;
  }
  __syncthreads();
}

// ------------------------------------------------------------ utilities -----
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}

template <typename T>
__device__ __forceinline__ T coord_dist(const double* coords, int n, int dim, int i, int j) {
  T s = T(0);
  for (int d = 0; d < dim; ++d) {
    const T a = T(coords[(int64_t)d * n + i]) - T(coords[(int64_t)d * n + j]);
    s += a * a;
  }
  return sqrt(s);
}

template <typename TS>
__device__ __forceinline__ TS point_dist(const DevCtx<TS>& c, int i, int j) {
  return coord_dist<TS>(c.coords, c.n, c.dim, i, j);
}

template <typename TS>
__device__ __forceinline__ int block_cols(const DevCtx<TS>& c, const BlockDesc& b, int bi) {
  return b.kind == BK_DENSE ? (b.r1 - b.r0) : c.rank[bi];
}

// W factor (|sigma| x cols, ld |sigma|) of an off-diagonal block.
template <typename TS>
__device__ __forceinline__ TS* block_w(const DevCtx<TS>& c, const BlockDesc& b) {
  return b.kind == BK_DENSE ? c.L + b.loff : c.L + b.loff + (int64_t)(b.r1 - b.r0) * c.R;
}

// ------------------------------------------------------------ kernels -------
template <typename T>
__global__ void __launch_bounds__(NT) k_matern(const double* h, int64_t count, MaternParams mp, double* out) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < count) out[i] = double(matern_value<T>(T(h[i]), mp));
}

__global__ void __launch_bounds__(NT) k_gather_coords(const double* pts, const int32_t* perm, int32_t n, int32_t dim,
                                                      double* coords) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n)
    for (int d = 0; d < dim; ++d) coords[(int64_t)d * n + i] = pts[(int64_t)perm[i] * dim + d];
}

__global__ void __launch_bounds__(NT) k_gather(const double* z, const int32_t* perm, int32_t n, double* v) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n) v[i] = z[perm[i]];
}

__global__ void __launch_bounds__(NT) k_scatter(const double* v, const int32_t* perm, int32_t n, double* z) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n) z[perm[i]] = v[i];
}

__global__ void __launch_bounds__(NT) k_check_finite(const double* x, int64_t count, int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < count && !isfinite(x[i])) atomicOr(flag, 1);
}

// Dense blocks of C~ (eq. (2) plus tau^2 on the diagonal). One workgroup per
// block; diagonal leaves in float64, off-diagonal blocks in TS, stored
// transposed (entry (i,j) at j + i*k) so that writes are contiguous in j.
template <typename TS>
__global__ void __launch_bounds__(NT) k_assemble_dense(DevCtx<TS> c) {
  const BlockDesc b = c.blocks[blockIdx.x];
  const MaternParams mp = c.mp[b.prob];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  if (b.kind == BK_DIAG) {
    double* Dg = c.D + b.loff;
    for (int e = threadIdx.x; e < m * k; e += NT) {
      const int i = e % m, j = e / m;
      double v = matern_value<double>(coord_dist<double>(c.coords, c.n, c.dim, b.r0 + i, b.c0 + j), mp);
      if (i == j) v += mp.tau2;
      Dg[e] = v;
    }
  } else {
    TS* W = c.L + b.loff;
    for (int e = threadIdx.x; e < m * k; e += NT) {
      const int j = e % k, i = e / k;
      W[e] = matern_value<TS>(point_dist<TS>(c, b.r0 + i, b.c0 + j), mp);
    }
  }
}

// Adaptive cross approximation with partial pivoting of one admissible block
// per workgroup: U0 W0^T ~ C_b built from single rows and columns of C_b.
// First row: block row 0; column pivot: largest |residual row entry|; next row:
// largest |entry| of the new column among unused rows (ties: lowest index);
// a vanishing residual row moves to the next unused row; stop when
// |u_k| |w_k| <= eps |S_k|_F (recursive Frobenius estimate of S_k = sum u_l w_l^T),
// at the rank cap, or after four consecutive vanishing rows.
template <typename TS>
__global__ void __launch_bounds__(NT) k_aca(DevCtx<TS> c, int32_t first, TS eps) {
  __shared__ TS red[NT];
  __shared__ TS shv[NT / 64];
  __shared__ int shi[NT / 64];
  __shared__ TS dots[2][64];
  const int bi = first + blockIdx.x;
  const BlockDesc b = c.blocks[bi];
  const MaternParams mp = c.mp[b.prob];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0, Ra = c.Ra;
  TS* U = c.A + b.aoff;
  TS* W = U + (int64_t)m * Ra;
  TS* used = c.S + b.soff;     // row flags (sketch scratch is free until the factorisation)
  for (int i = threadIdx.x; i < m; i += NT) used[i] = TS(0);
  __syncthreads();
  const TS tiny = sizeof(TS) == 8 ? TS(1e-300) : TS(1e-35);
  const TS rel_tiny = sizeof(TS) == 8 ? TS(1e-15) : TS(1e-7);
  int rank = 0, istar = 0, zero_run = 0, nused = 0;
  TS frob2 = TS(0), pivmax = TS(0);
  bool conv = false;
  while (rank < Ra && nused < m) {
    if (threadIdx.x == 0) used[istar] = TS(1);
    ++nused;
    TS* wr = W + (int64_t)rank * k;
    TS bv = TS(-1);
    int bj = -1;
    for (int j = threadIdx.x; j < k; j += NT) {
      TS v = matern_value<TS>(point_dist<TS>(c, b.r0 + istar, b.c0 + j), mp);
      // sequential update (same order, same bits), unrolled so that the loads are in flight together
#pragma unroll 8
      for (int l = 0; l < rank; ++l) v -= U[istar + (int64_t)l * m] * W[j + (int64_t)l * k];
      wr[j] = v;
      const TS a = fabs(v);
      if (bj < 0 || a > bv) { bv = a; bj = j; }
    }
    TS vmax;
    int jmax;
    block_argmax<TS>(bv, bj, shv, shi, vmax, jmax);
    if (!(vmax > tiny) || vmax <= rel_tiny * pivmax) {
      if (++zero_run >= 4) { conv = true; break; }
      // next unused row in index order
      int cand = -1;
      for (int i = threadIdx.x; i < m; i += NT)
        if (used[i] == TS(0)) { cand = i; break; }
      TS dummy;
      int nxt;
      block_argmax<TS>(cand >= 0 ? TS(-cand) : TS(-1e30), cand, shv, shi, dummy, nxt);
      if (nxt < 0) { conv = true; break; }
      istar = nxt;
      continue;
    }
    zero_run = 0;
    if (vmax > pivmax) pivmax = vmax;
    const TS piv = wr[jmax];
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += NT) wr[j] = wr[j] / piv;
    TS* uc = U + (int64_t)rank * m;
    for (int i = threadIdx.x; i < m; i += NT) {
      TS v = matern_value<TS>(point_dist<TS>(c, b.r0 + i, b.c0 + jmax), mp);
#pragma unroll 8
      for (int l = 0; l < rank; ++l) v -= U[i + (int64_t)l * m] * W[jmax + (int64_t)l * k];
      uc[i] = v;
    }
    __syncthreads();
    TS pu = TS(0), pw = TS(0);
    for (int i = threadIdx.x; i < m; i += NT) pu += uc[i] * uc[i];
    for (int j = threadIdx.x; j < k; j += NT) pw += wr[j] * wr[j];
    const TS nu2 = block_sum<TS>(pu, shv);
    const TS nw2 = block_sum<TS>(pw, shv);
    TS cross = TS(0);
    if (rank > 0) {
      wg_gemm_tn<TS, TS, TS>(m, rank, 1, U, m, uc, m, dots[0], red);
      wg_gemm_tn<TS, TS, TS>(k, rank, 1, W, k, wr, k, dots[1], red);
      for (int l = 0; l < rank; ++l) cross += dots[0][l] * dots[1][l];
    }
    frob2 += TS(2) * cross + nu2 * nw2;
    ++rank;
    // relative accuracy eps, tightened to the problem's absolute floor when that is smaller
    TS thr = eps * eps * frob2;
    if (mp.abs_tol > 0.0) thr = fmin(thr, TS(mp.abs_tol * mp.abs_tol));
    if (nu2 * nw2 <= thr) { conv = true; break; }
    if (nused >= m) { conv = true; break; }
    TS bu = TS(-1);
    int bu_i = -1;
    for (int i = threadIdx.x; i < m; i += NT) {
      if (used[i] != TS(0)) continue;
      const TS a = fabs(uc[i]);
      if (bu_i < 0 || a > bu) { bu = a; bu_i = i; }
    }
    TS dummy;
    block_argmax<TS>(bu, bu_i, shv, shi, dummy, istar);
    if (istar < 0) { conv = true; break; }
  }
  if (threadIdx.x == 0) {
    c.arank[bi] = rank;
    if (!conv) atomicAdd(&c.status[2], 1);
  }
}

// ------------------------------------------------------------ tile GEMM -----
// One workgroup accumulates a 128 x 128 tile on the matrix cores: wave w owns
// the 64 x 64 quadrant at rows 64 (w & 1), columns 64 (w >> 1), as 4 x 4
// blocks of 16 x 16 held in the MFMA output layout (lane l, element v: column
// l & 15 of the block, row 4 (l >> 4) + v for float, (l >> 4) + 4 v for
// double, as measured on gfx950). tile_mma adds A B^T where A
// (tile rows x K) and B (tile columns x K) are read through Op views, element
// (r, k) at p[r * rs + k * ks] for rows v0 <= r < v1 (zero outside), staged
// through LDS in chunks of KC along K with loads ordered along the
// unit-stride index; each 16 x 16 x 4 step is one v_mfma_f64_16x16x4f64 (or
// v_mfma_f32_16x16x4f32 for float), lane l supplying A(row l & 15, k l >> 4)
// and B(column l & 15, k l >> 4).
constexpr int KC = 16;
constexpr int LDT = TILE + 2;

typedef double hmle_d4 __attribute__((ext_vector_type(4)));
typedef float hmle_f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaVec;
template <>
struct MfmaVec<double> {
  typedef hmle_d4 type;
  static __device__ __forceinline__ type mma(double a, double b, type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row within the 16 x 16 block of output element v of lane l
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct MfmaVec<float> {
  typedef hmle_f4 type;
  static __device__ __forceinline__ type mma(float a, float b, type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

template <typename T>
struct Tile {
  typename MfmaVec<T>::type v[4][4];
};

template <typename T>
struct Op {
  const T* p;
  int64_t rs, ks;
  int v0, v1;
};

template <typename T>
__device__ __forceinline__ Op<T> op(const T* p, int64_t rs, int64_t ks, int v0, int v1) {
  Op<T> o;
  o.p = p; o.rs = rs; o.ks = ks; o.v0 = v0; o.v1 = v1;
  return o;
}

template <typename T>
__device__ __forceinline__ void tile_zero(Tile<T>& a) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) a.v[r][c][v] = T(0);
}

// stage_rows with every load of the thread issued before its first LDS store
// (one load-store pair at a time waits out each load). Costs a register per
// staged element and thread; used by the kernels that run few workgroups per
// compute unit, where registers do not limit occupancy.
template <int KCX, int ROWS, typename T, typename TO>
__device__ __forceinline__ void stage_rows_batched(T* s, int lds, const Op<TO>& o, int k0, int K) {
  constexpr int PER = (ROWS * KCX + NT - 1) / NT;
  T v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * NT;
    int r, kk;
    if (o.ks == 1) { kk = e % KCX; r = e / KCX; }
    else { r = e % ROWS; kk = e / ROWS; }
    const int k = k0 + kk;
    v[u] = (e < ROWS * KCX && r >= o.v0 && r < o.v1 && k < K)
               ? T(o.p[r * o.rs + (o.ks == 1 ? (int64_t)k : (int64_t)k * o.ks)]) : T(0);
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < ROWS * KCX) {
      if (o.ks == 1) s[(e % KCX) * lds + e / KCX] = v[u];
      else s[(e / ROWS) * lds + e % ROWS] = v[u];
    }
  }
}

template <int KCX, typename T, typename TO>
__device__ __forceinline__ void tile_stage(T* s, const Op<TO>& o, int k0, int K) {
  if (o.ks == 1) {
    for (int e = threadIdx.x; e < TILE * KCX; e += NT) {
      const int kk = e % KCX, r = e / KCX;
      const int k = k0 + kk;
      s[kk * LDT + r] = (r >= o.v0 && r < o.v1 && k < K) ? T(o.p[r * o.rs + k]) : T(0);
    }
  } else {
    for (int e = threadIdx.x; e < TILE * KCX; e += NT) {
      const int r = e % TILE, kk = e / TILE;
      const int k = k0 + kk;
      s[kk * LDT + r] = (r >= o.v0 && r < o.v1 && k < K) ? T(o.p[r * o.rs + (int64_t)k * o.ks]) : T(0);
    }
  }
}

template <int KCX = KC, bool BATCH = false, typename T, typename TA, typename TB>
__device__ void tile_mma(Tile<T>& acc, int K, const Op<TA>& A, const Op<TB>& B, T* sA, T* sB) {
  static_assert(KCX % 4 == 0, "the K chunk must be a multiple of the matrix-core K");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rq = 64 * (w & 1) + (lane & 15), cq = 64 * (w >> 1) + (lane & 15), kl = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += KCX) {
    __syncthreads();
    if (BATCH) {
      stage_rows_batched<KCX, TILE>(sA, LDT, A, k0, K);
      stage_rows_batched<KCX, TILE>(sB, LDT, B, k0, K);
    } else {
      tile_stage<KCX>(sA, A, k0, K);
      tile_stage<KCX>(sB, B, k0, K);
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < KCX; kq += 4) {
      T a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = sA[(kq + kl) * LDT + rq + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = sB[(kq + kl) * LDT + cq + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc.v[r][c] = MfmaVec<T>::mma(a[r], b[c], acc.v[r][c]);
    }
  }
  __syncthreads();
}

// d(i, j) at d[i * rs + j * cs] for i < M, j < N; mode 0: set, 1: add, 2: subtract.
template <typename T, typename TD>
__device__ __forceinline__ void tile_store(const Tile<T>& acc, int M, int N, TD* d, int64_t rs, int64_t cs,
                                           int mode) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = 64 * (w & 1), j0 = 64 * (w >> 1) + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + 16 * c;
      if (j >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 16 * r + MfmaVec<T>::row(lane, v);
        if (i >= M) continue;
        TD* q = d + i * rs + j * cs;
        if (mode == 0) *q = TD(acc.v[r][c][v]);
        else if (mode == 1) *q += TD(acc.v[r][c][v]);
        else *q -= TD(acc.v[r][c][v]);
      }
    }
}

// out(p, q) (+)= sum_k A(p, k) B(q, k) for p < P <= 64, q < Q <= 64 and any K
// (operand rows outside [v0, v1) read as zero),
// into LDS (ld 64). Threads own 4 x 4 output blocks; the 256 threads form
// 256 / (ceil(P/4) ceil(Q/4)) groups that split each staged K chunk; the group
// partials are summed in group order. ws: 4096 elements of LDS.
// BATCH: the staging issues every load of a thread (at most 16 per operand:
// kc * (SP + SQ) <= 4096) before its LDS stores; for kernels whose occupancy
// does not hinge on registers.
template <typename T, bool BATCH = false, typename TA, typename TB>
__device__ void wg_gemm_small(int P, int Q, int K, const Op<TA>& A, const Op<TB>& B, T* out, bool add, T* ws) {
  const int nP = (P + 3) >> 2, nQ = (Q + 3) >> 2;
  const int Tg = nP * nQ;
  if (Tg == 0) return;
  const int G = NT / Tg;
  const int SP = 4 * nP, SQ = 4 * nQ;
  const int KCH = 4096 / (SP + SQ);
  T* As = ws;
  T* Bs = ws + KCH * SP;
  const int g = threadIdx.x / Tg, lt = threadIdx.x % Tg;
  const int pi = lt % nP, qi = lt / nP;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
  for (int k0 = 0; k0 < K; k0 += KCH) {
    const int kc = min(KCH, K - k0);
    __syncthreads();
    if (BATCH) {
      T va[16], vb[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = threadIdx.x + u * NT;
        int kk, p;
        if (A.ks == 1) { kk = e % kc; p = e / kc; }
        else { p = e % SP; kk = e / SP; }
        va[u] = (e < kc * SP && p < P && p >= A.v0 && p < A.v1)
                    ? T(A.p[p * A.rs + (A.ks == 1 ? (int64_t)(k0 + kk) : (int64_t)(k0 + kk) * A.ks)]) : T(0);
        int kq, q;
        if (B.ks == 1) { kq = e % kc; q = e / kc; }
        else { q = e % SQ; kq = e / SQ; }
        vb[u] = (e < kc * SQ && q < Q && q >= B.v0 && q < B.v1)
                    ? T(B.p[q * B.rs + (B.ks == 1 ? (int64_t)(k0 + kq) : (int64_t)(k0 + kq) * B.ks)]) : T(0);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = threadIdx.x + u * NT;
        if (e < kc * SP) As[A.ks == 1 ? (e % kc) * SP + e / kc : e] = va[u];
        if (e < kc * SQ) Bs[B.ks == 1 ? (e % kc) * SQ + e / kc : e] = vb[u];
      }
    } else {
      if (A.ks == 1) {
        for (int e = threadIdx.x; e < kc * SP; e += NT) {
          const int kk = e % kc, p = e / kc;
          As[kk * SP + p] = (p < P && p >= A.v0 && p < A.v1) ? T(A.p[p * A.rs + (k0 + kk)]) : T(0);
        }
      } else {
        for (int e = threadIdx.x; e < kc * SP; e += NT) {
          const int p = e % SP, kk = e / SP;
          As[kk * SP + p] = (p < P && p >= A.v0 && p < A.v1) ? T(A.p[p * A.rs + (int64_t)(k0 + kk) * A.ks]) : T(0);
        }
      }
      if (B.ks == 1) {
        for (int e = threadIdx.x; e < kc * SQ; e += NT) {
          const int kk = e % kc, q = e / kc;
          Bs[kk * SQ + q] = (q < Q && q >= B.v0 && q < B.v1) ? T(B.p[q * B.rs + (k0 + kk)]) : T(0);
        }
      } else {
        for (int e = threadIdx.x; e < kc * SQ; e += NT) {
          const int q = e % SQ, kk = e / SQ;
          Bs[kk * SQ + q] = (q < Q && q >= B.v0 && q < B.v1) ? T(B.p[q * B.rs + (int64_t)(k0 + kk) * B.ks]) : T(0);
        }
      }
    }
    __syncthreads();
    if (g < G) {
      for (int kk = g; kk < kc; kk += G) {
        T a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As[kk * SP + 4 * pi + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Bs[kk * SQ + 4 * qi + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
      }
    }
  }
  __syncthreads();
  if (g < G) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) ws[(g * Tg + lt) * 16 + i * 4 + j] = acc[i][j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < P * Q; e += NT) {
    const int p = e % P, q = e / P;
    const int l = (p >> 2) + (q >> 2) * nP, sub = (p & 3) * 4 + (q & 3);
    T s = T(0);
    for (int gg = 0; gg < G; ++gg) s += ws[(gg * Tg + l) * 16 + sub];
    if (add) out[p + q * 64] += s;
    else out[p + q * 64] = s;
  }
  __syncthreads();
}

// Views of an off-diagonal block x restricted to rows from row0 and columns
// from col0 (global indices): dense L_x(i, a) = W[a + i * ldw]; low-rank
// L_x = U W^T with U(i, l) = U[i + l * ldu], W(a, l) = W[a + l * ldw].
template <typename TS>
struct Piece {
  bool lr;
  int rank;
  const TS* U;
  int64_t ldu;
  const TS* W;
  int64_t ldw;
};

template <typename TS>
__device__ __forceinline__ Piece<TS> make_piece(const DevCtx<TS>& c, const BlockDesc& x, int xi, int row0, int col0) {
  Piece<TS> q;
  const int64_t mx = x.r1 - x.r0, kx = x.c1 - x.c0;
  q.lr = x.kind == BK_LOWRANK;
  if (q.lr) {
    q.rank = c.rank[xi];
    q.U = c.L + x.loff + (row0 - x.r0);
    q.ldu = mx;
    q.W = c.L + x.loff + mx * c.R + (col0 - x.c0);
    q.ldw = kx;
  } else {
    q.rank = 0;
    q.U = nullptr;
    q.ldu = 0;
    q.W = c.L + x.loff + (col0 - x.c0) + (int64_t)(row0 - x.r0) * kx;
    q.ldw = kx;
  }
  return q;
}

// LDS scratch shared by the pair kernels.
constexpr int KCP = 12;   // K chunk of the pair kernels: a multiple of the matrix-core K (4); two chunks fit in 4096

template <typename TS>
struct PairLds {
  TS ws[4096];          // staging of tile_mma (sA | sB) and workspace of wg_gemm_small
  TS sM[64 * TILE];     // intermediates: up to 64 x 128 or 128 x 64
};


// acc(i, j) += sum_a L_x(i, a) L_y(j, a) over a in [0, nw) for tile rows
// [rv0, rv1) and columns [cv0, cv1); px, py are views whose row 0 is tile row
// 0 / tile column 0.
template <typename TS>
__device__ void pair_product_tile(Tile<TS>& acc, const Piece<TS>& px, const Piece<TS>& py, int rv0, int rv1, int cv0,
                                  int cv1, int nw, const TS* G, int gld, PairLds<TS>& L) {
  TS* sA = L.ws;
  TS* sB = L.ws + KCP * LDT;
  if (!px.lr && !py.lr) {
    tile_mma<KCP, true>(acc, nw, op(px.W, px.ldw, 1, rv0, rv1), op(py.W, py.ldw, 1, cv0, cv1), sA, sB);
  } else if (px.lr && !py.lr) {
    // M(l, j) = sum_a W_x(a, l) L_y(j, a) (two 64-column halves); acc += U_x M
    for (int h = 0; h < 2; ++h)
      wg_gemm_small<TS>(px.rank, 64, nw, op(px.W, px.ldw, 1, 0, px.rank),
                        op(py.W + (int64_t)(64 * h) * py.ldw, py.ldw, 1, cv0 - 64 * h, cv1 - 64 * h),
                        L.sM + 64 * 64 * h, false, L.ws);
    tile_mma<KCP, true>(acc, px.rank, op(px.U, 1, px.ldu, rv0, rv1), op<TS>(L.sM, 64, 1, 0, TILE), sA, sB);
  } else if (!px.lr && py.lr) {
    // M(i, q) = sum_a L_x(i, a) W_y(a, q) (two 64-row halves, stored as M^T); acc += M U_y^T
    for (int h = 0; h < 2; ++h)
      wg_gemm_small<TS>(py.rank, 64, nw, op(py.W, py.ldw, 1, 0, py.rank),
                        op(px.W + (int64_t)(64 * h) * px.ldw, px.ldw, 1, rv0 - 64 * h, rv1 - 64 * h),
                        L.sM + 64 * 64 * h, false, L.ws);
    tile_mma<KCP, true>(acc, py.rank, op<TS>(L.sM, 64, 1, 0, TILE), op(py.U, 1, py.ldu, cv0, cv1), sA, sB);
  } else {
    // M = G U_y^T with the cached Gram matrix G = W_x^T W_y, acc += U_x M
    for (int h = 0; h < 2; ++h)
      wg_gemm_small<TS>(px.rank, 64, py.rank, op<TS>(G, 1, gld, 0, px.rank),
                        op(py.U + 64 * h, 1, py.ldu, cv0 - 64 * h, cv1 - 64 * h), L.sM + 64 * 64 * h, false, L.ws);
    tile_mma<KCP, true>(acc, px.rank, op(px.U, 1, px.ldu, rv0, rv1), op<TS>(L.sM, 64, 1, 0, TILE), sA, sB);
  }
}

// Cached Gram matrices of low-rank pairs, one per workgroup: G = W_x[w]^T W_y[w]
// (rank_x x rank_y, ld R), computed once both blocks are final.
template <typename TS>
__global__ void __launch_bounds__(NT) k_gram(DevCtx<TS> c, const PairDesc* items) {
  __shared__ TS ws[4096];
  __shared__ TS sG[64 * 64];
  const PairDesc g = items[blockIdx.x];
  const BlockDesc x = c.blocks[g.x], y = c.blocks[g.y];
  const Piece<TS> px = make_piece(c, x, g.x, x.r0, g.w0);
  const Piece<TS> py = make_piece(c, y, g.y, y.r0, g.w0);
  wg_gemm_small<TS, true>(px.rank, py.rank, g.w1 - g.w0, op(px.W, px.ldw, 1, 0, px.rank), op(py.W, py.ldw, 1, 0, py.rank),
                    sG, false, ws);
  TS* G = c.gram + (int64_t)g.rx0 * c.R * c.R;
  for (int e = threadIdx.x; e < px.rank * py.rank; e += NT) {
    const int l = e % px.rank, q = e / px.rank;
    G[l + q * c.R] = sG[l + q * 64];
  }
}

// Dense targets, one workgroup per chunk of pairs: the chunk's sum of
// L_x[rx, w] L_y[ry, w]^T goes to its partial buffer in the target's own
// layout (diagonal: i + j*m; off-diagonal, transposed: j + i*k).
template <typename TS>
__global__ void __launch_bounds__(NT) k_dpairs(DevCtx<TS> c, const ChunkDesc* chunks, TS* part) {
  __shared__ PairLds<TS> L;
  const ChunkDesc ch = chunks[blockIdx.x];
  const BlockDesc b = c.blocks[ch.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const bool diag = b.kind == BK_DIAG;
  TS* P = part + ch.poff;
  for (int tr = 0; tr < m; tr += TILE) {
    for (int tc = 0; tc < k; tc += TILE) {
      Tile<TS> acc;
      tile_zero(acc);
      const int T_r0 = b.r0 + tr, T_c0 = b.c0 + tc;
      for (int q = ch.pair_lo; q < ch.pair_hi; ++q) {
        const PairDesc pr = c.pairs[q];
        const int rv0 = max(pr.rx0 - T_r0, 0), rv1 = min(pr.rx1 - T_r0, TILE);
        const int cv0 = max(pr.ry0 - T_c0, 0), cv1 = min(pr.ry1 - T_c0, TILE);
        if (rv0 >= rv1 || cv0 >= cv1) continue;
        const Piece<TS> px = make_piece(c, c.blocks[pr.x], pr.x, T_r0, pr.w0);
        const Piece<TS> py = make_piece(c, c.blocks[pr.y], pr.y, T_c0, pr.w0);
        const TS* G = pr.gram >= 0 ? c.gram + (int64_t)pr.gram * c.R * c.R : nullptr;
        pair_product_tile(acc, px, py, rv0, rv1, cv0, cv1, pr.w1 - pr.w0, G, c.R, L);
      }
      const int M = min(TILE, m - tr), N = min(TILE, k - tc);
      if (diag) tile_store(acc, M, N, P + tr + (int64_t)tc * m, 1, m, 0);
      else tile_store(acc, M, N, P + tc + (int64_t)tr * k, k, 1, 0);
    }
  }
}

// Dense targets: subtract the partial sums in chunk order.
template <typename TS>
__global__ void __launch_bounds__(NT) k_dreduce(DevCtx<TS> c, const TargetDesc* targets, const ChunkDesc* chunks,
                                                const TS* part) {
  const TargetDesc td = targets[blockIdx.x];
  if (td.chunk_lo == td.chunk_hi) return;
  const BlockDesc b = c.blocks[td.b];
  const int64_t mk = (int64_t)(b.r1 - b.r0) * (b.c1 - b.c0);
  for (int64_t e = (int64_t)blockIdx.y * NT + threadIdx.x; e < mk; e += (int64_t)gridDim.y * NT) {
    TS s = TS(0);
    // sequential sum in chunk order; unrolled so that several loads are in flight
#pragma unroll 8
    for (int q = td.chunk_lo; q < td.chunk_hi; ++q) s += part[chunks[q].poff + e];
    if (b.kind == BK_DIAG) c.D[b.loff + e] -= double(s);
    else c.L[b.loff + e] -= s;
  }
}



// Input-side products of a sketch pass: G = U_blk[r0:r1]^T X[r0:r1] (rank x
// ncol) into slot `slot` of gbuf (64 x 64 each, ld 64). Pass 1: X = the
// target's test matrix (rows of its columns); pass 2: its range basis Q.
template <typename TS>
__global__ void __launch_bounds__(NT) k_rG(DevCtx<TS> c, const GItem* items, int pass, TS* gbuf, TS* gseg) {
  __shared__ TS ws[4096];   // the product's staging only: it writes its rank x ncol result straight to the slot
  const GItem it = items[blockIdx.x];
  const BlockDesc b = c.blocks[it.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int ncol = pass == 1 ? min(c.R, min(m, k)) : c.rank[it.b];
  TS* G = it.part < 0 ? gbuf + (int64_t)it.slot * 4096 : gseg + (int64_t)it.part * 4096;
  if (it.blk < 0) {
    // rows [r0, r1) of the base factor and of the test matrix / range basis
    const int ka = c.arank[it.b];
    const TS* U0 = c.A + b.aoff;
    const TS* W0 = U0 + (int64_t)m * c.Ra;
    const int nr = it.r1 - it.r0;
    if (pass == 1)
      wg_gemm_small<TS, true>(ka, ncol, nr, op(W0 + it.r0, (int64_t)k, 1, 0, ka),
                        op(c.S + b.soff + (int64_t)(m + k) * c.R + it.r0, (int64_t)k, 1, 0, ncol), G, false, ws);
    else
      wg_gemm_small<TS, true>(ka, ncol, nr, op(U0 + it.r0, (int64_t)m, 1, 0, ka),
                        op(c.S + b.soff + it.r0, (int64_t)m, 1, 0, ncol), G, false, ws);
    return;
  }
  const BlockDesc p = c.blocks[it.blk];
  const TS* X = pass == 1 ? c.S + b.soff + (int64_t)(m + k) * c.R + (it.r0 - b.c0) : c.S + b.soff + (it.r0 - b.r0);
  const int64_t ldx = pass == 1 ? k : m;
  const int rk = c.rank[it.blk];
  const TS* U = c.L + p.loff + (it.r0 - p.r0);
  wg_gemm_small<TS, true>(rk, ncol, it.r1 - it.r0, op(U, (int64_t)(p.r1 - p.r0), 1, 0, rk), op(X, ldx, 1, 0, ncol), G,
                    false, ws);
}

// Segmented input-side products: slot = sum of the partials [lo, hi) in
// segment order over the valid extent (rank x ncol, ld 64). blockIdx.y picks
// 8 of the 64 columns.
template <typename TS>
__global__ void __launch_bounds__(NT) k_rG_fin(DevCtx<TS> c, const GFin* fins, int pass, TS* gbuf, const TS* gseg) {
  const GFin f = fins[blockIdx.x];
  const BlockDesc b = c.blocks[f.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int ncol = pass == 1 ? min(c.R, min(m, k)) : c.rank[f.b];
  const int rows = f.blk < 0 ? c.arank[f.b] : c.rank[f.blk];
  const int l = threadIdx.x & 63, cc = 8 * blockIdx.y + (threadIdx.x >> 6);
  TS* G = gbuf + (int64_t)f.slot * 4096;
  for (int c2 = cc; c2 < 8 * blockIdx.y + 8; c2 += NT / 64) {
    if (l >= rows || c2 >= ncol) continue;
    const int e = l + 64 * c2;
    TS s = TS(0);
#pragma unroll 8
    for (int q = f.lo; q < f.hi; ++q) s += gseg[(int64_t)q * 4096 + e];
    G[e] = s;
  }
}



// ---------------------------------------------------------------------------
// Rank-revealing QR of the low-rank targets' sketches through Gram matrices,
// split over 128-row tiles so that a large target spreads over many
// workgroups:
//   per tile    G_t = X[tile]^T X[tile] (float64 partial Gram matrices);
//   per target  G = sum of its tiles' G_t in tile order, pivoted Cholesky
//               G(Pi, Pi) = T^T T stopped when the trace of the remaining
//               Schur complement is <= tol^2 trace(G) (that trace is the
//               squared Frobenius norm of what the kept columns miss, as in
//               column-pivoted QR); X = Q Rm with Rm = T Pi^T (rows in pivot
//               order, columns in X's order) and Q = X Ri, Ri = Pi T^{-1};
//   per tile    Q[tile] = X[tile] Ri and its partial Gram matrix;
//   per target  second pass Q^T Q = R2^T R2 (unpivoted; restores the
//               orthogonality lost to squaring the condition number),
//               Ri2 = R2^{-1}, Rm <- R2 Rm;
//   per tile    Q[tile] <- Q[tile] Ri2.
// Per-target results live in qbuf (Ri and Rm, 64 x 64 float64 each) and qint
// (kq after the first pass, the column count, kq after the second pass).
constexpr int QB_DBL = 2 * 64 * 64;
constexpr int QB_INT = 4;

template <typename T, int NC>
struct TileN {
  T v[8][NC];
};

template <int KCX, int ROWS, typename T, typename TO>
__device__ __forceinline__ void stage_rows(T* s, int lds, const Op<TO>& o, int k0, int K) {
  if (o.ks == 1) {
    for (int e = threadIdx.x; e < ROWS * KCX; e += NT) {
      const int kk = e % KCX, r = e / KCX;
      const int k = k0 + kk;
      s[kk * lds + r] = (r >= o.v0 && r < o.v1 && k < K) ? T(o.p[r * o.rs + k]) : T(0);
    }
  } else {
    for (int e = threadIdx.x; e < ROWS * KCX; e += NT) {
      const int r = e % ROWS, kk = e / ROWS;
      const int k = k0 + kk;
      s[kk * lds + r] = (r >= o.v0 && r < o.v1 && k < K) ? T(o.p[r * o.rs + (int64_t)k * o.ks]) : T(0);
    }
  }
}

// acc(r, c) += sum_k A(r, k) B(c, k) for the 128 tile rows and 16 NC columns;
// thread t owns rows (t & 15) + 16 i and columns (t >> 4) + 16 j. K is staged
// KCX at a time (sA: KCX x LDT, sB: KCX x (16 NC + 2)); with inner dimensions
// of a leaf width or a rank the loop is bound by the latency of each chunk's
// loads, so the kernels on the step's critical path stage wide chunks.
template <int KCX = KC, bool BATCH = false, int NC, typename T, typename TA, typename TB>
__device__ void tile_mma_n(TileN<T, NC>& acc, int K, const Op<TA>& A, const Op<TB>& B, T* sA, T* sB) {
  constexpr int LB = 16 * NC + 2;
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
  for (int k0 = 0; k0 < K; k0 += KCX) {
    __syncthreads();
    if (BATCH) {
      stage_rows_batched<KCX, TILE>(sA, LDT, A, k0, K);
      stage_rows_batched<KCX, 16 * NC>(sB, LB, B, k0, K);
    } else {
      stage_rows<KCX, TILE>(sA, LDT, A, k0, K);
      stage_rows<KCX, 16 * NC>(sB, LB, B, k0, K);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KCX; ++kk) {
      T a[8], b[NC];
#pragma unroll
      for (int r = 0; r < 8; ++r) a[r] = sA[kk * LDT + ti + 16 * r];
#pragma unroll
      for (int c2 = 0; c2 < NC; ++c2) b[c2] = sB[kk * LB + tj + 16 * c2];
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2) acc.v[r][c2] += a[r] * b[c2];
    }
  }
  __syncthreads();
}

template <typename T, int NC>
__device__ __forceinline__ void tilen_zero(TileN<T, NC>& a) {
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2) a.v[r][c2] = T(0);
}

// Narrow tile on the matrix cores: acc(r, c) += sum_k A(r, k) B(c, k) for the
// 128 tile rows and 16 NC columns, operands staged as in tile_mma_n. Wave w
// owns rows 32 w .. 32 w + 31 as 2 x NC blocks of 16 x 16; each block is
// computed transposed (B as the matrix cores' first operand), so that lane l,
// element v of block (rb, cb) holds row 32 w + 16 rb + (l & 15) and column
// 16 cb + MfmaVec<T>::row(l, v): sixteen consecutive rows per column, as the
// plain narrow tile. Per four K steps a lane reads 2 + NC LDS values for 2 NC
// 16 x 16 x 4 products, against 4 (8 + NC) for the plain tile's 32 NC
// multiply-adds, whose K loop is bound by LDS bandwidth.
template <typename T, int NC = 2>
struct TileM {
  typename MfmaVec<T>::type v[2][NC];
};

template <typename T, int NC>
__device__ __forceinline__ void tilem_zero(TileM<T, NC>& a) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) a.v[rb][cb][v] = T(0);
}

// row and column of element v of block (rb, cb) of this lane
__device__ __forceinline__ int tilem_row(int rb) { return 32 * (threadIdx.x >> 6) + 16 * rb + (threadIdx.x & 15); }
template <typename T>
__device__ __forceinline__ int tilem_col(int cb, int v) { return 16 * cb + MfmaVec<T>::row(threadIdx.x & 63, v); }

template <int KCX, bool BATCH = true, typename T, int NC, typename TA, typename TB>
__device__ void tile_mma_m(TileM<T, NC>& acc, int K, const Op<TA>& A, const Op<TB>& B, T* sA, T* sB) {
  static_assert(KCX % 4 == 0, "the K chunk must be a multiple of the matrix-core K");
  constexpr int LB = 16 * NC + 2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rl = 32 * w + (lane & 15), cl = lane & 15, kl = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += KCX) {
    __syncthreads();
    if (BATCH) {
      stage_rows_batched<KCX, TILE>(sA, LDT, A, k0, K);
      stage_rows_batched<KCX, 16 * NC>(sB, LB, B, k0, K);
    } else {
      stage_rows<KCX, TILE>(sA, LDT, A, k0, K);
      stage_rows<KCX, 16 * NC>(sB, LB, B, k0, K);
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < KCX; kq += 4) {
      T a[2], b[NC];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) a[rb] = sA[(kq + kl) * LDT + rl + 16 * rb];
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) b[cb] = sB[(kq + kl) * LB + cl + 16 * cb];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) acc.v[rb][cb] = MfmaVec<T>::mma(b[cb], a[rb], acc.v[rb][cb]);
    }
  }
  __syncthreads();
}

// gp (ld R) = float64 Gram matrix of the nr x ncol tile in sY (ld 129, rows
// nr .. 127 zero, ncol <= 64) on the float64 matrix cores: the 16 x 16 blocks
// on and above the diagonal are dealt to the waves (block w + 4 j), each a sum
// over the rows in steps of 4; an entry above the diagonal is written to both
// of its places and one below the diagonal of a diagonal block is not written,
// so that gp is exactly symmetric.
template <typename T>
__device__ __forceinline__ void sy_gram(int nr, int ncol, const T* sY, double* gp, int R) {
  const int nB = (ncol + 15) >> 4, nb = nB * (nB + 1) / 2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, kl = lane >> 4;
  const int nr4 = (nr + 3) & ~3;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    int bi = w + 4 * j;
    if (bi >= nb) break;
    // block bi in the order (0,0), (0,1), (1,1), (0,2), ... (row block pb <= column block qb)
    int qb = 0;
    while (bi > qb) { bi -= qb + 1; ++qb; }
    const int pb = bi;
    hmle_d4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = 0.0;
    const T* yp = sY + (TILE + 1) * (16 * pb + li);
    const T* yq = sY + (TILE + 1) * (16 * qb + li);
    for (int k = kl; k < nr4; k += 4) acc = MfmaVec<double>::mma(double(yq[k]), double(yp[k]), acc);
    const int p = 16 * pb + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 16 * qb + MfmaVec<double>::row(lane, v);
      if (p < ncol && q < ncol && p <= q) {
        gp[p + (int64_t)R * q] = acc[v];
        gp[q + (int64_t)R * p] = acc[v];
      }
    }
  }
  __syncthreads();
}

// Store the tile (nr x ncol) to d (ld rows) and, when gp is given, its
// float64 Gram matrix (ncol x ncol, ld R) through LDS (sY: 129 x 16 NC).
template <typename T, int NC>
__device__ void tilen_store_gram(const TileN<T, NC>& acc, int nr, int ncol, T* d, int64_t ld, T* sY, double* gp,
                                 int R) {
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int i = ti + 16 * r;
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2) {
      const int j = tj + 16 * c2;
      if (i < nr && j < ncol) d[i + (int64_t)j * ld] = acc.v[r][c2];
      if (gp) sY[i + (TILE + 1) * j] = (i < nr) ? acc.v[r][c2] : T(0);
    }
  }
  if (!gp) return;
  __syncthreads();
  sy_gram(nr, ncol, sY, gp, R);
}

// Store the matrix-core tile (nr x ncol) to d (ld rows) and, when gp is given,
// its float64 Gram matrix as tilen_store_gram does.
template <typename T, int NC>
__device__ void tilem_store_gram(const TileM<T, NC>& acc, int nr, int ncol, T* d, int64_t ld, T* sY, double* gp,
                                 int R) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tilem_row(rb), j = tilem_col<T>(cb, v);
        if (i < nr && j < ncol) d[i + (int64_t)j * ld] = acc.v[rb][cb][v];
        if (gp) sY[i + (TILE + 1) * j] = (i < nr) ? acc.v[rb][cb][v] : T(0);
      }
  if (!gp) return;
  __syncthreads();
  sy_gram(nr, ncol, sY, gp, R);
}

// K chunk of the per-tile products of the truncation (inner dimension <= 16 NC):
// one chunk at rank 32, two at rank 64 (where a wider chunk would not leave room
// for a second workgroup per compute unit)
template <int NC>
constexpr int sum_kc() { return NC <= 2 ? 32 : 16; }

template <typename TS, int NC>
struct SumLds {
  TS sA[sum_kc<NC>() * LDT];
  TS sB[sum_kc<NC>() * (16 * NC + 2)];
  TS sY[(TILE + 1) * 16 * NC];
};


// Sketch pass of the low-rank targets: one chunk (pairs sharing their output
// block q) per workgroup. Pass 1 multiplies S_b by the test matrix X = Omega
// (output side x, input side y of each pair), pass 2 S_b^T by the range basis
// X = Q (output y, input x). Per pair, with p the input block and w the shared
// columns:
//   low-rank q, low-rank p:  H += (W_q^T W_p from the cache) G_p, G_p = U_p^T X;
//   low-rank q, dense p:     H += W_q[w]^T V,  V = L_p[rows, w]^T X[rows];
//   dense q:                 rows_q += L_q[rows, w] M,  M = W_p[w] G_p or V;
// H (rank_q x c) accumulates in LDS, the rows of a dense q in a register tile
// of the chunk; the chunk writes its compact negated output -H or -rows.
constexpr int RP_KC = 32;   // K chunk of the sketch-pass tile products

template <typename TS, int NC>
struct RpassLds {
  static constexpr int WC = 64;   // columns w per slice
  static constexpr int NST = RP_KC * LDT + RP_KC * (16 * NC + 2), NW = WC * 16 * NC;
  // sA | sB of the tile products, or W_q[w] (w rows x rank_q, ld WC) / the cached Gram
  // matrix (ld 64): never live at the same time (a product ends with a barrier before
  // W_q is staged, and the next product starts with one after it is read), so they
  // share the space: the LDS of three workgroups fits a compute unit at rank 32 (the
  // registers hold two)
  TS stage[NST > NW ? NST : NW];
  TS sM[WC * 16 * NC];      // V or M (w rows x c, ld WC), or staged G_p (ld 64)
  TS sH[64 * 16 * NC];      // H (rank_q x c, ld 64)
};

// Two waves per SIMD: at rank 32 the registers are held to 256 (a 12-byte spill)
// so that two workgroups share a compute unit; the rank-64 instance needs more
// than 256 with any tile and runs one wave per SIMD (the compiler says it cannot
// meet the target there).
template <typename TS, int NC>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) k_rpass(DevCtx<TS> c, const ChunkDesc* chunks, const RPairDesc* rp, int pass,
                                              const TS* gbuf, TS* part) {
  __shared__ RpassLds<TS, NC> L;
  constexpr int WC = RpassLds<TS, NC>::WC;
  TS* const sA = L.stage;
  TS* const sB = L.stage + RP_KC * LDT;
  TS* const sW = L.stage;
  const ChunkDesc ch = chunks[blockIdx.x];
  const BlockDesc b = c.blocks[ch.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int ncol = pass == 1 ? min(c.R, min(m, k)) : c.rank[ch.b];
  TS* P = part + ch.poff;
  if (ncol == 0) return;
  const TS* X = pass == 1 ? c.S + b.soff + (int64_t)(m + k) * c.R : c.S + b.soff;
  const int64_t ldx = pass == 1 ? k : m;
  const int xbase = pass == 1 ? b.c0 : b.r0;
  const RPairDesc r0p = rp[ch.pair_lo];
  const int qb = pass == 1 ? r0p.x : r0p.y;
  const BlockDesc qd = c.blocks[qb];
  const int rq0 = pass == 1 ? r0p.rx0 : r0p.ry0, rq1 = pass == 1 ? r0p.rx1 : r0p.ry1;
  const bool qlr = qd.kind == BK_LOWRANK;
  const int nq = rq1 - rq0;
  const int rkq = qlr ? c.rank[qb] : 0;
  for (int e = threadIdx.x; e < 64 * 16 * NC; e += NT) L.sH[e] = TS(0);
  // row tiles of a dense output block (one unless it has more than 128 rows)
  for (int r0 = 0; r0 < (qlr ? 1 : nq); r0 += TILE) {
    TileM<TS, NC> acc;
    tilem_zero(acc);
    for (int q = ch.pair_lo; q < ch.pair_hi; ++q) {
      const RPairDesc pr = rp[q];
      const int pb = pass == 1 ? pr.y : pr.x;
      const int rp0 = pass == 1 ? pr.ry0 : pr.rx0, rp1 = pass == 1 ? pr.ry1 : pr.rx1;
      const BlockDesc pd = c.blocks[pb];
      const Piece<TS> pp = make_piece(c, pd, pb, rp0, pr.w0);
      const Piece<TS> pq = make_piece(c, qd, qb, rq0, pr.w0);
      const int nw = pr.w1 - pr.w0, np = rp1 - rp0;
      const TS* Gp = pr.gslot >= 0 ? gbuf + (int64_t)pr.gslot * 4096 : nullptr;
      const TS* Xp = X + (rp0 - xbase);
      if (qlr && pp.lr) {
        // H += Gram_qp G_p: Gram x_y is cached as rank_x x rank_y (ld R)
        const TS* Gxy = c.gram + (int64_t)pr.gram * c.R * c.R;
        const int rpk = pp.rank;
        __syncthreads();
        for (int e = threadIdx.x; e < rkq * rpk; e += NT) {
          const int l = e % rkq, kk = e / rkq;
          sW[l + 64 * kk] = pass == 1 ? Gxy[l + (int64_t)c.R * kk] : Gxy[kk + (int64_t)c.R * l];
        }
        for (int e = threadIdx.x; e < rpk * ncol; e += NT) {
          const int kk = e % rpk, cc = e / rpk;
          L.sM[kk + 64 * cc] = Gp[kk + 64 * cc];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < rkq * ncol; e += NT) {
          const int l = e % rkq, cc = e / rkq;
          TS s = TS(0);
          for (int kk = 0; kk < rpk; ++kk) s += sW[l + 64 * kk] * L.sM[kk + 64 * cc];
          L.sH[l + 64 * cc] += s;
        }
        continue;
      }
      for (int a0 = 0; a0 < nw; a0 += WC) {
        const int na = min(WC, nw - a0);
        // V = L_p[rows, w]^T X (dense p) or M = W_p[w] G_p (low-rank p): na x ncol into sM
        TileM<TS, NC> t;
        tilem_zero(t);
        if (pp.lr)
          tile_mma_m<RP_KC, false>(t, pp.rank, op(pp.W + a0, 1, pp.ldw, 0, na), op(Gp, 64, 1, 0, ncol), sA, sB);
        else
          tile_mma_m<RP_KC, false>(t, np, op(pp.W + a0, 1, pp.ldw, 0, na), op(Xp, ldx, 1, 0, ncol), sA, sB);
        tilem_store_gram<TS, NC>(t, na, ncol, L.sM, WC, nullptr, nullptr, 0);
        __syncthreads();
        if (qlr) {
          // H += W_q[w]^T V
          for (int e = threadIdx.x; e < na * rkq; e += NT) {
            const int a = e % na, l = e / na;
            sW[a + WC * l] = pq.W[a0 + a + (int64_t)l * pq.ldw];
          }
          __syncthreads();
          for (int e = threadIdx.x; e < rkq * ncol; e += NT) {
            const int l = e % rkq, cc = e / rkq;
            TS s = TS(0);
            for (int a = 0; a < na; ++a) s += sW[a + WC * l] * L.sM[a + WC * cc];
            L.sH[l + 64 * cc] += s;
          }
          __syncthreads();
        } else {
          // rows_q += L_q[rows, w] M (this row tile)
          tile_mma_m<RP_KC, false>(acc, na, op(pq.W + a0 + (int64_t)r0 * pq.ldw, pq.ldw, 1, 0, min(TILE, nq - r0)),
                                op<TS>(L.sM, WC, 1, 0, ncol), sA, sB);
        }
      }
    }
    if (!qlr) {
      // negated touched rows (nq x ncol, ld nq)
      const int nr = min(TILE, nq - r0);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < NC; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = tilem_row(rb), j = tilem_col<TS>(cb, v);
            if (i < nr && j < ncol) P[r0 + i + (int64_t)j * nq] = -acc.v[rb][cb][v];
          }
    }
  }
  if (qlr) {
    __syncthreads();
    for (int e = threadIdx.x; e < rkq * ncol; e += NT) {
      const int l = e % rkq, cc = e / rkq;
      P[l + cc * c.R] = -L.sH[l + cc * 64];
    }
  }
}

// Accumulator of the sketch sums: the matrix-core narrow tile, except for
// float64 at rank 64, which takes the vector tile and so keeps two waves per
// SIMD (the matrix-core accumulators take it past 256 registers).
template <typename TS, int NC>
using RsumAcc = typename std::conditional<NC == 2 || sizeof(TS) == 4, TileM<TS, NC>, TileN<TS, NC>>::type;

// K steps [0, KCX) of a staged chunk (sA: KCX x LDT, sB: KCX x (16 NC + 2)) into the tile
template <int KCX, typename T, int NC>
__device__ __forceinline__ void tile_kloop(TileM<T, NC>& t, const T* sA, const T* sB) {
  constexpr int LB = 16 * NC + 2;
  const int lane = threadIdx.x & 63;
  const int rl = 32 * (threadIdx.x >> 6) + (lane & 15), cl = lane & 15, kl = lane >> 4;
#pragma unroll
  for (int kq = 0; kq < KCX; kq += 4) {
    T a[2], b[NC];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) a[rb] = sA[(kq + kl) * LDT + rl + 16 * rb];
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) b[cb] = sB[(kq + kl) * LB + cl + 16 * cb];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) t.v[rb][cb] = MfmaVec<T>::mma(b[cb], a[rb], t.v[rb][cb]);
  }
}
template <int KCX, typename T, int NC>
__device__ __forceinline__ void tile_kloop(TileN<T, NC>& t, const T* sA, const T* sB) {
  constexpr int LB = 16 * NC + 2;
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
#pragma unroll 4
  for (int kk = 0; kk < KCX; ++kk) {
    T a[8], b[NC];
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = sA[kk * LDT + ti + 16 * r];
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2) b[c2] = sB[kk * LB + tj + 16 * c2];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int c2 = 0; c2 < NC; ++c2) t.v[r][c2] += a[r] * b[c2];
  }
}

// f(row, column, element) over the 8 NC elements of this thread's share of the tile, in a fixed order
template <typename T, int NC, typename F>
__device__ __forceinline__ void tile_elems(TileM<T, NC>& t, F f) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T x = t.v[rb][cb][v];   // a vector element binds no reference: through a copy
        f(tilem_row(rb), tilem_col<T>(cb, v), x);
        t.v[rb][cb][v] = x;
      }
}
template <typename T, int NC, typename F>
__device__ __forceinline__ void tile_elems(TileN<T, NC>& t, F f) {
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2) f(ti + 16 * r, tj + 16 * c2, t.v[r][c2]);
}

// Low-rank targets: 128-row tile tl of the sketch sum after pass `pass`
//   pass 1: Y[tile] = U0[tile] (W0^T Omega) + sum over chunks q of U_q[tile rows] (-H_q) (+ dense rows)
//   pass 2: B^T[tile] = W0[tile] (U0^T Q) + ... (the same with the roles of rows and columns exchanged)
// where -H_q are the chunks' compact outputs; writes the tile and its Gram
// partial gp[tile] (ncol x ncol, ld R). The tile's chunk entries are read into
// LDS at once; consecutive entries of one low-rank output block form a group
// (their -H summed in entry order), and the base term and all groups make one
// product over the concatenated inner dimension (the groups' ranks), staged
// 32 columns at a time whatever group each column belongs to.
constexpr int RS_MAXE = 256;   // tile entries per round
constexpr int RS_MAXG = 64;    // groups per round

template <typename TS, int NC, int RS_KC>
struct RsumLds {
  TS sA[RS_KC * LDT];
  TS sB[RS_KC * (16 * NC + 2)];
  TileChunk ents[RS_MAXE];
  const TS* gU[RS_MAXG];
  int64_t gld[RS_MAXG];
  int gqb[RS_MAXG], gv0[RS_MAXG], gv1[RS_MAXG], ge0[RS_MAXG], ge1[RS_MAXG], gk[RS_MAXG + 1];
  int colg[RS_KC], coll[RS_KC];
  int ngroups, consumed;
};

// RS_KC: inner-dimension columns per staged chunk (the sum_kc tile shape; 16 keeps the
// LDS small enough for more workgroups per compute unit, 32 halves the chunk count)
template <typename TS, int NC, int RS_KC>
__global__ void __launch_bounds__(NT) k_rsum(DevCtx<TS> c, const RTargetDesc* targets, const RowTile* tiles,
                                             const TileSeg* segs, const TileChunk* tents, const TS* part,
                                             const TS* gbuf, int pass, TS* spart) {
  __shared__ RsumLds<TS, NC, RS_KC> L;
  constexpr int LB = 16 * NC + 2;
  const TileSeg sg = segs[blockIdx.x];
  const RowTile tl = tiles[sg.tile];
  const RTargetDesc td = targets[tl.t];
  const BlockDesc b = c.blocks[td.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int ncol = pass == 1 ? min(c.R, min(m, k)) : c.rank[td.b];
  if (ncol == 0) return;
  const int rows = pass == 1 ? m : k;
  const int nr = min(TILE, rows - tl.r0);
  const int obase = pass == 1 ? b.r0 : b.c0;
  const int t0 = obase + tl.r0, t1 = t0 + nr;       // global rows of the tile
  const int ka = c.arank[td.b];
  const TS* U0 = c.A + b.aoff;
  const TS* base = pass == 1 ? U0 : U0 + (int64_t)m * c.Ra;    // U0 rows (pass 1) or W0 rows (pass 2)
  const TS* G = gbuf + (int64_t)(pass == 1 ? td.gb1 : td.gb2) * 4096;
  TS* out = pass == 1 ? c.S + b.soff : c.S + b.soff + (int64_t)m * c.R;
  RsumAcc<TS, NC> t;
  tile_elems(t, [](int, int, TS& x) { x = TS(0); });
  int e0 = sg.eb;
  bool first = sg.first != 0;
  do {
    const int ne = min(RS_MAXE, sg.ee - e0);
    for (int i = threadIdx.x; i < ne; i += NT) L.ents[i] = tents[e0 + i];
    __syncthreads();
    // groups: the base term (first round), then runs of entries of one low-rank output block
    if (threadIdx.x == 0) {
      int g = 0;
      if (first) {
        L.gqb[0] = -1;
        L.ge0[0] = L.ge1[0] = 0;
        g = 1;
      }
      int i = 0;
      for (; i < ne; ++i) {
        if (!L.ents[i].lr) continue;
        if (g > (first ? 1 : 0) && L.gqb[g - 1] == L.ents[i].qb && L.ge1[g - 1] == i) {
          L.ge1[g - 1] = i + 1;
          continue;
        }
        if (g == RS_MAXG) break;
        L.gqb[g] = L.ents[i].qb;
        L.ge0[g] = i;
        L.ge1[g] = i + 1;
        ++g;
      }
      L.ngroups = g;
      L.consumed = i;
    }
    __syncthreads();
    const int ng = L.ngroups, consumed = L.consumed;
    for (int g = threadIdx.x; g < ng; g += NT) {
      const int qb = L.gqb[g];
      if (qb < 0) {
        L.gU[g] = base + tl.r0;
        L.gld[g] = rows;
        L.gv0[g] = 0;
        L.gv1[g] = nr;
        L.gk[g + 1] = ka;
      } else {
        const BlockDesc qd = c.blocks[qb];
        const TileChunk en = L.ents[L.ge0[g]];
        L.gU[g] = c.L + qd.loff + (t0 - qd.r0);      // row 0 of the tile
        L.gld[g] = qd.r1 - qd.r0;
        L.gv0[g] = max(en.rq0, t0) - t0;
        L.gv1[g] = min(en.rq1, t1) - t0;
        L.gk[g + 1] = c.rank[qb];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      L.gk[0] = 0;
      for (int g = 0; g < ng; ++g) L.gk[g + 1] += L.gk[g];
    }
    __syncthreads();
    const int K = L.gk[ng];
    for (int k0 = 0; k0 < K; k0 += RS_KC) {
      if (threadIdx.x < RS_KC) {
        const int kv = k0 + threadIdx.x;
        int g = -1;
        if (kv < K) {
          g = 0;
          while (L.gk[g + 1] <= kv) ++g;
        }
        L.colg[threadIdx.x] = g;
        L.coll[threadIdx.x] = g >= 0 ? kv - L.gk[g] : 0;
      }
      __syncthreads();
      {
        // every load of the thread first, then the LDS stores (few workgroups run per compute
        // unit here, so the registers this takes cost no occupancy)
        constexpr int PER = TILE * RS_KC / NT;
        static_assert(TILE * RS_KC % NT == 0, "whole staging rounds");
        TS va[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int e = threadIdx.x + u * NT;
          const int r = e % TILE, kk = e / TILE;
          const int g = L.colg[kk];
          va[u] = (g >= 0 && r >= L.gv0[g] && r < L.gv1[g]) ? L.gU[g][r + (int64_t)L.coll[kk] * L.gld[g]] : TS(0);
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int e = threadIdx.x + u * NT;
          L.sA[(e / TILE) * LDT + e % TILE] = va[u];
        }
      }
      for (int e = threadIdx.x; e < 16 * NC * RS_KC; e += NT) {
        const int kk = e % RS_KC, cc = e / RS_KC;
        const int g = L.colg[kk], l = L.coll[kk];
        TS v = TS(0);
        if (g >= 0 && cc < ncol) {
          if (L.gqb[g] < 0) v = G[l + 64 * cc];
          else
            for (int i = L.ge0[g]; i < L.ge1[g]; ++i) v += part[L.ents[i].poff + l + (int64_t)c.R * cc];
        }
        L.sB[kk * LB + cc] = v;
      }
      __syncthreads();
      tile_kloop<RS_KC>(t, L.sA, L.sB);
      __syncthreads();
    }
    // dense output blocks: negated touched rows (nq x ncol, ld nq) added in registers
    for (int i = 0; i < consumed; ++i) {
      const TileChunk en = L.ents[i];
      if (en.lr) continue;
      const int nq = en.rq1 - en.rq0;
      const TS* P = part + en.poff;
      // the entry's values for this thread's tile elements, all loads first
      TS pv[8 * NC];
      int u = 0;
      tile_elems(t, [&](int i, int j, TS&) {
        const int gi = t0 + i;
        pv[u++] = (gi >= en.rq0 && gi < en.rq1 && gi < t1 && j < ncol) ? P[(gi - en.rq0) + (int64_t)j * nq] : TS(0);
      });
      u = 0;
      tile_elems(t, [&](int, int, TS& x) { x += pv[u++]; });
    }
    __syncthreads();
    e0 += consumed;
    first = false;
  } while (e0 < sg.ee);
  // partial tile of this segment (128 x 16 NC, ld 128)
  TS* sp = spart + (int64_t)blockIdx.x * TILE * 64;
  tile_elems(t, [&](int i, int j, TS& x) { sp[i + TILE * j] = x; });
}

// Finish of the sketch sums: a tile is the sum of its segments' partial
// tiles (segment order); writes the tile and its Gram partial.
template <typename TS, int NC>
__global__ void __launch_bounds__(NT) k_rsum_fin(DevCtx<TS> c, const RTargetDesc* targets, const RowTile* tiles,
                                                 const TS* spart, int pass, double* gpart) {
  __shared__ TS sY[(TILE + 1) * 16 * NC];
  const RowTile tl = tiles[blockIdx.x];
  const RTargetDesc td = targets[tl.t];
  const BlockDesc b = c.blocks[td.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int ncol = pass == 1 ? min(c.R, min(m, k)) : c.rank[td.b];
  if (ncol == 0) return;
  const int rows = pass == 1 ? m : k;
  const int nr = min(TILE, rows - tl.r0);
  TS* out = pass == 1 ? c.S + b.soff : c.S + b.soff + (int64_t)m * c.R;
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
  TileN<TS, NC> t;
  tilen_zero(t);
  // several segments' loads in flight before their sums (which keep segment order)
  constexpr int SG = NC <= 2 ? 4 : 2;
  int sgi = tl.sb;
  for (; sgi + SG <= tl.se; sgi += SG) {
    TS pv[SG][8][NC];
#pragma unroll
    for (int s = 0; s < SG; ++s) {
      const TS* sp = spart + (int64_t)(sgi + s) * TILE * 64;
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2) pv[s][r][c2] = sp[ti + 16 * r + TILE * (tj + 16 * c2)];
    }
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2) t.v[r][c2] += pv[s][r][c2];
  }
  for (; sgi < tl.se; ++sgi) {
    const TS* sp = spart + (int64_t)sgi * TILE * 64;
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int c2 = 0; c2 < NC; ++c2) t.v[r][c2] += sp[ti + 16 * r + TILE * (tj + 16 * c2)];
  }
  tilen_store_gram(t, nr, ncol, out + tl.r0, rows, sY, gpart + (int64_t)blockIdx.x * c.R * c.R, c.R);
}


// Lane l's value of x, read by the whole wave (l the same in every lane).
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long bits = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)bits, l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One step of a wave reduction through the data-parallel-primitive lane moves:
// the value and lane index of the source lane given by CTRL (rows of 16 lanes;
// lanes without a source, or in rows outside ROWMASK, see their own pair), kept
// when larger, or equal with a lower index.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ void argmax_step(double& v, int& idx) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  const int oi = __builtin_amdgcn_update_dpp(idx, idx, CTRL, ROWMASK, 0xf, false);
  const double ov = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
}

// Largest value over the wave, ties to the lowest lane; returns the lane (and
// the value in best), the same in every lane. Prefix form: row shifts by 1, 2,
// 4 and 8 leave each row's result in its lane 15, the row broadcasts 15 and 31
// carry it across rows into lane 63, which is read back by every lane. The
// combination (larger value, else lower index) is associative and
// commutative, so the order of combination does not change the result.
__device__ __forceinline__ int wave_argmax(double v, double& best) {
  int idx = threadIdx.x & 63;
  argmax_step<0x111, 0xf>(v, idx);   // row_shr:1
  argmax_step<0x112, 0xf>(v, idx);   // row_shr:2
  argmax_step<0x114, 0xf>(v, idx);   // row_shr:4
  argmax_step<0x118, 0xf>(v, idx);   // row_shr:8
  argmax_step<0x142, 0xa>(v, idx);   // row_bcast:15 into rows 1 and 3
  argmax_step<0x143, 0xc>(v, idx);   // row_bcast:31 into rows 2 and 3
  best = readlane_f64(v, 63);
  return __builtin_amdgcn_readlane(idx, 63);
}

struct QrLds {
  double G[64 * 65];
  double T[64 * 65];
  double colp[64];
  int perm[64];
};

// Orders the LDS accesses of one wave around a point where lanes start to
// read what other lanes wrote.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum of the tile partials [tlo, thi) of an n x n Gram matrix into G (LDS, ld 65):
// per element four running sums over the tiles t = tlo + 4i + r, added as
// (s0 + s1) + (s2 + s3). A thread takes four of its elements at once, so that
// sixteen loads are in flight (a large target has hundreds of tiles).
__device__ __forceinline__ void gram_reduce(const double* gpart, int tlo, int thi, int n, int R, double* G) {
  const int64_t RR = (int64_t)R * R;
  const int nn = n * n;
  constexpr int EG = 4;
  for (int e0 = threadIdx.x; e0 < nn; e0 += EG * NT) {
    const double* g[EG];
    bool act[EG];
    int gi[EG];
    double s[EG][4];
#pragma unroll
    for (int j = 0; j < EG; ++j) {
      const int e = e0 + j * NT;
      act[j] = e < nn;
      const int p = act[j] ? e % n : 0, q = act[j] ? e / n : 0;   // element (0, 0) stands in: in bounds
      g[j] = gpart + p + (int64_t)R * q;
      gi[j] = p + 65 * q;
#pragma unroll
      for (int r = 0; r < 4; ++r) s[j][r] = 0.0;
    }
    int t = tlo;
    for (; t + 4 <= thi; t += 4) {
      double v[EG][4];
#pragma unroll
      for (int j = 0; j < EG; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[j][r] = act[j] ? g[j][(t + r) * RR] : 0.0;
#pragma unroll
      for (int j = 0; j < EG; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) s[j][r] += v[j][r];
    }
#pragma unroll
    for (int j = 0; j < EG; ++j) {
      if (!act[j]) continue;
      if (t < thi) s[j][0] += g[j][t * RR];
      if (t + 1 < thi) s[j][1] += g[j][(t + 1) * RR];
      if (t + 2 < thi) s[j][2] += g[j][(t + 2) * RR];
      G[gi[j]] = (s[j][0] + s[j][1]) + (s[j][2] + s[j][3]);
    }
  }
  __syncthreads();
}

// Pivoted Cholesky of the n x n Gram matrix in G (ld 65) by one wave: lane j
// keeps column j in registers; step kk picks the largest remaining diagonal
// (ties to the lowest index), stops when the remaining trace is <= tol^2
// trace(G) or the pivot is not positive, and writes row kk of the factor (in
// the original column order) to T. Returns the number of steps; perm in LDS.
// Inlined into its kernels, so that G, T, perm and colp are known to be LDS
// (a call would pass them as generic pointers).
template <int NR>
__device__ __forceinline__ int wave_pivoted_cholesky(const double* G, int n, double tol, double abs2, double* T,
                                                     int* perm, double* colp, bool pivot) {
  const int lane = threadIdx.x & 63;
  const bool mine = lane < n;
  double g[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) g[i] = (mine && i < n) ? G[i + 65 * lane] : 0.0;
  double diag = mine ? G[lane * 66] : 0.0;
  const double trace = wave_sum_f64(diag);
  // trace of the remaining Schur complement: each step removes the squared
  // norm of the new factor row, which every lane reads anyway
  double rem = trace;
  // stop at the relative accuracy tol, or at the absolute floor abs2 (> 0) when that is smaller
  const double thr = abs2 > 0.0 ? fmin(tol * tol * trace, abs2) : tol * tol * trace;
  bool used = false;
  int kq = 0;
  for (int kk = 0; kk < n; ++kk) {
    int p = kk;
    double best;
    if (pivot) {
      p = wave_argmax((mine && !used) ? diag : -1.0, best);
      if (!(rem > thr)) break;
    } else {
      best = readlane_f64(diag, kk);
    }
    if (!(best > 0.0)) break;
    const double r = sqrt(best);
    // the pivot lane publishes its column: G(p, lane) = G(lane, p) (symmetry)
    if (lane == p) {
#pragma unroll
      for (int i = 0; i < NR; ++i) colp[i] = g[i];
    }
    wave_sync();
    double rk = 0.0;
    if (mine && !used && (pivot || lane >= kk)) rk = (lane == p) ? r : colp[lane] / r;
    T[kk + 65 * lane] = rk;
    if (lane == p) used = true;
    if (lane == 0) perm[kk] = p;
    wave_sync();
    double row2 = 0.0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const double ti = T[kk + 65 * i];
      g[i] -= ti * rk;
      row2 += ti * ti;
    }
    rem -= row2;
    diag -= rk * rk;
    kq = kk + 1;
    wave_sync();
  }
  return kq;
}

// Column `lane` of the inverse of the kq x kq upper-triangular matrix U held
// in LDS (U(i, l) at U[i + 65 l]) into x (LDS, the lane's own column x[i + 65
// lane]), by back substitution; the inner sums run in four interleaved
// partial sums (fixed order) so that their loads overlap.
__device__ __forceinline__ void wave_triu_inverse(const double* U, int kq, double* x) {
  const int lane = threadIdx.x & 63;
  if (lane >= kq) return;
  double* xc = x + 65 * lane;
  for (int i = lane; i >= 0; --i) {
    double s0 = (i == lane) ? 1.0 : 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int l = i + 1;
    for (; l + 3 <= lane; l += 4) {
      s0 -= U[i + 65 * l] * xc[l];
      s1 -= U[i + 65 * (l + 1)] * xc[l + 1];
      s2 -= U[i + 65 * (l + 2)] * xc[l + 2];
      s3 -= U[i + 65 * (l + 3)] * xc[l + 3];
    }
    for (; l <= lane; ++l) s0 -= U[i + 65 * l] * xc[l];
    xc[i] = ((s0 + s1) + (s2 + s3)) / U[i + 65 * i];
  }
}

// First pass of the per-target QR (see above), wave 0 after the reduction.
template <typename TS, int NR>
__global__ void __launch_bounds__(NT) k_qchol(DevCtx<TS> c, const RTargetDesc* targets, int pass, double tol,
                                              const double* gpart, double* qbuf, int* qint) {
  __shared__ QrLds L;
  const RTargetDesc td = targets[blockIdx.x];
  const BlockDesc b = c.blocks[td.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int ncol = pass == 1 ? min(c.R, min(m, k)) : c.rank[td.b];
  int* qi = qint + (int64_t)blockIdx.x * QB_INT;
  double* Ri = qbuf + (int64_t)blockIdx.x * QB_DBL;
  double* Rm = Ri + 64 * 64;
  if (ncol == 0) {
    if (threadIdx.x == 0) { qi[0] = 0; qi[1] = 0; qi[2] = 0; }
    return;
  }
  gram_reduce(gpart, pass == 1 ? td.t1lo : td.t2lo, pass == 1 ? td.t1hi : td.t2hi, ncol, c.R, L.G);
  if (threadIdx.x >= 64) return;   // one wave from here on: no workgroup barriers below
  const int lane = threadIdx.x;
  const bool mine = lane < ncol;
  // absolute floor of the problem: pass 2 truncates B^T, whose trailing trace is the squared
  // truncation error; pass 1 ranks the sketch Y = S Omega (+-1 entries, ncol columns), whose
  // residual is about ncol times that of S, to 1/100 of the floor like the relative tolerance
  const double at = c.mp[b.prob].abs_tol;
  const double abs2 = pass == 1 ? 1e-4 * at * at * ncol : at * at;
  const int kq = wave_pivoted_cholesky<NR>(L.G, ncol, tol, abs2, L.T, L.perm, L.colp, true);
  // Rm = rows 0..kq of T Pi^T (ld 64); Ri = Pi T^{-1}: column `lane` of T^{-1}
  // by back substitution, scattered to the rows perm[0..kq)
  for (int l = 0; l < kq; ++l) Rm[l + 64 * lane] = mine ? L.T[l + 65 * lane] : 0.0;
  for (int i = 0; i < ncol; ++i) Ri[i + 64 * lane] = 0.0;
  wave_sync();
  // U = T Pi (pivot order, upper triangular) into G's space, then its inverse over T
  if (lane < kq) {
    const int pc = L.perm[lane];
    for (int i = 0; i < kq; ++i) L.G[i + 65 * lane] = L.T[i + 65 * pc];
  }
  wave_sync();
  wave_triu_inverse(L.G, kq, L.T);
  if (lane < kq)
    for (int i = 0; i <= lane; ++i) Ri[L.perm[i] + 64 * lane] = L.T[i + 65 * lane];
  if (lane == 0) { qi[0] = kq; qi[1] = ncol; qi[2] = kq; }
}

// Q[tile] = X[tile] Ri (ncol -> kq columns, in place) and its Gram partial.
template <typename TS, int NC>
__global__ void __launch_bounds__(NT) k_qapply(DevCtx<TS> c, const RTargetDesc* targets, const RowTile* tiles,
                                               int pass, const double* qbuf, const int* qint, double* gpart) {
  __shared__ SumLds<TS, NC> L;
  const RowTile tl = tiles[blockIdx.x];
  const RTargetDesc td = targets[tl.t];
  const BlockDesc b = c.blocks[td.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int* qi = qint + (int64_t)tl.t * QB_INT;
  const int kq = qi[0], ncol = qi[1];
  if (kq == 0) return;
  const int rows = pass == 1 ? m : k;
  const int nr = min(TILE, rows - tl.r0);
  TS* X = (pass == 1 ? c.S + b.soff : c.S + b.soff + (int64_t)m * c.R) + tl.r0;
  const double* Ri = qbuf + (int64_t)tl.t * QB_DBL;
  TileM<TS, NC> t;
  tilem_zero(t);
  tile_mma_m<sum_kc<NC>()>(t, ncol, op<TS>(X, 1, (int64_t)rows, 0, nr), op<double>(Ri, 64, 1, 0, kq), L.sA, L.sB);
  tilem_store_gram(t, nr, kq, X, rows, L.sY, gpart + (int64_t)blockIdx.x * c.R * c.R, c.R);
}

// Second pass: Q^T Q = R2^T R2 without pivoting (stops at a non-positive
// pivot: kq2 columns kept), Ri2 = R2^{-1} into Ri's slot, Rm <- R2 Rm; the
// kept width becomes the block's rank.
template <typename TS, int NR>
__global__ void __launch_bounds__(NT) k_qchol2(DevCtx<TS> c, const RTargetDesc* targets, int pass,
                                               const double* gpart, double* qbuf, int* qint) {
  __shared__ QrLds L;
  const RTargetDesc td = targets[blockIdx.x];
  int* qi = qint + (int64_t)blockIdx.x * QB_INT;
  const int kq = qi[0], ncol = qi[1];
  double* Ri = qbuf + (int64_t)blockIdx.x * QB_DBL;
  double* Rm = Ri + 64 * 64;
  if (kq == 0) {
    if (threadIdx.x == 0) {
      qi[2] = 0;
      c.rank[td.b] = 0;
      if (pass == 1) c.rank1[td.b] = 0;
    }
    return;
  }
  gram_reduce(gpart, pass == 1 ? td.t1lo : td.t2lo, pass == 1 ? td.t1hi : td.t2hi, kq, c.R, L.G);
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const int kq2 = wave_pivoted_cholesky<NR>(L.G, kq, 0.0, 0.0, L.T, L.perm, L.colp, false);
  wave_sync();
  // new Rm = R2 Rm (kq2 x ncol): lane owns column `lane`, staged in its G column
  if (pass == 2 && lane < ncol) {
    double* col = L.G + 65 * lane;
    for (int l = 0; l < kq; ++l) col[l] = Rm[l + 64 * lane];
    for (int kk = 0; kk < kq2; ++kk) {
      double s0 = 0.0, s1 = 0.0;
      int l = kk;
      for (; l + 1 < kq; l += 2) {
        s0 += L.T[kk + 65 * l] * col[l];
        s1 += L.T[kk + 65 * (l + 1)] * col[l + 1];
      }
      if (l < kq) s0 += L.T[kk + 65 * l] * col[l];
      Rm[kk + 64 * lane] = s0 + s1;
    }
    for (int kk = kq2; kk < 64; ++kk) Rm[kk + 64 * lane] = 0.0;
  }
  // Ri2 = R2^{-1} (kq x kq2, rows >= kq2 zero): the inverse columns over G
  for (int i = 0; i < kq; ++i) Ri[i + 64 * lane] = 0.0;
  wave_sync();
  wave_triu_inverse(L.T, kq2, L.G);
  if (lane < kq2)
    for (int i = 0; i <= lane; ++i) Ri[i + 64 * lane] = L.G[i + 65 * lane];
  if (lane == 0) {
    qi[2] = kq2;
    c.rank[td.b] = kq2;
    if (pass == 1) c.rank1[td.b] = kq2;
    if (pass == 2 && kq2 >= c.R) atomicAdd(&c.status[1], 1);
  }
}

// Pass 1 finish: Q[tile] <- Q[tile] Ri2 (kq -> kq2 columns, in place).
template <typename TS, int NC>
__global__ void __launch_bounds__(NT) k_qapply2(DevCtx<TS> c, const RTargetDesc* targets, const RowTile* tiles,
                                                const double* qbuf, const int* qint) {
  __shared__ SumLds<TS, NC> L;
  const RowTile tl = tiles[blockIdx.x];
  const RTargetDesc td = targets[tl.t];
  const BlockDesc b = c.blocks[td.b];
  const int m = b.r1 - b.r0;
  const int* qi = qint + (int64_t)tl.t * QB_INT;
  const int kq = qi[0], kq2 = qi[2];
  if (kq2 == 0) return;
  const int nr = min(TILE, m - tl.r0);
  TS* X = c.S + b.soff + tl.r0;
  const double* Ri = qbuf + (int64_t)tl.t * QB_DBL;
  TileM<TS, NC> t;
  tilem_zero(t);
  tile_mma_m<sum_kc<NC>()>(t, kq, op<TS>(X, 1, (int64_t)m, 0, nr), op<double>(Ri, 64, 1, 0, kq2), L.sA, L.sB);
  tilem_store_gram<TS, NC>(t, nr, kq2, X, m, L.sY, nullptr, c.R);
}

// Truncation finish (after the second pass on B^T): the first n2 workgroups
// write W[tile] = Q2[tile] Ri2 (k rows), the others U[tile] = Q1[tile] Rm^T
// (m rows, Rm = kr x kq1 with columns in Q1's order): L_b = U W^T.
template <typename TS, int NC>
__global__ void __launch_bounds__(NT) k_qfin(DevCtx<TS> c, const RTargetDesc* targets, const RowTile* tiles2, int n2,
                                             const RowTile* tiles1, const double* qbuf, const int* qint) {
  __shared__ SumLds<TS, NC> L;
  const bool wpart = (int)blockIdx.x < n2;
  const RowTile tl = wpart ? tiles2[blockIdx.x] : tiles1[blockIdx.x - n2];
  const RTargetDesc td = targets[tl.t];
  const BlockDesc b = c.blocks[td.b];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int* qi = qint + (int64_t)tl.t * QB_INT;
  const int kq = qi[0], kq1 = qi[1], kr = qi[2];
  if (kr == 0) return;
  const double* Ri = qbuf + (int64_t)tl.t * QB_DBL;
  const double* Rm = Ri + 64 * 64;
  TS* Ul = c.L + b.loff;
  TS* Wl = Ul + (int64_t)m * c.R;
  TileM<TS, NC> t;
  tilem_zero(t);
  if (wpart) {
    const int nr = min(TILE, k - tl.r0);
    const TS* Q2 = c.S + b.soff + (int64_t)m * c.R + tl.r0;
    tile_mma_m<sum_kc<NC>()>(t, kq, op<TS>(Q2, 1, (int64_t)k, 0, nr), op<double>(Ri, 64, 1, 0, kr), L.sA, L.sB);
    tilem_store_gram<TS, NC>(t, nr, kr, Wl + tl.r0, k, L.sY, nullptr, c.R);
  } else {
    const int nr = min(TILE, m - tl.r0);
    const TS* Q1 = c.S + b.soff + tl.r0;
    tile_mma_m<sum_kc<NC>()>(t, kq1, op<TS>(Q1, 1, (int64_t)m, 0, nr), op<double>(Rm, 1, 64, 0, kr), L.sA, L.sB);
    tilem_store_gram<TS, NC>(t, nr, kr, Ul + tl.r0, m, L.sY, nullptr, c.R);
  }
}


// Cholesky of diagonal leaf j and the inverse of its factor, in float64. The
// leaf (padded with the identity to M, the next multiple of 32) sits in LDS
// (column-major, ld PLD) and is factorised by 32-column blocks, right-looking:
//   one wave factorises the 32 x 32 diagonal block from registers (lane r
//     holds row r of the remaining symmetric matrix; each step's column goes
//     through LDS and is read back as broadcasts; no workgroup barrier) and,
//     in the same sweep, inverts its factor (lanes 32..63, a column each); the
//     factor goes to the diagonal pool and its inverse X_kk replaces it in LDS;
//   all waves form the panel L_ik = A_ik X_kk^T and the trailing update
//     A_ij -= L_ik L_jk^T (lower triangle) with 4 x 4 register blocks.
// The inverse X = L^{-1} is then built in place from the right, block
// column by block column: T = X[below, below] L[below, k] (kept in the free
// upper triangle), X[below, k] = -T X_kk.
constexpr int PLD = TILE + 1;

// The 32 x 32 diagonal block at (o, o), by one wave: lane r < 32 holds row r
// of the remaining symmetric block (its lower part is what counts), lane
// 32 + c column c of X_kk = L_kk^{-1}, starting from the identity. Step i: the
// pivot is lane i's entry (i, i); every lane turns its entry i into s --
// row lanes r > i: L(r, i) = A(r, i) / L(i, i), lane i: L(i, i), rows above: 0;
// inverse lanes: X(i, c) / L(i, i) -- the row lanes publish L(., i) in LDS,
// and every lane subtracts s L(q, i) from its entries q > i: the Schur update
// of its row (s = L(r, i)), or the forward substitution of its column of
// X_kk (s = X(i, c)). L(., i) is read back as broadcasts, one per entry.
__device__ __forceinline__ bool potrf_diag32(double* A, int o, int m, double* Dg, int* pst, double* pval,
                                             int leaf, double* colb) {
  const int lane = threadIdx.x & 63;
  const bool fac = lane < 32;
  const int rc = lane & 31;   // row (factor lanes) or column (inverse lanes)
  double v[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    // the lower triangle holds the remaining matrix; entry (rc, q) by symmetry
    const int rr = max(rc, q), cc = min(rc, q);
    v[q] = fac ? A[o + rr + PLD * (o + cc)] : (q == rc ? 1.0 : 0.0);
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const double piv = readlane_f64(v[i], i);
    if (!(piv > 0.0)) {
      if (lane == 0 && o + i < m && atomicCAS(pst, 0, leaf + 1) == 0) *pval = piv;
      return false;
    }
    // 1/sqrt(piv): hardware estimate and two Newton steps
    double rd = __builtin_amdgcn_rsq(piv);
    rd = rd * (1.5 - 0.5 * piv * rd * rd);
    rd = rd * (1.5 - 0.5 * piv * rd * rd);
    const double sc = v[i] * rd;
    const double sv = fac ? (rc > i ? sc : (rc == i ? piv * rd : 0.0)) : sc;
    v[i] = sv;
    if (fac) colb[rc] = sv;
    wave_sync();
    // all reads of the column first, then the updates: the reads are in flight together
    double cb[32];
#pragma unroll
    for (int q = i + 1; q < 32; ++q) cb[q] = colb[q];
#pragma unroll
    for (int q = i + 1; q < 32; ++q) v[q] -= sv * cb[q];
    wave_sync();
  }
  // the factor block (zeros above, row by row) to the pool, X_kk (column by
  // column) in its place in LDS
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    if (fac) {
      if (o + rc < m && o + q < m) Dg[(o + rc) + (int64_t)(o + q) * m] = q <= rc ? v[q] : 0.0;
    } else {
      A[o + q + PLD * (o + rc)] = v[q];
    }
  }
  return true;
}

// One workgroup per compute unit (its LDS holds the whole leaf), so one wave per
// SIMD: the register budget of a single wave is available.
template <typename TS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_potrf(DevCtx<TS> c, const int32_t* leaves) {
  __shared__ double A[TILE * PLD];
  __shared__ double colb[32];   // the broadcast column of the diagonal-block sweep
  __shared__ int fail;
  const int j = leaves[blockIdx.x];
  const int m = c.leaf_hi[j] - c.leaf_lo[j];
  const int M = (m + 31) & ~31;
  const BlockDesc b = c.blocks[c.leaf_diag[j]];
  int* const pst = c.pstatus + b.prob;
  double* const pval = c.pstatus_val + b.prob;
  double* Dg = c.D + b.loff;
  double* Xg = c.inv + c.leaf_inv_off[j];
  const int t = threadIdx.x;
  const int ti = t & (TILE - 1), tc = t >> 7;   // row, and column parity of the IO loops
#pragma unroll 8
  for (int jj = tc; jj < M; jj += 2)
    if (ti < M && ti >= jj) A[ti + PLD * jj] = (ti < m && jj < m) ? Dg[ti + (int64_t)jj * m] : (ti == jj ? 1.0 : 0.0);
  if (t == 0) fail = 0;
  __syncthreads();
  for (int o = 0; o < M; o += 32) {
    if (t < 64 && !potrf_diag32(A, o, m, Dg, pst, pval, j, colb) && t == 0) fail = 1;
    __syncthreads();
    if (fail) return;
    const int r0 = o + 32, nrb = (M - r0) >> 2;
    if (nrb == 0) break;
    // panel rows r0.. : L(i, o + c) = sum_k A(i, o + k) X_kk(c, k)
    {
      const int rb = t >> 3, cb = t & 7;
      double acc[4][4] = {};
      if (rb < nrb) {
#pragma unroll 4
        for (int k = 0; k < 32; ++k) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = A[r0 + 4 * rb + u + PLD * (o + k)];
#pragma unroll
          for (int v = 0; v < 4; ++v) bv[v] = A[o + 4 * cb + v + PLD * (o + k)];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
      }
      __syncthreads();
      if (rb < nrb) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) A[r0 + 4 * rb + u + PLD * (o + 4 * cb + v)] = acc[u][v];
      }
      __syncthreads();
    }
    // trailing update, lower triangle: A(i, j) -= sum_k L(i, o + k) L(j, o + k)
    const int nblk = nrb * (nrb + 1) / 2;
    for (int q = t; q < nblk; q += NT) {
      int bi = (int)((sqrtf(8.0f * q + 1.0f) - 1.0f) * 0.5f);
      while (bi * (bi + 1) / 2 > q) --bi;
      while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
      const int bj = q - bi * (bi + 1) / 2;
      double acc[4][4] = {};
#pragma unroll 4
      for (int k = 0; k < 32; ++k) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = A[r0 + 4 * bi + u + PLD * (o + k)];
#pragma unroll
        for (int v = 0; v < 4; ++v) bv[v] = A[r0 + 4 * bj + v + PLD * (o + k)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (bi > bj || u >= v) A[r0 + 4 * bi + u + PLD * (r0 + 4 * bj + v)] -= acc[u][v];
    }
    __syncthreads();
  }
  // off-diagonal blocks of the factor (the diagonal blocks went out with their wave)
#pragma unroll 8
  for (int jj = tc; jj < m; jj += 2)
    if (ti < m && (ti >> 5) != (jj >> 5)) Dg[ti + (int64_t)jj * m] = ti > jj ? A[ti + PLD * jj] : 0.0;
  // inverse, block columns from the right
  for (int o = M - 64; o >= 0; o -= 32) {
    const int r0 = o + 32, nrb = (M - r0) >> 2;
    const int rb = t >> 3, cb = t & 7;
    // T(r, c) = sum_{s <= r} X(r0 + r, r0 + s) L(r0 + s, o + c), stored at (c, r0 + r)
    {
      double acc[4][4] = {};
      if (rb < nrb) {
#pragma unroll 4
        for (int s = 0; s < 4 * rb + 4; ++s) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = A[r0 + 4 * rb + u + PLD * (r0 + s)];
#pragma unroll
          for (int v = 0; v < 4; ++v) bv[v] = A[r0 + s + PLD * (o + 4 * cb + v)];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) A[4 * cb + v + PLD * (r0 + 4 * rb + u)] = acc[u][v];
      }
      __syncthreads();
    }
    // X(r0 + r, o + c) = -sum_k T(r, k) X_kk(k, c)
    {
      double acc[4][4] = {};
      if (rb < nrb) {
#pragma unroll 4
        for (int k = 0; k < 32; ++k) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = A[k + PLD * (r0 + 4 * rb + u)];
#pragma unroll
          for (int v = 0; v < 4; ++v) bv[v] = A[o + k + PLD * (o + 4 * cb + v)];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) A[r0 + 4 * rb + u + PLD * (o + 4 * cb + v)] = -acc[u][v];
      }
      __syncthreads();
    }
  }
#pragma unroll 8
  for (int jj = tc; jj < m; jj += 2)
    if (ti < m) Xg[ti + (int64_t)jj * m] = ti >= jj ? A[ti + PLD * jj] : 0.0;
}

// Column solve at step s (leaf j = the problem's s-th leaf), 32 columns of W_b
// from c0: W_b[leaf rows] <- L_jj^{-1} W_b[leaf rows] (product with the
// inverted leaf on a narrow tile).
template <typename TS>
__global__ void __launch_bounds__(NT) k_trsm(DevCtx<TS> c, int s, const InnerDesc* items) {
  // the whole leaf width in two chunks (one workgroup per compute unit; a step has few of them)
  constexpr int KT = 64;
  __shared__ double sA[KT * LDT], sB[KT * 34];
  const InnerDesc it = items[blockIdx.x];
  const BlockDesc b = c.blocks[it.b];
  const int j = c.prob_leaf0[b.prob] + s;
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const int ncol = min(32, block_cols(c, b, it.b) - it.c0);
  if (ncol <= 0) return;
  const int64_t ldw = b.c1 - b.c0;
  TS* Ws = block_w(c, b) + (lo - b.c0) + (int64_t)it.c0 * ldw;
  const double* X = c.inv + c.leaf_inv_off[j];
  TileM<double> t;
  tilem_zero(t);
  tile_mma_m<KT>(t, nl, op(X, 1, (int64_t)nl, 0, nl), op<TS>(Ws, ldw, 1, 0, ncol), sA, sB);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tilem_row(rb), jj = tilem_col<double>(cb, v);
        if (i < nl && jj < ncol) Ws[i + (int64_t)jj * ldw] = TS(t.v[rb][cb][v]);
      }
}

// Inner update at step s (leaf j of the block's problem), rows [r0, r0 + 128)
// of x and 32 columns of W_b from c0: W_b[rows of x] -= L_x[:, leaf j] W_b[leaf rows].
template <typename TS>
__global__ void __launch_bounds__(NT) k_inner(DevCtx<TS> c, int s, const InnerDesc* items) {
  constexpr int KI = 32;   // four chunks over a leaf width, two workgroups per compute unit
  __shared__ TS sA[KI * LDT], sB[KI * 34];
  __shared__ TS sH[64 * 32];
  const InnerDesc it = items[blockIdx.x];
  const BlockDesc b = c.blocks[it.b], x = c.blocks[it.x];
  const int j = c.prob_leaf0[b.prob] + s;
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const int ncol = min(32, block_cols(c, b, it.b) - it.c0);
  if (ncol <= 0) return;
  const int64_t ldw = b.c1 - b.c0;
  TS* Wb = block_w(c, b) + (int64_t)it.c0 * ldw;
  const TS* T = Wb + (lo - b.c0);
  const int r0 = it.r0, nr = min(TILE, x.r1 - x.r0 - r0);
  TS* out = Wb + (x.r0 - b.c0) + r0;
  const Piece<TS> px = make_piece(c, x, it.x, x.r0, lo);
  TileM<TS> t;
  if (px.lr) {
    // H = W_x[leaf rows]^T T (rank x ncol, ld 64) into LDS
    tilem_zero(t);
    tile_mma_m<KI>(t, nl, op(px.W, px.ldw, 1, 0, px.rank), op(T, ldw, 1, 0, ncol), sA, sB);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = tilem_row(rb), jj = tilem_col<TS>(cb, v);
          if (i < px.rank && jj < ncol) sH[i + 64 * jj] = t.v[rb][cb][v];
        }
    __syncthreads();
  }
  tilem_zero(t);
  if (px.lr) tile_mma_m<KI>(t, px.rank, op(px.U + r0, 1, px.ldu, 0, nr), op<TS>(sH, 64, 1, 0, ncol), sA, sB);
  else tile_mma_m<KI>(t, nl, op(px.W + (int64_t)r0 * px.ldw, px.ldw, 1, 0, nr), op(T, ldw, 1, 0, ncol), sA, sB);
  // read-modify-write of the 16 elements: all loads first (a store between two loads would have
  // to wait for the load before it, the compiler cannot tell that the elements are distinct)
  TS ov[2][2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tilem_row(rb), jj = tilem_col<TS>(cb, v);
        ov[rb][cb][v] = (i < nr && jj < ncol) ? out[i + (int64_t)jj * ldw] : TS(0);
      }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tilem_row(rb), jj = tilem_col<TS>(cb, v);
        if (i < nr && jj < ncol) out[i + (int64_t)jj * ldw] = ov[rb][cb][v] - t.v[rb][cb][v];
      }
}

// One forward-substitution step s. The first n_leaves workgroups write
// vout[leaf j] = L_jj^{-1} v[leaf j] for the step's leaves; each of the others
// takes rows [r0, r1) of one block x in column j of its problem, forms the
// same L_jj^{-1} v[leaf j] and subtracts L_x[rows, leaf j] times it.
template <typename TS>
__global__ void __launch_bounds__(NT) k_solve_step(DevCtx<TS> c, int s, const int32_t* leaves, int n_leaves,
                                                    const InnerDesc* items, double* v, double* vout) {
  __shared__ double t[TILE], vj[TILE];
  __shared__ double h[64];
  const bool own = (int)blockIdx.x < n_leaves;
  const InnerDesc it = own ? InnerDesc{-1, -1, 0, 0} : items[blockIdx.x - n_leaves];
  const int bi = it.b;
  const int j = own ? leaves[blockIdx.x] : c.prob_leaf0[c.blocks[bi].prob] + s;
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const double* X = c.inv + c.leaf_inv_off[j];
  for (int a = threadIdx.x; a < nl; a += NT) t[a] = v[lo + a];
  __syncthreads();
  for (int i = threadIdx.x; i < nl; i += NT) {
    double acc = 0.0;
    for (int a = 0; a <= i; ++a) acc += X[i + a * nl] * t[a];
    vj[i] = acc;
  }
  __syncthreads();
  if (own) {
    for (int i = threadIdx.x; i < nl; i += NT) vout[lo + i] = vj[i];
    return;
  }
  const BlockDesc x = c.blocks[bi];
  const int64_t mx = x.r1 - x.r0, kx = x.c1 - x.c0;
  if (x.kind == BK_DENSE) {
    const TS* W = c.L + x.loff + (lo - x.c0);
    for (int i = it.r0 + threadIdx.x; i < it.c0; i += NT) {
      double s = 0.0;
      for (int a = 0; a < nl; ++a) s += double(W[a + i * kx]) * vj[a];
      v[x.r0 + i] -= s;
    }
  } else {
    const int rk = c.rank[bi];
    const TS* U = c.L + x.loff;
    const TS* W = U + mx * c.R + (lo - x.c0);
    for (int l = threadIdx.x; l < rk; l += NT) {
      double s = 0.0;
      for (int a = 0; a < nl; ++a) s += double(W[a + l * kx]) * vj[a];
      h[l] = s;
    }
    __syncthreads();
    for (int i = it.r0 + threadIdx.x; i < it.c0; i += NT) {
      double s = 0.0;
      for (int l = 0; l < rk; ++l) s += double(U[i + l * mx]) * h[l];
      v[x.r0 + i] -= s;
    }
  }
}

// Backward substitution L~^T w = v (the second half of a solve with C~), step
// s of a single problem, in two launches. Part: workgroup q takes rows
// [r0, r1) of one block x in column j (leaf j = step s) and writes
// part[q][a] = sum_i L_x[i, leaf column a] w[x.r0 + i]; the rows of x lie after
// leaf j, so their w is already final.
template <typename TS>
__global__ void __launch_bounds__(NT) k_bsolve_part(DevCtx<TS> c, int s, const InnerDesc* items, const double* w,
                                                     double* part) {
  __shared__ double red[NT];
  __shared__ double u[64];
  const InnerDesc it = items[blockIdx.x];
  const BlockDesc x = c.blocks[it.b];
  const int j = c.prob_leaf0[x.prob] + s;
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const int64_t mx = x.r1 - x.r0, kx = x.c1 - x.c0;
  double* p = part + (int64_t)blockIdx.x * TILE;
  const int t = threadIdx.x;
  if (x.kind == BK_DENSE) {
    // thread (a, g): column a, every other row from g; the two halves added in order
    const TS* W = c.L + x.loff + (lo - x.c0);
    const int a = t & (TILE - 1), g = t >> 7;
    double acc = 0.0;
    if (a < nl)
      for (int i = it.r0 + g; i < it.c0; i += 2) acc += double(W[a + (int64_t)i * kx]) * w[x.r0 + i];
    red[t] = acc;
    __syncthreads();
    if (t < nl) p[t] = red[t] + red[t + TILE];
  } else {
    // u = U_x[rows]^T w[rows] (fixed-order tree per column), then W_x[leaf] u
    const int rk = c.rank[it.b];
    const TS* U = c.L + x.loff;
    const TS* Wl = U + mx * c.R + (lo - x.c0);
    for (int l = 0; l < rk; ++l) {
      double acc = 0.0;
      for (int i = it.r0 + t; i < it.c0; i += NT) acc += double(U[i + (int64_t)l * mx]) * w[x.r0 + i];
      red[t] = acc;
      __syncthreads();
      for (int h = NT / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
      }
      if (t == 0) u[l] = red[0];
      __syncthreads();
    }
    for (int a = t; a < nl; a += NT) {
      double acc = 0.0;
      for (int l = 0; l < rk; ++l) acc += double(Wl[a + (int64_t)l * kx]) * u[l];
      p[a] = acc;
    }
  }
}

// Finish of step s: w[leaf j] = L_jj^{-T} (v[leaf j] - the parts in item order).
template <typename TS>
__global__ void __launch_bounds__(NT) k_bsolve_fin(DevCtx<TS> c, const int32_t* leaves, int n_items,
                                                    const double* part, const double* v, double* w) {
  __shared__ double tt[TILE];
  const int j = leaves[blockIdx.x];
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const double* X = c.inv + c.leaf_inv_off[j];
  for (int a = threadIdx.x; a < nl; a += NT) {
    double s = v[lo + a];
    for (int q = 0; q < n_items; ++q) s -= part[(int64_t)q * TILE + a];
    tt[a] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nl; i += NT) {
    double acc = 0.0;
    for (int a = i; a < nl; ++a) acc += X[a + (int64_t)i * nl] * tt[a];
    w[lo + i] = acc;
  }
}

// Kriging mean at m new points: z2[k] = sum_j M(|s2_k - s1_j|) w[j] over all n1
// training points (coordinates c1 dim-major in the internal order, w =
// C~^{-1} z1 in the same order), the Matern covariance without nugget.
// PRED_P points per workgroup; each thread sums a strided share of the
// training points, the shares are added by a fixed-order tree.
constexpr int PRED_P = 16;
__global__ void __launch_bounds__(NT) k_predict(const double* c1, const double* w, int n1, const double* p2, int64_t m,
                                                int dim, MaternParams mp, double* z2) {
  __shared__ double q[PRED_P * 3];
  __shared__ double red[NT];
  const int64_t k0 = (int64_t)blockIdx.x * PRED_P;
  const int np = (int)min<int64_t>(PRED_P, m - k0);
  const int t = threadIdx.x;
  for (int e = t; e < np * dim; e += NT) q[e] = p2[k0 * dim + e];
  __syncthreads();
  for (int k = 0; k < np; ++k) {
    const double qx = q[k * dim], qy = q[k * dim + 1], qz = dim == 3 ? q[k * dim + 2] : 0.0;
    double acc = 0.0;
    for (int jj = t; jj < n1; jj += NT) {
      const double dx = qx - c1[jj], dy = qy - c1[(int64_t)n1 + jj];
      const double dz = dim == 3 ? qz - c1[2 * (int64_t)n1 + jj] : 0.0;
      acc += matern_value<double>(sqrt(dx * dx + dy * dy + dz * dz), mp) * w[jj];
    }
    red[t] = acc;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
      if (t < h) red[t] += red[t + h];
      __syncthreads();
    }
    if (t == 0) z2[k0 + k] = red[0];
    __syncthreads();
  }
}

// Kriging variance at new points, 32 at a time: the columns B[:, k] =
// P c(s_k) (Matern covariance of the new point s_k with every training point,
// internal order, no nugget), the forward substitution of all 32 columns
// together, and var_k = sigma^2 - |L~^{-1} P c(s_k)|^2.
constexpr int VAR_K = 32;

__global__ void __launch_bounds__(NT) k_cross_cols(const double* c1, int n1, const double* p2, int kk, int dim,
                                                   MaternParams mp, double* B) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)n1 * VAR_K) return;
  const int jj = (int)(e % n1), k = (int)(e / n1);
  double v = 0.0;
  if (k < kk) {
    const double dx = p2[k * dim] - c1[jj], dy = p2[k * dim + 1] - c1[(int64_t)n1 + jj];
    const double dz = dim == 3 ? p2[k * dim + 2] - c1[2 * (int64_t)n1 + jj] : 0.0;
    v = matern_value<double>(sqrt(dx * dx + dy * dy + dz * dz), mp);
  }
  B[e] = v;
}

// One forward-substitution step for VAR_K right-hand sides (V and Vout: n x
// VAR_K column-major, ld n); the work split is that of k_solve_step, with each
// item's rows further split over gridDim.y workgroups (blockIdx.y).
template <typename TS>
__global__ void __launch_bounds__(NT) k_solve_step_multi(DevCtx<TS> c, int s, const int32_t* leaves, int n_leaves,
                                                          const InnerDesc* items, double* V, double* Vout) {
  constexpr int LD = VAR_K + 1;
  __shared__ double tv[TILE * LD], xv[TILE * LD];
  __shared__ double h[64 * LD];
  const bool own = (int)blockIdx.x < n_leaves;
  if (own && blockIdx.y > 0) return;
  InnerDesc it = own ? InnerDesc{-1, -1, 0, 0} : items[blockIdx.x - n_leaves];
  if (!own) {
    const int per = (it.c0 - it.r0 + (int)gridDim.y - 1) / (int)gridDim.y;
    const int a0 = it.r0 + (int)blockIdx.y * per;
    it.c0 = min(it.c0, a0 + per);
    it.r0 = a0;
    if (it.r0 >= it.c0) return;
  }
  const int bi = it.b;
  const int j = own ? leaves[blockIdx.x] : c.prob_leaf0[c.blocks[bi].prob] + s;
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const int64_t n = c.n;
  const double* X = c.inv + c.leaf_inv_off[j];
  for (int e = threadIdx.x; e < nl * VAR_K; e += NT) {
    const int a = e % nl, k = e / nl;
    tv[a * LD + k] = V[lo + a + (int64_t)k * n];
  }
  __syncthreads();
  // xv = L_jj^{-1} V[leaf, :]: thread (row i, half g of the columns), one load
  // of X per 16 products
  static_assert(NT == 2 * TILE, "two threads per leaf row");
  {
    const int i = threadIdx.x & (TILE - 1), g = threadIdx.x >> 7;
    if (i < nl) {
      double acc[VAR_K / 2];
#pragma unroll
      for (int q = 0; q < VAR_K / 2; ++q) acc[q] = 0.0;
      for (int a = 0; a <= i; ++a) {
        const double xa = X[i + a * nl];
#pragma unroll
        for (int q = 0; q < VAR_K / 2; ++q) acc[q] += xa * tv[a * LD + (VAR_K / 2) * g + q];
      }
#pragma unroll
      for (int q = 0; q < VAR_K / 2; ++q) xv[i * LD + (VAR_K / 2) * g + q] = acc[q];
    }
  }
  __syncthreads();
  if (own) {
    for (int e = threadIdx.x; e < nl * VAR_K; e += NT) {
      const int i = e % nl, k = e / nl;
      Vout[lo + i + (int64_t)k * n] = xv[i * LD + k];
    }
    return;
  }
  const BlockDesc x = c.blocks[bi];
  const int64_t mx = x.r1 - x.r0, kx = x.c1 - x.c0;
  const int k = threadIdx.x & (VAR_K - 1), rg = threadIdx.x / VAR_K;
  constexpr int RG = NT / VAR_K;
  if (x.kind == BK_DENSE) {
    const TS* W = c.L + x.loff + (lo - x.c0);
    for (int i = it.r0 + rg; i < it.c0; i += RG) {
      double acc = 0.0;
      for (int a = 0; a < nl; ++a) acc += double(W[a + (int64_t)i * kx]) * xv[a * LD + k];
      V[x.r0 + i + (int64_t)k * n] -= acc;
    }
  } else {
    const int rk = c.rank[bi];
    const TS* U = c.L + x.loff;
    const TS* W = U + mx * c.R + (lo - x.c0);
    for (int e = threadIdx.x; e < rk * VAR_K; e += NT) {
      const int l = e % rk, kq = e / rk;
      double acc = 0.0;
      for (int a = 0; a < nl; ++a) acc += double(W[a + (int64_t)l * kx]) * xv[a * LD + kq];
      h[l * LD + kq] = acc;
    }
    __syncthreads();
    for (int i = it.r0 + rg; i < it.c0; i += RG) {
      double acc = 0.0;
      for (int l = 0; l < rk; ++l) acc += double(U[i + (int64_t)l * mx]) * h[l * LD + k];
      V[x.r0 + i + (int64_t)k * n] -= acc;
    }
  }
}

// var[k] = sigma^2 - sum_j Vout[j, k]^2 for k < kk (fixed-order tree per column).
__global__ void __launch_bounds__(NT) k_var_finish(const double* Vout, int64_t n, int kk, double sigma2, double* var) {
  __shared__ double red[NT];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int64_t jj = threadIdx.x; jj < n; jj += NT) {
    const double v = Vout[jj + (int64_t)k * n];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && k < kk) var[k] = sigma2 - red[0];
}

// Test matrices of the low-rank target sketches: +-1 entries from a counter
// hash of (block, entry), drawn once per problem (k x R per block); the block
// enters through its index in its own problem, so a problem of a batch draws
// the same test matrices as alone.
template <typename TS>
__global__ void __launch_bounds__(NT) k_gen_omega(DevCtx<TS> c, int32_t first, uint32_t seed) {
  const int bi = first + blockIdx.x;
  const BlockDesc b = c.blocks[bi];
  const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
  TS* Om = c.S + b.soff + (m + k) * c.R;
  const uint32_t bs = mix32(seed ^ mix32((uint32_t)b.sid * 2654435761u));
  for (int64_t e = threadIdx.x; e < k * c.R; e += NT) Om[e] = (mix32(bs + (uint32_t)e) & 1u) ? TS(1) : TS(-1);
}

// Sampler, part 1: h_b = W_b^T w[sigma_b] for every low-rank block.
template <typename TS>
__global__ void __launch_bounds__(NT) k_sample_h(DevCtx<TS> c, int32_t first, const double* w, double* h) {
  __shared__ double sh[NT / 64];
  const int bi = first + blockIdx.x;
  const BlockDesc b = c.blocks[bi];
  const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int rk = c.rank[bi];
  const TS* W = c.L + b.loff + m * c.R;
  for (int l = 0; l < rk; ++l) {
    double s = 0.0;
    for (int j = threadIdx.x; j < k; j += NT) s += double(W[j + l * k]) * w[b.c0 + j];
    s = block_sum<double>(s, sh);
    if (threadIdx.x == 0) h[(int64_t)blockIdx.x * c.R + l] = s;
  }
}

// Sampler, part 2: y[leaf i] = L_ii w[leaf i] + sum over the row panel of leaf i.
template <typename TS>
__global__ void __launch_bounds__(NT) k_sample_rows(DevCtx<TS> c, int32_t n_dense, const int32_t* rowp_beg,
                                                     const int32_t* rowp, const double* w, const double* h, double* y) {
  const int j = blockIdx.x;
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const BlockDesc d = c.blocks[c.leaf_diag[j]];
  const double* Dg = c.D + d.loff;
  for (int r = threadIdx.x; r < nl; r += NT) {
    double acc = 0.0;
    for (int a = 0; a <= r; ++a) acc += Dg[r + a * nl] * w[lo + a];
    for (int q = rowp_beg[j]; q < rowp_beg[j + 1]; ++q) {
      const int bi = rowp[q];
      const BlockDesc b = c.blocks[bi];
      const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
      const int64_t rr = lo + r - b.r0;
      if (b.kind == BK_DENSE) {
        const TS* W = c.L + b.loff + rr * k;
        for (int64_t jj = 0; jj < k; ++jj) acc += double(W[jj]) * w[b.c0 + jj];
      } else {
        const int rk = c.rank[bi];
        const TS* U = c.L + b.loff;
        const double* hb = h + (int64_t)(bi - n_dense) * c.R;
        for (int l = 0; l < rk; ++l) acc += double(U[rr + l * m]) * hb[l];
      }
    }
    y[lo + r] = acc;
  }
}

// H-matrix-vector product y = C~ x of the assembled matrix (before the
// factorisation), part 1: for every low-rank block b = U0 W0^T (cross
// approximation, rank arank[b]) the two short vectors
//   h[b][0:Ra]  = W0^T x[columns of b]   (for y[rows]    += U0 h),
//   h[b][Ra:2Ra] = U0^T x[rows of b]     (for y[columns] += W0 h, the mirrored block).
template <typename TS>
__global__ void __launch_bounds__(NT) k_mv_lr(DevCtx<TS> c, int32_t first, const double* x, double* h) {
  __shared__ double sh[NT / 64];
  const int bi = first + blockIdx.x;
  const BlockDesc b = c.blocks[bi];
  const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int rk = c.arank[bi];
  const TS* U = c.A + b.aoff;
  const TS* W = U + m * c.Ra;
  double* hb = h + (int64_t)blockIdx.x * 2 * c.Ra;
  for (int l = 0; l < rk; ++l) {
    double s = 0.0, t = 0.0;
    for (int64_t j = threadIdx.x; j < k; j += NT) s += double(W[j + l * k]) * x[b.c0 + j];
    for (int64_t i = threadIdx.x; i < m; i += NT) t += double(U[i + l * m]) * x[b.r0 + i];
    s = block_sum<double>(s, sh);
    t = block_sum<double>(t, sh);
    if (threadIdx.x == 0) { hb[l] = s; hb[c.Ra + l] = t; }
  }
}

// Part 2, one workgroup per leaf i and one thread per row r of it:
//   y[r] = D_ii[r, :] x[leaf]                                  (diagonal leaf, full square)
//        + sum over blocks b whose rows hold leaf i   of C_b[r, :] x[columns of b]
//        + sum over blocks b whose columns hold leaf i of C_b[:, r]^T x[rows of b],
// the last sum being the upper triangle by symmetry; lists in a fixed order.
template <typename TS>
__global__ void __launch_bounds__(NT) k_mv_rows(DevCtx<TS> c, int32_t n_dense, const int32_t* rowp_beg,
                                                 const int32_t* rowp, const int32_t* colp_beg, const int32_t* colp,
                                                 const double* x, const double* h, double* y) {
  const int j = blockIdx.x;
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const BlockDesc d = c.blocks[c.leaf_diag[j]];
  const double* Dg = c.D + d.loff;
  for (int r = threadIdx.x; r < nl; r += NT) {
    double acc = 0.0;
    for (int a = 0; a < nl; ++a) acc += Dg[r + a * nl] * x[lo + a];
    for (int q = rowp_beg[j]; q < rowp_beg[j + 1]; ++q) {
      const int bi = rowp[q];
      const BlockDesc b = c.blocks[bi];
      const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
      const int64_t rr = lo + r - b.r0;
      if (b.kind == BK_DENSE) {
        const TS* W = c.L + b.loff + rr * k;
        for (int64_t jj = 0; jj < k; ++jj) acc += double(W[jj]) * x[b.c0 + jj];
      } else {
        const int rk = c.arank[bi];
        const TS* U = c.A + b.aoff;
        const double* hb = h + (int64_t)(bi - n_dense) * 2 * c.Ra;
        for (int l = 0; l < rk; ++l) acc += double(U[rr + l * m]) * hb[l];
      }
    }
    for (int q = colp_beg[j]; q < colp_beg[j + 1]; ++q) {
      const int bi = colp[q];
      const BlockDesc b = c.blocks[bi];
      const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
      const int64_t cc = lo + r - b.c0;
      if (b.kind == BK_DENSE) {
        const TS* W = c.L + b.loff + cc;
        for (int64_t i = 0; i < m; ++i) acc += double(W[i * k]) * x[b.r0 + i];
      } else {
        const int rk = c.arank[bi];
        const TS* W = c.A + b.aoff + m * c.Ra;
        const double* hb = h + (int64_t)(bi - n_dense) * 2 * c.Ra + c.Ra;
        for (int l = 0; l < rk; ++l) acc += double(W[cc + l * k]) * hb[l];
      }
    }
    y[lo + r] = acc;
  }
}

// Assembly reuse (theta changes only in sigma^2 and tau^2): the saved
// off-diagonal dense entries scaled by s = sigma1^2 / sigma0^2, the saved
// diagonal leaves as s (D0 - tau0^2 I) + tau1^2 I, and the cross-approximation
// factors U0 of every low-rank block scaled by f (in place).
template <typename TS>
__global__ void __launch_bounds__(NT) k_scale_copy(const TS* src, TS* dst, int64_t count, double s) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < count; e += (int64_t)gridDim.x * NT)
    dst[e] = TS(s * double(src[e]));
}

template <typename TS>
__global__ void __launch_bounds__(NT) k_rescale_diag(DevCtx<TS> c, const double* Dsave, double s, double t0,
                                                     double t1) {
  const int j = blockIdx.x;
  const BlockDesc b = c.blocks[c.leaf_diag[j]];
  const int m = b.r1 - b.r0;
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const bool d = e % m == e / m;
    c.D[b.loff + e] = s * (Dsave[b.loff + e] - (d ? t0 : 0.0)) + (d ? t1 : 0.0);
  }
}

template <typename TS>
__global__ void __launch_bounds__(NT) k_scale_lr(DevCtx<TS> c, int32_t first, double f) {
  const BlockDesc b = c.blocks[first + blockIdx.x];
  const int64_t cnt = (int64_t)(b.r1 - b.r0) * c.Ra;
  TS* U = c.A + b.aoff;
  for (int64_t e = threadIdx.x; e < cnt; e += NT) U[e] = TS(f * double(U[e]));
}

// Transposed factor product y = L~^T x (internal order), part 1: for every
// low-rank block of the factor, L_b = U W^T, the short vector g_b = U^T x[rows of b].
template <typename TS>
__global__ void __launch_bounds__(NT) k_lt_h(DevCtx<TS> c, int32_t first, const double* x, double* g) {
  __shared__ double sh[NT / 64];
  const int bi = first + blockIdx.x;
  const BlockDesc b = c.blocks[bi];
  const int64_t m = b.r1 - b.r0;
  const int rk = c.rank[bi];
  const TS* U = c.L + b.loff;
  for (int l = 0; l < rk; ++l) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += NT) s += double(U[i + l * m]) * x[b.r0 + i];
    s = block_sum<double>(s, sh);
    if (threadIdx.x == 0) g[(int64_t)blockIdx.x * c.R + l] = s;
  }
}

// Part 2, one workgroup per leaf j and one thread per column cc of it:
//   y[cc] = sum_{r >= cc} L_jj[r, cc] x[leaf j rows r]
//         + sum over off-diagonal blocks b whose columns hold leaf j of L_b[:, cc]^T x[rows of b],
// dense blocks from their transposed storage, low-rank ones as W[cc, :] g_b; lists in a fixed order.
template <typename TS>
__global__ void __launch_bounds__(NT) k_lt_cols(DevCtx<TS> c, int32_t n_dense, const int32_t* colp_beg,
                                                 const int32_t* colp, const double* x, const double* g, double* y) {
  const int j = blockIdx.x;
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const BlockDesc d = c.blocks[c.leaf_diag[j]];
  const double* Dg = c.D + d.loff;
  for (int cc = threadIdx.x; cc < nl; cc += NT) {
    double acc = 0.0;
    for (int r = cc; r < nl; ++r) acc += Dg[r + cc * nl] * x[lo + r];
    for (int q = colp_beg[j]; q < colp_beg[j + 1]; ++q) {
      const int bi = colp[q];
      const BlockDesc b = c.blocks[bi];
      const int64_t m = b.r1 - b.r0, k = b.c1 - b.c0;
      const int64_t cb = lo + cc - b.c0;
      if (b.kind == BK_DENSE) {
        const TS* W = c.L + b.loff + cb;
        for (int64_t i = 0; i < m; ++i) acc += double(W[i * k]) * x[b.r0 + i];
      } else {
        const int rk = c.rank[bi];
        const TS* W = c.L + b.loff + m * c.R + cb;
        const double* gb = g + (int64_t)(bi - n_dense) * c.R;
        for (int l = 0; l < rk; ++l) acc += double(W[l * k]) * gb[l];
      }
    }
    y[lo + cc] = acc;
  }
}

// Expected squared errors for one new point k (column k of the cross
// covariances): out[k] = |y|^2 - 2 w . ct + var, with w = C~_a^{-1} c_a (the
// kriging weights of the estimated model), ct the true model's cross
// covariance and y = L~_t^T w; one workgroup, sums in a fixed order.
__global__ void __launch_bounds__(NT) k_eta_point(const double* w, const double* ct, const double* y, int64_t n,
                                                  double var, double* out) {
  __shared__ double sh[NT / 64];
  double a = 0.0, q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    a += w[i] * ct[i];
    q += y[i] * y[i];
  }
  a = block_sum<double>(a, sh);
  q = block_sum<double>(q, sh);
  if (threadIdx.x == 0) *out = q - 2.0 * a + var;
}

// MLOE and MMOM (eqs. (5), (6)) from the per-point expected squared errors,
// means over the m points in index order.
__global__ void __launch_bounds__(NT) k_mloe_final(const double* e_ta, const double* e_tt, const double* e_aa,
                                                   int64_t m, double* out) {
  __shared__ double sh[NT / 64];
  double a = 0.0, b = 0.0;
  for (int64_t k = threadIdx.x; k < m; k += NT) {
    a += e_ta[k] / e_tt[k] - 1.0;
    b += e_aa[k] / e_ta[k] - 1.0;
  }
  a = block_sum<double>(a, sh);
  b = block_sum<double>(b, sh);
  if (threadIdx.x == 0) { out[0] = a / (double)m; out[1] = b / (double)m; }
}

__global__ void __launch_bounds__(NT) k_add_scalar(double* x, int64_t count, double v) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e < count) x[e] += v;
}

// Per-leaf partial sums: partial[2j] = 2 sum log L_ii, partial[2j+1] = sum v_i^2.
__global__ void __launch_bounds__(NT) k_reduce_leaf(const double* D, const int64_t* diag_off, const int32_t* leaf_lo,
                                                    const int32_t* leaf_hi, const double* v, double* partial) {
  __shared__ double sh[NT / 64];
  const int j = blockIdx.x;
  const int lo = leaf_lo[j], m = leaf_hi[j] - lo;
  const double* Dg = D + diag_off[j];
  double a = 0.0, q = 0.0;
  for (int i = threadIdx.x; i < m; i += NT) {
    a += log(Dg[i + (int64_t)i * m]);
    q += v[lo + i] * v[lo + i];
  }
  a = block_sum<double>(a, sh);
  q = block_sum<double>(q, sh);
  if (threadIdx.x == 0) { partial[2 * j] = 2.0 * a; partial[2 * j + 1] = q; }
}

// One workgroup per problem: sums the partials of its leaves in leaf order.
__global__ void __launch_bounds__(NT) k_reduce_final(const double* partial, const int32_t* prob_leaf0, double* out) {
  __shared__ double sh[NT / 64];
  const int p = blockIdx.x;
  double a = 0.0, q = 0.0;
  for (int j = prob_leaf0[p] + threadIdx.x; j < prob_leaf0[p + 1]; j += NT) {
    a += partial[2 * j];
    q += partial[2 * j + 1];
  }
  a = block_sum<double>(a, sh);
  q = block_sum<double>(q, sh);
  if (threadIdx.x == 0) { out[2 * p] = a; out[2 * p + 1] = q; }
}

__global__ void __launch_bounds__(NT) k_zero_i32(int32_t* x, int32_t count) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < count) x[i] = 0;
}

// ------------------------------------------------------------ launchers -----
template <typename TS>
void launch_assemble(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, double eps, hipStream_t st) {
  if (n_dense > 0) HMLE_LAUNCH(k_assemble_dense<TS>, dim3(n_dense), dim3(NT), 0, st, c);
  if (n_lowrank > 0) HMLE_LAUNCH(k_aca<TS>, dim3(n_lowrank), dim3(NT), 0, st, c, n_dense, TS(eps));
}

template <typename TS>
void launch_step_dense(const DevCtx<TS>& c, const StepLists& sl, hipStream_t st) {
  if (sl.n_dchunks > 0) HMLE_LAUNCH(k_dpairs<TS>, dim3(sl.n_dchunks), dim3(NT), 0, st, c, sl.dchunks, (TS*)sl.dpart);
  if (sl.n_dtargets > 0)
    HMLE_LAUNCH(k_dreduce<TS>, dim3(sl.n_dtargets, 16), dim3(NT), 0, st, c, sl.dtargets, sl.dchunks,
                       (const TS*)sl.dpart);
}

template <typename TS, int NC>
void step_lowrank_nc(const DevCtx<TS>& c, const StepLists& sl, double eps, hipStream_t st, hipEvent_t* ev) {
  TS* gbuf = (TS*)sl.gbuf;
  TS* rpart = (TS*)sl.rpart;
  const dim3 blk(NT);
  // pass 1: range sketch Y = S_b Omega and its orthonormal basis Q (rank-revealing to 1e-2 eps)
  HMLE_LAUNCH(k_rG<TS>, dim3(sl.n_g1), blk, 0, st, c, sl.g1, 1, gbuf, (TS*)sl.gseg);
  if (sl.n_gf1 > 0)
    HMLE_LAUNCH(k_rG_fin<TS>, dim3(sl.n_gf1, 8), blk, 0, st, c, sl.gf1, 1, gbuf, (const TS*)sl.gseg);
  if (ev) (void)hipEventRecord(ev[0], st);
  if (sl.n_r1chunks > 0)
    HMLE_LAUNCH((k_rpass<TS, NC>), dim3(sl.n_r1chunks), blk, 0, st, c, sl.r1chunks, sl.rpairs1, 1,
                       (const TS*)gbuf, rpart);
  if (ev) (void)hipEventRecord(ev[1], st);
  if (c.sum_kc == 32)
    HMLE_LAUNCH((k_rsum<TS, NC, 32>), dim3(sl.n_sg1), blk, 0, st, c, sl.rtargets, sl.tiles1, sl.sg1, sl.tc1,
                (const TS*)rpart, (const TS*)gbuf, 1, (TS*)sl.spart);
  else
    HMLE_LAUNCH((k_rsum<TS, NC, 16>), dim3(sl.n_sg1), blk, 0, st, c, sl.rtargets, sl.tiles1, sl.sg1, sl.tc1,
                (const TS*)rpart, (const TS*)gbuf, 1, (TS*)sl.spart);
  HMLE_LAUNCH((k_rsum_fin<TS, NC>), dim3(sl.n_t1), blk, 0, st, c, sl.rtargets, sl.tiles1, (const TS*)sl.spart,
                     1, sl.gpart);
  HMLE_LAUNCH((k_qchol<TS, 16 * NC>), dim3(sl.n_rtargets), blk, 0, st, c, sl.rtargets, 1, 0.01 * eps,
                     (const double*)sl.gpart, sl.qbuf, sl.qint);
  HMLE_LAUNCH((k_qapply<TS, NC>), dim3(sl.n_t1), blk, 0, st, c, sl.rtargets, sl.tiles1, 1,
                     (const double*)sl.qbuf, (const int*)sl.qint, sl.gpart);
  HMLE_LAUNCH((k_qchol2<TS, 16 * NC>), dim3(sl.n_rtargets), blk, 0, st, c, sl.rtargets, 1, (const double*)sl.gpart,
                     sl.qbuf, sl.qint);
  HMLE_LAUNCH((k_qapply2<TS, NC>), dim3(sl.n_t1), blk, 0, st, c, sl.rtargets, sl.tiles1,
                     (const double*)sl.qbuf, (const int*)sl.qint);
  // pass 2: B^T = S_b^T Q, truncated to eps: S_b ~ (Q Rm^T) Q2^T
  HMLE_LAUNCH(k_rG<TS>, dim3(sl.n_g2), blk, 0, st, c, sl.g2, 2, gbuf, (TS*)sl.gseg);
  if (sl.n_gf2 > 0)
    HMLE_LAUNCH(k_rG_fin<TS>, dim3(sl.n_gf2, 8), blk, 0, st, c, sl.gf2, 2, gbuf, (const TS*)sl.gseg);
  if (ev) (void)hipEventRecord(ev[2], st);
  if (sl.n_r2chunks > 0)
    HMLE_LAUNCH((k_rpass<TS, NC>), dim3(sl.n_r2chunks), blk, 0, st, c, sl.r2chunks, sl.rpairs2, 2,
                       (const TS*)gbuf, rpart);
  if (ev) (void)hipEventRecord(ev[3], st);
  if (c.sum_kc == 32)
    HMLE_LAUNCH((k_rsum<TS, NC, 32>), dim3(sl.n_sg2), blk, 0, st, c, sl.rtargets, sl.tiles2, sl.sg2, sl.tc2,
                (const TS*)rpart, (const TS*)gbuf, 2, (TS*)sl.spart);
  else
    HMLE_LAUNCH((k_rsum<TS, NC, 16>), dim3(sl.n_sg2), blk, 0, st, c, sl.rtargets, sl.tiles2, sl.sg2, sl.tc2,
                (const TS*)rpart, (const TS*)gbuf, 2, (TS*)sl.spart);
  HMLE_LAUNCH((k_rsum_fin<TS, NC>), dim3(sl.n_t2), blk, 0, st, c, sl.rtargets, sl.tiles2, (const TS*)sl.spart,
                     2, sl.gpart);
  HMLE_LAUNCH((k_qchol<TS, 16 * NC>), dim3(sl.n_rtargets), blk, 0, st, c, sl.rtargets, 2, eps, (const double*)sl.gpart,
                     sl.qbuf, sl.qint);
  HMLE_LAUNCH((k_qapply<TS, NC>), dim3(sl.n_t2), blk, 0, st, c, sl.rtargets, sl.tiles2, 2,
                     (const double*)sl.qbuf, (const int*)sl.qint, sl.gpart);
  HMLE_LAUNCH((k_qchol2<TS, 16 * NC>), dim3(sl.n_rtargets), blk, 0, st, c, sl.rtargets, 2, (const double*)sl.gpart,
                     sl.qbuf, sl.qint);
  HMLE_LAUNCH((k_qfin<TS, NC>), dim3(sl.n_t2 + sl.n_t1), blk, 0, st, c, sl.rtargets, sl.tiles2, sl.n_t2,
                     sl.tiles1, (const double*)sl.qbuf, (const int*)sl.qint);
}

template <typename TS>
void launch_step_lowrank(const DevCtx<TS>& c, const StepLists& sl, double eps, hipStream_t st, hipEvent_t* ev) {
  if (sl.n_rtargets == 0) {
    if (ev)
      for (int i = 0; i < 4; ++i) (void)hipEventRecord(ev[i], st);
    return;
  }
  if (c.R <= 32) step_lowrank_nc<TS, 2>(c, sl, eps, st, ev);
  else step_lowrank_nc<TS, 4>(c, sl, eps, st, ev);
}

template <typename TS>
void launch_step_diag(const DevCtx<TS>& c, const StepLists& sl, hipStream_t st) {
  if (sl.n_leaves > 0) HMLE_LAUNCH(k_potrf<TS>, dim3(sl.n_leaves), dim3(NT), 0, st, c, sl.leaves);
}

template <typename TS>
void launch_step_cols(const DevCtx<TS>& c, int32_t s, const StepLists& sl, hipStream_t st) {
  if (sl.n_tsolve > 0) HMLE_LAUNCH(k_trsm<TS>, dim3(sl.n_tsolve), dim3(NT), 0, st, c, s, sl.tsolve);
  if (sl.n_inner > 0) HMLE_LAUNCH(k_inner<TS>, dim3(sl.n_inner), dim3(NT), 0, st, c, s, sl.inner);
  if (sl.n_grams > 0) HMLE_LAUNCH(k_gram<TS>, dim3(sl.n_grams), dim3(NT), 0, st, c, sl.grams);
}

#define HMLE_INST_STEP(TS)                                                                          \
  template void launch_step_dense<TS>(const DevCtx<TS>&, const StepLists&, hipStream_t);           \
  template void launch_step_lowrank<TS>(const DevCtx<TS>&, const StepLists&, double, hipStream_t, hipEvent_t*); \
  template void launch_step_diag<TS>(const DevCtx<TS>&, const StepLists&, hipStream_t);            \
  template void launch_step_cols<TS>(const DevCtx<TS>&, int32_t, const StepLists&, hipStream_t);
HMLE_INST_STEP(double)
HMLE_INST_STEP(float)

template <typename TS>
void launch_dense_pairs(const DevCtx<TS>& c, const StepLists& sl, hipStream_t st) {
  if (sl.n_dchunks > 0) HMLE_LAUNCH(k_dpairs<TS>, dim3(sl.n_dchunks), dim3(NT), 0, st, c, sl.dchunks, (TS*)sl.dpart);
}
template void launch_dense_pairs<double>(const DevCtx<double>&, const StepLists&, hipStream_t);
template void launch_dense_pairs<float>(const DevCtx<float>&, const StepLists&, hipStream_t);

template <typename TS>
void launch_dense_reduce(const DevCtx<TS>& c, const StepLists& sl, hipStream_t st) {
  if (sl.n_dtargets > 0)
    HMLE_LAUNCH(k_dreduce<TS>, dim3(sl.n_dtargets, 16), dim3(NT), 0, st, c, sl.dtargets, sl.dchunks,
                       (const TS*)sl.dpart);
}
template void launch_dense_reduce<double>(const DevCtx<double>&, const StepLists&, hipStream_t);
template void launch_dense_reduce<float>(const DevCtx<float>&, const StepLists&, hipStream_t);

template <typename TS>
void launch_gen_omega(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, hipStream_t st) {
  if (n_lowrank > 0) HMLE_LAUNCH(k_gen_omega<TS>, dim3(n_lowrank), dim3(NT), 0, st, c, n_dense, 0x9e3779b9u);
}
template void launch_gen_omega<double>(const DevCtx<double>&, int32_t, int32_t, hipStream_t);
template void launch_gen_omega<float>(const DevCtx<float>&, int32_t, int32_t, hipStream_t);

template <typename TS>
void launch_solve_step(const DevCtx<TS>& c, int32_t s, const int32_t* leaves, int32_t n_leaves, const InnerDesc* items,
                       int32_t n_items, double* v, hipStream_t st) {
  // v holds [running right-hand side | solution]
  if (n_leaves + n_items > 0)
    HMLE_LAUNCH(k_solve_step<TS>, dim3(n_leaves + n_items), dim3(NT), 0, st, c, s, leaves, n_leaves, items, v,
                       v + c.n);
}

template <typename TS>
void launch_sample(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, int32_t n_leaves, const int32_t* rowp_beg,
                   const int32_t* rowp, const double* w, double* h, double* y, hipStream_t st) {
  if (n_lowrank > 0) HMLE_LAUNCH(k_sample_h<TS>, dim3(n_lowrank), dim3(NT), 0, st, c, n_dense, w, h);
  HMLE_LAUNCH(k_sample_rows<TS>, dim3(n_leaves), dim3(NT), 0, st, c, n_dense, rowp_beg, rowp, w, h, y);
}

void launch_matern(const double* h, int64_t count, const MaternParams& mp, int precision, double* out,
                   hipStream_t st) {
  if (count <= 0) return;
  const dim3 g((unsigned)((count + NT - 1) / NT));
  if (precision == 0) HMLE_LAUNCH(k_matern<double>, g, dim3(NT), 0, st, h, count, mp, out);
  else HMLE_LAUNCH(k_matern<float>, g, dim3(NT), 0, st, h, count, mp, out);
}

void launch_gather_coords(const double* pts, const int32_t* perm, int32_t n, int32_t dim, double* coords,
                          hipStream_t st) {
  HMLE_LAUNCH(k_gather_coords, dim3((n + NT - 1) / NT), dim3(NT), 0, st, pts, perm, n, dim, coords);
}
void launch_gather(const double* z, const int32_t* perm, int32_t n, double* v, hipStream_t st) {
  HMLE_LAUNCH(k_gather, dim3((n + NT - 1) / NT), dim3(NT), 0, st, z, perm, n, v);
}
void launch_scatter(const double* v, const int32_t* perm, int32_t n, double* z, hipStream_t st) {
  HMLE_LAUNCH(k_scatter, dim3((n + NT - 1) / NT), dim3(NT), 0, st, v, perm, n, z);
}
void launch_check_finite(const double* x, int64_t count, int32_t* flag, hipStream_t st) {
  if (count <= 0) return;
  HMLE_LAUNCH(k_check_finite, dim3((unsigned)((count + NT - 1) / NT)), dim3(NT), 0, st, x, count, flag);
}
void launch_reduce(const double* D, const int64_t* diag_off, const int32_t* leaf_lo, const int32_t* leaf_hi,
                   int32_t n_leaves, const int32_t* prob_leaf0, int32_t n_probs, const double* v, double* partial,
                   double* out, hipStream_t st) {
  HMLE_LAUNCH(k_reduce_leaf, dim3(n_leaves), dim3(NT), 0, st, D, diag_off, leaf_lo, leaf_hi, v, partial);
  HMLE_LAUNCH(k_reduce_final, dim3(n_probs), dim3(NT), 0, st, partial, prob_leaf0, out);
}
void launch_zero_i32(int32_t* x, int32_t count, hipStream_t st) {
  if (count > 0) HMLE_LAUNCH(k_zero_i32, dim3((count + NT - 1) / NT), dim3(NT), 0, st, x, count);
}

template void launch_assemble<double>(const DevCtx<double>&, int32_t, int32_t, double, hipStream_t);
template void launch_assemble<float>(const DevCtx<float>&, int32_t, int32_t, double, hipStream_t);
template <typename TS>
void launch_factor_t_product(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, int32_t n_leaves,
                             const int32_t* colp_beg, const int32_t* colp, const double* x, double* g, double* y,
                             hipStream_t st) {
  HMLE_LAUNCH(k_lt_h<TS>, dim3(n_lowrank), dim3(NT), 0, st, c, n_dense, x, g);
  HMLE_LAUNCH(k_lt_cols<TS>, dim3(n_leaves), dim3(NT), 0, st, c, n_dense, colp_beg, colp, x, (const double*)g, y);
}
template void launch_factor_t_product<double>(const DevCtx<double>&, int32_t, int32_t, int32_t, const int32_t*,
                                              const int32_t*, const double*, double*, double*, hipStream_t);
template void launch_factor_t_product<float>(const DevCtx<float>&, int32_t, int32_t, int32_t, const int32_t*,
                                             const int32_t*, const double*, double*, double*, hipStream_t);

void launch_cross_cols(const double* coords, int32_t n, const double* p2, int32_t kk, int32_t dim,
                       const MaternParams& mp, double* B, hipStream_t st) {
  const int64_t tot = (int64_t)n * VAR_K;
  HMLE_LAUNCH(k_cross_cols, dim3((unsigned)((tot + NT - 1) / NT)), dim3(NT), 0, st, coords, n, p2, kk, dim, mp, B);
}

void launch_eta_point(const double* w, const double* ct, const double* y, int64_t n, double var, double* out,
                      hipStream_t st) {
  HMLE_LAUNCH(k_eta_point, dim3(1), dim3(NT), 0, st, w, ct, y, n, var, out);
}

void launch_mloe_final(const double* e_ta, const double* e_tt, const double* e_aa, int64_t m, double* out,
                       hipStream_t st) {
  HMLE_LAUNCH(k_mloe_final, dim3(1), dim3(NT), 0, st, e_ta, e_tt, e_aa, m, out);
}

void launch_add_scalar(double* x, int64_t count, double v, hipStream_t st) {
  if (count > 0) HMLE_LAUNCH(k_add_scalar, dim3((unsigned)((count + NT - 1) / NT)), dim3(NT), 0, st, x, count, v);
}

template <typename TS>
void launch_rescale(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, int32_t n_leaves, const TS* Lsave,
                    int64_t l_dense, const double* Dsave, double s, double t0, double t1, double f, hipStream_t st) {
  const int g = (int)std::min<int64_t>(4096, (l_dense + NT - 1) / NT);
  HMLE_LAUNCH(k_scale_copy<TS>, dim3(g), dim3(NT), 0, st, Lsave, c.L, l_dense, s);
  HMLE_LAUNCH(k_rescale_diag<TS>, dim3(n_leaves), dim3(NT), 0, st, c, Dsave, s, t0, t1);
  HMLE_LAUNCH(k_scale_lr<TS>, dim3(n_lowrank), dim3(NT), 0, st, c, n_dense, f);
}
template void launch_rescale<double>(const DevCtx<double>&, int32_t, int32_t, int32_t, const double*, int64_t,
                                     const double*, double, double, double, double, hipStream_t);
template void launch_rescale<float>(const DevCtx<float>&, int32_t, int32_t, int32_t, const float*, int64_t,
                                    const double*, double, double, double, double, hipStream_t);

template <typename TS>
void launch_matvec(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, int32_t n_leaves, const int32_t* rowp_beg,
                   const int32_t* rowp, const int32_t* colp_beg, const int32_t* colp, const double* x, double* h,
                   double* y, hipStream_t st) {
  HMLE_LAUNCH(k_mv_lr<TS>, dim3(n_lowrank), dim3(NT), 0, st, c, n_dense, x, h);
  HMLE_LAUNCH(k_mv_rows<TS>, dim3(n_leaves), dim3(NT), 0, st, c, n_dense, rowp_beg, rowp, colp_beg, colp, x, h, y);
}
template void launch_matvec<double>(const DevCtx<double>&, int32_t, int32_t, int32_t, const int32_t*, const int32_t*,
                                    const int32_t*, const int32_t*, const double*, double*, double*, hipStream_t);
template void launch_matvec<float>(const DevCtx<float>&, int32_t, int32_t, int32_t, const int32_t*, const int32_t*,
                                   const int32_t*, const int32_t*, const double*, double*, double*, hipStream_t);

template void launch_sample<double>(const DevCtx<double>&, int32_t, int32_t, int32_t, const int32_t*, const int32_t*,
                                    const double*, double*, double*, hipStream_t);
template void launch_sample<float>(const DevCtx<float>&, int32_t, int32_t, int32_t, const int32_t*, const int32_t*,
                                   const double*, double*, double*, hipStream_t);
template void launch_solve_step<double>(const DevCtx<double>&, int32_t, const int32_t*, int32_t, const InnerDesc*,
                                         int32_t, double*, hipStream_t);
template void launch_solve_step<float>(const DevCtx<float>&, int32_t, const int32_t*, int32_t, const InnerDesc*, int32_t,
                                        double*, hipStream_t);

template <typename TS>
void launch_bsolve_step(const DevCtx<TS>& c, int32_t s, const int32_t* leaves, int32_t n_leaves, const InnerDesc* items,
                        int32_t n_items, double* part, const double* v, double* w, hipStream_t st) {
  if (n_items > 0) HMLE_LAUNCH(k_bsolve_part<TS>, dim3(n_items), dim3(NT), 0, st, c, s, items, (const double*)w, part);
  if (n_leaves > 0)
    HMLE_LAUNCH(k_bsolve_fin<TS>, dim3(n_leaves), dim3(NT), 0, st, c, leaves, n_items, (const double*)part, v, w);
}
template void launch_bsolve_step<double>(const DevCtx<double>&, int32_t, const int32_t*, int32_t, const InnerDesc*,
                                         int32_t, double*, const double*, double*, hipStream_t);
template void launch_bsolve_step<float>(const DevCtx<float>&, int32_t, const int32_t*, int32_t, const InnerDesc*,
                                        int32_t, double*, const double*, double*, hipStream_t);

void launch_predict(const double* c1, const double* w, int32_t n1, const double* p2, int64_t m, int32_t dim,
                    const MaternParams& mp, double* z2, hipStream_t st) {
  if (m > 0)
    HMLE_LAUNCH(k_predict, dim3((unsigned)((m + PRED_P - 1) / PRED_P)), dim3(NT), 0, st, c1, w, n1, p2, m, dim,
                       mp, z2);
}

template <typename TS>
void launch_predict_var(const DevCtx<TS>& c, int32_t n_steps, const int32_t* step_leaf, const int32_t* step_leaf_beg,
                        const InnerDesc* fsolve, const int32_t* fsolve_beg, const double* p2, int32_t kk,
                        const MaternParams& mp, double sigma2, double* V, double* Vout, double* var, hipStream_t st) {
  const int64_t tot = (int64_t)c.n * VAR_K;
  HMLE_LAUNCH(k_cross_cols, dim3((unsigned)((tot + NT - 1) / NT)), dim3(NT), 0, st, c.coords, c.n, p2, kk, c.dim,
                     mp, V);
  for (int32_t j = 0; j < n_steps; ++j) {
    const int32_t nlv = step_leaf_beg[j + 1] - step_leaf_beg[j];
    const int32_t ni = fsolve_beg[j + 1] - fsolve_beg[j];
    if (nlv + ni > 0)
      HMLE_LAUNCH(k_solve_step_multi<TS>, dim3(nlv + ni, 8), dim3(NT), 0, st, c, j, step_leaf + step_leaf_beg[j],
                         nlv, fsolve + fsolve_beg[j], V, Vout);
  }
  HMLE_LAUNCH(k_var_finish, dim3(VAR_K), dim3(NT), 0, st, (const double*)Vout, (int64_t)c.n, kk, sigma2, var);
}
template void launch_predict_var<double>(const DevCtx<double>&, int32_t, const int32_t*, const int32_t*,
                                         const InnerDesc*, const int32_t*, const double*, int32_t,
                                         const MaternParams&, double, double*, double*, double*, hipStream_t);
template void launch_predict_var<float>(const DevCtx<float>&, int32_t, const int32_t*, const int32_t*,
                                        const InnerDesc*, const int32_t*, const double*, int32_t,
                                        const MaternParams&, double, double*, double*, double*, hipStream_t);

}  // namespace hmle
