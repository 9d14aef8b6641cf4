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
//                2 sum log L_ii and v^T v (Section 2, "Storage and complexity").
//
// Every reduction runs in a fixed order, so results are bit-reproducible.
#include <hip/hip_runtime.h>

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

// Element L_x[row, col] (global indices) of an off-diagonal block.
template <typename TS>
__device__ __forceinline__ TS piece_elem(const DevCtx<TS>& c, const BlockDesc& x, int rank, int row, int col) {
  const int64_t k = x.c1 - x.c0;
  if (x.kind == BK_DENSE) return c.L[x.loff + (col - x.c0) + (int64_t)(row - x.r0) * k];
  const int64_t m = x.r1 - x.r0;
  const TS* U = c.L + x.loff;
  const TS* W = U + m * c.R;
  TS s = TS(0);
  for (int l = 0; l < rank; ++l) s += U[(row - x.r0) + l * m] * W[(col - x.c0) + l * k];
  return s;
}

// out (|w| x ncol, ld ldo) = L_y[ry0:ry1, w0:w1]^T X, X: |ry| x ncol (ld ldx).
template <typename TS>
__device__ void wg_piece_T(const DevCtx<TS>& c, const BlockDesc& y, int ranky, int ry0, int ry1, int w0, int w1,
                           const TS* X, int64_t ldx, int ncol, TS* out, int64_t ldo, TS* G, TS* red) {
  const int nr = ry1 - ry0, nw = w1 - w0;
  const int64_t ky = y.c1 - y.c0;
  if (y.kind == BK_DENSE) {
    const TS* W = c.L + y.loff;
    for (int e = threadIdx.x; e < nw * ncol; e += NT) {
      const int a = e % nw, cc = e / nw;
      const TS* wp = W + (w0 + a - y.c0) + (int64_t)(ry0 - y.r0) * ky;
      const TS* xp = X + (int64_t)cc * ldx;
      TS s = TS(0);
      for (int i = 0; i < nr; ++i) s += wp[(int64_t)i * ky] * xp[i];
      out[a + (int64_t)cc * ldo] = s;
    }
  } else {
    const int64_t my = y.r1 - y.r0;
    const TS* U = c.L + y.loff;
    const TS* W = U + my * c.R;
    wg_gemm_tn<TS, TS, TS>(nr, ranky, ncol, U + (ry0 - y.r0), my, X, ldx, G, red);
    for (int e = threadIdx.x; e < nw * ncol; e += NT) {
      const int a = e % nw, cc = e / nw;
      TS s = TS(0);
      for (int l = 0; l < ranky; ++l) s += W[(w0 + a - y.c0) + l * ky] * G[l + cc * ranky];
      out[a + (int64_t)cc * ldo] = s;
    }
  }
  __syncthreads();
}

// out[0:|rx|, :] -= L_x[rx0:rx1, w0:w1] T, T: |w| x ncol (ld ldt), out ld ldo.
template <typename TS, typename TT>
__device__ void wg_piece_N_sub(const DevCtx<TS>& c, const BlockDesc& x, int rankx, int rx0, int rx1, int w0, int w1,
                               const TT* T, int64_t ldt, int ncol, TS* out, int64_t ldo, TS* H, TS* red) {
  const int nr = rx1 - rx0, nw = w1 - w0;
  const int64_t kx = x.c1 - x.c0;
  if (x.kind == BK_DENSE) {
    const TS* W = c.L + x.loff;
    for (int e = threadIdx.x; e < nr * ncol; e += NT) {
      const int i = e % nr, cc = e / nr;
      const TS* wp = W + (w0 - x.c0) + (int64_t)(rx0 + i - x.r0) * kx;
      const TT* tp = T + (int64_t)cc * ldt;
      TS s = TS(0);
      for (int a = 0; a < nw; ++a) s += wp[a] * TS(tp[a]);
      out[i + (int64_t)cc * ldo] -= s;
    }
  } else {
    const int64_t mx = x.r1 - x.r0;
    const TS* U = c.L + x.loff;
    const TS* W = U + mx * c.R;
    wg_gemm_tn<TS, TT, TS>(nw, rankx, ncol, W + (w0 - x.c0), kx, T, ldt, H, red);
    for (int e = threadIdx.x; e < nr * ncol; e += NT) {
      const int i = e % nr, cc = e / nr;
      TS s = TS(0);
      for (int l = 0; l < rankx; ++l) s += U[(rx0 + i - x.r0) + l * mx] * H[l + cc * rankx];
      out[i + (int64_t)cc * ldo] -= s;
    }
  }
  __syncthreads();
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
__global__ void __launch_bounds__(NT) k_assemble_dense(DevCtx<TS> c, MaternParams mp) {
  const BlockDesc b = c.blocks[blockIdx.x];
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
__global__ void __launch_bounds__(NT) k_aca(DevCtx<TS> c, int32_t first, MaternParams mp, TS eps) {
  __shared__ TS red[NT];
  __shared__ TS shv[NT / 64];
  __shared__ int shi[NT / 64];
  __shared__ TS dots[2][64];
  const int bi = first + blockIdx.x;
  const BlockDesc b = c.blocks[bi];
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
    if (nu2 * nw2 <= eps * eps * frob2) { conv = true; break; }
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

// External update of dense targets (diagonal leaves and dense off-diagonal
// blocks): S_b = C_b - sum over pairs L_x[rx, w] L_y[ry, w]^T. One workgroup
// per target; 128 x 128 output tiles held in registers, the two factor pieces
// staged through LDS in chunks of CH columns.
template <typename TS>
__global__ void __launch_bounds__(NT) k_ext_dense(DevCtx<TS> c, const int32_t* ids) {
  __shared__ TS As[TILE * (CH + 1)];
  __shared__ TS Bs[TILE * (CH + 1)];
  const int bi = ids[blockIdx.x];
  const BlockDesc b = c.blocks[bi];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int64_t p0 = c.pair_beg[bi], p1 = c.pair_beg[bi + 1];
  const int ti_ = threadIdx.x & (TILE - 1), tg = threadIdx.x >> 7;
  for (int64_t p = p0; p < p1; ++p) {
    const PairDesc pr = c.pairs[p];
    const BlockDesc x = c.blocks[pr.x], y = c.blocks[pr.y];
    const int rkx = x.kind == BK_LOWRANK ? c.rank[pr.x] : 0;
    const int rky = y.kind == BK_LOWRANK ? c.rank[pr.y] : 0;
    for (int ti = pr.rx0; ti < pr.rx1; ti += TILE) {
      for (int tj = pr.ry0; tj < pr.ry1; tj += TILE) {
        const int ni = min(TILE, pr.rx1 - ti), nj = min(TILE, pr.ry1 - tj);
        TS acc[TILE / 2];
#pragma unroll
        for (int q = 0; q < TILE / 2; ++q) acc[q] = TS(0);
        for (int w = pr.w0; w < pr.w1; w += CH) {
          const int nw = min(CH, pr.w1 - w);
          __syncthreads();
          for (int e = threadIdx.x; e < TILE * CH; e += NT) {
            const int r = e / CH, cc = e % CH;
            As[r * (CH + 1) + cc] = (r < ni && cc < nw) ? piece_elem(c, x, rkx, ti + r, w + cc) : TS(0);
            Bs[r * (CH + 1) + cc] = (r < nj && cc < nw) ? piece_elem(c, y, rky, tj + r, w + cc) : TS(0);
          }
          __syncthreads();
          if (ti_ < ni) {
#pragma unroll
            for (int q = 0; q < TILE / 2; ++q) {
              const int j = tg + 2 * q;
              TS s = TS(0);
#pragma unroll
              for (int cc = 0; cc < CH; ++cc) s += As[ti_ * (CH + 1) + cc] * Bs[j * (CH + 1) + cc];
              acc[q] += s;
            }
          }
        }
        if (ti_ < ni) {
          const int gi = ti + ti_ - b.r0;
#pragma unroll
          for (int q = 0; q < TILE / 2; ++q) {
            const int j = tg + 2 * q;
            if (j < nj) {
              const int gj = tj + j - b.c0;
              if (b.kind == BK_DIAG) c.D[b.loff + gi + (int64_t)gj * m] -= double(acc[q]);
              else c.L[b.loff + gj + (int64_t)gi * k] -= acc[q];
            }
          }
        }
      }
    }
  }
}

// Pass 1 of the low-rank target update: Y = S_b Omega with
// S_b = U0 W0^T - sum over pairs L_x[rx,w] L_y[ry,w]^T and a +-1 test matrix.
template <typename TS>
__global__ void __launch_bounds__(NT) k_sketch1(DevCtx<TS> c, const int32_t* ids, uint32_t seed) {
  __shared__ TS G[64 * TILE];
  __shared__ TS red[NT];
  const int bi = ids[blockIdx.x];
  const BlockDesc b = c.blocks[bi];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int re = min(c.R, min(m, k));
  TS* Y = c.S + b.soff;
  TS* Om = c.S + b.soff + (int64_t)m * c.R;
  TS* tmp = c.tmp + (int64_t)blockIdx.x * c.tmp_stride;
  const uint32_t bs = mix32(seed ^ mix32((uint32_t)bi * 2654435761u));
  for (int e = threadIdx.x; e < k * re; e += NT) Om[e] = (mix32(bs + (uint32_t)e) & 1u) ? TS(1) : TS(-1);
  __syncthreads();
  const int ka = c.arank[bi];
  const TS* U0 = c.A + b.aoff;
  const TS* W0 = U0 + (int64_t)m * c.Ra;
  wg_gemm_tn<TS, TS, TS>(k, ka, re, W0, k, Om, k, G, red);
  for (int e = threadIdx.x; e < m * re; e += NT) {
    const int i = e % m, cc = e / m;
    TS s = TS(0);
    for (int l = 0; l < ka; ++l) s += U0[i + (int64_t)l * m] * G[l + cc * ka];
    Y[e] = s;
  }
  __syncthreads();
  for (int64_t p = c.pair_beg[bi]; p < c.pair_beg[bi + 1]; ++p) {
    const PairDesc pr = c.pairs[p];
    const BlockDesc x = c.blocks[pr.x], y = c.blocks[pr.y];
    const int rkx = x.kind == BK_LOWRANK ? c.rank[pr.x] : 0;
    const int rky = y.kind == BK_LOWRANK ? c.rank[pr.y] : 0;
    const int nw = pr.w1 - pr.w0;
    wg_piece_T(c, y, rky, pr.ry0, pr.ry1, pr.w0, pr.w1, Om + (pr.ry0 - b.c0), k, re, tmp, nw, G, red);
    wg_piece_N_sub<TS, TS>(c, x, rkx, pr.rx0, pr.rx1, pr.w0, pr.w1, tmp, nw, re, Y + (pr.rx0 - b.r0), m, G, red);
  }
}

// Column-pivoted QR (modified Gram-Schmidt with one re-orthogonalisation of
// each pivot column) of A (rows x ncol, ld rows) in place, stopped when the
// Frobenius norm of the remaining columns is <= tol times the initial one.
// On return A[:, 0:kq] holds orthonormal columns, Rm (kq x ncol, ld 64) the
// triangular factor of the permuted columns, perm the column order.
template <typename TS>
__device__ int wg_cpqr(TS* A, int rows, int ncol, TS tol, TS* Rm, int* perm, TS* nrm2, TS* dots, TS* red) {
  for (int cc = threadIdx.x; cc < ncol; cc += NT) perm[cc] = cc;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) Rm[e] = TS(0);
  // initial column norms
  for (int cc = 0; cc < ncol; ++cc) {
    TS s = TS(0);
    const TS* a = A + (int64_t)cc * rows;
    for (int i = threadIdx.x; i < rows; i += NT) s += a[i] * a[i];
    s = block_sum<TS>(s, red);
    if (threadIdx.x == 0) nrm2[cc] = s;
  }
  __syncthreads();
  TS total = TS(0);
  for (int cc = 0; cc < ncol; ++cc) total += nrm2[cc];
  int kq = 0;
  for (int i = 0; i < ncol; ++i) {
    TS rem = TS(0);
    int p = i;
    for (int cc = i; cc < ncol; ++cc) {
      rem += nrm2[cc];
      if (nrm2[cc] > nrm2[p]) p = cc;
    }
    if (!(rem > tol * tol * total) || !(total > TS(0))) break;
    __syncthreads();
    if (p != i) {
      TS* a = A + (int64_t)i * rows;
      TS* bcol = A + (int64_t)p * rows;
      for (int r = threadIdx.x; r < rows; r += NT) { const TS t = a[r]; a[r] = bcol[r]; bcol[r] = t; }
      if (threadIdx.x == 0) {
        const TS t = nrm2[i]; nrm2[i] = nrm2[p]; nrm2[p] = t;
        const int tp = perm[i]; perm[i] = perm[p]; perm[p] = tp;
      }
      for (int l = threadIdx.x; l < i; l += NT) { const TS t = Rm[l + 64 * i]; Rm[l + 64 * i] = Rm[l + 64 * p]; Rm[l + 64 * p] = t; }
      __syncthreads();
    }
    TS* ai = A + (int64_t)i * rows;
    // re-orthogonalise against the previous q's
    if (i > 0) {
      wg_gemm_tn<TS, TS, TS>(rows, i, 1, A, rows, ai, rows, dots, red);
      for (int r = threadIdx.x; r < rows; r += NT) {
        TS s = TS(0);
        for (int l = 0; l < i; ++l) s += A[r + (int64_t)l * rows] * dots[l];
        ai[r] -= s;
      }
      if (threadIdx.x < i) Rm[threadIdx.x + 64 * i] += dots[threadIdx.x];
      __syncthreads();
    }
    TS s = TS(0);
    for (int r = threadIdx.x; r < rows; r += NT) s += ai[r] * ai[r];
    const TS nr = sqrt(block_sum<TS>(s, red));
    if (!(nr > TS(0))) break;
    const TS inv = TS(1) / nr;
    for (int r = threadIdx.x; r < rows; r += NT) ai[r] *= inv;
    if (threadIdx.x == 0) Rm[i + 64 * i] = nr;
    __syncthreads();
    kq = i + 1;
    // project the remaining columns
    const int rest = ncol - i - 1;
    if (rest > 0) {
      TS* ar = A + (int64_t)(i + 1) * rows;
      wg_gemm_tn<TS, TS, TS>(rows, rest, 1, ar, rows, ai, rows, dots, red);
      for (int e = threadIdx.x; e < rows * rest; e += NT) {
        const int r = e % rows, cc = e / rows;
        ar[r + (int64_t)cc * rows] -= dots[cc] * ai[r];
      }
      if (threadIdx.x < rest) Rm[i + 64 * (i + 1 + threadIdx.x)] = dots[threadIdx.x];
      __syncthreads();
      for (int cc = 0; cc < rest; ++cc) {
        TS s2 = TS(0);
        const TS* a = ar + (int64_t)cc * rows;
        for (int r = threadIdx.x; r < rows; r += NT) s2 += a[r] * a[r];
        s2 = block_sum<TS>(s2, red);
        if (threadIdx.x == 0) nrm2[i + 1 + cc] = s2;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  return kq;
}

// Orthonormal basis Q of the sketch Y (in place); its width goes to rank[b].
template <typename TS>
__global__ void __launch_bounds__(NT) k_sketch_qr(DevCtx<TS> c, const int32_t* ids, TS tol) {
  __shared__ TS Rm[64 * 64];
  __shared__ int perm[64];
  __shared__ TS nrm2[64], dots[64], red[NT];
  const int bi = ids[blockIdx.x];
  const BlockDesc b = c.blocks[bi];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int re = min(c.R, min(m, k));
  const int kq = wg_cpqr<TS>(c.S + b.soff, m, re, tol, Rm, perm, nrm2, dots, red);
  if (threadIdx.x == 0) c.rank[bi] = kq;
}

// Pass 2: B^T = S_b^T Q (k x kq) into the sketch scratch, then truncation:
// CPQR of B^T to the block accuracy eps gives B^T Pi = Q2 R, so
// S_b ~ (Q Pi R^T) Q2^T: U = Q Pi R^T, W = Q2, rank = columns kept.
template <typename TS>
__global__ void __launch_bounds__(NT) k_sketch2(DevCtx<TS> c, const int32_t* ids, TS eps) {
  __shared__ TS G[64 * TILE];
  __shared__ TS red[NT];
  __shared__ TS Rm[64 * 64];
  __shared__ int perm[64];
  __shared__ TS nrm2[64], dots[64];
  const int bi = ids[blockIdx.x];
  const BlockDesc b = c.blocks[bi];
  const int m = b.r1 - b.r0, k = b.c1 - b.c0;
  const int kq = c.rank[bi];
  TS* Q = c.S + b.soff;
  TS* Bt = c.S + b.soff + (int64_t)m * c.R;
  TS* tmp = c.tmp + (int64_t)blockIdx.x * c.tmp_stride;
  const int ka = c.arank[bi];
  const TS* U0 = c.A + b.aoff;
  const TS* W0 = U0 + (int64_t)m * c.Ra;
  TS* Ul = c.L + b.loff;
  TS* Wl = Ul + (int64_t)m * c.R;
  if (kq == 0) {
    if (threadIdx.x == 0) c.rank[bi] = 0;
    return;
  }
  wg_gemm_tn<TS, TS, TS>(m, ka, kq, U0, m, Q, m, G, red);
  for (int e = threadIdx.x; e < k * kq; e += NT) {
    const int j = e % k, cc = e / k;
    TS s = TS(0);
    for (int l = 0; l < ka; ++l) s += W0[j + (int64_t)l * k] * G[l + cc * ka];
    Bt[e] = s;
  }
  __syncthreads();
  for (int64_t p = c.pair_beg[bi]; p < c.pair_beg[bi + 1]; ++p) {
    const PairDesc pr = c.pairs[p];
    const BlockDesc x = c.blocks[pr.x], y = c.blocks[pr.y];
    const int rkx = x.kind == BK_LOWRANK ? c.rank[pr.x] : 0;
    const int rky = y.kind == BK_LOWRANK ? c.rank[pr.y] : 0;
    const int nw = pr.w1 - pr.w0;
    wg_piece_T(c, x, rkx, pr.rx0, pr.rx1, pr.w0, pr.w1, Q + (pr.rx0 - b.r0), m, kq, tmp, nw, G, red);
    wg_piece_N_sub<TS, TS>(c, y, rky, pr.ry0, pr.ry1, pr.w0, pr.w1, tmp, nw, kq, Bt + (pr.ry0 - b.c0), k, G, red);
  }
  const int kr = wg_cpqr<TS>(Bt, k, kq, eps, Rm, perm, nrm2, dots, red);
  for (int e = threadIdx.x; e < k * kr; e += NT) Wl[e] = Bt[e];
  for (int e = threadIdx.x; e < m * kr; e += NT) {
    const int i = e % m, l = e / m;
    TS s = TS(0);
    for (int cc = l; cc < kq; ++cc) s += Q[i + (int64_t)perm[cc] * m] * Rm[l + 64 * cc];
    Ul[e] = s;
  }
  if (threadIdx.x == 0) {
    c.rank[bi] = kr;
    if (kr >= c.R) atomicAdd(&c.status[1], 1);
  }
}

// Cholesky of diagonal leaf j in LDS (float64) and the inverse of the factor.
template <typename TS>
__global__ void __launch_bounds__(NT) k_potrf(DevCtx<TS> c, int j) {
  __shared__ double A[TILE * TILE];
  __shared__ int fail;
  const int lo = c.leaf_lo[j], m = c.leaf_hi[j] - lo;
  const BlockDesc b = c.blocks[c.leaf_diag[j]];
  double* Dg = c.D + b.loff;
  for (int e = threadIdx.x; e < m * m; e += NT) A[e] = Dg[e];
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  for (int kk = 0; kk < m; ++kk) {
    if (threadIdx.x == 0) {
      const double piv = A[kk + kk * m];
      if (!(piv > 0.0)) {
        fail = 1;
        if (atomicCAS(&c.status[0], 0, j + 1) == 0) c.status_val[0] = piv;
      } else {
        A[kk + kk * m] = sqrt(piv);
      }
    }
    __syncthreads();
    if (fail) break;
    const double d = A[kk + kk * m];
    for (int i = kk + 1 + threadIdx.x; i < m; i += NT) A[i + kk * m] /= d;
    __syncthreads();
    const int nt = m - kk - 1;
    for (int e = threadIdx.x; e < nt * nt; e += NT) {
      const int i = kk + 1 + e % nt, jj = kk + 1 + e / nt;
      if (i >= jj) A[i + jj * m] -= A[i + kk * m] * A[jj + kk * m];
    }
    __syncthreads();
  }
  if (fail) return;
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int i = e % m, jj = e / m;
    Dg[e] = (i >= jj) ? A[e] : 0.0;
  }
  double* X = c.inv + c.leaf_inv_off[j];
  for (int cc = threadIdx.x; cc < m; cc += NT) {
    for (int i = 0; i < cc; ++i) X[i + cc * m] = 0.0;
    X[cc + cc * m] = 1.0 / A[cc + cc * m];
    for (int i = cc + 1; i < m; ++i) {
      double s = 0.0;
      for (int l = cc; l < i; ++l) s += A[i + l * m] * X[l + cc * m];
      X[i + cc * m] = -s / A[i + i * m];
    }
  }
}

// Column solve at leaf j: W_b[leaf rows] <- L_jj^{-1} W_b[leaf rows].
template <typename TS>
__global__ void __launch_bounds__(NT) k_trsm(DevCtx<TS> c, int j, const int32_t* ids) {
  __shared__ TS T[TILE * CH];
  const int bi = ids[blockIdx.x];
  const BlockDesc b = c.blocks[bi];
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const int ncol = block_cols(c, b, bi);
  const int64_t ldw = b.c1 - b.c0;
  TS* Ws = block_w(c, b) + (lo - b.c0);
  const double* X = c.inv + c.leaf_inv_off[j];
  for (int c0 = 0; c0 < ncol; c0 += CH) {
    const int nc = min(CH, ncol - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < nl * nc; e += NT) {
      const int a = e % nl, cc = e / nl;
      T[a + cc * TILE] = Ws[a + (int64_t)(c0 + cc) * ldw];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nl * nc; e += NT) {
      const int i = e % nl, cc = e / nl;
      double s = 0.0;
      for (int a = 0; a <= i; ++a) s += X[i + a * nl] * double(T[a + cc * TILE]);
      Ws[i + (int64_t)(c0 + cc) * ldw] = TS(s);
    }
  }
}

// Inner update at leaf j: W_b[rows of x] -= L_x[:, leaf j] W_b[leaf rows].
template <typename TS>
__global__ void __launch_bounds__(NT) k_inner(DevCtx<TS> c, int j, const InnerDesc* items) {
  __shared__ TS H[64 * TILE];
  __shared__ TS red[NT];
  const InnerDesc it = items[blockIdx.x];
  const BlockDesc b = c.blocks[it.b], x = c.blocks[it.x];
  const int lo = c.leaf_lo[j], hi = c.leaf_hi[j];
  const int ncol = block_cols(c, b, it.b);
  const int64_t ldw = b.c1 - b.c0;
  TS* Wb = block_w(c, b);
  const int rkx = x.kind == BK_LOWRANK ? c.rank[it.x] : 0;
  wg_piece_N_sub<TS, TS>(c, x, rkx, x.r0, x.r1, lo, hi, Wb + (lo - b.c0), ldw, ncol, Wb + (x.r0 - b.c0), ldw, H, red);
}

// One forward-substitution step: vout[leaf j] = L_jj^{-1} v[leaf j]; every
// block x in column j subtracts L_x[:, leaf j] vout[leaf j] from its rows.
template <typename TS>
__global__ void __launch_bounds__(NT) k_solve_step(DevCtx<TS> c, int j, const int32_t* ids, int n_ids, double* v,
                                                    double* vout) {
  __shared__ double t[TILE], vj[TILE];
  __shared__ double h[64];
  const int lo = c.leaf_lo[j], nl = c.leaf_hi[j] - lo;
  const double* X = c.inv + c.leaf_inv_off[j];
  for (int a = threadIdx.x; a < nl; a += NT) t[a] = v[lo + a];
  __syncthreads();
  for (int i = threadIdx.x; i < nl; i += NT) {
    double s = 0.0;
    for (int a = 0; a <= i; ++a) s += X[i + a * nl] * t[a];
    vj[i] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < nl; i += NT) vout[lo + i] = vj[i];
  if (n_ids == 0) return;
  const int bi = ids[blockIdx.x];
  const BlockDesc x = c.blocks[bi];
  const int64_t mx = x.r1 - x.r0, kx = x.c1 - x.c0;
  if (x.kind == BK_DENSE) {
    const TS* W = c.L + x.loff + (lo - x.c0);
    for (int i = threadIdx.x; i < mx; i += NT) {
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
    for (int i = threadIdx.x; i < mx; i += NT) {
      double s = 0.0;
      for (int l = 0; l < rk; ++l) s += double(U[i + l * mx]) * h[l];
      v[x.r0 + i] -= s;
    }
  }
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

__global__ void __launch_bounds__(NT) k_reduce_final(const double* partial, int nl, double* out) {
  __shared__ double sh[NT / 64];
  double a = 0.0, q = 0.0;
  for (int j = threadIdx.x; j < nl; j += NT) { a += partial[2 * j]; q += partial[2 * j + 1]; }
  a = block_sum<double>(a, sh);
  q = block_sum<double>(q, sh);
  if (threadIdx.x == 0) { out[0] = a; out[1] = q; }
}

// ------------------------------------------------------------ launchers -----
template <typename TS>
void launch_assemble(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, const MaternParams& mp, double eps,
                     hipStream_t st) {
  if (n_dense > 0) hipLaunchKernelGGL(k_assemble_dense<TS>, dim3(n_dense), dim3(NT), 0, st, c, mp);
  if (n_lowrank > 0) hipLaunchKernelGGL(k_aca<TS>, dim3(n_lowrank), dim3(NT), 0, st, c, n_dense, mp, TS(eps));
}

template <typename TS>
void launch_factor_step(const DevCtx<TS>& c, int32_t j, const StepLists& sl, double eps, hipStream_t st) {
  if (sl.n_ext_dense > 0) hipLaunchKernelGGL(k_ext_dense<TS>, dim3(sl.n_ext_dense), dim3(NT), 0, st, c, sl.ext_dense);
  if (sl.n_ext_lr > 0) {
    hipLaunchKernelGGL(k_sketch1<TS>, dim3(sl.n_ext_lr), dim3(NT), 0, st, c, sl.ext_lr, 0x9e3779b9u);
    hipLaunchKernelGGL(k_sketch_qr<TS>, dim3(sl.n_ext_lr), dim3(NT), 0, st, c, sl.ext_lr, TS(0.01 * eps));
    hipLaunchKernelGGL(k_sketch2<TS>, dim3(sl.n_ext_lr), dim3(NT), 0, st, c, sl.ext_lr, TS(eps));
  }
  hipLaunchKernelGGL(k_potrf<TS>, dim3(1), dim3(NT), 0, st, c, j);
  if (sl.n_active > 0) hipLaunchKernelGGL(k_trsm<TS>, dim3(sl.n_active), dim3(NT), 0, st, c, j, sl.active);
  if (sl.n_inner > 0) hipLaunchKernelGGL(k_inner<TS>, dim3(sl.n_inner), dim3(NT), 0, st, c, j, sl.inner);
}

template <typename TS>
void launch_solve_step(const DevCtx<TS>& c, int32_t j, const int32_t* active, int32_t n_active, double* v,
                       hipStream_t st) {
  // v holds [running right-hand side | solution]
  hipLaunchKernelGGL(k_solve_step<TS>, dim3(n_active > 0 ? n_active : 1), dim3(NT), 0, st, c, j, active, n_active, v,
                     v + c.n);
}

template <typename TS>
void launch_sample(const DevCtx<TS>& c, int32_t n_dense, int32_t n_lowrank, int32_t n_leaves, const int32_t* rowp_beg,
                   const int32_t* rowp, const double* w, double* h, double* y, hipStream_t st) {
  if (n_lowrank > 0) hipLaunchKernelGGL(k_sample_h<TS>, dim3(n_lowrank), dim3(NT), 0, st, c, n_dense, w, h);
  hipLaunchKernelGGL(k_sample_rows<TS>, dim3(n_leaves), dim3(NT), 0, st, c, n_dense, rowp_beg, rowp, w, h, y);
}

void launch_matern(const double* h, int64_t count, const MaternParams& mp, int precision, double* out,
                   hipStream_t st) {
  if (count <= 0) return;
  const dim3 g((unsigned)((count + NT - 1) / NT));
  if (precision == 0) hipLaunchKernelGGL(k_matern<double>, g, dim3(NT), 0, st, h, count, mp, out);
  else hipLaunchKernelGGL(k_matern<float>, g, dim3(NT), 0, st, h, count, mp, out);
}

void launch_gather_coords(const double* pts, const int32_t* perm, int32_t n, int32_t dim, double* coords,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_gather_coords, dim3((n + NT - 1) / NT), dim3(NT), 0, st, pts, perm, n, dim, coords);
}
void launch_gather(const double* z, const int32_t* perm, int32_t n, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3((n + NT - 1) / NT), dim3(NT), 0, st, z, perm, n, v);
}
void launch_scatter(const double* v, const int32_t* perm, int32_t n, double* z, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3((n + NT - 1) / NT), dim3(NT), 0, st, v, perm, n, z);
}
void launch_check_finite(const double* x, int64_t count, int32_t* flag, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((count + NT - 1) / NT)), dim3(NT), 0, st, x, count, flag);
}
void launch_reduce(const double* D, const int64_t* diag_off, const int32_t* leaf_lo, const int32_t* leaf_hi,
                   int32_t n_leaves, const double* v, int32_t n, double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_leaf, dim3(n_leaves), dim3(NT), 0, st, D, diag_off, leaf_lo, leaf_hi, v, partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(NT), 0, st, partial, n_leaves, out);
}

template void launch_assemble<double>(const DevCtx<double>&, int32_t, int32_t, const MaternParams&, double, hipStream_t);
template void launch_assemble<float>(const DevCtx<float>&, int32_t, int32_t, const MaternParams&, double, hipStream_t);
template void launch_factor_step<double>(const DevCtx<double>&, int32_t, const StepLists&, double, hipStream_t);
template void launch_factor_step<float>(const DevCtx<float>&, int32_t, const StepLists&, double, hipStream_t);
template void launch_sample<double>(const DevCtx<double>&, int32_t, int32_t, int32_t, const int32_t*, const int32_t*,
                                    const double*, double*, double*, hipStream_t);
template void launch_sample<float>(const DevCtx<float>&, int32_t, int32_t, int32_t, const int32_t*, const int32_t*,
                                   const double*, double*, double*, hipStream_t);
template void launch_solve_step<double>(const DevCtx<double>&, int32_t, const int32_t*, int32_t, double*, hipStream_t);
template void launch_solve_step<float>(const DevCtx<float>&, int32_t, const int32_t*, int32_t, double*, hipStream_t);

}  // namespace hmle
