// Learned starting point for the optimiser: empirical-variogram features of a
// field and the fully connected tanh network (the network family of Section 4,
// trained with Adam as in Section 6) that maps them to a parameter guess.
//
// Features: for the pairs i < j of the points used, bin b = floor(64 h) for
// pair distance h < 1/2; gamma_b = sum of (z_i - z_j)^2 / (2 count_b);
// feature b = log(max(gamma_b, 1e-30)) (0 for an empty bin), feature 32 =
// log(points used). The bin is the largest k with k^2 <= 4096 h^2, h^2
// formed without fused multiply-adds, so it is decided exactly.
//
// Network: 33 -> 128 -> 128 -> 128 -> 4, tanh hidden layers, linear output,
// y = x W^T + b per layer, float32. Inputs enter standardised, the outputs
// are standardised log(sigma2, range, nu, tau2); loss = mean squared error.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>

#include "common.hpp"
#include "learned.hpp"

namespace hmle {

namespace {

constexpr int VNT = 256;   // threads of a variogram workgroup
constexpr int VT = 128;    // points per tile side
constexpr int NB = 32;     // distance bins

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Squared distance with every product and sum rounded on its own.
__device__ __forceinline__ double pair_h2(const double* a, const double* b, int dim) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int k = 0; k < dim; ++k) {
    const double d = a[k] - b[k];
    s = s + d * d;
  }
  return s;
}

// Largest k with k^2 <= 4096 h2, or -1 when k >= 32 (distance >= 1/2).
__device__ __forceinline__ int pair_bin(double h2) {
  const double s = 4096.0 * h2;
  if (!(s < 1024.0)) return -1;
  int b = (int)sqrt(s);
  if ((double)(b + 1) * (double)(b + 1) <= s) ++b;
  if ((double)b * (double)b > s) --b;
  return b < NB ? b : -1;
}

// One tile (I, J), I <= J, of the pair triangle of problem blockIdx.y: per-bin
// sums and counts of its pairs into part[(q * max_tiles + tile) * 64 + ...].
// Each thread owns one row i and half of the tile's columns and keeps its 32
// bins in registers; the workgroup then reduces them in a fixed order.
__global__ void __launch_bounds__(VNT) k_variogram(const double* pts, const double* z, const int64_t* offs,
                                                   const int32_t* sel, const int64_t* soffs, int dim, int max_tiles,
                                                   double* part) {
  __shared__ double sp[VT * 3], sz[VT];
  __shared__ double wsum[VNT / 64][2 * NB];
  const int q = blockIdx.y;
  const int64_t base = offs[q];
  const int64_t m = sel ? soffs[q + 1] - soffs[q] : offs[q + 1] - offs[q];
  const int nt = (int)((m + VT - 1) / VT);
  int tile = blockIdx.x;
  if (tile >= nt * (nt + 1) / 2) return;
  int I = 0;
  while (tile >= nt - I) { tile -= nt - I; ++I; }
  const int J = I + tile;
  auto point = [&](int64_t local) -> int64_t { return base + (sel ? (int64_t)sel[soffs[q] + local] : local); };
  for (int a = threadIdx.x; a < VT; a += VNT) {
    const int64_t j = (int64_t)J * VT + a;
    if (j < m) {
      const int64_t g = point(j);
      for (int k = 0; k < dim; ++k) sp[a * 3 + k] = pts[g * dim + k];
      sz[a] = z[g];
    }
  }
  __syncthreads();
  double acc[NB], cnt[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) { acc[k] = 0.0; cnt[k] = 0.0; }
  const int64_t i = (int64_t)I * VT + (threadIdx.x & (VT - 1));
  if (i < m) {
    const int64_t g = point(i);
    double pi[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) pi[k] = pts[g * dim + k];
    const double zi = z[g];
    const int a0 = (threadIdx.x >> 7) * (VT / 2);
    for (int a = a0; a < a0 + VT / 2; ++a) {
      const int64_t j = (int64_t)J * VT + a;
      if (j >= m || (I == J && j <= i)) continue;
      const int b = pair_bin(pair_h2(pi, sp + a * 3, dim));
      if (b < 0) continue;
      const double d = zi - sz[a];
      const double d2 = d * d;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        acc[k] += (b == k) ? d2 : 0.0;
        cnt[k] += (b == k) ? 1.0 : 0.0;
      }
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const double s = wave_sum_d(acc[k]);
    const double c = wave_sum_d(cnt[k]);
    if (lane == 0) { wsum[w][k] = s; wsum[w][NB + k] = c; }
  }
  __syncthreads();
  if (threadIdx.x < 2 * NB) {
    double s = 0.0;
    for (int v = 0; v < VNT / 64; ++v) s += wsum[v][threadIdx.x];
    part[((int64_t)q * max_tiles + blockIdx.x) * 2 * NB + threadIdx.x] = s;
  }
}

// Features of problem blockIdx.x from its tiles' partial sums (tile order).
__global__ void __launch_bounds__(64) k_variogram_final(const int64_t* offs, const int64_t* soffs, const int32_t* sel,
                                                        int max_tiles, const double* part, float* out) {
  const int q = blockIdx.x;
  const int64_t m = sel ? soffs[q + 1] - soffs[q] : offs[q + 1] - offs[q];
  const int nt = (int)((m + VT - 1) / VT);
  const int ntiles = nt * (nt + 1) / 2;
  const int k = threadIdx.x;
  if (k < NB) {
    double s = 0.0, c = 0.0;
    for (int t = 0; t < ntiles; ++t) {
      s += part[((int64_t)q * max_tiles + t) * 2 * NB + k];
      c += part[((int64_t)q * max_tiles + t) * 2 * NB + NB + k];
    }
    out[(int64_t)q * N_FEAT + k] = c > 0.0 ? (float)log(fmax(s / (2.0 * c), 1e-30)) : 0.0f;
  } else if (k == NB) {
    out[(int64_t)q * N_FEAT + NB] = (float)log((double)m);
  }
}

// ------------------------------------------------------------- network -----
constexpr int MNT = 256;   // threads of a network workgroup
constexpr int MR = 64;     // rows per workgroup

// X0[r] = (x[idx ? idx[r] : r] - mu) / sd
__global__ void __launch_bounds__(MNT) k_mlp_input(const float* x, const int32_t* idx, int rows, const float* norm,
                                                   float* X0) {
  const int e = blockIdx.x * MNT + threadIdx.x;
  if (e >= rows * N_FEAT) return;
  const int r = e / N_FEAT, i = e % N_FEAT;
  const int64_t src = idx ? idx[r] : r;
  X0[e] = (x[src * N_FEAT + i] - norm[i]) / norm[N_FEAT + i];
}

// Y = act(X W^T + b) for MR rows per workgroup; X: rows x IN, W: OUT x IN.
template <int IN, int OUT, bool TANH>
__global__ void __launch_bounds__(MNT) k_mlp_fwd(const float* X, const float* W, const float* bias, float* Y,
                                                 int rows) {
  __shared__ float Xs[MR][IN + 1];
  __shared__ float Ws[OUT][IN + 1];
  const int r0 = blockIdx.x * MR;
  for (int e = threadIdx.x; e < MR * IN; e += MNT) {
    const int r = e / IN, i = e % IN;
    Xs[r][i] = (r0 + r < rows) ? X[(int64_t)(r0 + r) * IN + i] : 0.0f;
  }
  for (int e = threadIdx.x; e < OUT * IN; e += MNT) Ws[e / IN][e % IN] = W[e];
  __syncthreads();
  constexpr int PER = (OUT + 3) / 4;
  const int r = threadIdx.x & (MR - 1), cg = threadIdx.x >> 6;
  float acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int o = cg + 4 * k;
    acc[k] = (o < OUT) ? bias[o] : 0.0f;
  }
  for (int i = 0; i < IN; ++i) {
    const float xv = Xs[r][i];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int o = cg + 4 * k;
      if (o < OUT) acc[k] += xv * Ws[o][i];
    }
  }
  if (r0 + r < rows) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int o = cg + 4 * k;
      if (o < OUT) Y[(int64_t)(r0 + r) * OUT + o] = TANH ? tanhf(acc[k]) : acc[k];
    }
  }
}

// Output layer error: G = 2 (Y - t) / (rows * 4) with t the standardised log
// targets; loss[0] = mean squared error (one workgroup, fixed order).
__global__ void __launch_bounds__(MNT) k_mlp_loss(const float* Y, const float* lt, const int32_t* idx, int rows,
                                                  const float* norm, float* G, float* loss) {
  __shared__ float red[MNT / 64];
  const float* mu = norm + 2 * N_FEAT;
  const float* sd = mu + N_OUT;
  const float scale = 2.0f / (float)(rows * N_OUT);
  float s = 0.0f;
  for (int e = threadIdx.x; e < rows * N_OUT; e += MNT) {
    const int r = e / N_OUT, k = e % N_OUT;
    const int64_t src = idx ? idx[r] : r;
    const float t = (lt[src * N_OUT + k] - mu[k]) / sd[k];
    const float d = Y[e] - t;
    G[e] = scale * d;
    s += d * d;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int v = 0; v < MNT / 64; ++v) t += red[v];
    loss[0] = t / (float)(rows * N_OUT);
  }
}

// Error at the previous layer's activations:
// Gp[r][i] = (sum_o G[r][o] W[o][i]) * (1 - H[r][i]^2)   (H = tanh activations)
template <int IN, int OUT>
__global__ void __launch_bounds__(MNT) k_mlp_bwd_data(const float* G, const float* W, const float* H, float* Gp,
                                                      int rows) {
  __shared__ float Gs[MR][OUT + 1];
  __shared__ float Ws[OUT][IN + 1];
  const int r0 = blockIdx.x * MR;
  for (int e = threadIdx.x; e < MR * OUT; e += MNT) {
    const int r = e / OUT, o = e % OUT;
    Gs[r][o] = (r0 + r < rows) ? G[(int64_t)(r0 + r) * OUT + o] : 0.0f;
  }
  for (int e = threadIdx.x; e < OUT * IN; e += MNT) Ws[e / IN][e % IN] = W[e];
  __syncthreads();
  constexpr int PER = (IN + 3) / 4;
  const int r = threadIdx.x & (MR - 1), cg = threadIdx.x >> 6;
  float acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = 0.0f;
  for (int o = 0; o < OUT; ++o) {
    const float gv = Gs[r][o];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = cg + 4 * k;
      if (i < IN) acc[k] += gv * Ws[o][i];
    }
  }
  if (r0 + r < rows) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = cg + 4 * k;
      if (i < IN) {
        const float h = H[(int64_t)(r0 + r) * IN + i];
        Gp[(int64_t)(r0 + r) * IN + i] = acc[k] * (1.0f - h * h);
      }
    }
  }
}

// Weight and bias gradients of one layer, one output unit o per workgroup:
// gW[o][i] = sum_r G[r][o] X[r][i], gb[o] = sum_r G[r][o] (rows in order).
__global__ void __launch_bounds__(MNT) k_mlp_bwd_weight(const float* G, const float* X, int rows, int in, int out,
                                                        float* gW, float* gb) {
  const int o = blockIdx.x;
  const int i = threadIdx.x;
  if (i > in) return;
  float s = 0.0f;
  if (i < in) {
    for (int r = 0; r < rows; ++r) s += G[(int64_t)r * out + o] * X[(int64_t)r * in + i];
    gW[(int64_t)o * in + i] = s;
  } else {
    for (int r = 0; r < rows; ++r) s += G[(int64_t)r * out + o];
    gb[o] = s;
  }
}

// Predicted log parameters: out = Y * sd_y + mu_y.
__global__ void __launch_bounds__(MNT) k_mlp_output(const float* Y, const float* norm, int rows, float* out) {
  const int e = blockIdx.x * MNT + threadIdx.x;
  if (e >= rows * N_OUT) return;
  const int k = e % N_OUT;
  out[e] = Y[e] * norm[2 * N_FEAT + N_OUT + k] + norm[2 * N_FEAT + k];
}

// Adam (bias-corrected): c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void __launch_bounds__(MNT) k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float c1,
                                              float c2) {
  const int e = blockIdx.x * MNT + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = 0.9f * m[e] + 0.1f * gi;
  const float vi = 0.999f * v[e] + 0.001f * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// Column means and standard deviations (population) of a rows x cols float
// array, accumulated in float64; out[c], out[cols + c]. A column whose
// deviation is below 1e-6 gets the scale `flat` instead.
__global__ void __launch_bounds__(MNT) k_col_stats(const float* a, int64_t rows, int cols, float flat, float* out) {
  __shared__ double red[MNT / 64];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += MNT) s += a[r * cols + c];
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double mean = 0.0;
  for (int v = 0; v < MNT / 64; ++v) mean += red[v];
  mean /= (double)rows;
  __syncthreads();
  double q = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += MNT) {
    const double d = a[r * cols + c] - mean;
    q += d * d;
  }
  q = wave_sum_d(q);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int v = 0; v < MNT / 64; ++v) t += red[v];
    out[c] = (float)mean;
    const double sd = sqrt(t / (double)rows);
    out[cols + c] = sd < 1e-6 ? flat : (float)sd;
  }
}

}  // namespace

// ------------------------------------------------------------ launchers -----
void launch_variogram(const double* pts, const double* z, const int64_t* offs, const int32_t* sel,
                      const int64_t* soffs, int32_t count, int32_t dim, int32_t max_tiles, double* part, float* out,
                      hipStream_t st) {
  HMLE_LAUNCH(k_variogram, dim3(max_tiles, count), dim3(VNT), 0, st, pts, z, offs, sel, soffs, dim, max_tiles,
                     part);
  HMLE_LAUNCH(k_variogram_final, dim3(count), dim3(64), 0, st, offs, soffs, sel, max_tiles, part, out);
}

int32_t variogram_tiles(int64_t m) {
  const int64_t nt = (m + VT - 1) / VT;
  return (int32_t)(nt * (nt + 1) / 2);
}

// Fixed device workspace of the allocation-free variogram call: one array per
// GPU, alive until the process ends. Host code never passes the array's name
// to a kernel (on the host it is only a stand-in symbol): it looks up the
// array's device address once per device and uses that address.
static __device__ __align__(256) unsigned char scratch[VARIO_SCRATCH_BYTES];

hipError_t variogram_scratch(void** ptr) {
  static std::mutex mu;
  static std::map<int, void*> addr;   // device id -> address of that device's array
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = addr.emplace(dev, p).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

void launch_mlp_forward(const MlpBuffers& b, const float* x, const int32_t* idx, int32_t rows, hipStream_t st) {
  const int g = (rows + MR - 1) / MR;
  HMLE_LAUNCH(k_mlp_input, dim3((rows * N_FEAT + MNT - 1) / MNT), dim3(MNT), 0, st, x, idx, rows, b.norm, b.X0);
  HMLE_LAUNCH((k_mlp_fwd<N_FEAT, N_HID, true>), dim3(g), dim3(MNT), 0, st, b.X0, b.params + OFF_W1,
                     b.params + OFF_B1, b.H1, rows);
  HMLE_LAUNCH((k_mlp_fwd<N_HID, N_HID, true>), dim3(g), dim3(MNT), 0, st, b.H1, b.params + OFF_W2,
                     b.params + OFF_B2, b.H2, rows);
  HMLE_LAUNCH((k_mlp_fwd<N_HID, N_HID, true>), dim3(g), dim3(MNT), 0, st, b.H2, b.params + OFF_W3,
                     b.params + OFF_B3, b.H3, rows);
  HMLE_LAUNCH((k_mlp_fwd<N_HID, N_OUT, false>), dim3(g), dim3(MNT), 0, st, b.H3, b.params + OFF_W4,
                     b.params + OFF_B4, b.Y, rows);
}

void launch_mlp_backward(const MlpBuffers& b, const float* lt, const int32_t* idx, int32_t rows, hipStream_t st) {
  const int g = (rows + MR - 1) / MR;
  float* gr = b.grad;
  HMLE_LAUNCH(k_mlp_loss, dim3(1), dim3(MNT), 0, st, b.Y, lt, idx, rows, b.norm, b.G4, b.loss);
  HMLE_LAUNCH(k_mlp_bwd_weight, dim3(N_OUT), dim3(MNT), 0, st, b.G4, b.H3, rows, N_HID, N_OUT, gr + OFF_W4,
                     gr + OFF_B4);
  HMLE_LAUNCH((k_mlp_bwd_data<N_HID, N_OUT>), dim3(g), dim3(MNT), 0, st, b.G4, b.params + OFF_W4, b.H3, b.Ga,
                     rows);
  HMLE_LAUNCH(k_mlp_bwd_weight, dim3(N_HID), dim3(MNT), 0, st, b.Ga, b.H2, rows, N_HID, N_HID, gr + OFF_W3,
                     gr + OFF_B3);
  HMLE_LAUNCH((k_mlp_bwd_data<N_HID, N_HID>), dim3(g), dim3(MNT), 0, st, b.Ga, b.params + OFF_W3, b.H2, b.Gb,
                     rows);
  HMLE_LAUNCH(k_mlp_bwd_weight, dim3(N_HID), dim3(MNT), 0, st, b.Gb, b.H1, rows, N_HID, N_HID, gr + OFF_W2,
                     gr + OFF_B2);
  HMLE_LAUNCH((k_mlp_bwd_data<N_HID, N_HID>), dim3(g), dim3(MNT), 0, st, b.Gb, b.params + OFF_W2, b.H1, b.Ga,
                     rows);
  HMLE_LAUNCH(k_mlp_bwd_weight, dim3(N_HID), dim3(MNT), 0, st, b.Ga, b.X0, rows, N_FEAT, N_HID, gr + OFF_W1,
                     gr + OFF_B1);
}

void launch_mlp_output(const MlpBuffers& b, int32_t rows, float* out, hipStream_t st) {
  HMLE_LAUNCH(k_mlp_output, dim3((rows * N_OUT + MNT - 1) / MNT), dim3(MNT), 0, st, b.Y, b.norm, rows, out);
}

void launch_adam(const MlpBuffers& b, float lr, float c1, float c2, hipStream_t st) {
  HMLE_LAUNCH(k_adam, dim3((N_PARAMS + MNT - 1) / MNT), dim3(MNT), 0, st, b.params, b.grad, b.m, b.v,
                     (int)N_PARAMS, lr, c1, c2);
}

void launch_col_stats(const float* a, int64_t rows, int32_t cols, float flat, float* out, hipStream_t st) {
  HMLE_LAUNCH(k_col_stats, dim3(cols), dim3(MNT), 0, st, a, rows, cols, flat, out);
}

}  // namespace hmle
