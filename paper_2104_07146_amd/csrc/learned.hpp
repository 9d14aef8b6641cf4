// Launch interface of the learned-start kernels (variogram features and the
// start-proposal network).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hmle {

constexpr int N_FEAT = 33;    // 32 variogram bins + log(points used)
constexpr int N_HID = 128;
constexpr int N_OUT = 4;      // standardised log(sigma2, range, nu, tau2)
// flat parameter layout: W1 (128 x 33), b1, W2 (128 x 128), b2, W3, b3, W4 (4 x 128), b4
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = OFF_W1 + N_HID * N_FEAT;
constexpr int64_t OFF_W2 = OFF_B1 + N_HID;
constexpr int64_t OFF_B2 = OFF_W2 + N_HID * N_HID;
constexpr int64_t OFF_W3 = OFF_B2 + N_HID;
constexpr int64_t OFF_B3 = OFF_W3 + N_HID * N_HID;
constexpr int64_t OFF_W4 = OFF_B3 + N_HID;
constexpr int64_t OFF_B4 = OFF_W4 + N_OUT * N_HID;
constexpr int64_t N_PARAMS = OFF_B4 + N_OUT;
constexpr int N_NORM = 2 * N_FEAT + 2 * N_OUT;   // mu_x, sd_x, mu_y, sd_y

// Device buffers of a network (weights, Adam moments, gradient, activations
// for up to `cap` rows).
struct MlpBuffers {
  float *params, *m, *v, *grad, *norm, *loss;
  float *X0, *H1, *H2, *H3, *Y, *G4, *Ga, *Gb;
  int32_t cap;
};

// part: count * max_tiles * 64 doubles of scratch; out: count * 33 floats.
void launch_variogram(const double* pts, const double* z, const int64_t* offs, const int32_t* sel,
                      const int64_t* soffs, int32_t count, int32_t dim, int32_t max_tiles, double* part, float* out,
                      hipStream_t st);
int32_t variogram_tiles(int64_t m);   // pair tiles of m points
// Size of the fixed device workspace of hmle_variogram_noalloc, and its
// address on the current device (looked up once per device, then cached).
constexpr size_t VARIO_SCRATCH_BYTES = (size_t)16 << 20;
hipError_t variogram_scratch(void** ptr);
// forward pass of `rows` rows x[idx[r]] (idx may be NULL: rows 0..rows-1); outputs in b.Y
void launch_mlp_forward(const MlpBuffers& b, const float* x, const int32_t* idx, int32_t rows, hipStream_t st);
// loss of b.Y against log targets lt[idx[r]] and the gradient of every parameter into b.grad
void launch_mlp_backward(const MlpBuffers& b, const float* lt, const int32_t* idx, int32_t rows, hipStream_t st);
// de-standardised outputs (log parameters) of the last forward pass
void launch_mlp_output(const MlpBuffers& b, int32_t rows, float* out, hipStream_t st);
void launch_adam(const MlpBuffers& b, float lr, float c1, float c2, hipStream_t st);
void launch_col_stats(const float* a, int64_t rows, int32_t cols, float flat, float* out, hipStream_t st);

}  // namespace hmle
