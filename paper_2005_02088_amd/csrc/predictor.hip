// Learned contention predictor: forward, backward (per-minibatch gradient) and Adam
// kernels for the MLP 16 -> 64 (ReLU) -> 64 (ReLU) -> 1, FP32.
//
// Parameter buffer: W1[16][64], b1[64], W2[64][64], b2[64], W3[64][1], b3[1]
// (weights [in, out]). Loss L = mean over the minibatch of (yhat - y)^2.
// The gradient kernel gives each workgroup 64 rows; it writes a partial gradient
// per workgroup, and the reduce kernel adds the partials in workgroup order, so
// results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace camelot {

constexpr int kPIn = CAMELOT_PRED_NIN, kPH = CAMELOT_PRED_NHID;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kPIn * kPH, kOffW2 = kOffB1 + kPH,
              kOffB2 = kOffW2 + kPH * kPH, kOffW3 = kOffB2 + kPH, kOffB3 = kOffW3 + kPH,
              kNParams = kOffB3 + 1;
static_assert(kNParams == CAMELOT_PRED_NPARAMS, "parameter layout");
constexpr int kPRows = 64;   // rows per workgroup

// yhat for m rows; one thread per row, parameters staged in LDS.
extern "C" __global__ __launch_bounds__(kThreads) void camelot_pred_forward(const float* params, const float* x,
                                                                          int m, float* yhat) {
  __shared__ float P[kNParams];
  for (int i = threadIdx.x; i < kNParams; i += kThreads) P[i] = params[i];
  __syncthreads();
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= m) return;
  float xi[kPIn];
#pragma unroll
  for (int k = 0; k < kPIn; ++k) xi[k] = x[(int64_t)r * kPIn + k];
  float h1[kPH];
  for (int j = 0; j < kPH; ++j) {
    float z = P[kOffB1 + j];
#pragma unroll
    for (int k = 0; k < kPIn; ++k) z = fmaf(xi[k], P[kOffW1 + k * kPH + j], z);
    h1[j] = fmaxf(z, 0.f);
  }
  float y = P[kOffB3];
  for (int j = 0; j < kPH; ++j) {
    float z = P[kOffB2 + j];
    for (int i = 0; i < kPH; ++i) z = fmaf(h1[i], P[kOffW2 + i * kPH + j], z);
    y = fmaf(fmaxf(z, 0.f), P[kOffW3 + j], y);
  }
  yhat[r] = y;
}

// Partial gradient of workgroup g over rows [64 g, 64 g + 64) of the minibatch
// (row r of the minibatch is x[idx[r]] when idx != nullptr). partial: [nwg][kNParams + 1],
// the extra slot holds the partial sum of squared errors.
extern "C" __global__ __launch_bounds__(kThreads) void camelot_pred_grad_partial(
    const float* params, const float* x, const float* y, const int32_t* idx, int m, float* partial) {
  __shared__ float P[kNParams];
  __shared__ float X[kPRows][kPIn];
  __shared__ float Z1[kPRows][kPH];
  __shared__ float Z2[kPRows][kPH];
  __shared__ float D2[kPRows][kPH];
  __shared__ float D1[kPRows][kPH];
  __shared__ float DY[kPRows];
  __shared__ float SE[kPRows];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * kPRows;
  const int nr = min(kPRows, m - r0);
  float* G = partial + (int64_t)blockIdx.x * (kNParams + 1);
  for (int i = tid; i < kNParams; i += kThreads) P[i] = params[i];
  for (int i = tid; i < kPRows * kPIn; i += kThreads) {
    const int r = i / kPIn, k = i - r * kPIn;
    float v = 0.f;
    if (r < nr) {
      const int64_t src = idx ? (int64_t)idx[r0 + r] : (int64_t)(r0 + r);
      v = x[src * kPIn + k];
    }
    X[r][k] = v;
  }
  __syncthreads();
  // z1 = X W1 + b1
  for (int i = tid; i < kPRows * kPH; i += kThreads) {
    const int r = i / kPH, j = i - r * kPH;
    float z = P[kOffB1 + j];
#pragma unroll
    for (int k = 0; k < kPIn; ++k) z = fmaf(X[r][k], P[kOffW1 + k * kPH + j], z);
    Z1[r][j] = z;
  }
  __syncthreads();
  // z2 = relu(z1) W2 + b2
  for (int i = tid; i < kPRows * kPH; i += kThreads) {
    const int r = i / kPH, j = i - r * kPH;
    float z = P[kOffB2 + j];
    for (int q = 0; q < kPH; ++q) z = fmaf(fmaxf(Z1[r][q], 0.f), P[kOffW2 + q * kPH + j], z);
    Z2[r][j] = z;
  }
  __syncthreads();
  // yhat, dL/dyhat = 2 (yhat - y) / m
  if (tid < kPRows) {
    const int r = tid;
    float dy = 0.f, se = 0.f;
    if (r < nr) {
      float yh = P[kOffB3];
      for (int j = 0; j < kPH; ++j) yh = fmaf(fmaxf(Z2[r][j], 0.f), P[kOffW3 + j], yh);
      const int64_t src = idx ? (int64_t)idx[r0 + r] : (int64_t)(r0 + r);
      const float e = yh - y[src];
      dy = 2.f * e / (float)m;
      se = e * e;
    }
    DY[r] = dy;
    SE[r] = se;
  }
  __syncthreads();
  // dz2 = dy w3^T * (z2 > 0)
  for (int i = tid; i < kPRows * kPH; i += kThreads) {
    const int r = i / kPH, j = i - r * kPH;
    D2[r][j] = Z2[r][j] > 0.f ? DY[r] * P[kOffW3 + j] : 0.f;
  }
  __syncthreads();
  // dz1 = dz2 W2^T * (z1 > 0)
  for (int i = tid; i < kPRows * kPH; i += kThreads) {
    const int r = i / kPH, q = i - r * kPH;
    float s = 0.f;
    for (int j = 0; j < kPH; ++j) s = fmaf(D2[r][j], P[kOffW2 + q * kPH + j], s);
    D1[r][q] = Z1[r][q] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // parameter gradients (sums over this workgroup's rows, in row order)
  for (int p = tid; p < kNParams + 1; p += kThreads) {
    float g = 0.f;
    if (p < kOffB1) {                       // W1[k][j]
      const int k = p / kPH, j = p - k * kPH;
      for (int r = 0; r < kPRows; ++r) g = fmaf(X[r][k], D1[r][j], g);
    } else if (p < kOffW2) {                // b1[j]
      const int j = p - kOffB1;
      for (int r = 0; r < kPRows; ++r) g += D1[r][j];
    } else if (p < kOffB2) {                // W2[q][j]
      const int q = (p - kOffW2) / kPH, j = (p - kOffW2) - q * kPH;
      for (int r = 0; r < kPRows; ++r) g = fmaf(fmaxf(Z1[r][q], 0.f), D2[r][j], g);
    } else if (p < kOffW3) {                // b2[j]
      const int j = p - kOffB2;
      for (int r = 0; r < kPRows; ++r) g += D2[r][j];
    } else if (p < kOffB3) {                // W3[j]
      const int j = p - kOffW3;
      for (int r = 0; r < kPRows; ++r) g = fmaf(fmaxf(Z2[r][j], 0.f), DY[r], g);
    } else if (p == kOffB3) {               // b3
      for (int r = 0; r < kPRows; ++r) g += DY[r];
    } else {                                // squared-error sum
      for (int r = 0; r < kPRows; ++r) g += SE[r];
    }
    G[p] = g;
  }
}

// grad[p] = sum over workgroups (in order) of partial[g][p]; loss = SE sum / m.
extern "C" __global__ __launch_bounds__(kThreads) void camelot_pred_grad_reduce(const float* partial, int nwg,
                                                                              int m, float* grad,
                                                                              float* loss) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p > kNParams) return;
  float s = 0.f;
  for (int g = 0; g < nwg; ++g) s += partial[(int64_t)g * (kNParams + 1) + p];
  if (p < kNParams) grad[p] = s;
  else if (loss) *loss = s / (float)m;
}

// Adam (Kingma & Ba): bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t from the host.
extern "C" __global__ __launch_bounds__(kThreads) void camelot_pred_adam(float* params, const float* grad,
                                                                       float* m1, float* m2, float lr,
                                                                       float c1, float c2) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= kNParams) return;
  const float g = grad[p];
  const float a = 0.9f * m1[p] + 0.1f * g;
  const float b = 0.999f * m2[p] + 0.001f * g * g;
  m1[p] = a;
  m2[p] = b;
  const float mh = a / c1, vh = b / c2;
  params[p] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

}  // namespace camelot
