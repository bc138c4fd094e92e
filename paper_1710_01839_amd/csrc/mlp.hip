// Run-time model kernels: a F -> H -> H -> 1 perceptron (ReLU, FP32),
// forward, loss gradient and Adam.  Parameters are one flat FP32 array:
// W1 (H x F), b1 (H), W2 (H x H), b2 (H), W3 (H), b3 (1), row-major.
// Every reduction runs in a fixed order, so results are deterministic.
#include "mlp_internal.hpp"

namespace mpg {
namespace {

constexpr int H = kMlpHidden;

struct Offs {
  int W1, b1, W2, b2, W3, b3, P;
  __host__ __device__ explicit Offs(int F)
      : W1(0), b1(H * F), W2(H * F + H), b2(H * F + H + H * H), W3(H * F + 2 * H + H * H),
        b3(H * F + 3 * H + H * H), P(H * F + 3 * H + H * H + 1) {}
};

// wave64 butterfly sum (fixed order)
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One row per 64-thread workgroup; thread j owns hidden unit j.
__global__ __launch_bounds__(64) void mlp_forward_kernel(const float* __restrict__ prm,
                                                         const float* __restrict__ X, int rows,
                                                         int F, float* __restrict__ out) {
  __shared__ float h1[H];
  const int r = blockIdx.x, j = threadIdx.x;
  if (r >= rows) return;
  const Offs o(F);
  const float* x = X + (size_t)r * F;
  float z = prm[o.b1 + j];
  for (int f = 0; f < F; ++f) z += prm[o.W1 + j * F + f] * x[f];
  h1[j] = z > 0.f ? z : 0.f;
  __syncthreads();
  float z2 = prm[o.b2 + j];
  for (int i = 0; i < H; ++i) z2 += prm[o.W2 + j * H + i] * h1[i];
  const float h2 = z2 > 0.f ? z2 : 0.f;
  const float y = wave_sum(prm[o.W3 + j] * h2) + prm[o.b3];
  if (j == 0) out[r] = y;
}

// Gradient of mean((y - t)^2) over a chunk of rows.  Threads 0..63 run the
// forward and backward pass of one row at a time through LDS; all 256
// threads then add that row's contribution to the parameters they own
// (p = tid, tid + 256, ...).  partial[chunk][p] receives the chunk's sum;
// partial[chunk][P] the chunk's sum of squared residuals.
constexpr int kGradThreads = 256;
constexpr int kMaxOwned = 32;  // P <= 256 * 32
__global__ __launch_bounds__(kGradThreads) void mlp_grad_kernel(const float* __restrict__ prm,
                                                                const float* __restrict__ X,
                                                                const float* __restrict__ t,
                                                                int rows, int F, int chunk,
                                                                float* __restrict__ partial) {
  __shared__ float x_s[kMlpMaxFeatures], z1[H], h1[H], z2[H], h2[H], dz2[H], dz1[H];
  __shared__ float dy_s, res2_s;
  const Offs o(F);
  const int tid = threadIdx.x;
  float acc[kMaxOwned];
#pragma unroll
  for (int q = 0; q < kMaxOwned; ++q) acc[q] = 0.f;
  float loss = 0.f;
  const int r0 = blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
  for (int r = r0; r < r1; ++r) {
    if (tid < F) x_s[tid] = X[(size_t)r * F + tid];
    __syncthreads();
    if (tid < H) {
      float z = prm[o.b1 + tid];
      for (int f = 0; f < F; ++f) z += prm[o.W1 + tid * F + f] * x_s[f];
      z1[tid] = z;
      h1[tid] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    if (tid < H) {
      float z = prm[o.b2 + tid];
      for (int i = 0; i < H; ++i) z += prm[o.W2 + tid * H + i] * h1[i];
      z2[tid] = z;
      h2[tid] = z > 0.f ? z : 0.f;
      const float y = wave_sum(prm[o.W3 + tid] * h2[tid]) + prm[o.b3];
      if (tid == 0) {
        const float res = y - t[r];
        dy_s = 2.f * res / (float)rows;
        res2_s = res * res;
      }
    }
    __syncthreads();
    const float dy = dy_s;
    if (tid == 0) loss += res2_s;
    if (tid < H) dz2[tid] = z2[tid] > 0.f ? dy * prm[o.W3 + tid] : 0.f;
    __syncthreads();
    if (tid < H) {
      float d = 0.f;
      for (int j = 0; j < H; ++j) d += prm[o.W2 + j * H + tid] * dz2[j];
      dz1[tid] = z1[tid] > 0.f ? d : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxOwned; ++q) {
      const int p = tid + q * kGradThreads;
      if (p >= o.P) break;
      float g;
      if (p < o.b1) g = dz1[p / F] * x_s[p % F];
      else if (p < o.W2) g = dz1[p - o.b1];
      else if (p < o.b2) g = dz2[(p - o.W2) / H] * h1[(p - o.W2) % H];
      else if (p < o.W3) g = dz2[p - o.b2];
      else if (p < o.b3) g = dy * h2[p - o.W3];
      else g = dy;
      acc[q] += g;
    }
    __syncthreads();
  }
  float* dst = partial + (size_t)blockIdx.x * (o.P + 1);
#pragma unroll
  for (int q = 0; q < kMaxOwned; ++q) {
    const int p = tid + q * kGradThreads;
    if (p < o.P) dst[p] = acc[q];
  }
  if (tid == 0) dst[o.P] = loss;
}

// grad[p] = sum over chunks (in order) of partial[c][p]; grad[P] = mean
// squared residual.  losses (nullable) receives the loss at `epoch`.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partial,
                                                         int chunks, int P, int rows,
                                                         float* __restrict__ grad,
                                                         float* __restrict__ losses, int epoch) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > P) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += partial[(size_t)c * (P + 1) + p];
  if (p == P) {
    s /= (float)rows;
    if (losses) losses[epoch] = s;
  }
  grad[p] = s;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ prm,
                                                       const float* __restrict__ grad,
                                                       float* __restrict__ m, float* __restrict__ v,
                                                       int P, float lr, float b1, float b2,
                                                       float eps, float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  prm[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace

int mlp_num_params(int F) { return Offs(F).P; }

hipError_t launch_mlp_forward(const float* prm, const float* X, int rows, int F, float* out,
                              hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(rows), dim3(64), 0, s, prm, X, rows, F, out);
  return hipGetLastError();
}

int mlp_grad_chunks(int rows) { return (rows + kMlpChunk - 1) / kMlpChunk; }

hipError_t launch_mlp_grad(const float* prm, const float* X, const float* t, int rows, int F,
                           float* partial, float* grad, float* losses, int epoch, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int chunks = mlp_grad_chunks(rows);
  const int P = mlp_num_params(F);
  if (P > kGradThreads * kMaxOwned || F > kMlpMaxFeatures) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(chunks), dim3(kGradThreads), 0, s, prm, X, t, rows, F,
                     kMlpChunk, partial);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((P + 1 + 255) / 256), dim3(256), 0, s, partial,
                     chunks, P, rows, grad, losses, epoch);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* prm, const float* grad, float* m, float* v, int P, float lr,
                           int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((P + 255) / 256), dim3(256), 0, s, prm, grad, m, v, P,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace mpg
