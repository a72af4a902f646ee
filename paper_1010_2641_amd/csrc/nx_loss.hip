// nx_loss.hip -- intensity misfit and adjoint seed for fitting a model to measured
// intensities I:  e_k = |A_k|^2 - I_k,  L = sum_k e_k^2,  G_k = 4 e_k A_k.
//
// Memory-bound elementwise pass: e is formed in FP64 from the FP32 inputs (the
// squares of FP32 values are exact in FP64), G is rounded once to FP32, and L is
// reduced deterministically: each of a fixed number of work-groups sums a fixed
// grid-stride subset with a fixed tree, and one work-group then sums the partials
// in index order.
#include "nx_internal.h"

namespace nx {
namespace {

// Fixed-shape tree reduction of one double per thread over a 256-thread group.
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(kThreads) void loss_partial_kernel(const float2* __restrict__ A,
                                                                const float* __restrict__ I,
                                                                int64_t K, float2* __restrict__ G,
                                                                double* __restrict__ partial) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < K;
       k += int64_t(gridDim.x) * kThreads) {
    const float2 a = A[k];
    const double re = a.x, im = a.y;
    const double e = (re * re + im * im) - static_cast<double>(I[k]);
    acc += e * e;
    if (G) G[k] = make_float2(static_cast<float>(4.0 * e * re), static_cast<float>(4.0 * e * im));
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void loss_final_kernel(const double* __restrict__ partial,
                                                              int nb, double* __restrict__ L) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) acc += partial[b];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) L[0] = s;
}

// Small point counts: the whole misfit in one work-group of kSmallThreads (the same
// per-point arithmetic, each thread summing a fixed stride of points, then a fixed tree),
// one dispatch instead of two.
constexpr int kSmallThreads = 1024;

__global__ __launch_bounds__(kSmallThreads) void loss_small_kernel(const float2* __restrict__ A,
                                                                   const float* __restrict__ I,
                                                                   int64_t K, float2* __restrict__ G,
                                                                   double* __restrict__ L) {
  __shared__ double sh[kSmallThreads];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < K; k += kSmallThreads) {
    const float2 a = A[k];
    const double re = a.x, im = a.y;
    const double e = (re * re + im * im) - static_cast<double>(I[k]);
    acc += e * e;
    if (G) G[k] = make_float2(static_cast<float>(4.0 * e * re), static_cast<float>(4.0 * e * im));
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
#pragma unroll
  for (int w = kSmallThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) L[0] = sh[0];
}

}  // namespace

hipError_t launch_loss(const float* A, const float* I, int64_t K, double* L, float* G,
                       double* partial, hipStream_t st) {
  if (K <= kLossSmall) {
    loss_small_kernel<<<1, kSmallThreads, 0, st>>>(reinterpret_cast<const float2*>(A), I, K,
                                              reinterpret_cast<float2*>(G), L);
    return hipGetLastError();
  }
  int64_t nb = (K + kThreads - 1) / kThreads;
  if (nb < 1) nb = 1;
  if (nb > kLossBlocks) nb = kLossBlocks;
  loss_partial_kernel<<<static_cast<unsigned>(nb), kThreads, 0, st>>>(
      reinterpret_cast<const float2*>(A), I, K, reinterpret_cast<float2*>(G), partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  loss_final_kernel<<<1, kThreads, 0, st>>>(partial, static_cast<int>(nb), L);
  return hipGetLastError();
}

}  // namespace nx
