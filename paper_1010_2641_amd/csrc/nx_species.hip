// nx_species.hip -- the per-point steps of the species-factorised sum.  Section 4.2 of
// Favre-Nicolin et al. (2010) groups the atoms of one type, evaluates
// sum_j exp(2 i pi S.r_j) per group, and multiplies each group sum by that type's
// scattering factor at S (which may depend on |S| and on the energy):
//     A_k = sum_s fs[s][k] * sum_{j in s} exp(2 i pi S_k . r_j).
// The group sums come from the forward kernel with f_j = 1 as (sum, comp) states; these
// kernels combine them (in FP64, rounded once), form the per-type adjoint seeds and the
// gradient with respect to the per-type factors.  All three are memory-bound elementwise
// passes over the points.
#include "nx_internal.h"

namespace nx {
namespace {

__global__ __launch_bounds__(kThreads) void species_combine_kernel(SpeciesStates ss,
                                                                   const float2* __restrict__ fs,
                                                                   int64_t K,
                                                                   float2* __restrict__ A,
                                                                   float2* __restrict__ As) {
  const int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (k >= K) return;
  double ar = 0.0, ai = 0.0;
  for (int s = 0; s < ss.n; ++s) {
    const float4* st = static_cast<const float4*>(ss.state[s]);
    double sr = 0.0, si = 0.0;
    for (int sp = 0; sp < ss.nsplit[s]; ++sp) {
      const float4 v = st[int64_t(sp) * K + k];
      sr += static_cast<double>(v.x) + static_cast<double>(v.z);
      si += static_cast<double>(v.y) + static_cast<double>(v.w);
    }
    if (As) As[int64_t(s) * K + k] = make_float2(static_cast<float>(sr), static_cast<float>(si));
    double fr = 1.0, fi = 0.0;
    if (fs) {
      const float2 f = fs[int64_t(s) * K + k];
      fr = f.x;
      fi = f.y;
    }
    ar += fr * sr - fi * si;
    ai += fr * si + fi * sr;
  }
  A[k] = make_float2(static_cast<float>(ar), static_cast<float>(ai));
}

__global__ __launch_bounds__(kThreads) void species_seed_kernel(const float2* __restrict__ G,
                                                                const float2* __restrict__ fs,
                                                                int64_t K,
                                                                float2* __restrict__ seed) {
  const int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (k >= K) return;
  const float2 g = G[k];
  if (!fs) {
    seed[k] = g;
    return;
  }
  const float2 f = fs[k];
  // G conj(f)
  const double gr = g.x, gi = g.y, fr = f.x, fi = f.y;
  seed[k] = make_float2(static_cast<float>(gr * fr + gi * fi), static_cast<float>(gi * fr - gr * fi));
}

__global__ __launch_bounds__(kThreads) void species_gradf_kernel(const float2* __restrict__ G,
                                                                 const float2* __restrict__ As,
                                                                 int64_t K,
                                                                 float2* __restrict__ out) {
  const int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (k >= K) return;
  // dL/dfs = G conj(A_s)
  const double gr = G[k].x, gi = G[k].y, ar = As[k].x, ai = As[k].y;
  out[k] = make_float2(static_cast<float>(gr * ar + gi * ai), static_cast<float>(gi * ar - gr * ai));
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_species_combine(const SpeciesStates& ss, const float* fs, int64_t k, float* A,
                                  float* A_species, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  species_combine_kernel<<<blocks_for(k), kThreads, 0, st>>>(
      ss, reinterpret_cast<const float2*>(fs), k, reinterpret_cast<float2*>(A),
      reinterpret_cast<float2*>(A_species));
  return hipGetLastError();
}

hipError_t launch_species_seed(const float* G, const float* fs_s, int64_t k, float* seed,
                               hipStream_t st) {
  if (k <= 0) return hipSuccess;
  species_seed_kernel<<<blocks_for(k), kThreads, 0, st>>>(
      reinterpret_cast<const float2*>(G), reinterpret_cast<const float2*>(fs_s), k,
      reinterpret_cast<float2*>(seed));
  return hipGetLastError();
}

hipError_t launch_species_gradf(const float* G, const float* A_s, int64_t k, float* grad_fs_s,
                                hipStream_t st) {
  if (k <= 0) return hipSuccess;
  species_gradf_kernel<<<blocks_for(k), kThreads, 0, st>>>(
      reinterpret_cast<const float2*>(G), reinterpret_cast<const float2*>(A_s), k,
      reinterpret_cast<float2*>(grad_fs_s));
  return hipGetLastError();
}

}  // namespace nx
