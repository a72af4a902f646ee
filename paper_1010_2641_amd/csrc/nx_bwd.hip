// nx_bwd.hip -- adjoint of the direct scattering sum with respect to the atom
// positions.  For a real loss L(A) with seed G_k = dL/dRe A_k + i dL/dIm A_k, the
// chain rule through Eq. 2 of Favre-Nicolin et al. (2010) gives
//     dL/dr_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k . r_j)
//             = -2 pi sum_k S_k v_jk,   v_jk = Im( f_j conj(G_k) exp(2 i pi S_k . r_j) )
// so each atom carries three real sums (one per coordinate).  In the FP64-phase mode
// the seed is taken in polar form, conj(G_k) = |G_k| exp(2 i pi delta_k): delta_k
// joins the FP64 phase and |G_k| is folded into S_k, so that
//     v_jk = |G_k| Im( f_j exp(2 i pi (S_k . r_j + delta_k)) ) = |G_k| (fr s + fi c)
// costs two FP32 operations (none for f_j = 1) on top of the phase and sin/cos.
//
// Layout: every lane owns Q atoms and keeps their position and the T sums in
// registers; the points are streamed as packed wave-uniform records through the
// scalar load path (the paper's alternative of parallelising over atoms and sharing
// the reflection coordinates, Section 2.2).  The phases are recomputed, never stored.
//
// Per (point, atom) pair, FP64-phase mode: FP64 phase and reduction (as in the
// forward) with delta_k, FP32 v_sin/v_cos, T_d += (|G_k| S_kd) v with FP32 fma into
// per-group partials folded into (sum, comp) pairs by an error-free two-sum every GRP
// points.
// FP32 mode: the paper's FP32 arithmetic with plain sums.
#include "nx_internal.h"

namespace nx {
namespace {

__device__ __forceinline__ void two_sum_acc(float& s, float& c, float g) {
  const float t = s + g;
  const float bp = t - s;
  const float ap = t - bp;
  c += (s - ap) + (g - bp);
  s = t;
}

template <int MODE> struct PointOf;
template <> struct PointOf<kF32> { using type = PointF32; };
template <> struct PointOf<kPH64> { using type = PointPH; };

constexpr float kTwoPi = 6.283185307179586f;

// v = Im(f conj(G) (c + i s)) for the lane's atom; f = 1 when FK == 0.
//   conj(G) (c + i s) = (gr c + gi s) + i (gr s - gi c)
template <int FK>
__device__ __forceinline__ float adj_weight(float gr, float gi, float fr, float fi, float c,
                                            float s) {
  const float wim = __builtin_fmaf(-gi, c, gr * s);
  if constexpr (FK == 0) {
    return wim;
  } else {
    const float wre = __builtin_fmaf(gi, s, gr * c);
    return __builtin_fmaf(fi, wre, fr * wim);
  }
}

// One FP64-phase point record as three 16-byte words (the wave-uniform address lets
// the compiler fetch them with scalar loads), unpacked into named fields.
struct PtRegs { double sx, sy, sz, delta; float gsx, gsy, gsz; };

__device__ __forceinline__ PtRegs load_point(const PointPH* __restrict__ rec, int k) {
  const uint4* w = reinterpret_cast<const uint4*>(rec + k);
  const uint4 a = w[0], b = w[1], c = w[2];
  PtRegs r;
  r.sx = __hiloint2double(static_cast<int>(a.y), static_cast<int>(a.x));
  r.sy = __hiloint2double(static_cast<int>(a.w), static_cast<int>(a.z));
  r.sz = __hiloint2double(static_cast<int>(b.y), static_cast<int>(b.x));
  r.delta = __hiloint2double(static_cast<int>(b.w), static_cast<int>(b.z));
  r.gsx = __uint_as_float(c.x);
  r.gsy = __uint_as_float(c.y);
  r.gsz = __uint_as_float(c.z);
  return r;
}

// (c, s) of exp(2 i pi psi), psi = S.r + delta (delta includes the 1/2 of RED == 1).
// The seed phase enters as the addend of the first fma: with delta copied once per point
// into a VGPR pair (shared by the lane's Q atoms), each pair saves an FP64 add.
template <int RED>
__device__ __forceinline__ void cis_ph64_pt(const PtRegs& a, double dv, double x, double y,
                                            double z, float& c, float& s) {
  const double ph = __builtin_fma(a.sz, z, __builtin_fma(a.sy, y, __builtin_fma(a.sx, x, dv)));
  float tf;
  if constexpr (RED == 0) tf = static_cast<float>(ph - __builtin_rint(ph));
  else tf = static_cast<float>(__builtin_amdgcn_fract(ph));
  c = __builtin_amdgcn_cosf(tf);
  s = __builtin_amdgcn_sinf(tf);
}

// v / |G| = Im(f (c + i s)) = fr s + fi c; s for f = 1.
template <int FK>
__device__ __forceinline__ float adj_im(float fr, float fi, float c, float s) {
  if constexpr (FK == 0) return s;
  else return __builtin_fmaf(fi, c, fr * s);
}

// Adjoint over points [k_begin + sp*per_split, ...) for Q atoms per lane.
// Grid: blocks_n * nsplit; blockIdx = sp * blocks_n + nb.
// part layout: [sp][coordinate][sum | comp][N] floats.
template <int MODE, int Q, int FK, int GRP, int RED>
__global__ __launch_bounds__(kThreads) void bwd_kernel(
    const typename PointOf<MODE>::type* __restrict__ rec, int k_begin, int k_end, int per_split,
    const float* __restrict__ xyz, const float* __restrict__ f, int64_t N, int blocks_n,
    float* __restrict__ part, float* __restrict__ grad, int carry_in, int direct) {
  using RReg = typename std::conditional<MODE == kPH64, double, float>::type;
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int nb = lb % blocks_n;
  const int sp = lb / blocks_n;
  const int64_t j0 = int64_t(nb) * (kThreads * Q) + threadIdx.x;

  RReg x[Q], y[Q], z[Q];
  float fr[Q], fi[Q];
  float sum[Q][3], cmp[Q][3];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    const int64_t jj = j < N ? j : N - 1;
    x[q] = static_cast<RReg>(xyz[3 * jj]);
    y[q] = static_cast<RReg>(xyz[3 * jj + 1]);
    z[q] = static_cast<RReg>(xyz[3 * jj + 2]);
    fr[q] = (FK && f) ? f[2 * jj] : 1.f;
    fi[q] = (FK && f) ? f[2 * jj + 1] : 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (carry_in && j < N) {
        sum[q][d] = part[((int64_t(sp) * 3 + d) * 2 + 0) * N + j];
        cmp[q][d] = part[((int64_t(sp) * 3 + d) * 2 + 1) * N + j];
      } else {
        sum[q][d] = 0.f;
        cmp[q][d] = 0.f;
      }
    }
  }

  const int k0 = k_begin + sp * per_split;
  const int k1 = min(k0 + per_split, k_end);

  if constexpr (MODE == kF32) {
    // the paper's FP32 arithmetic with plain running sums
    for (int k = k0; k < k1; ++k) {
      const PointF32 a = rec[k];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const float ph = __builtin_fmaf(a.sz, z[q], __builtin_fmaf(a.sy, y[q], a.sx * x[q]));
        const float u = __builtin_amdgcn_fractf(ph);
        const float c = __builtin_amdgcn_cosf(u);
        const float s = __builtin_amdgcn_sinf(u);
        const float v = adj_weight<FK>(a.gr, a.gi, fr[q], fi[q], c, s);
        sum[q][0] = __builtin_fmaf(v, a.sx, sum[q][0]);
        sum[q][1] = __builtin_fmaf(v, a.sy, sum[q][1]);
        sum[q][2] = __builtin_fmaf(v, a.sz, sum[q][2]);
      }
    }
  } else {
    // sign of the RED == 1 terms, applied once per group (see cis_ph64_pt)
    constexpr float SGN = (RED == 1) ? -1.f : 1.f;
    int k = k0;
    while (k < k1) {
      const int kend = (k + GRP <= k1) ? k + GRP : k1;
      float g[Q][3];
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[q][d] = 0.f;
      if (kend - k == GRP) {
#pragma unroll
        for (int u = 0; u < GRP; ++u) {
          const PtRegs a = load_point(rec, k + u);
          const double dv = a.delta;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            float c, s;
            cis_ph64_pt<RED>(a, dv, x[q], y[q], z[q], c, s);
            const float v = adj_im<FK>(fr[q], fi[q], c, s);
            g[q][0] = __builtin_fmaf(v, a.gsx, g[q][0]);
            g[q][1] = __builtin_fmaf(v, a.gsy, g[q][1]);
            g[q][2] = __builtin_fmaf(v, a.gsz, g[q][2]);
          }
        }
      } else {
        for (int kk = k; kk < kend; ++kk) {
          const PtRegs a = load_point(rec, kk);
          const double dv = a.delta;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            float c, s;
            cis_ph64_pt<RED>(a, dv, x[q], y[q], z[q], c, s);
            const float v = adj_im<FK>(fr[q], fi[q], c, s);
            g[q][0] = __builtin_fmaf(v, a.gsx, g[q][0]);
            g[q][1] = __builtin_fmaf(v, a.gsy, g[q][1]);
            g[q][2] = __builtin_fmaf(v, a.gsz, g[q][2]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int d = 0; d < 3; ++d) two_sum_acc(sum[q][d], cmp[q][d], SGN * g[q][d]);
      k = kend;
    }
  }

#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    if (j < N) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (direct) {
          grad[3 * j + d] = -kTwoPi * (sum[q][d] + cmp[q][d]);
        } else {
          part[((int64_t(sp) * 3 + d) * 2 + 0) * N + j] = sum[q][d];
          part[((int64_t(sp) * 3 + d) * 2 + 1) * N + j] = cmp[q][d];
        }
      }
    }
  }
}

// All-FP64 adjoint.  part layout: [sp][coordinate][N] doubles.
template <int Q, int FK>
__global__ __launch_bounds__(kThreads) void bwd_f64_kernel(
    const PointF64* __restrict__ rec, int k_begin, int k_end, int per_split,
    const double* __restrict__ xyz, const double* __restrict__ f, int64_t N, int blocks_n,
    double* __restrict__ part, double* __restrict__ grad, int carry_in, int direct) {
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int nb = lb % blocks_n;
  const int sp = lb / blocks_n;
  const int64_t j0 = int64_t(nb) * (kThreads * Q) + threadIdx.x;
  double x[Q], y[Q], z[Q], fr[Q], fi[Q], T[Q][3];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    const int64_t jj = j < N ? j : N - 1;
    x[q] = xyz[3 * jj]; y[q] = xyz[3 * jj + 1]; z[q] = xyz[3 * jj + 2];
    fr[q] = (FK && f) ? f[2 * jj] : 1.0;
    fi[q] = (FK && f) ? f[2 * jj + 1] : 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      T[q][d] = (carry_in && j < N) ? part[(int64_t(sp) * 3 + d) * N + j] : 0.0;
  }
  const int k0 = k_begin + sp * per_split;
  const int k1 = min(k0 + per_split, k_end);
  for (int k = k0; k < k1; ++k) {
    const PointF64 a = rec[k];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double ph = __builtin_fma(a.sz, z[q], __builtin_fma(a.sy, y[q], a.sx * x[q]));
      const double t = ph - __builtin_rint(ph);
      double s, c;
      sincospi(2.0 * t, &s, &c);
      double v = __builtin_fma(-a.gi, c, a.gr * s);                  // Im conj(G) e^{i theta}
      if constexpr (FK) v = __builtin_fma(fi[q], __builtin_fma(a.gi, s, a.gr * c), fr[q] * v);
      T[q][0] = __builtin_fma(v, a.sx, T[q][0]);
      T[q][1] = __builtin_fma(v, a.sy, T[q][1]);
      T[q][2] = __builtin_fma(v, a.sz, T[q][2]);
    }
  }
  constexpr double kTwoPiD = 6.283185307179586476925286766559;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    if (j < N) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (direct) grad[3 * j + d] = -kTwoPiD * T[q][d];
        else part[(int64_t(sp) * 3 + d) * N + j] = T[q][d];
      }
    }
  }
}

// Combine the split partials of every atom in split order, then grad = -2 pi T.
__global__ __launch_bounds__(kThreads) void bwd_reduce_kernel(const float* __restrict__ part,
                                                              int nsplit, int64_t N,
                                                              float* __restrict__ grad) {
  const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (j >= N) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float s = 0.f, cm = 0.f;
    for (int sp = 0; sp < nsplit; ++sp) {
      two_sum_acc(s, cm, part[((int64_t(sp) * 3 + d) * 2 + 0) * N + j]);
      cm += part[((int64_t(sp) * 3 + d) * 2 + 1) * N + j];
    }
    grad[3 * j + d] = -kTwoPi * (s + cm);
  }
}

__global__ __launch_bounds__(kThreads) void bwd_reduce_f64_kernel(const double* __restrict__ part,
                                                                  int nsplit, int64_t N,
                                                                  double* __restrict__ grad) {
  const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (j >= N) return;
  constexpr double kTwoPiD = 6.283185307179586476925286766559;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += part[(int64_t(sp) * 3 + d) * N + j];
    grad[3 * j + d] = -kTwoPiD * s;
  }
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void pack_points_kernel(const void* __restrict__ S_v,
                                                               const void* __restrict__ G_v,
                                                               int64_t n, void* __restrict__ rec_v,
                                                               double offset) {
  for (int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * kThreads) {
    if constexpr (MODE == kF64) {
      const double* S = static_cast<const double*>(S_v);
      const double* G = static_cast<const double*>(G_v);
      PointF64 r;
      r.sx = S[3 * k]; r.sy = S[3 * k + 1]; r.sz = S[3 * k + 2];
      r.gr = G[2 * k]; r.gi = G[2 * k + 1]; r.pad = 0.0;
      static_cast<PointF64*>(rec_v)[k] = r;
    } else {
      const float* S = static_cast<const float*>(S_v);
      const float* G = static_cast<const float*>(G_v);
      if constexpr (MODE == kPH64) {
        // conj(G) = |G| exp(2 i pi delta): delta = -arg(G) / (2 pi) in FP64 (plus the
        // reduction offset of the variant), |G| S rounded once to FP32
        PointPH r;
        const double sx = S[3 * k], sy = S[3 * k + 1], sz = S[3 * k + 2];
        const double gr = G[2 * k], gi = G[2 * k + 1];
        const double m = sqrt(gr * gr + gi * gi);
        r.sx = sx; r.sy = sy; r.sz = sz;
        r.delta = -atan2(gi, gr) * 0.15915494309189533577 + offset;
        r.gsx = static_cast<float>(m * sx);
        r.gsy = static_cast<float>(m * sy);
        r.gsz = static_cast<float>(m * sz);
        r.pad = 0.f;
        static_cast<PointPH*>(rec_v)[k] = r;
      } else {
        PointF32 r;
        r.sx = S[3 * k]; r.sy = S[3 * k + 1]; r.sz = S[3 * k + 2];
        r.gr = G[2 * k]; r.gi = G[2 * k + 1];
        r.pad0 = r.pad1 = r.pad2 = 0.f;
        static_cast<PointF32*>(rec_v)[k] = r;
      }
    }
  }
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<unsigned>(b);
}

template <int MODE, int Q, int FK>
hipError_t bwd_dispatch(const Plan& p, const void* rec, int64_t k_begin, int64_t k_end,
                        int64_t per_split, const void* xyz, const void* f, void* partial,
                        void* grad, int carry_in, int direct, hipStream_t st) {
  using PT = typename PointOf<MODE>::type;
  const dim3 grid(static_cast<unsigned>(p.blocks * p.nsplit));
  const auto* r = static_cast<const PT*>(rec);
  const auto* x = static_cast<const float*>(xyz);
  const auto* ff = static_cast<const float*>(f);
  auto* pa = static_cast<float*>(partial);
  auto* g = static_cast<float*>(grad);
  if constexpr (MODE == kF32) {
    bwd_kernel<MODE, Q, FK, 16, 0><<<grid, kThreads, 0, st>>>(
        r, int(k_begin), int(k_end), int(per_split), x, ff, p.lanes, int(p.blocks), pa, g, carry_in, direct);
  } else {
    if (p.grp == 16 && p.red == 0)
      bwd_kernel<MODE, Q, FK, 16, 0><<<grid, kThreads, 0, st>>>(
          r, int(k_begin), int(k_end), int(per_split), x, ff, p.lanes, int(p.blocks), pa, g, carry_in, direct);
    else if (p.grp == 16)
      bwd_kernel<MODE, Q, FK, 16, 1><<<grid, kThreads, 0, st>>>(
          r, int(k_begin), int(k_end), int(per_split), x, ff, p.lanes, int(p.blocks), pa, g, carry_in, direct);
    else if (p.red == 0)
      bwd_kernel<MODE, Q, FK, 32, 0><<<grid, kThreads, 0, st>>>(
          r, int(k_begin), int(k_end), int(per_split), x, ff, p.lanes, int(p.blocks), pa, g, carry_in, direct);
    else
      bwd_kernel<MODE, Q, FK, 32, 1><<<grid, kThreads, 0, st>>>(
          r, int(k_begin), int(k_end), int(per_split), x, ff, p.lanes, int(p.blocks), pa, g, carry_in, direct);
  }
  return hipGetLastError();
}

template <int MODE>
hipError_t bwd_dispatch_q(const Plan& p, const void* rec, int64_t k_begin, int64_t k_end,
                          int64_t per_split, const void* xyz, const void* f, void* partial,
                          void* grad, int carry_in, int direct, hipStream_t st) {
  if (p.per_lane == 4)
    return p.fk ? bwd_dispatch<MODE, 4, 1>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st)
                : bwd_dispatch<MODE, 4, 0>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st);
  if (p.per_lane == 2)
    return p.fk ? bwd_dispatch<MODE, 2, 1>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st)
                : bwd_dispatch<MODE, 2, 0>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st);
  return p.fk ? bwd_dispatch<MODE, 1, 1>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st)
              : bwd_dispatch<MODE, 1, 0>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st);
}

template <int Q, int FK>
hipError_t bwd_f64_launch(const Plan& p, const void* rec, int64_t k_begin, int64_t k_end,
                          int64_t per_split, const void* xyz, const void* f, void* partial,
                          void* grad, int carry_in, int direct, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(p.blocks * p.nsplit));
  bwd_f64_kernel<Q, FK><<<grid, kThreads, 0, st>>>(
      static_cast<const PointF64*>(rec), int(k_begin), int(k_end), int(per_split),
      static_cast<const double*>(xyz), static_cast<const double*>(f), p.lanes, int(p.blocks),
      static_cast<double*>(partial), static_cast<double*>(grad), carry_in, direct);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pack_points(int mode, int red, const void* S, const void* G, int64_t k,
                              void* rec, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  const unsigned g = grid_for(k);
  const double offset = red == 1 ? 0.5 : 0.0;
  if (mode == kF64) pack_points_kernel<kF64><<<g, kThreads, 0, st>>>(S, G, k, rec, 0.0);
  else if (mode == kPH64) pack_points_kernel<kPH64><<<g, kThreads, 0, st>>>(S, G, k, rec, offset);
  else pack_points_kernel<kF32><<<g, kThreads, 0, st>>>(S, G, k, rec, 0.0);
  return hipGetLastError();
}

hipError_t launch_bwd_chunk(const Plan& p, const void* rec, int64_t k_begin, int64_t k_end,
                            int64_t per_split, const void* xyz, const void* f, void* partial,
                            void* grad, int carry_in, int direct, hipStream_t st) {
  if (p.mode == kF64) {
    if (p.per_lane == 2)
      return p.fk ? bwd_f64_launch<2, 1>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st)
                  : bwd_f64_launch<2, 0>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st);
    return p.fk ? bwd_f64_launch<1, 1>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st)
                : bwd_f64_launch<1, 0>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st);
  }
  if (p.mode == kPH64)
    return bwd_dispatch_q<kPH64>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st);
  return bwd_dispatch_q<kF32>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, st);
}

hipError_t launch_bwd_reduce(const Plan& p, const void* partial, const void* /*f*/, void* grad,
                             hipStream_t st) {
  const int64_t N = p.lanes;
  const unsigned g = static_cast<unsigned>((N + kThreads - 1) / kThreads);
  if (p.mode == kF64)
    bwd_reduce_f64_kernel<<<g, kThreads, 0, st>>>(static_cast<const double*>(partial), p.nsplit, N,
                                                 static_cast<double*>(grad));
  else
    bwd_reduce_kernel<<<g, kThreads, 0, st>>>(static_cast<const float*>(partial), p.nsplit, N,
                                             static_cast<float*>(grad));
  return hipGetLastError();
}

}  // namespace nx
