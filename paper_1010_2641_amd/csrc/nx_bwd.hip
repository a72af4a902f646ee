// nx_bwd.hip -- adjoint of the direct scattering sum.  For a real loss L(A) with seed
// G_k = dL/dRe A_k + i dL/dIm A_k, the chain rule through Eq. 2 of Favre-Nicolin et al.
// (2010) gives, for the positions,
//     dL/dr_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k . r_j)
//             = -2 pi sum_k S_k v_jk,   v_jk = Im( f_j conj(G_k) exp(2 i pi S_k . r_j) )
// (three real sums per atom), and for the factors (torch's convention for a complex
// parameter, dL/dRe f + i dL/dIm f)
//     dL/df_j = conj(W_j),   W_j = sum_k conj(G_k) exp(2 i pi S_k . r_j)
// (one complex sum per atom, computed only when asked for).
//
// In the FP64-phase mode both factors are taken in polar form, conj(G_k) =
// |G_k| exp(2 i pi delta_k) and f_j = |f_j| exp(2 i pi alpha_j): delta_k and alpha_j ride in
// the FP64 phase psi = S_k.r_j + delta_k + alpha_j, |G_k| is folded into S_k, and |f_j|
// leaves the sums altogether, so that
//     dL/dr_j = -2 pi |f_j| sum_k |G_k| S_k sin(2 pi psi)          (sin only), and
//     W_j = exp(-2 i pi alpha_j) sum_k |G_k| exp(2 i pi psi);
// |f_j| and the rotation by arg f_j are applied once per atom to the finished sums.
//
// Layout: every lane owns Q atoms and keeps their position and the sums in registers;
// the points are wave-uniform records (the paper's alternative of parallelising over
// atoms and sharing the reflection coordinates, Section 2.2).  bwd_kernel streams them
// through the scalar load path; bwd_split_kernel (the FP64-phase default) stages their
// phase part in LDS tiles and reads the rest with scalar loads.  The phases are recomputed, never stored.  Sums are
// accumulated in FP32 per group of GRP points and folded into (sum, comp) pairs by
// Kahan's compensated addition.  FP32 mode: the paper's FP32 arithmetic with plain sums.
#include "nx_internal.h"

namespace nx {
namespace {

// Knuth's two-sum: s + g = t + err exactly; err is added into the compensation word
// (the split reduction, once per split and output).
__device__ __forceinline__ void two_sum_acc(float& s, float& c, float g) {
  const float t = s + g;
  const float bp = t - s;
  const float ap = t - bp;
  c += (s - ap) + (g - bp);
  s = t;
}

// Kahan's compensated addition with the correction kept as the error to add (sum + comp
// is the running total): the error of s + y is recovered exactly while |s| >= |y|, which
// holds once the running sum exceeds one group partial.  Four FP32 operations.
__device__ __forceinline__ void kahan_acc(float& s, float& c, float g) {
  const float y = g + c;
  const float t = s + y;
  c = y - (t - s);
  s = t;
}

template <int MODE> struct PointOf;
template <> struct PointOf<kF32> { using type = PointF32; };
template <> struct PointOf<kPH64> { using type = PointPH; };

constexpr float kTwoPi = 6.283185307179586f;
constexpr double kTwoPiD = 6.283185307179586476925286766559;
constexpr double kInvTwoPiD = 0.15915494309189533577;

// arg(f) in cycles, FP64 (0 for f = 0, whose signed zeros carry no angle).
__device__ __forceinline__ double arg_cycles(float fr, float fi) {
  if (fr == 0.f && fi == 0.f) return 0.0;
  return atan2(static_cast<double>(fi), static_cast<double>(fr)) * kInvTwoPiD;
}

// Sums carried per atom: 3 position components, plus Re W and Im W with GF.
template <bool GF> struct NSum { static constexpr int value = GF ? 5 : 3; };

// FP32 mode: w = conj(G) (c + i s) = (gr c + gi s) + i (gr s - gi c);
// v = Im(f w) = fr Im w + fi Re w (f = 1 when FK == 0).
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
struct PtRegs { double sx, sy, sz, delta; float gsx, gsy, gsz, gmag; };

__device__ __forceinline__ PtRegs load_point(const PointPH* __restrict__ rec, int k) {
  const uint4* w = reinterpret_cast<const uint4*>(rec + k);
  const uint4 a = w[0], b = w[1], c = w[2];
  PtRegs r;
  r.sx = __hiloint2double(static_cast<int>(a.y), static_cast<int>(a.x));
  r.delta = __hiloint2double(static_cast<int>(a.w), static_cast<int>(a.z));
  r.sy = __hiloint2double(static_cast<int>(b.y), static_cast<int>(b.x));
  r.sz = __hiloint2double(static_cast<int>(b.w), static_cast<int>(b.z));
  r.gsx = __uint_as_float(c.x);
  r.gsy = __uint_as_float(c.y);
  r.gsz = __uint_as_float(c.z);
  r.gmag = __uint_as_float(c.w);
  return r;
}

// The same record with its phase part (sx, delta, sy, sz: the first two words) taken
// from an LDS tile and its last word (|G| S, |G|) from the record itself (scalar loads).
// The tile is read as two (double, double) pairs, which the compiler turns into two
// 16-byte LDS reads per point (read as 32-bit words the same bytes took three reads and
// the adjoint was 3-4.5 % slower).
__device__ __forceinline__ PtRegs load_point_split(const uint4* sd, int u,
                                                   const PointPH* __restrict__ rec, int k) {
  const uint4* w = reinterpret_cast<const uint4*>(rec + k);
  const double2* sdd = reinterpret_cast<const double2*>(sd);
  const double2 a = sdd[2 * u], b = sdd[2 * u + 1];
  const uint4 c = w[2];
  PtRegs r;
  r.sx = a.x;
  r.delta = a.y;
  r.sy = b.x;
  r.sz = b.y;
  r.gsx = __uint_as_float(c.x);
  r.gsy = __uint_as_float(c.y);
  r.gsz = __uint_as_float(c.z);
  r.gmag = __uint_as_float(c.w);
  return r;
}

// The FP64-phase record of point k, with the seed in polar form conj(G) = |G| exp(2 i pi
// delta): delta = -arg(G) / (2 pi) in FP64 (plus kPhaseShift and the reduction offset of the
// variant: `offset`); |G| S
// and |G| rounded once to FP32.  The pack kernel writes it to the workspace; the adjoint of
// small calls forms it while staging its tile, so that both give the same record.
__device__ __forceinline__ PointPH make_point_ph(const float* __restrict__ S,
                                                const float* __restrict__ G, int64_t k,
                                                double offset) {
  PointPH r;
  const double sx = S[3 * k], sy = S[3 * k + 1], sz = S[3 * k + 2];
  const double gr = G[2 * k], gi = G[2 * k + 1];
  const double m = sqrt(gr * gr + gi * gi);
  r.sx = sx; r.sy = sy; r.sz = sz;
  r.delta = -atan2(gi, gr) * 0.15915494309189533577 + offset;
  r.gsx = static_cast<float>(m * sx);
  r.gsy = static_cast<float>(m * sy);
  r.gsz = static_cast<float>(m * sz);
  r.gmag = static_cast<float>(m);
  return r;
}

// |v| as FP32, +inf when v is not finite (the fixed-point tile bounds).
__device__ __forceinline__ float bound_abs(double v) {
  const float a = static_cast<float>(fabs(v));
  return a <= 3.402823466e38f ? a : __builtin_inff();
}

// Largest v over the wavefront.
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// A whole record from an LDS tile of 48-byte records (the inline form of small calls):
// the phase part as two (double, double) pairs, the rest as one 16-byte word.
__device__ __forceinline__ PtRegs load_point_lds(const uint4* sd, int u) {
  const double2* sdd = reinterpret_cast<const double2*>(sd);
  const double2 a = sdd[3 * u], b = sdd[3 * u + 1];
  const uint4 c = sd[3 * u + 2];
  PtRegs r;
  r.sx = a.x;
  r.delta = a.y;
  r.sy = b.x;
  r.sz = b.y;
  r.gsx = __uint_as_float(c.x);
  r.gsy = __uint_as_float(c.y);
  r.gsz = __uint_as_float(c.z);
  r.gmag = __uint_as_float(c.w);
  return r;
}

// (c, s) of exp(2 i pi psi), psi = S.r + delta + alpha (delta includes kPhaseShift and the
// 1/2 of RED == 1; alpha = arg f in cycles, absent for f = 1).  The seed angle enters as
// the addend of the first fma, the atom's angle as one FP64 add.  RED 0 centred, 1 fract,
// 2 the fixed-point read of the low word (where the tile's bound holds; see kPhaseShift),
// 3 its fallback: centred with rint, then the low word of the turn plus kPhaseShift.
template <int RED>
__device__ __forceinline__ void cis_turn_pt(double ph, float& c, float& s) {
  float tf;
  if constexpr (RED == 0) tf = static_cast<float>(ph - __builtin_rint(ph));
  else if constexpr (RED == 1) tf = static_cast<float>(__builtin_amdgcn_fract(ph));
  else if constexpr (RED == 2) tf = static_cast<float>(__double2loint(ph)) * 0x1.0p-32f;
  else tf = static_cast<float>(__double2loint((ph - __builtin_rint(ph)) + kPhaseShift)) * 0x1.0p-32f;
  c = __builtin_amdgcn_cosf(tf);
  s = __builtin_amdgcn_sinf(tf);
}
template <int RED, int FK>
__device__ __forceinline__ void cis_ph64_pt(const PtRegs& a, double x, double y, double z,
                                            double al, float& c, float& s) {
  double ph = __builtin_fma(a.sz, z, __builtin_fma(a.sy, y, __builtin_fma(a.sx, x, a.delta)));
  if constexpr (FK != 0) ph += al;
  cis_turn_pt<RED>(ph, c, s);
}

// One point's contribution to the FP64-phase group partials g[0..NS).
template <bool GF>
__device__ __forceinline__ void ph64_pair(float* g, const PtRegs& a, float c, float s) {
  g[0] = __builtin_fmaf(s, a.gsx, g[0]);
  g[1] = __builtin_fmaf(s, a.gsy, g[1]);
  g[2] = __builtin_fmaf(s, a.gsz, g[2]);
  if constexpr (GF) {
    g[3] = __builtin_fmaf(a.gmag, c, g[3]);
    g[4] = __builtin_fmaf(a.gmag, s, g[4]);
  }
}

// Writes the outputs of one atom from its total sums T[0..NS).  POLAR (FP64-phase mode
// with complex f): the sums hold sin and exp of the phase shifted by arg f_j and no
// |f_j|, so dL/dr = -2 pi |f| T and dL/df = conj(W) = (f / |f|) conj(T3 + i T4), formed in
// FP64 and rounded once.
template <bool GF, bool POLAR>
__device__ __forceinline__ void write_out(float* grad, float* gradf, int64_t j, const float* T,
                                          const float* __restrict__ f) {
  if constexpr (POLAR) {
    const double fr = f[2 * j], fi = f[2 * j + 1];
    const double m = sqrt(fr * fr + fi * fi);
    if (grad) {
#pragma unroll
      for (int d = 0; d < 3; ++d) grad[3 * j + d] = static_cast<float>(-kTwoPiD * m * T[d]);
    }
    if constexpr (GF) {
      const double t3 = T[3], t4 = T[4];
      if (m > 0.0) {
        gradf[2 * j] = static_cast<float>((fr * t3 + fi * t4) / m);
        gradf[2 * j + 1] = static_cast<float>((fi * t3 - fr * t4) / m);
      } else {
        gradf[2 * j] = T[3];
        gradf[2 * j + 1] = -T[4];
      }
    }
  } else {
    if (grad) {
      grad[3 * j] = -kTwoPi * T[0];
      grad[3 * j + 1] = -kTwoPi * T[1];
      grad[3 * j + 2] = -kTwoPi * T[2];
    }
    if constexpr (GF) {
      gradf[2 * j] = T[3];          // dL/df = conj(W)
      gradf[2 * j + 1] = -T[4];
    }
  }
}

// Adjoint over points [k_begin + sp*per_split, ...) for Q atoms per lane.
// Grid: blocks_n * nsplit; logical block = sp * blocks_n + nb (XCD-major order).
// part layout: [sp][sum index][sum | comp][N] floats.
template <int MODE, int Q, int FK, int GRP, int RED, bool GF>
__global__ __launch_bounds__(kThreads) void bwd_kernel(
    const typename PointOf<MODE>::type* __restrict__ rec, int k_begin, int k_end, int per_split,
    const float* __restrict__ xyz, const float* __restrict__ f, int64_t N, int blocks_n,
    float* __restrict__ part, float* __restrict__ grad, float* __restrict__ gradf, int carry_in,
    int direct) {
  constexpr int NS = NSum<GF>::value;
  using RReg = typename std::conditional<MODE == kPH64, double, float>::type;
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int nb = lb % blocks_n;
  const int sp = lb / blocks_n;
  const int64_t j0 = int64_t(nb) * (kThreads * Q) + threadIdx.x;

  RReg x[Q], y[Q], z[Q];
  float fr[Q], fi[Q];
  double al[Q];
  float sum[Q][NS], cmp[Q][NS];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    const int64_t jj = j < N ? j : N - 1;
    x[q] = static_cast<RReg>(xyz[3 * jj]);
    y[q] = static_cast<RReg>(xyz[3 * jj + 1]);
    z[q] = static_cast<RReg>(xyz[3 * jj + 2]);
    fr[q] = (FK && f) ? f[2 * jj] : 1.f;
    fi[q] = (FK && f) ? f[2 * jj + 1] : 0.f;
    al[q] = (MODE == kPH64 && FK) ? arg_cycles(fr[q], fi[q]) : 0.0;
#pragma unroll
    for (int d = 0; d < NS; ++d) {
      if (carry_in && j < N) {
        sum[q][d] = part[((int64_t(sp) * NS + d) * 2 + 0) * N + j];
        cmp[q][d] = part[((int64_t(sp) * NS + d) * 2 + 1) * N + j];
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
        if constexpr (GF) {
          sum[q][3] += __builtin_fmaf(a.gi, s, a.gr * c);
          sum[q][4] += __builtin_fmaf(-a.gi, c, a.gr * s);
        }
      }
    }
  } else {
    // sign of the RED == 1 terms, applied once per group (see cis_ph64_pt)
    constexpr float SGN = (RED == 1) ? -1.f : 1.f;
    int k = k0;
    while (k < k1) {
      const int kend = (k + GRP <= k1) ? k + GRP : k1;
      float g[Q][NS];
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int d = 0; d < NS; ++d) g[q][d] = 0.f;
      if (kend - k == GRP) {
#pragma unroll
        for (int u = 0; u < GRP; ++u) {
          const PtRegs a = load_point(rec, k + u);
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            float c, s;
            cis_ph64_pt<RED, FK>(a, x[q], y[q], z[q], al[q], c, s);
            ph64_pair<GF>(g[q], a, c, s);
          }
        }
      } else {
        for (int kk = k; kk < kend; ++kk) {
          const PtRegs a = load_point(rec, kk);
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            float c, s;
            cis_ph64_pt<RED, FK>(a, x[q], y[q], z[q], al[q], c, s);
            ph64_pair<GF>(g[q], a, c, s);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int d = 0; d < NS; ++d) kahan_acc(sum[q][d], cmp[q][d], SGN * g[q][d]);
      k = kend;
    }
  }

#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    if (j < N) {
      if (direct) {
        float T[NS];
#pragma unroll
        for (int d = 0; d < NS; ++d) T[d] = sum[q][d] + cmp[q][d];
        write_out<GF, MODE == kPH64 && FK != 0>(grad, gradf, j, T, f);
      } else {
#pragma unroll
        for (int d = 0; d < NS; ++d) {
          part[((int64_t(sp) * NS + d) * 2 + 0) * N + j] = sum[q][d];
          part[((int64_t(sp) * NS + d) * 2 + 1) * N + j] = cmp[q][d];
        }
      }
    }
  }
}

// FP64-phase adjoint with the phase part of each point (sx, delta, sy, sz: 32 bytes)
// staged in an LDS tile and the rest of the record (|G| S, |G|) read with scalar loads:
// the phase's fma chain then takes its point values from VGPRs.  Groups and compensation are those of bwd_kernel
// (tiles are whole groups), so the result is bitwise the same.
//
// RED 2: each wave checks the fixed-point bound for every tile, (|x| + |y| + |z|) of its
// atoms times the tile's largest |S| component (the bounds of the at most two pack blocks
// the tile overlaps, `bnd`), and takes the fallback (variant 3, same records) for a tile
// where some lane fails it.
//
// INL (small calls): no packed records; each thread forms its whole record of the tile from
// S and G while staging it (make_point_ph, as the pack kernel does) and every field is read
// back from LDS, which saves the pack dispatch when few work-groups share each record; the
// tile's bound is then reduced over its own points.
template <int Q, int FK, int GRP, int RED, bool GF, bool INL>
__global__ __launch_bounds__(kThreads) void bwd_split_kernel(
    const PointPH* __restrict__ rec, int k_begin, int k_end, int per_split,
    const float* __restrict__ xyz, const float* __restrict__ f, int64_t N, int blocks_n,
    float* __restrict__ part, float* __restrict__ grad, float* __restrict__ gradf, int carry_in,
    int direct, const float* __restrict__ S, const float* __restrict__ G,
    const float* __restrict__ bnd) {
  static_assert(kThreads % GRP == 0, "tiles must hold whole groups");
  constexpr int NS = NSum<GF>::value;
  constexpr float SGN = (RED == 1) ? -1.f : 1.f;
  constexpr int W = INL ? 3 : 2;            // 16-byte words per point in the LDS tile
  __shared__ uint4 sd[W * kThreads];
  __shared__ float wmax[kThreads / 64];
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int nb = lb % blocks_n;
  const int sp = lb / blocks_n;
  const int64_t j0 = int64_t(nb) * (kThreads * Q) + threadIdx.x;
  double x[Q], y[Q], z[Q], al[Q];
  float sum[Q][NS], cmp[Q][NS];
  float r1 = 0.f;                           // the lane's |x| + |y| + |z| (largest over q)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    const int64_t jj = j < N ? j : N - 1;
    x[q] = xyz[3 * jj];
    y[q] = xyz[3 * jj + 1];
    z[q] = xyz[3 * jj + 2];
    r1 = fmaxf(r1, bound_abs(fabs(x[q]) + fabs(y[q]) + fabs(z[q])));
    al[q] = (FK && f) ? arg_cycles(f[2 * jj], f[2 * jj + 1]) : 0.0;
#pragma unroll
    for (int d = 0; d < NS; ++d) {
      if (carry_in && j < N) {
        sum[q][d] = part[((int64_t(sp) * NS + d) * 2 + 0) * N + j];
        cmp[q][d] = part[((int64_t(sp) * NS + d) * 2 + 1) * N + j];
      } else {
        sum[q][d] = 0.f;
        cmp[q][d] = 0.f;
      }
    }
  }
  // the groups of one tile (points t0 .. t0 + nt), reduced with the variant R
  auto run_tile = [&](auto red_c, int t0, int nt) {
    constexpr int R = decltype(red_c)::value;
    for (int u0 = 0; u0 < nt; u0 += GRP) {
      const int ue = (u0 + GRP <= nt) ? u0 + GRP : nt;
      float g[Q][NS];
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int d = 0; d < NS; ++d) g[q][d] = 0.f;
      if (ue - u0 == GRP) {
#pragma unroll
        for (int u = 0; u < GRP; ++u) {
          const PtRegs a = INL ? load_point_lds(sd, u0 + u) : load_point_split(sd, u0 + u, rec, t0 + u0 + u);
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            float c, s;
            cis_ph64_pt<R, FK>(a, x[q], y[q], z[q], al[q], c, s);
            ph64_pair<GF>(g[q], a, c, s);
          }
        }
      } else {
        for (int u = u0; u < ue; ++u) {
          const PtRegs a = INL ? load_point_lds(sd, u) : load_point_split(sd, u, rec, t0 + u);
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            float c, s;
            cis_ph64_pt<R, FK>(a, x[q], y[q], z[q], al[q], c, s);
            ph64_pair<GF>(g[q], a, c, s);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int d = 0; d < NS; ++d) kahan_acc(sum[q][d], cmp[q][d], SGN * g[q][d]);
    }
  };
  const int k0 = k_begin + sp * per_split;
  const int k1 = min(k0 + per_split, k_end);
  for (int t0 = k0; t0 < k1; t0 += kThreads) {
    const int nt = min(kThreads, k1 - t0);
    __syncthreads();                        // the previous tile is no longer read
    float sm = 0.f;
    if (int(threadIdx.x) < nt) {
      if constexpr (INL) {
        const PointPH r = make_point_ph(S, G, t0 + threadIdx.x, kPhaseShift + (RED == 1 ? 0.5 : 0.0));
        const uint4* w = reinterpret_cast<const uint4*>(&r);
        sd[3 * threadIdx.x] = w[0];
        sd[3 * threadIdx.x + 1] = w[1];
        sd[3 * threadIdx.x + 2] = w[2];
        sm = fmaxf(bound_abs(r.sx), fmaxf(bound_abs(r.sy), bound_abs(r.sz)));
      } else {
        const uint4* w = reinterpret_cast<const uint4*>(rec + t0 + threadIdx.x);
        sd[2 * threadIdx.x] = w[0];
        sd[2 * threadIdx.x + 1] = w[1];
      }
    }
    if constexpr (INL && RED == 2) {
      sm = wave_max(sm);
      if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = sm;
    }
    __syncthreads();
    if constexpr (RED == 2) {
      float st;
      if constexpr (INL) {
        st = wmax[0];
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) st = fmaxf(st, wmax[w]);
      } else {
        st = fmaxf(bnd[t0 / kThreads], bnd[(t0 + nt - 1) / kThreads]);
      }
      if (__all(r1 * st < kFixedPhaseBound)) run_tile(std::integral_constant<int, 2>{}, t0, nt);
      else run_tile(std::integral_constant<int, 3>{}, t0, nt);
    } else {
      run_tile(std::integral_constant<int, RED>{}, t0, nt);
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    if (j < N) {
      if (direct) {
        float T[NS];
#pragma unroll
        for (int d = 0; d < NS; ++d) T[d] = sum[q][d] + cmp[q][d];
        write_out<GF, FK != 0>(grad, gradf, j, T, f);
      } else {
#pragma unroll
        for (int d = 0; d < NS; ++d) {
          part[((int64_t(sp) * NS + d) * 2 + 0) * N + j] = sum[q][d];
          part[((int64_t(sp) * NS + d) * 2 + 1) * N + j] = cmp[q][d];
        }
      }
    }
  }
}

// FP64-phase adjoint over a grid whose rows hold a multiple of 64 points: 64-point groups,
// each one row's run of consecutive points (groups start at multiples of 64 from the
// grid's start).  Per lane atom, c0 = o.r + arg f / 2 pi + kPhaseShift and c_d = e_d.r in
// FP64, and w - 1 = exp(2 i pi c1) - 1 in FP32 (formed in FP64).  A group takes the phase
// factor E = exp(2 i pi (S.r + arg f / 2 pi)) of its first point exactly (the FP64 phase
// fma(i1, c1, c0 + i2 c2 + i3 c3), the fixed-point read under the per-tile range check or
// variant 3, hardware cos and sin) and steps it along the row, E <- E + E (w - 1) (four
// FP32 fma; the small w - 1 keeps the rounding of w out of the steps where step1.r is
// small).  Per point: v = Im(conj(G) E) = Re G Im E - Im G Re E, a0 += v and a1 += u v
// (u the point's place in the group); per group: T_d += S0_d a0 + e1_d a1 (S0 the
// group's first point), Kahan-compensated across groups as in bwd_split_kernel.  The
// point records (PointRow) come with scalar loads; no LDS.  Outputs as bwd_split_kernel.
template <int Q, int FK>
__global__ __launch_bounds__(kThreads) void bwd_rows_kernel(
    const PointRow* __restrict__ rec, const float4* __restrict__ grp, const float* __restrict__ bnd,
    int k_begin, int k_end, int per_split, const float* __restrict__ xyz, const float* __restrict__ f,
    int64_t N, int blocks_n, float* __restrict__ part, float* __restrict__ grad, int carry_in, int direct,
    GridDef g) {
  constexpr int GRP = kRowGroup;
  constexpr int NS = 3;
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int nb = lb % blocks_n;
  const int sp = lb / blocks_n;
  const int64_t j0 = int64_t(nb) * (kThreads * Q) + threadIdx.x;
  double c0[Q], c1[Q], c2[Q], c3[Q];
  float wr[Q], wi[Q];                       // w - 1
  float sum[Q][NS], cmp[Q][NS];
  float r1 = 0.f;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    const int64_t jj = j < N ? j : N - 1;
    const double x = xyz[3 * jj], y = xyz[3 * jj + 1], z = xyz[3 * jj + 2];
    r1 = fmaxf(r1, bound_abs(fabs(x) + fabs(y) + fabs(z)));
    const double al = (FK && f) ? arg_cycles(f[2 * jj], f[2 * jj + 1]) : 0.0;
    c0[q] = __builtin_fma(g.o[2], z, __builtin_fma(g.o[1], y, __builtin_fma(g.o[0], x, al + kPhaseShift)));
    c1[q] = __builtin_fma(g.e1[2], z, __builtin_fma(g.e1[1], y, g.e1[0] * x));
    c2[q] = __builtin_fma(g.e2[2], z, __builtin_fma(g.e2[1], y, g.e2[0] * x));
    c3[q] = __builtin_fma(g.e3[2], z, __builtin_fma(g.e3[1], y, g.e3[0] * x));
    // w - 1 = (cos 2 pi t - 1, sin 2 pi t), t = c1 mod 1, with cos 2 pi t - 1 = -2 sin^2 pi t
    const double t = c1[q] - __builtin_rint(c1[q]);
    const double h = sinpi(t);
    wr[q] = static_cast<float>(-2.0 * h * h);
    wi[q] = static_cast<float>(sinpi(2.0 * t));
#pragma unroll
    for (int d = 0; d < NS; ++d) {
      if (carry_in && j < N) {
        sum[q][d] = part[((int64_t(sp) * NS + d) * 2 + 0) * N + j];
        cmp[q][d] = part[((int64_t(sp) * NS + d) * 2 + 1) * N + j];
      } else {
        sum[q][d] = 0.f;
        cmp[q][d] = 0.f;
      }
    }
  }
  const float e1x = static_cast<float>(g.e1[0]), e1y = static_cast<float>(g.e1[1]),
              e1z = static_cast<float>(g.e1[2]);
  auto run_tile = [&](auto red_c, int t0, int nt) {
    constexpr int R = decltype(red_c)::value;
    for (int u0 = 0; u0 < nt; u0 += GRP) {
      const int ue = (u0 + GRP <= nt) ? u0 + GRP : nt;
      const uint32_t k = static_cast<uint32_t>(t0 + u0);     // the group's first point
      const uint32_t row = k / static_cast<uint32_t>(g.n1);
      const double d1 = static_cast<double>(k - row * static_cast<uint32_t>(g.n1));
      const double d2 = static_cast<double>(row % static_cast<uint32_t>(g.n2)),
                   d3 = static_cast<double>(row / static_cast<uint32_t>(g.n2));
      float er[Q], ei[Q], a0[Q], a1[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const double b = __builtin_fma(d3, c3[q], __builtin_fma(d2, c2[q], c0[q]));
        cis_turn_pt<R>(__builtin_fma(d1, c1[q], b), er[q], ei[q]);
        a0[q] = 0.f;
        a1[q] = 0.f;
      }
      auto point = [&](int u, bool step) {
        const PointRow r = rec[t0 + u];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const float v = __builtin_fmaf(r.gr, ei[q], r.ngi * er[q]);
          a0[q] += v;
          a1[q] = __builtin_fmaf(r.u, v, a1[q]);
          if (step) {
            const float nr = __builtin_fmaf(er[q], wr[q], __builtin_fmaf(-ei[q], wi[q], er[q]));
            const float ni = __builtin_fmaf(er[q], wi[q], __builtin_fmaf(ei[q], wr[q], ei[q]));
            er[q] = nr;
            ei[q] = ni;
          }
        }
      };
      if (ue - u0 == GRP) {
#pragma unroll
        for (int u = 0; u < GRP; ++u) point(u0 + u, u + 1 < GRP);
      } else {
        for (int u = u0; u < ue; ++u) point(u, true);
      }
      const float4 s0 = grp[k / GRP];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        kahan_acc(sum[q][0], cmp[q][0], __builtin_fmaf(s0.x, a0[q], e1x * a1[q]));
        kahan_acc(sum[q][1], cmp[q][1], __builtin_fmaf(s0.y, a0[q], e1y * a1[q]));
        kahan_acc(sum[q][2], cmp[q][2], __builtin_fmaf(s0.z, a0[q], e1z * a1[q]));
      }
    }
  };
  const int k0 = k_begin + sp * per_split;
  const int k1 = min(k0 + per_split, k_end);
  for (int t0 = k0; t0 < k1; t0 += kThreads) {
    const int nt = min(kThreads, k1 - t0);
    const float st = fmaxf(bnd[t0 / kThreads], bnd[(t0 + nt - 1) / kThreads]);
    if (__all(r1 * st < kFixedPhaseBound)) run_tile(std::integral_constant<int, 2>{}, t0, nt);
    else run_tile(std::integral_constant<int, 3>{}, t0, nt);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    if (j < N) {
      if (direct) {
        float T[NS];
#pragma unroll
        for (int d = 0; d < NS; ++d) T[d] = sum[q][d] + cmp[q][d];
        write_out<false, FK != 0>(grad, nullptr, j, T, f);
      } else {
#pragma unroll
        for (int d = 0; d < NS; ++d) {
          part[((int64_t(sp) * NS + d) * 2 + 0) * N + j] = sum[q][d];
          part[((int64_t(sp) * NS + d) * 2 + 1) * N + j] = cmp[q][d];
        }
      }
    }
  }
}

// All-FP64 adjoint.  part layout: [sp][sum index][N] doubles.
template <int Q, int FK, bool GF>
__global__ __launch_bounds__(kThreads) void bwd_f64_kernel(
    const PointF64* __restrict__ rec, int k_begin, int k_end, int per_split,
    const double* __restrict__ xyz, const double* __restrict__ f, int64_t N, int blocks_n,
    double* __restrict__ part, double* __restrict__ grad, double* __restrict__ gradf, int carry_in,
    int direct) {
  constexpr int NS = NSum<GF>::value;
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int nb = lb % blocks_n;
  const int sp = lb / blocks_n;
  const int64_t j0 = int64_t(nb) * (kThreads * Q) + threadIdx.x;
  double x[Q], y[Q], z[Q], fr[Q], fi[Q], T[Q][NS];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    const int64_t jj = j < N ? j : N - 1;
    x[q] = xyz[3 * jj]; y[q] = xyz[3 * jj + 1]; z[q] = xyz[3 * jj + 2];
    fr[q] = (FK && f) ? f[2 * jj] : 1.0;
    fi[q] = (FK && f) ? f[2 * jj + 1] : 0.0;
#pragma unroll
    for (int d = 0; d < NS; ++d)
      T[q][d] = (carry_in && j < N) ? part[(int64_t(sp) * NS + d) * N + j] : 0.0;
  }
  const int k0 = k_begin + sp * per_split;
  const int k1 = min(k0 + per_split, k_end);
  for (int k = k0; k < k1; ++k) {
    const PointF64 a = rec[k];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double ph = __builtin_fma(a.sz, z[q], __builtin_fma(a.sy, y[q], a.sx * x[q]));
      double s, c;
      cis_f64(ph, c, s);
      const double wre = __builtin_fma(a.gi, s, a.gr * c);      // conj(G) e^{i theta}
      const double wim = __builtin_fma(-a.gi, c, a.gr * s);
      double v = wim;
      if constexpr (FK) v = __builtin_fma(fi[q], wre, fr[q] * wim);
      T[q][0] = __builtin_fma(v, a.sx, T[q][0]);
      T[q][1] = __builtin_fma(v, a.sy, T[q][1]);
      T[q][2] = __builtin_fma(v, a.sz, T[q][2]);
      if constexpr (GF) {
        T[q][3] += wre;
        T[q][4] += wim;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t j = j0 + int64_t(q) * kThreads;
    if (j < N) {
      if (direct) {
        if (grad) {
#pragma unroll
          for (int d = 0; d < 3; ++d) grad[3 * j + d] = -kTwoPiD * T[q][d];
        }
        if constexpr (GF) {
          gradf[2 * j] = T[q][3];
          gradf[2 * j + 1] = -T[q][4];
        }
      } else {
#pragma unroll
        for (int d = 0; d < NS; ++d) part[(int64_t(sp) * NS + d) * N + j] = T[q][d];
      }
    }
  }
}

// Combine the split partials of every atom in a fixed order (deterministic): G lanes of
// one wave serve one atom (G a power of two up to 64, about a quarter of the splits); lane i
// folds splits i, i + G, ... of each sum in sequence with Knuth's two-sum, then the lanes'
// states meet in a butterfly in which both partners fold the lower lane's state first (a
// fixed tree), and lane 0 writes the atom's outputs.  Few splits take G = 1.  A wave
// serves 64 / G consecutive atoms side by side (its lane w: atom w % (64 / G), split lane
// w / (64 / G)), so that each load reads a run of consecutive atoms of G split rows.
template <int G, bool GF, bool POLAR>
__global__ __launch_bounds__(kThreads) void bwd_reduce_kernel(const float* __restrict__ part,
                                                              int nsplit, int64_t N,
                                                              const float* __restrict__ f,
                                                              float* __restrict__ grad,
                                                              float* __restrict__ gradf) {
  static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "G: a power of two within a wave");
  constexpr int NS = NSum<GF>::value;
  constexpr int OPW = 64 / G;               // atoms per wave, side by side
  const int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  const int w = static_cast<int>(t & 63);
  const int64_t j = (t >> 6) * OPW + (w % OPW);
  const int lane = w / OPW;
  float T[NS];
#pragma unroll
  for (int d = 0; d < NS; ++d) {
    float s = 0.f, cm = 0.f;
    if (j < N) {
#pragma unroll 4
      for (int sp = lane; sp < nsplit; sp += G) {
        two_sum_acc(s, cm, part[((int64_t(sp) * NS + d) * 2 + 0) * N + j]);
        cm += part[((int64_t(sp) * NS + d) * 2 + 1) * N + j];
      }
    }
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
      const float os = __shfl_xor(s, off * OPW), oc = __shfl_xor(cm, off * OPW);
      const bool upper = (lane & off) != 0;    // the partner is the lower lane: fold it first
      float a = upper ? os : s, ac = upper ? oc : cm;
      const float b = upper ? s : os, bc = upper ? cm : oc;
      two_sum_acc(a, ac, b);
      s = a;
      cm = ac + bc;
    }
    T[d] = s + cm;
  }
  if (j < N && lane == 0) write_out<GF, POLAR>(grad, gradf, j, T, f);
}

template <bool GF>
__global__ __launch_bounds__(kThreads) void bwd_reduce_f64_kernel(const double* __restrict__ part,
                                                                  int nsplit, int64_t N,
                                                                  double* __restrict__ grad,
                                                                  double* __restrict__ gradf) {
  constexpr int NS = NSum<GF>::value;
  const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (j >= N) return;
  double T[NS];
#pragma unroll
  for (int d = 0; d < NS; ++d) {
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += part[(int64_t(sp) * NS + d) * N + j];
    T[d] = s;
  }
  if (grad) {
#pragma unroll
    for (int d = 0; d < 3; ++d) grad[3 * j + d] = -kTwoPiD * T[d];
  }
  if constexpr (GF) {
    gradf[2 * j] = T[3];
    gradf[2 * j + 1] = -T[4];
  }
}

// FP64-phase point records, grid-stride over blocks of 256 points, with each block's
// largest |S| component in bnd[block] (the adjoint's tile bound).
__global__ __launch_bounds__(kThreads) void pack_points_ph_kernel(const float* __restrict__ S,
                                                                  const float* __restrict__ G,
                                                                  int64_t n, PointPH* __restrict__ rec,
                                                                  float* __restrict__ bnd,
                                                                  double offset) {
  __shared__ float wmax[kThreads / 64];
  for (int64_t b = blockIdx.x; b * kThreads < n; b += gridDim.x) {
    const int64_t k = b * kThreads + threadIdx.x;
    float sm = 0.f;
    if (k < n) {
      const PointPH r = make_point_ph(S, G, k, offset);
      rec[k] = r;
      sm = fmaxf(bound_abs(r.sx), fmaxf(bound_abs(r.sy), bound_abs(r.sz)));
    }
    sm = wave_max(sm);
    __syncthreads();                      // wmax of the previous block is read
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = sm;
    __syncthreads();
    if (threadIdx.x == 0) {
      float bm = wmax[0];
#pragma unroll
      for (int w = 1; w < kThreads / 64; ++w) bm = fmaxf(bm, wmax[w]);
      bnd[b] = bm;
    }
  }
}

// Point k of a grid: S (FP64) and the row part R = o + i2 e2 + i3 e3.
__device__ __forceinline__ void grid_point_rows(const GridDef& g, int64_t k, double* S, double* R) {
  // (counts and indices stay below 2^30: 32-bit index arithmetic)
  const uint32_t ku = static_cast<uint32_t>(k), n1 = static_cast<uint32_t>(g.n1),
                 n2 = static_cast<uint32_t>(g.n2);
  const uint32_t row = ku / n1;
  const double d1 = static_cast<double>(ku - row * n1), d2 = static_cast<double>(row % n2),
               d3 = static_cast<double>(row / n2);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    R[d] = __builtin_fma(d3, g.e3[d], __builtin_fma(d2, g.e2[d], g.o[d]));
    S[d] = __builtin_fma(d1, g.e1[d], R[d]);
  }
}

// Point records of a grid, grid-stride over blocks of 256 points, and each block's bound
// in bnd[block] (the largest |S| component, for the rows form also of the row part):
// ROWS, the records of bwd_rows_kernel (PointRow, and the group's first point S0 in
// grp[k / 64]); otherwise PointPH for the general kernels, with the FP64 grid point and
// the seed's phase and modulus as pack_points_ph_kernel forms them.
template <bool ROWS>
__global__ __launch_bounds__(kThreads) void pack_points_grid_kernel(GridDef g, const float* __restrict__ G,
                                                                    int64_t n, void* __restrict__ rec_v,
                                                                    float4* __restrict__ grp,
                                                                    float* __restrict__ bnd) {
  __shared__ float wmax[kThreads / 64];
  for (int64_t b = blockIdx.x; b * kThreads < n; b += gridDim.x) {
    const int64_t k = b * kThreads + threadIdx.x;
    float sm = 0.f;
    if (k < n) {
      double S[3], R[3];
      grid_point_rows(g, k, S, R);
      sm = fmaxf(bound_abs(S[0]), fmaxf(bound_abs(S[1]), bound_abs(S[2])));
      const float gr = G[2 * k], gi = G[2 * k + 1];
      if constexpr (ROWS) {
        sm = fmaxf(sm, fmaxf(bound_abs(R[0]), fmaxf(bound_abs(R[1]), bound_abs(R[2]))));
        PointRow r;
        r.gr = gr;
        r.ngi = -gi;
        r.u = static_cast<float>(k % kRowGroup);
        r.pad = 0.f;
        static_cast<PointRow*>(rec_v)[k] = r;
        if (k % kRowGroup == 0)
          grp[k / kRowGroup] = make_float4(static_cast<float>(S[0]), static_cast<float>(S[1]),
                                           static_cast<float>(S[2]), 0.f);
      } else {
        const double m = sqrt(double(gr) * gr + double(gi) * gi);
        PointPH r;
        r.sx = S[0]; r.sy = S[1]; r.sz = S[2];
        r.delta = -atan2(double(gi), double(gr)) * 0.15915494309189533577 + kPhaseShift;
        r.gsx = static_cast<float>(m * S[0]);
        r.gsy = static_cast<float>(m * S[1]);
        r.gsz = static_cast<float>(m * S[2]);
        r.gmag = static_cast<float>(m);
        static_cast<PointPH*>(rec_v)[k] = r;
      }
    }
    sm = wave_max(sm);
    __syncthreads();                      // wmax of the previous block is read
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = sm;
    __syncthreads();
    if (threadIdx.x == 0) {
      float bm = wmax[0];
#pragma unroll
      for (int w = 1; w < kThreads / 64; ++w) bm = fmaxf(bm, wmax[w]);
      bnd[b] = bm;
    }
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
        static_cast<PointPH*>(rec_v)[k] = make_point_ph(S, G, k, offset);
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

struct BwdArgs {
  const void* rec; int64_t k_begin, k_end, per_split;
  const void* xyz; const void* f; void* partial; void* grad; void* gradf;
  int carry_in, direct;
  const void* S; const void* G;            // the inline form's record sources
};

template <int MODE, int Q, int FK, bool GF>
hipError_t bwd_dispatch(const Plan& p, const BwdArgs& b, hipStream_t st) {
  using PT = typename PointOf<MODE>::type;
  const dim3 grid(static_cast<unsigned>(p.blocks * p.nsplit));
  const auto* r = static_cast<const PT*>(b.rec);
  const auto* x = static_cast<const float*>(b.xyz);
  const auto* ff = static_cast<const float*>(b.f);
  auto* pa = static_cast<float*>(b.partial);
  auto* g = static_cast<float*>(b.grad);
  auto* gf = static_cast<float*>(b.gradf);
  const int k0 = int(b.k_begin), k1 = int(b.k_end), per = int(b.per_split), nblk = int(p.blocks);
  if constexpr (MODE == kF32) {
    bwd_kernel<MODE, Q, FK, 16, 0, GF><<<grid, kThreads, 0, st>>>(
        r, k0, k1, per, x, ff, p.lanes, nblk, pa, g, gf, b.carry_in, b.direct);
  } else {
    if (p.lds && (p.red == 1 || p.red == 2) && (p.grp == 64 || p.grp == 32 || p.grp == 16)) {
      const float* bnd = (p.inl || !r) ? nullptr
          : reinterpret_cast<const float*>(reinterpret_cast<const char*>(r) + point_bound_offset(p.stream));
      const auto* S = static_cast<const float*>(b.S);
      const auto* G = static_cast<const float*>(b.G);
      auto launch = [&](auto grp_c, auto red_c, auto inl_c) {
        constexpr bool I = decltype(inl_c)::value;
        bwd_split_kernel<I ? 1 : Q, FK, decltype(grp_c)::value, decltype(red_c)::value, GF, I>
            <<<grid, kThreads, 0, st>>>(I ? nullptr : r, k0, k1, per, x, ff, p.lanes, nblk, pa, g, gf,
                                        b.carry_in, b.direct, I ? S : nullptr, I ? G : nullptr, bnd);
      };
      using R1 = std::integral_constant<int, 1>;
      using R2 = std::integral_constant<int, 2>;
      using NoInl = std::integral_constant<bool, false>;
      if constexpr (Q == 1) {
        if (p.inl && p.grp == 64 && p.red == 2) {       // records formed while staging (small calls)
          launch(std::integral_constant<int, 64>{}, R2{}, std::integral_constant<bool, true>{});
          return hipGetLastError();
        }
      }
      if (p.grp == 64) {
        if (p.red == 2) launch(std::integral_constant<int, 64>{}, R2{}, NoInl{});
        else launch(std::integral_constant<int, 64>{}, R1{}, NoInl{});
      } else if (p.grp == 32) {
        if (p.red == 2) launch(std::integral_constant<int, 32>{}, R2{}, NoInl{});
        else launch(std::integral_constant<int, 32>{}, R1{}, NoInl{});
      } else {
        if (p.red == 2) launch(std::integral_constant<int, 16>{}, R2{}, NoInl{});
        else launch(std::integral_constant<int, 16>{}, R1{}, NoInl{});
      }
      return hipGetLastError();
    }
    if (p.grp == 64 && p.red == 0)
      bwd_kernel<MODE, Q, FK, 64, 0, GF><<<grid, kThreads, 0, st>>>(
          r, k0, k1, per, x, ff, p.lanes, nblk, pa, g, gf, b.carry_in, b.direct);
    else if (p.grp == 64)
      bwd_kernel<MODE, Q, FK, 64, 1, GF><<<grid, kThreads, 0, st>>>(
          r, k0, k1, per, x, ff, p.lanes, nblk, pa, g, gf, b.carry_in, b.direct);
    else if (p.grp == 16 && p.red == 0)
      bwd_kernel<MODE, Q, FK, 16, 0, GF><<<grid, kThreads, 0, st>>>(
          r, k0, k1, per, x, ff, p.lanes, nblk, pa, g, gf, b.carry_in, b.direct);
    else if (p.grp == 16)
      bwd_kernel<MODE, Q, FK, 16, 1, GF><<<grid, kThreads, 0, st>>>(
          r, k0, k1, per, x, ff, p.lanes, nblk, pa, g, gf, b.carry_in, b.direct);
    else if (p.red == 0)
      bwd_kernel<MODE, Q, FK, 32, 0, GF><<<grid, kThreads, 0, st>>>(
          r, k0, k1, per, x, ff, p.lanes, nblk, pa, g, gf, b.carry_in, b.direct);
    else
      bwd_kernel<MODE, Q, FK, 32, 1, GF><<<grid, kThreads, 0, st>>>(
          r, k0, k1, per, x, ff, p.lanes, nblk, pa, g, gf, b.carry_in, b.direct);
  }
  return hipGetLastError();
}

template <int MODE, int Q, bool GF>
hipError_t bwd_dispatch_fk(const Plan& p, const BwdArgs& b, hipStream_t st) {
  return p.fk ? bwd_dispatch<MODE, Q, 1, GF>(p, b, st) : bwd_dispatch<MODE, Q, 0, GF>(p, b, st);
}

template <int MODE, bool GF>
hipError_t bwd_dispatch_q(const Plan& p, const BwdArgs& b, hipStream_t st) {
  if (p.per_lane == 4) return bwd_dispatch_fk<MODE, 4, GF>(p, b, st);
  if (p.per_lane == 2) return bwd_dispatch_fk<MODE, 2, GF>(p, b, st);
  return bwd_dispatch_fk<MODE, 1, GF>(p, b, st);
}

template <int Q, int FK, bool GF>
hipError_t bwd_f64_launch(const Plan& p, const BwdArgs& b, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(p.blocks * p.nsplit));
  bwd_f64_kernel<Q, FK, GF><<<grid, kThreads, 0, st>>>(
      static_cast<const PointF64*>(b.rec), int(b.k_begin), int(b.k_end), int(b.per_split),
      static_cast<const double*>(b.xyz), static_cast<const double*>(b.f), p.lanes, int(p.blocks),
      static_cast<double*>(b.partial), static_cast<double*>(b.grad), static_cast<double*>(b.gradf),
      b.carry_in, b.direct);
  return hipGetLastError();
}

template <bool GF>
hipError_t bwd_f64_dispatch(const Plan& p, const BwdArgs& b, hipStream_t st) {
  if (p.per_lane == 2)
    return p.fk ? bwd_f64_launch<2, 1, GF>(p, b, st) : bwd_f64_launch<2, 0, GF>(p, b, st);
  return p.fk ? bwd_f64_launch<1, 1, GF>(p, b, st) : bwd_f64_launch<1, 0, GF>(p, b, st);
}

template <int G>
void bwd_reduce_launch(bool gf, bool polar, int nsplit, int64_t N, const float* pa, const float* ff,
                       float* g0, float* g1, hipStream_t st) {
  const int64_t waves = (N + 64 / G - 1) / (64 / G);
  const unsigned g = static_cast<unsigned>((waves * 64 + kThreads - 1) / kThreads);
  if (gf && polar) bwd_reduce_kernel<G, true, true><<<g, kThreads, 0, st>>>(pa, nsplit, N, ff, g0, g1);
  else if (gf) bwd_reduce_kernel<G, true, false><<<g, kThreads, 0, st>>>(pa, nsplit, N, ff, g0, g1);
  else if (polar) bwd_reduce_kernel<G, false, true><<<g, kThreads, 0, st>>>(pa, nsplit, N, ff, g0, g1);
  else bwd_reduce_kernel<G, false, false><<<g, kThreads, 0, st>>>(pa, nsplit, N, ff, g0, g1);
}

}  // namespace

hipError_t launch_pack_points(int mode, int red, const void* S, const void* G, int64_t k,
                              void* rec, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  const unsigned g = grid_for(k);
  const double offset = kPhaseShift + (red == 1 ? 0.5 : 0.0);
  if (mode == kF64) pack_points_kernel<kF64><<<g, kThreads, 0, st>>>(S, G, k, rec, 0.0);
  else if (mode == kPH64)
    pack_points_ph_kernel<<<g, kThreads, 0, st>>>(
        static_cast<const float*>(S), static_cast<const float*>(G), k, static_cast<PointPH*>(rec),
        reinterpret_cast<float*>(static_cast<char*>(rec) + point_bound_offset(k)), offset);
  else pack_points_kernel<kF32><<<g, kThreads, 0, st>>>(S, G, k, rec, 0.0);
  return hipGetLastError();
}

hipError_t launch_pack_points_grid(const Plan& p, const GridDef& g, const float* G, void* rec,
                                   hipStream_t st) {
  const int64_t k = p.stream;
  if (k <= 0) return hipSuccess;
  char* base = static_cast<char*>(rec);
  if (p.grid == 2)
    pack_points_grid_kernel<true><<<grid_for(k), kThreads, 0, st>>>(
        g, G, k, rec, reinterpret_cast<float4*>(base + row_group_offset(k)),
        reinterpret_cast<float*>(base + row_bound_offset(k)));
  else
    pack_points_grid_kernel<false><<<grid_for(k), kThreads, 0, st>>>(
        g, G, k, rec, nullptr, reinterpret_cast<float*>(base + point_bound_offset(k)));
  return hipGetLastError();
}

namespace {
template <int Q, int FK>
void bwd_rows_launch(const Plan& p, const void* rec, int64_t k_begin, int64_t k_end, int64_t per_split,
                     const void* xyz, const void* f, void* partial, void* grad, int carry_in, int direct,
                     const GridDef& g, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(p.blocks * p.nsplit));
  const char* base = static_cast<const char*>(rec);
  bwd_rows_kernel<Q, FK><<<grid, kThreads, 0, st>>>(
      static_cast<const PointRow*>(rec), reinterpret_cast<const float4*>(base + row_group_offset(p.stream)),
      reinterpret_cast<const float*>(base + row_bound_offset(p.stream)), int(k_begin), int(k_end),
      int(per_split), static_cast<const float*>(xyz), static_cast<const float*>(f), p.lanes, int(p.blocks),
      static_cast<float*>(partial), static_cast<float*>(grad), carry_in, direct, g);
}
}  // namespace

hipError_t launch_bwd_chunk(const Plan& p, const void* rec, int64_t k_begin, int64_t k_end,
                            int64_t per_split, const void* xyz, const void* f, void* partial,
                            void* grad, void* gradf, int carry_in, int direct, hipStream_t st,
                            const void* S, const void* G, const GridDef* gd) {
  if (p.mode == kPH64 && p.grid == 2 && gd && !p.gf) {
#define NX_GRID_BWD(Q, FK) \
  bwd_rows_launch<Q, FK>(p, rec, k_begin, k_end, per_split, xyz, f, partial, grad, carry_in, direct, *gd, st)
    if (p.fk) {
      if (p.per_lane == 4) NX_GRID_BWD(4, 1);
      else if (p.per_lane == 2) NX_GRID_BWD(2, 1);
      else NX_GRID_BWD(1, 1);
    } else {
      if (p.per_lane == 4) NX_GRID_BWD(4, 0);
      else if (p.per_lane == 2) NX_GRID_BWD(2, 0);
      else NX_GRID_BWD(1, 0);
    }
#undef NX_GRID_BWD
    return hipGetLastError();
  }
  const BwdArgs b{rec, k_begin, k_end, per_split, xyz, f, partial, grad, gradf, carry_in, direct, S, G};
  if (p.mode == kF64) return p.gf ? bwd_f64_dispatch<true>(p, b, st) : bwd_f64_dispatch<false>(p, b, st);
  if (p.mode == kPH64) return p.gf ? bwd_dispatch_q<kPH64, true>(p, b, st) : bwd_dispatch_q<kPH64, false>(p, b, st);
  return p.gf ? bwd_dispatch_q<kF32, true>(p, b, st) : bwd_dispatch_q<kF32, false>(p, b, st);
}

hipError_t launch_bwd_reduce(const Plan& p, const void* partial, const void* f, void* grad,
                             void* gradf, hipStream_t st) {
  const int64_t N = p.lanes;
  const unsigned g = static_cast<unsigned>((N + kThreads - 1) / kThreads);
  if (p.mode == kF64) {
    if (p.gf)
      bwd_reduce_f64_kernel<true><<<g, kThreads, 0, st>>>(static_cast<const double*>(partial), p.nsplit, N,
                                                         static_cast<double*>(grad), static_cast<double*>(gradf));
    else
      bwd_reduce_f64_kernel<false><<<g, kThreads, 0, st>>>(static_cast<const double*>(partial), p.nsplit, N,
                                                          static_cast<double*>(grad), static_cast<double*>(gradf));
  } else {
    const auto* pa = static_cast<const float*>(partial);
    const auto* ff = static_cast<const float*>(f);
    auto* g0 = static_cast<float*>(grad);
    auto* g1 = static_cast<float*>(gradf);
    const bool polar = p.mode == kPH64 && p.fk;
    switch (reduce_lanes(p.nsplit, N)) {
      case 64: bwd_reduce_launch<64>(p.gf, polar, p.nsplit, N, pa, ff, g0, g1, st); break;
      case 32: bwd_reduce_launch<32>(p.gf, polar, p.nsplit, N, pa, ff, g0, g1, st); break;
      case 16: bwd_reduce_launch<16>(p.gf, polar, p.nsplit, N, pa, ff, g0, g1, st); break;
      case 8: bwd_reduce_launch<8>(p.gf, polar, p.nsplit, N, pa, ff, g0, g1, st); break;
      case 4: bwd_reduce_launch<4>(p.gf, polar, p.nsplit, N, pa, ff, g0, g1, st); break;
      default: bwd_reduce_launch<1>(p.gf, polar, p.nsplit, N, pa, ff, g0, g1, st); break;
    }
  }
  return hipGetLastError();
}

}  // namespace nx
