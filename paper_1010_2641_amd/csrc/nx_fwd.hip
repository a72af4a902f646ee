// nx_fwd.hip -- forward direct scattering sum (Eq. 2 of Favre-Nicolin et al. 2010):
//     A_k = sum_j f_j exp(2 i pi S_k . r_j)
//
// Layout on gfx950: every lane owns P points (coalesced rows of S, strided by the
// work-group size), keeps their S and complex accumulators in registers, and walks
// the atoms of its slice in order.  The atom index is uniform over the wavefront, so
// every packed atom record is a broadcast.  Two forms (the paper shares atom
// coordinates between threads through on-chip memory for the same reason, Section 2.2):
//   fwd_kernel     -- records fetched with scalar loads into SGPRs and used as SGPR
//                     operands: no LDS traffic, no barriers (the FP32 mode; in the
//                     FP64-phase mode the phase addend is a second scalar operand of an
//                     fma and costs two copies per atom);
//   fwd_lds_kernel -- records staged per work-group in LDS tiles and read back as
//                     broadcasts (the FP64-phase default).
// Both sum in the same order, so their results are bitwise equal.
//
// Per (atom, point) pair:
//   F32  : phase S.r with FP32 fma, v_fract_f32, v_sin_f32/v_cos_f32 (both take the
//          angle in turns), plain FP32 complex multiply-add -- the paper's arithmetic.
//   PH64 : phase with FP64 fma (the products of FP32 inputs are exact in FP64),
//          reduction modulo one cycle in FP64 (exact), one rounding to FP32, FP32
//          v_sin/v_cos.  A complex f_j is taken in polar form m_j exp(2 i pi alpha_j):
//          alpha_j (FP64, cycles) rides in the addend of the phase's first fma and the
//          term is m_j (cos + i sin), two FP32 fma instead of four.  Terms are summed in
//          quads of consecutive atoms, quads into a group partial, and every `GRP` atoms
//          the group partial is folded into a two-word (sum, comp) accumulator by
//          Kahan's compensated addition (so FP32 roundings happen only at the magnitude
//          of a group partial, never at that of the whole sum).
//          Every group also carries a pseudo-random eighth turn k/8 (k = 0..7, a hash
//          of the group's index): the records of its atoms add k/8 to the phase addend,
//          and the group partial is turned back by exp(-2 i pi k/8) inside the first
//          addition of the compensated fold (two fma instead of one add).  The error of
//          the hardware sin/cos is a fixed periodic function of the reduced phase; its
//          harmonic p adds up over the atoms like an amplitude at p S_k, coherently
//          wherever that amplitude is large.  Under the turns harmonic p picks up the
//          factor exp(2 i pi (p - 1) k/8) per group, so every harmonic but p = 1 (a
//          relative scale error) and p = 1 mod 8 (measured negligible) adds up
//          incoherently.
//   F64  : phase, reduction, sin/cos (cis_f64) and sums all in FP64.
#include <type_traits>

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

// Kahan's compensated addition, with the correction kept as the error to add (sum + comp
// is the running total): the error of s + y is recovered exactly while |s| >= |y|, which
// holds once the running sum exceeds one group partial.  Here the addend is a group
// partial turned by (ck + i sk), and the turn takes the place of the first addition
// (two fma per component instead of one add): five FP32 operations per component.
__device__ __forceinline__ void kahan_rot(float& sr, float& cr, float& si, float& ci, float gr,
                                          float gi, float ck, float sk) {
  const float yr = __builtin_fmaf(ck, gr, __builtin_fmaf(-sk, gi, cr));
  const float yi = __builtin_fmaf(ck, gi, __builtin_fmaf(sk, gr, ci));
  const float tr = sr + yr;
  cr = yr - (tr - sr);
  sr = tr;
  const float ti = si + yi;
  ci = yi - (ti - si);
  si = ti;
}

// SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014): 64 pseudo-random
// bits of a 64-bit key.  The atoms' roundings use keys 2j, the groups' turns keys 2g + 1.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// m >= 0 to FP32 by unbiased (stochastic) rounding: the FP32 value above m with
// probability equal to the fraction of the gap by which m exceeds the value below it,
// drawn from the top 53 bits of mix64(2 j).  The expected result is m, so the rounding
// errors of atoms with equal factors are independent and add up incoherently instead
// of as one relative error of their species' amplitude.
__device__ __forceinline__ float round_unbiased(double m, int64_t j) {
  float lo = static_cast<float>(m);
  if (static_cast<double>(lo) > m) lo = __uint_as_float(__float_as_uint(lo) - 1u);
  const float hi = __uint_as_float(__float_as_uint(lo) + 1u);
  const double t = (m - static_cast<double>(lo)) / (static_cast<double>(hi) - static_cast<double>(lo));
  const double u = static_cast<double>(mix64(2 * static_cast<uint64_t>(j)) >> 11) * 0x1.0p-53;
  return u < t ? hi : lo;
}

// Any finite v to FP32 by unbiased rounding (round_unbiased of |v|, the sign put back),
// drawn from mix64(key).
__device__ __forceinline__ float round_unbiased_signed(double v, uint64_t key) {
  const double a = fabs(v);
  float lo = static_cast<float>(a);
  if (static_cast<double>(lo) > a) lo = __uint_as_float(__float_as_uint(lo) - 1u);
  const float hi = __uint_as_float(__float_as_uint(lo) + 1u);
  const double t = (a - static_cast<double>(lo)) / (static_cast<double>(hi) - static_cast<double>(lo));
  const double u = static_cast<double>(mix64(key) >> 11) * 0x1.0p-53;
  const float r = u < t ? hi : lo;
  return v < 0.0 ? -r : r;
}

// The FP64-phase record of atom j (indices counted from the first atom of a plan, which
// starts the plan's first group):
//   a  = arg f in cycles (0 for f = 1 or f = 0) + offset (kPhaseShift, plus 1/2 for the
//        fract variant) + k/8,
//   m  = |f| from FP64, rounded without bias (1 for f = 1),
//   (ck, sk) = sgn exp(-2 i pi k/8) in FP32, sgn = -1 for the fract variant,
// with k = 0..7 the turn of the atom's group g = j / grp, from mix64(2 g + 1).  The pack
// kernel writes it to the workspace; the forward of small calls forms it while staging
// its tile, so that both give the same record.
__device__ __forceinline__ AtomPH make_atom_ph(const float* __restrict__ xyz,
                                               const float* __restrict__ f, int64_t j,
                                               double offset, int grp, float sgn) {
  AtomPH r;
  r.x = xyz[3 * j]; r.y = xyz[3 * j + 1]; r.z = xyz[3 * j + 2];       // exact widening
  double alpha = 0.0;
  r.m = 1.f;
  if (f) {
    const double fr = f[2 * j], fi = f[2 * j + 1];
    if (fr != 0.0 || fi != 0.0) alpha = atan2(fi, fr) * 0.15915494309189533577;
    r.m = round_unbiased(sqrt(fr * fr + fi * fi), j);
  }
  const uint64_t g = static_cast<uint64_t>(j / grp);
  const int k = static_cast<int>(mix64(2 * g + 1) & 7u);
  r.a = alpha + offset + 0.125 * k;
  r.ck = sgn * static_cast<float>(cospi(0.25 * k));
  r.sk = -sgn * static_cast<float>(sinpi(0.25 * k));
  r.rmax = 0.f;
  return r;
}

// |v| as FP32, +inf when v is not finite: the tile bounds of the fixed-point reduction
// treat coordinates that are not finite as unbounded (their tiles take the centred form).
__device__ __forceinline__ float bound_abs(double v) {
  const float a = static_cast<float>(fabs(v));
  return a <= 3.402823466e38f ? a : __builtin_inff();
}

// Largest v over the wavefront (the tile bounds).
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// FP64-phase atom records, grid-stride over the blocks of 256 atoms of one plan; every
// record of a block carries the block's largest coordinate magnitude (rmax).
__global__ __launch_bounds__(kThreads) void pack_atoms_ph_kernel(const float* __restrict__ xyz,
                                                                 const float* __restrict__ f,
                                                                 int64_t n, AtomPH* __restrict__ rec,
                                                                 double offset, int grp, float sgn) {
  __shared__ float wmax[kThreads / 64];
  for (int64_t b = blockIdx.x; b * kThreads < n; b += gridDim.x) {
    const int64_t j = b * kThreads + threadIdx.x;
    AtomPH r;
    float am = 0.f;
    if (j < n) {
      r = make_atom_ph(xyz, f, j, offset, grp, sgn);
      am = fmaxf(bound_abs(r.x), fmaxf(bound_abs(r.y), bound_abs(r.z)));
    }
    am = wave_max(am);
    __syncthreads();                      // wmax of the previous block is read
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = am;
    __syncthreads();
    float bm = wmax[0];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) bm = fmaxf(bm, wmax[w]);
    if (j < n) {
      r.rmax = bm;
      rec[j] = r;
    }
  }
}

template <int MODE> struct AtomOf;
template <> struct AtomOf<kF32> { using type = AtomF32; };
template <> struct AtomOf<kPH64> { using type = AtomPH; };

// exp(2 i pi psi) for the FP64-phase mode as (c, s) in FP32, psi = S.r + arg f + k/8 (the
// group's eighth turn); the record's addend is a = arg f + k/8 + kPhaseShift (an integer)
// + the variant's offset:
//   RED 0 (offset 0):   t = (S.r + a) - rint(S.r + a) in [-1/2, 1/2] (exact), rounded once
//                       to FP32;
//   RED 1 (offset 1/2): u = fract(S.r + a) = fract(psi + 1/2) in [0, 1) (exact), rounded
//                       once to FP32, so that exp(2 i pi u) = -exp(2 i pi psi); the records'
//                       turn-back factor carries the -1;
//   RED 2 (offset 0):   t from the low word of S.r + a read as a 32-bit fixed-point turn
//                       (see kPhaseShift): the RED 0 value but at exactly half a turn, where
//                       the tile's bound holds (the kernels check it per tile);
//   3 (RED 2's fallback for tiles out of that range): t = (S.r + a) - rint(S.r + a), then
//                       the low word of t + kPhaseShift read in the same way.
template <int RED>
__device__ __forceinline__ void cis_turn(double ph, float& c, float& s) {
  float tf;
  if constexpr (RED == 0) tf = static_cast<float>(ph - __builtin_rint(ph));
  else if constexpr (RED == 1) tf = static_cast<float>(__builtin_amdgcn_fract(ph));
  else if constexpr (RED == 2) tf = static_cast<float>(__double2loint(ph)) * 0x1.0p-32f;
  else tf = static_cast<float>(__double2loint((ph - __builtin_rint(ph)) + kPhaseShift)) * 0x1.0p-32f;
  c = __builtin_amdgcn_cosf(tf);
  s = __builtin_amdgcn_sinf(tf);
}
template <int RED>
__device__ __forceinline__ void cis_ph64(double sx, double sy, double sz, const AtomPH& a, float& c,
                                         float& s) {
  cis_turn<RED>(__builtin_fma(sz, a.z, __builtin_fma(sy, a.y, __builtin_fma(sx, a.x, a.a))), c, s);
}

// Point (i1, i2, i3) of a grid, and the row part o + i2 e2 + i3 e3, in FP64.
// (Counts and indices stay below 2^30, so the index arithmetic is 32-bit.)
__device__ __forceinline__ void grid_point(const GridDef& g, int64_t k, double* S, double* R) {
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

// FP64-phase terms: the first term of a running sum, and the sum plus one more term.
// f = 1 (FK == 0): c + i s; complex f: m (c + i s), its angle being in the phase.
template <int FK>
__device__ __forceinline__ void first_term(const AtomPH& a, float c, float s, float& gr, float& gi) {
  if constexpr (FK == 0) {
    gr = c;
    gi = s;
  } else {
    gr = a.m * c;
    gi = a.m * s;
  }
}
template <int FK>
__device__ __forceinline__ void add_term(const AtomPH& a, float c, float s, float& gr, float& gi) {
  if constexpr (FK == 0) {
    gr += c;
    gi += s;
  } else {
    gr = __builtin_fmaf(a.m, c, gr);
    gi = __builtin_fmaf(a.m, s, gi);
  }
}

// (gr, gi) += f * (c + i s) with FP32 fma; f = 1 when FK == 0 (the FP32 mode).
template <int FK>
__device__ __forceinline__ void cmac(float& gr, float& gi, float fr, float fi, float c, float s) {
  if constexpr (FK == 0) {
    gr += c;
    gi += s;
  } else {
    gr = __builtin_fmaf(fr, c, gr);
    gr = __builtin_fmaf(-fi, s, gr);
    gi = __builtin_fmaf(fr, s, gi);
    gi = __builtin_fmaf(fi, c, gi);
  }
}

// Forward sum over atoms [a_begin + sp*per_split, ...) for P points per lane.
// Grid: blocks_k * nsplit work-groups; blockIdx = sp * blocks_k + kb.
template <int MODE, int P, int FK, int GRP, int RED>
__global__ __launch_bounds__(kThreads) void fwd_kernel(
    const typename AtomOf<MODE>::type* __restrict__ rec, int a_begin, int a_end, int per_split,
    const float* __restrict__ S, int64_t K, int blocks_k, float4* __restrict__ part,
    float2* __restrict__ A, int carry_in, int direct) {
  using SReg = typename std::conditional<MODE == kPH64, double, float>::type;
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int kb = lb % blocks_k;
  const int sp = lb / blocks_k;
  const int64_t k0 = int64_t(kb) * (kThreads * P) + threadIdx.x;

  SReg sx[P], sy[P], sz[P];
  float sr[P], si[P], cr[P], ci[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t k = k0 + int64_t(p) * kThreads;
    const int64_t kk = k < K ? k : K - 1;     // lanes past the end compute a valid point, store nothing
    sx[p] = static_cast<SReg>(S[3 * kk]);
    sy[p] = static_cast<SReg>(S[3 * kk + 1]);
    sz[p] = static_cast<SReg>(S[3 * kk + 2]);
    if (carry_in && k < K) {
      const float4 st = part[int64_t(sp) * K + k];
      sr[p] = st.x; si[p] = st.y; cr[p] = st.z; ci[p] = st.w;
    } else {
      sr[p] = 0.f; si[p] = 0.f; cr[p] = 0.f; ci[p] = 0.f;
    }
  }

  const int j0 = a_begin + sp * per_split;
  const int j1 = min(j0 + per_split, a_end);

  if constexpr (MODE == kF32) {
    // The paper's arithmetic: FP32 phase, FP32 reduction, plain FP32 running sums.
    for (int j = j0; j < j1; ++j) {
      const AtomF32 a = rec[j];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const float ph = __builtin_fmaf(sz[p], a.z, __builtin_fmaf(sy[p], a.y, sx[p] * a.x));
        const float u = __builtin_amdgcn_fractf(ph);
        const float c = __builtin_amdgcn_cosf(u);
        const float s = __builtin_amdgcn_sinf(u);
        cmac<FK>(sr[p], si[p], a.fr, a.fi, c, s);
      }
    }
  } else {
    // Groups start at multiples of GRP from the first record packed for this plan (the
    // chunk and split boundaries are multiples of GRP), so every group's atoms share
    // one eighth turn; its turn-back factor is read from the group's first record.
    int j = j0;
    for (; j + GRP <= j1; j += GRP) {
      // Group partial: GRP/4 quads, each the running sum of 4 consecutive terms, are
      // added into the group sum; the group sum is then turned back and folded into
      // (sum, comp).
      const float ck = rec[j].ck, sk = rec[j].sk;
      float gr[P], gi[P];
#pragma unroll
      for (int q = 0; q < GRP / 4; ++q) {
        float qr[P], qi[P];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const auto a = rec[j + 4 * q + u];
#pragma unroll
          for (int p = 0; p < P; ++p) {
            float c, s;
            cis_ph64<RED>(sx[p], sy[p], sz[p], a, c, s);
            if (u == 0) first_term<FK>(a, c, s, qr[p], qi[p]);
            else add_term<FK>(a, c, s, qr[p], qi[p]);
          }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
          if (q == 0) { gr[p] = qr[p]; gi[p] = qi[p]; }
          else { gr[p] += qr[p]; gi[p] += qi[p]; }
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) kahan_rot(sr[p], cr[p], si[p], ci[p], gr[p], gi[p], ck, sk);
    }
    if (j < j1) {   // last, partial group: terms added one by one
      const float ck = rec[j].ck, sk = rec[j].sk;
      float gr[P], gi[P];
#pragma unroll
      for (int p = 0; p < P; ++p) { gr[p] = 0.f; gi[p] = 0.f; }
      for (; j < j1; ++j) {
        const auto a = rec[j];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          float c, s;
          cis_ph64<RED>(sx[p], sy[p], sz[p], a, c, s);
          add_term<FK>(a, c, s, gr[p], gi[p]);
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) kahan_rot(sr[p], cr[p], si[p], ci[p], gr[p], gi[p], ck, sk);
    }
  }

#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t k = k0 + int64_t(p) * kThreads;
    if (k < K) {
      if (direct) A[k] = make_float2(sr[p] + cr[p], si[p] + ci[p]);
      else part[int64_t(sp) * K + k] = make_float4(sr[p], si[p], cr[p], ci[p]);
    }
  }
}

// FP64-phase forward with the atom records staged through LDS: each work-group copies a
// tile of kThreads records into LDS (one record per thread, coalesced), and every wave
// then reads the records from LDS as broadcasts.  Groups, quads and compensation are
// those of fwd_kernel (tiles are whole groups), so the result is bitwise the same.
// (At least 5 waves per SIMD: without the bound the compiler keeps whole groups of
// records in flight, up to 130 VGPRs for two points per lane, and three waves per SIMD
// then hide the LDS latency worse; with it the same loop takes 52.)
//
// RED 2: each wave checks the fixed-point bound for every tile, (|Sx| + |Sy| + |Sz|) of
// its points times the tile's largest coordinate magnitude (the rmax of the tile's first
// and last records, which cover the at most two pack blocks the tile overlaps), and
// takes the fallback (variant 3, same records) for a tile where some lane fails it.
//
// INL (small calls): no packed records; each thread forms its record of the tile from
// xyz and f while staging it (make_atom_ph, as the pack kernel does), which saves the pack
// dispatch when few work-groups share each record; the tile's bound is then reduced over
// its own records.  The FP64 arctangent of the record needs more registers than 5 waves
// per SIMD leave, so this form is built for 4.
//
// GRID: the points are those of a grid (gd), formed in FP64 by each lane, instead of S.
template <int P, int FK, int GRP, int RED, bool INL, bool GRID = false>
__global__ __launch_bounds__(kThreads, INL ? 4 : 5) void fwd_lds_kernel(
    const AtomPH* __restrict__ rec, int a_begin, int a_end, int per_split,
    const float* __restrict__ S, int64_t K, int blocks_k, float4* __restrict__ part,
    float2* __restrict__ A, int carry_in, int direct, const float* __restrict__ xyz,
    const float* __restrict__ f, GridDef gd) {
  static_assert(kThreads % GRP == 0, "tiles must hold whole groups");
  using AT = AtomPH;
  __shared__ AT tile[kThreads];
  __shared__ float wmax[kThreads / 64];
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int kb = lb % blocks_k;
  const int sp = lb / blocks_k;
  const int64_t k0 = int64_t(kb) * (kThreads * P) + threadIdx.x;
  double sx[P], sy[P], sz[P];
  float sr[P], si[P], cr[P], ci[P];
  float s1 = 0.f;                           // the lane's |Sx| + |Sy| + |Sz| (largest over p)
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t k = k0 + int64_t(p) * kThreads;
    const int64_t kk = k < K ? k : K - 1;
    if constexpr (GRID) {    // the points of a grid, in FP64
      double G3[3], R3[3];
      grid_point(gd, kk, G3, R3);
      sx[p] = G3[0];
      sy[p] = G3[1];
      sz[p] = G3[2];
    } else {
      sx[p] = S[3 * kk];
      sy[p] = S[3 * kk + 1];
      sz[p] = S[3 * kk + 2];
    }
    s1 = fmaxf(s1, bound_abs(fabs(sx[p]) + fabs(sy[p]) + fabs(sz[p])));
    if (carry_in && k < K) {
      const float4 st = part[int64_t(sp) * K + k];
      sr[p] = st.x; si[p] = st.y; cr[p] = st.z; ci[p] = st.w;
    } else {
      sr[p] = 0.f; si[p] = 0.f; cr[p] = 0.f; ci[p] = 0.f;
    }
  }
  // the groups of one tile, reduced with the variant R
  auto run_tile = [&](auto red_c, int nt) {
    constexpr int R = decltype(red_c)::value;
    int u0 = 0;
    for (; u0 + GRP <= nt; u0 += GRP) {
      const float ck = tile[u0].ck, sk = tile[u0].sk;
      float gr[P], gi[P];
#pragma unroll
      for (int q = 0; q < GRP / 4; ++q) {
        float qr[P], qi[P];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const AT a = tile[u0 + 4 * q + u];
#pragma unroll
          for (int p = 0; p < P; ++p) {
            float c, s;
            cis_ph64<R>(sx[p], sy[p], sz[p], a, c, s);
            if (u == 0) first_term<FK>(a, c, s, qr[p], qi[p]);
            else add_term<FK>(a, c, s, qr[p], qi[p]);
          }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
          if (q == 0) { gr[p] = qr[p]; gi[p] = qi[p]; }
          else { gr[p] += qr[p]; gi[p] += qi[p]; }
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) kahan_rot(sr[p], cr[p], si[p], ci[p], gr[p], gi[p], ck, sk);
    }
    if (u0 < nt) {    // the split's last, partial group
      const float ck = tile[u0].ck, sk = tile[u0].sk;
      float gr[P], gi[P];
#pragma unroll
      for (int p = 0; p < P; ++p) { gr[p] = 0.f; gi[p] = 0.f; }
      for (int u = u0; u < nt; ++u) {
        const AT a = tile[u];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          float c, s;
          cis_ph64<R>(sx[p], sy[p], sz[p], a, c, s);
          add_term<FK>(a, c, s, gr[p], gi[p]);
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) kahan_rot(sr[p], cr[p], si[p], ci[p], gr[p], gi[p], ck, sk);
    }
  };
  const int j0 = a_begin + sp * per_split;
  const int j1 = min(j0 + per_split, a_end);
  for (int t0 = j0; t0 < j1; t0 += kThreads) {
    const int nt = min(kThreads, j1 - t0);
    __syncthreads();                        // the previous tile is no longer read
    float am = 0.f;
    if (int(threadIdx.x) < nt) {
      if constexpr (INL) {    // f = 1 (FK == 0): no factor to take apart
        const AT r = make_atom_ph(xyz, FK ? f : nullptr, t0 + threadIdx.x,
                                  kPhaseShift + (RED == 1 ? 0.5 : 0.0), GRP, RED == 1 ? -1.f : 1.f);
        tile[threadIdx.x] = r;
        am = fmaxf(bound_abs(r.x), fmaxf(bound_abs(r.y), bound_abs(r.z)));
      } else {
        tile[threadIdx.x] = rec[t0 + threadIdx.x];
      }
    }
    if constexpr (INL && RED == 2) {
      am = wave_max(am);
      if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = am;
    }
    __syncthreads();
    if constexpr (RED == 2) {
      float rt;
      if constexpr (INL) {
        rt = wmax[0];
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) rt = fmaxf(rt, wmax[w]);
      } else {
        rt = fmaxf(tile[0].rmax, tile[nt - 1].rmax);
      }
      if (__all(s1 * rt < kFixedPhaseBound)) run_tile(std::integral_constant<int, 2>{}, nt);
      else run_tile(std::integral_constant<int, 3>{}, nt);
    } else {
      run_tile(std::integral_constant<int, RED>{}, nt);
    }
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t k = k0 + int64_t(p) * kThreads;
    if (k < K) {
      if (direct) A[k] = make_float2(sr[p] + cr[p], si[p] + ci[p]);
      else part[int64_t(sp) * K + k] = make_float4(sr[p], si[p], cr[p], ci[p]);
    }
  }
}

// Grid atom records (AtomGrid): the AtomPH record of atom j (same addend, factor, turn
// and rounding) with its position folded into c0 = o.r + a and c_d = e_d.r, in FP64, and
// the steps exp(2 i pi c_d) - 1 that the plan's block shape takes (bit d - 1 of `steps`;
// the others are written as 0 and never read: each costs two FP64 sinpi and two
// roundings, most of the pack's time when the block has one point); rmax as in
// pack_atoms_ph_kernel.
__global__ __launch_bounds__(kThreads) void pack_atoms_grid_kernel(const float* __restrict__ xyz,
                                                                   const float* __restrict__ f,
                                                                   int64_t n, AtomGrid* __restrict__ rec,
                                                                   GridDef g, int grp, int steps) {
  __shared__ float wmax[kThreads / 64];
  for (int64_t b = blockIdx.x; b * kThreads < n; b += gridDim.x) {
    const int64_t j = b * kThreads + threadIdx.x;
    AtomGrid r;
    float am = 0.f;
    if (j < n) {
      const AtomPH a = make_atom_ph(xyz, f, j, kPhaseShift, grp, 1.f);
      r.c0 = __builtin_fma(g.o[2], a.z, __builtin_fma(g.o[1], a.y, __builtin_fma(g.o[0], a.x, a.a)));
      r.c1 = __builtin_fma(g.e1[2], a.z, __builtin_fma(g.e1[1], a.y, g.e1[0] * a.x));
      r.c2 = __builtin_fma(g.e2[2], a.z, __builtin_fma(g.e2[1], a.y, g.e2[0] * a.x));
      r.c3 = __builtin_fma(g.e3[2], a.z, __builtin_fma(g.e3[1], a.y, g.e3[0] * a.x));
      r.m = a.m;
      r.ck = a.ck;
      r.sk = a.sk;
      // exp(2 i pi c) - 1 = (-2 sin^2 pi t, sin 2 pi t), t = c mod 1, for c1, c2 and c3,
      // rounded without bias (keys of their own: j with a tag 1..6 in bits 60-62)
      const uint64_t key = static_cast<uint64_t>(j);
      r.wr = r.wi = r.vr = r.vi = r.xr = r.xi = 0.f;
      if (steps & 1) {
        const double t1 = r.c1 - __builtin_rint(r.c1), h1 = sinpi(t1);
        r.wr = round_unbiased_signed(-2.0 * h1 * h1, key | (1ull << 60));
        r.wi = round_unbiased_signed(sinpi(2.0 * t1), key | (2ull << 60));
      }
      if (steps & 2) {
        const double t2 = r.c2 - __builtin_rint(r.c2), h2 = sinpi(t2);
        r.vr = round_unbiased_signed(-2.0 * h2 * h2, key | (3ull << 60));
        r.vi = round_unbiased_signed(sinpi(2.0 * t2), key | (4ull << 60));
      }
      if (steps & 4) {
        const double t3 = r.c3 - __builtin_rint(r.c3), h3 = sinpi(t3);
        r.xr = round_unbiased_signed(-2.0 * h3 * h3, key | (5ull << 60));
        r.xi = round_unbiased_signed(sinpi(2.0 * t3), key | (6ull << 60));
      }
      r.pad0 = 0.f;
      r.pad1 = 0.f;
      am = fmaxf(bound_abs(a.x), fmaxf(bound_abs(a.y), bound_abs(a.z)));
    }
    am = wave_max(am);
    __syncthreads();                      // wmax of the previous block is read
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = am;
    __syncthreads();
    float bm = wmax[0];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) bm = fmaxf(bm, wmax[w]);
    if (j < n) {
      r.rmax = bm;
      rec[j] = r;
    }
  }
}

// FP64-phase forward over a grid whose rows hold a multiple of 64 points, a block of
// BA x BB x BC points per lane: (i1 + a, i2 + b, i3 + c), 0 <= a < BA, 0 <= b < BB,
// 0 <= c < BC (each 1 or 2), with i1 a multiple of BA, i2 of BB and i3 of BC.  Each wave
// covers 64 BA consecutive points of BB x BC rows (task t = 4 (work-group) + wave: segment
// t % (n1 / (64 BA)) of row block t / (n1 / (64 BA)); waves past the last task compute
// nothing that is written).
//
// The phase of atom j at point (i1, i2, i3) is i1 c1_j + b_j with the base row's term
// b = c0 + i2 c2 + i3 c3: the thread that stages atom j into the LDS tile forms b for the
// base rows of the work-group's 4 waves (two fma each; the rows' indices sit in LDS, not in
// registers), so the first point's phase is one FP64 fma instead of three.  Its phase
// factor E comes from the fixed-point read and hardware cos and sin; the block's other
// points take theirs by steps, E + E (s - 1) in FP32 (four fma) with the atom's steps
// w - 1, v - 1, x - 1 (along the row, to i2 + 1, to i3 + 1) from its record: (a, b, c) from
// (a, b, c - 1) by x, else from (a, b - 1, 0) by v, else from (a - 1, 0, 0) by w, at most
// three steps from E.  Groups, quads, eighth turns and compensation per point are those of
// fwd_lds_kernel; the range check covers every point of the block (its |S|_1 and that of
// its row parts o + i2 e2 + i3 e3, so that the row term stays in range too) and takes
// variant 3 for tiles out of range.  Built for 8 waves per SIMD with one or two points per
// lane, 5 with four, 3 with eight (no spills).
constexpr int block_waves(int p) { return p <= 2 ? 8 : p == 4 ? 5 : 3; }

template <int FK, int GRP, int BA, int BB, int BC>
__global__ __launch_bounds__(kThreads, block_waves(BA * BB * BC)) void fwd_block_kernel(
    const AtomGrid* __restrict__ rec, int a_begin, int a_end, int per_split, GridDef g, int64_t K,
    int blocks_k, float4* __restrict__ part, float2* __restrict__ A, int carry_in, int direct) {
  static_assert(kThreads % GRP == 0, "tiles must hold whole groups");
  constexpr int P = BA * BB * BC;
  // the tile holds the steps the shape uses, in the order w, v, x (32 or 48 B per atom:
  // with every step in every shape's record the compiler kept up to twice the registers)
  constexpr int NS = (BA == 2) + (BB == 2) + (BC == 2);
  // (the index of a step the shape does not take is 0: those branches never run)
  constexpr int IW = 0, IV = BB == 2 ? (BA == 2) : 0, IX = BC == 2 ? (BA == 2) + (BB == 2) : 0;
  // blocks of eight points keep each atom's c1 beside its row term per wave (one 16-byte
  // LDS read for the phase) and its factor before its steps: 49 LDS reads per 16 atoms
  // instead of 57, C2's forward 2.4 % faster with the same results; with four points the
  // larger staging cost more than it saved (C3, C4 2 % slower), and one or two points keep
  // the smaller tile of 8 waves per SIMD
  constexpr bool FUSE = P == 8;
  struct alignas(16) TileN { double c1; float m, ck, sk, rmax; float st[NS > 0 ? NS : 1][2]; };
  struct alignas(16) TileF { float m; float st[NS > 0 ? NS : 1][2]; float ck, sk, rmax; };
  using Tile = std::conditional_t<FUSE, TileF, TileN>;
  __shared__ Tile tile[kThreads];
  // the base row's term per wave and atom (and, with FUSE, the atom's c1 beside it)
  __shared__ std::conditional_t<FUSE, double2, double> rowb[kThreads / 64][kThreads];
  __shared__ double rowd[kThreads / 64][2];          // (i2, i3) of the waves' base rows
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int kb = lb % blocks_k;
  const int sp = lb / blocks_k;
  const int wave = threadIdx.x >> 6;
  const uint32_t n1 = static_cast<uint32_t>(g.n1), n2 = static_cast<uint32_t>(g.n2);
  const uint32_t segs = n1 / (64 * BA), ntask = static_cast<uint32_t>(K / (64 * P));
  uint32_t k0;
  {
    uint32_t t = static_cast<uint32_t>(kb) * 4 + wave;
    if (t >= ntask) t = ntask - 1;
    const uint32_t rb = t / segs, seg = t - rb * segs;
    const uint32_t nb2 = n2 / BB;
    const uint32_t i3 = BC * (rb / nb2), i2 = BB * (rb - (rb / nb2) * nb2);
    k0 = seg * (64 * BA) + BA * (threadIdx.x & 63) + n1 * (i2 + n2 * i3);
    if ((threadIdx.x & 63) == 0) {
      rowd[wave][0] = static_cast<double>(i2);
      rowd[wave][1] = static_cast<double>(i3);
    }
  }
  const bool live = static_cast<uint32_t>(kb) * 4 + wave < ntask;
  uint32_t kp[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int a = p % BA, b = (p / BA) % BB, c = p / (BA * BB);
    kp[p] = k0 + a + n1 * (b + n2 * c);
  }
  const double di1 = static_cast<double>(k0 % n1);
  float s1 = 0.f;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    double S3[3], R3[3];
    grid_point(g, kp[p], S3, R3);
    s1 = fmaxf(s1, fmaxf(bound_abs(fabs(S3[0]) + fabs(S3[1]) + fabs(S3[2])),
                         bound_abs(fabs(R3[0]) + fabs(R3[1]) + fabs(R3[2]))));
  }
  float sr[P], si[P], cr[P], ci[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    sr[p] = si[p] = cr[p] = ci[p] = 0.f;
    if (carry_in && live) {
      const float4 st = part[int64_t(sp) * K + kp[p]];
      sr[p] = st.x; si[p] = st.y; cr[p] = st.z; ci[p] = st.w;
    }
  }
  // one atom against the block's points; the terms (m-weighted for complex f) into
  // (r[p], im[p])
  auto block_terms = [&](auto red_c, int uu, float* r, float* im, bool first) {
    constexpr int R = decltype(red_c)::value;
    double ph;
    if constexpr (FUSE) {
      const double2 rc = rowb[wave][uu];
      ph = __builtin_fma(di1, rc.y, rc.x);
    } else {
      ph = __builtin_fma(di1, tile[uu].c1, rowb[wave][uu]);
    }
    float z[P][2];
    cis_turn<R>(ph, z[0][0], z[0][1]);
    // z <- z + z (s - 1) for a step s - 1 = (sr_, si_)
    auto step = [](const float* q, float sr_, float si_, float* o) {
      o[0] = __builtin_fmaf(q[0], sr_, __builtin_fmaf(-q[1], si_, q[0]));
      o[1] = __builtin_fmaf(q[0], si_, __builtin_fmaf(q[1], sr_, q[1]));
    };
#pragma unroll
    for (int p = 1; p < P; ++p) {
      const int a = p % BA, b = (p / BA) % BB, c = p / (BA * BB);
      if (c > 0) step(z[p - BA * BB], tile[uu].st[IX][0], tile[uu].st[IX][1], z[p]);
      else if (b > 0) step(z[p - BA], tile[uu].st[IV][0], tile[uu].st[IV][1], z[p]);
      else if (a > 0) step(z[p - 1], tile[uu].st[IW][0], tile[uu].st[IW][1], z[p]);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if constexpr (FK == 0) {
        if (first) { r[p] = z[p][0]; im[p] = z[p][1]; }
        else { r[p] += z[p][0]; im[p] += z[p][1]; }
      } else {
        const float m = tile[uu].m;
        if (first) { r[p] = m * z[p][0]; im[p] = m * z[p][1]; }
        else { r[p] = __builtin_fmaf(m, z[p][0], r[p]); im[p] = __builtin_fmaf(m, z[p][1], im[p]); }
      }
    }
  };
  auto run_tile = [&](auto red_c, int nt) {
    int u0 = 0;
    for (; u0 + GRP <= nt; u0 += GRP) {
      const float ck = tile[u0].ck, sk = tile[u0].sk;
      float gr[P], gi[P];
#pragma unroll
      for (int q = 0; q < GRP / 4; ++q) {
        float qr[P], qi[P];
#pragma unroll
        for (int u = 0; u < 4; ++u) block_terms(red_c, u0 + 4 * q + u, qr, qi, u == 0);
#pragma unroll
        for (int p = 0; p < P; ++p) {
          if (q == 0) { gr[p] = qr[p]; gi[p] = qi[p]; }
          else { gr[p] += qr[p]; gi[p] += qi[p]; }
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) kahan_rot(sr[p], cr[p], si[p], ci[p], gr[p], gi[p], ck, sk);
    }
    if (u0 < nt) {    // the split's last, partial group
      const float ck = tile[u0].ck, sk = tile[u0].sk;
      float gr[P], gi[P];
#pragma unroll
      for (int p = 0; p < P; ++p) { gr[p] = 0.f; gi[p] = 0.f; }
      for (int uu = u0; uu < nt; ++uu) {
        float r[P], im[P];
        block_terms(red_c, uu, r, im, true);
#pragma unroll
        for (int p = 0; p < P; ++p) { gr[p] += r[p]; gi[p] += im[p]; }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) kahan_rot(sr[p], cr[p], si[p], ci[p], gr[p], gi[p], ck, sk);
    }
  };
  const int j0 = a_begin + sp * per_split;
  const int j1 = min(j0 + per_split, a_end);
  for (int t0 = j0; t0 < j1; t0 += kThreads) {
    const int nt = min(kThreads, j1 - t0);
    __syncthreads();                        // the previous tile is no longer read
    if (int(threadIdx.x) < nt) {
      const AtomGrid a = rec[t0 + threadIdx.x];
      Tile t;
      if constexpr (!FUSE) t.c1 = a.c1;
      t.m = a.m;
      t.ck = a.ck;
      t.sk = a.sk;
      t.rmax = a.rmax;
      if constexpr (BA == 2) { t.st[IW][0] = a.wr; t.st[IW][1] = a.wi; }
      if constexpr (BB == 2) { t.st[IV][0] = a.vr; t.st[IV][1] = a.vi; }
      if constexpr (BC == 2) { t.st[IX][0] = a.xr; t.st[IX][1] = a.xi; }
      if constexpr (NS == 0) { t.st[0][0] = 0.f; t.st[0][1] = 0.f; }
      tile[threadIdx.x] = t;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) {
        const double b = __builtin_fma(rowd[w][1], a.c3, __builtin_fma(rowd[w][0], a.c2, a.c0));
        if constexpr (FUSE) rowb[w][threadIdx.x] = make_double2(b, a.c1);
        else rowb[w][threadIdx.x] = b;
      }
    }
    __syncthreads();
    const float rt = fmaxf(tile[0].rmax, tile[nt - 1].rmax);
    if (__all(s1 * rt < kFixedPhaseBound)) run_tile(std::integral_constant<int, 2>{}, nt);
    else run_tile(std::integral_constant<int, 3>{}, nt);
  }
  if (live) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (direct) A[kp[p]] = make_float2(sr[p] + cr[p], si[p] + ci[p]);
      else part[int64_t(sp) * K + kp[p]] = make_float4(sr[p], si[p], cr[p], ci[p]);
    }
  }
}

// All-FP64 forward: FP64 phase, reduction and sin/cos (cis_f64), FP64 sums.
template <int P, int FK>
__global__ __launch_bounds__(kThreads) void fwd_f64_kernel(
    const AtomF64* __restrict__ rec, int a_begin, int a_end, int per_split,
    const double* __restrict__ S, int64_t K, int blocks_k, double2* __restrict__ part,
    double2* __restrict__ A, int carry_in, int direct) {
  const int lb = xcd_major_block(blockIdx.x, gridDim.x);
  const int kb = lb % blocks_k;
  const int sp = lb / blocks_k;
  const int64_t k0 = int64_t(kb) * (kThreads * P) + threadIdx.x;
  double sx[P], sy[P], sz[P], ar[P], ai[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t k = k0 + int64_t(p) * kThreads;
    const int64_t kk = k < K ? k : K - 1;
    sx[p] = S[3 * kk]; sy[p] = S[3 * kk + 1]; sz[p] = S[3 * kk + 2];
    if (carry_in && k < K) {
      const double2 st = part[int64_t(sp) * K + k];
      ar[p] = st.x; ai[p] = st.y;
    } else {
      ar[p] = 0.0; ai[p] = 0.0;
    }
  }
  const int j0 = a_begin + sp * per_split;
  const int j1 = min(j0 + per_split, a_end);
  for (int j = j0; j < j1; ++j) {
    const AtomF64 a = rec[j];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const double ph = __builtin_fma(sz[p], a.z, __builtin_fma(sy[p], a.y, sx[p] * a.x));
      double s, c;
      cis_f64(ph, c, s);
      if constexpr (FK == 0) {
        ar[p] += c; ai[p] += s;
      } else {
        ar[p] = __builtin_fma(a.fr, c, __builtin_fma(-a.fi, s, ar[p]));
        ai[p] = __builtin_fma(a.fr, s, __builtin_fma(a.fi, c, ai[p]));
      }
    }
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t k = k0 + int64_t(p) * kThreads;
    if (k < K) {
      if (direct) A[k] = make_double2(ar[p], ai[p]);
      else part[int64_t(sp) * K + k] = make_double2(ar[p], ai[p]);
    }
  }
}

// Combine the split partials of every point in a fixed order (deterministic): G lanes
// of one wave serve one point (G a power of two up to 64, about a quarter of the splits);
// lane i folds splits i, i + G, i + 2G, ... in sequence with Knuth's two-sum, then the G
// states are combined by a butterfly in which both partners fold the lower lane's state
// first, so that every lane holds the same total and the order of the additions is a
// fixed tree.  Few splits take G = 1 (one thread per point, splits in sequence).  A wave
// serves 64 / G consecutive points side by side (its lane w: point w % (64 / G), split
// lane w / (64 / G)), so that each load reads whole runs of consecutive partial states.
template <int G>
__global__ __launch_bounds__(kThreads) void fwd_reduce_kernel(const float4* __restrict__ part,
                                                              int nsplit, int64_t K,
                                                              float2* __restrict__ A) {
  static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "G: a power of two within a wave");
  constexpr int OPW = 64 / G;               // outputs per wave, side by side
  const int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  const int w = static_cast<int>(t & 63);
  const int64_t k = (t >> 6) * OPW + (w % OPW);
  const int lane = w / OPW;
  float sr = 0.f, si = 0.f, cr = 0.f, ci = 0.f;
  if (k < K) {
#pragma unroll 4
    for (int sp = lane; sp < nsplit; sp += G) {
      const float4 st = part[int64_t(sp) * K + k];
      two_sum_acc(sr, cr, st.x);
      two_sum_acc(si, ci, st.y);
      cr += st.z;
      ci += st.w;
    }
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    const float osr = __shfl_xor(sr, off * OPW), osi = __shfl_xor(si, off * OPW);
    const float ocr = __shfl_xor(cr, off * OPW), oci = __shfl_xor(ci, off * OPW);
    const bool upper = (lane & off) != 0;      // the partner is the lower lane: fold it first
    float ar = upper ? osr : sr, ai = upper ? osi : si, ac = upper ? ocr : cr, aci = upper ? oci : ci;
    const float br = upper ? sr : osr, bi = upper ? si : osi, bc = upper ? cr : ocr, bci = upper ? ci : oci;
    two_sum_acc(ar, ac, br);
    two_sum_acc(ai, aci, bi);
    sr = ar; si = ai;
    cr = ac + bc;
    ci = aci + bci;
  }
  if (k < K && lane == 0) A[k] = make_float2(sr + cr, si + ci);
}

__global__ __launch_bounds__(kThreads) void fwd_reduce_f64_kernel(const double2* __restrict__ part,
                                                                  int nsplit, int64_t K,
                                                                  double2* __restrict__ A) {
  const int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (k >= K) return;
  double sr = 0.0, si = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) {
    const double2 st = part[int64_t(sp) * K + k];
    sr += st.x;
    si += st.y;
  }
  A[k] = make_double2(sr, si);
}

// Atom records of the FP32 mode and the all-FP64 path (grid-stride over atoms).
template <int MODE>
__global__ __launch_bounds__(kThreads) void pack_atoms_kernel(const void* __restrict__ xyz_v,
                                                              const void* __restrict__ f_v,
                                                              int64_t n, void* __restrict__ rec_v) {
  for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n;
       j += int64_t(gridDim.x) * kThreads) {
    if constexpr (MODE == kF64) {
      const double* xyz = static_cast<const double*>(xyz_v);
      const double* f = static_cast<const double*>(f_v);
      AtomF64 r;
      r.x = xyz[3 * j]; r.y = xyz[3 * j + 1]; r.z = xyz[3 * j + 2];
      r.fr = f ? f[2 * j] : 1.0;
      r.fi = f ? f[2 * j + 1] : 0.0;
      r.pad = 0.0;
      static_cast<AtomF64*>(rec_v)[j] = r;
    } else {
      const float* xyz = static_cast<const float*>(xyz_v);
      const float* f = static_cast<const float*>(f_v);
      AtomF32 r;
      r.x = xyz[3 * j]; r.y = xyz[3 * j + 1]; r.z = xyz[3 * j + 2];
      r.fr = f ? f[2 * j] : 1.f;
      r.fi = f ? f[2 * j + 1] : 0.f;
      r.pad0 = r.pad1 = r.pad2 = 0.f;
      static_cast<AtomF32*>(rec_v)[j] = r;
    }
  }
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<unsigned>(b);
}

template <int MODE, int P, int FK>
hipError_t fwd_dispatch_red(const Plan& p, const void* rec, int64_t a_begin, int64_t a_end,
                            int64_t per_split, const void* S, void* partial, void* A,
                            int carry_in, int direct, hipStream_t st, int red, const float* xyz,
                            const float* f, const GridDef* gd) {
  using AT = typename AtomOf<MODE>::type;
  const dim3 grid(static_cast<unsigned>(p.blocks * p.nsplit));
  const auto* r = static_cast<const AT*>(rec);
  const auto* s = static_cast<const float*>(S);
  auto* pa = static_cast<float4*>(partial);
  auto* a = static_cast<float2*>(A);
  if constexpr (MODE == kF32) {   // plain FP32 sums: no groups, no reduction variants
    fwd_kernel<MODE, P, FK, 16, 0><<<grid, kThreads, 0, st>>>(
        r, int(a_begin), int(a_end), int(per_split), s, p.lanes, int(p.blocks), pa, a, carry_in, direct);
    return hipGetLastError();
  }
  if constexpr (MODE == kPH64) {
    if (gd) {       // grid points: the plan takes one point per lane, LDS tiles, RED 2
      if constexpr (P == 1) {
        if (p.inl && red == 2) {    // small calls: atom records formed while staging
          if (p.grp == 16)
            fwd_lds_kernel<1, FK, 16, 2, true, true><<<grid, kThreads, 0, st>>>(
                nullptr, int(a_begin), int(a_end), int(per_split), nullptr, p.lanes, int(p.blocks), pa,
                a, carry_in, direct, xyz, f, *gd);
          else
            fwd_lds_kernel<1, FK, 8, 2, true, true><<<grid, kThreads, 0, st>>>(
                nullptr, int(a_begin), int(a_end), int(per_split), nullptr, p.lanes, int(p.blocks), pa,
                a, carry_in, direct, xyz, f, *gd);
          return hipGetLastError();
        }
        if (p.grp == 16)
          fwd_lds_kernel<1, FK, 16, 2, false, true><<<grid, kThreads, 0, st>>>(
              r, int(a_begin), int(a_end), int(per_split), nullptr, p.lanes, int(p.blocks), pa, a,
              carry_in, direct, nullptr, nullptr, *gd);
        else
          fwd_lds_kernel<1, FK, 8, 2, false, true><<<grid, kThreads, 0, st>>>(
              r, int(a_begin), int(a_end), int(per_split), nullptr, p.lanes, int(p.blocks), pa, a,
              carry_in, direct, nullptr, nullptr, *gd);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    }
    if (p.lds && (p.grp == 16 || p.grp == 8)) {
      // records formed while staging (small calls): one point per lane, the fixed-point
      // reduction
      const bool inl = P == 1 && p.inl && red == 2;
      auto launch = [&](auto grp_c, auto red_c, auto inl_c) {
        fwd_lds_kernel<P, FK, decltype(grp_c)::value, decltype(red_c)::value, decltype(inl_c)::value>
            <<<grid, kThreads, 0, st>>>(decltype(inl_c)::value ? nullptr : r, int(a_begin), int(a_end),
                                        int(per_split), s, p.lanes, int(p.blocks), pa, a, carry_in,
                                        direct, xyz, f, GridDef{});
      };
      using I16 = std::integral_constant<int, 16>;
      using I8 = std::integral_constant<int, 8>;
      using R0 = std::integral_constant<int, 0>;
      using R1 = std::integral_constant<int, 1>;
      using R2 = std::integral_constant<int, 2>;
      using NoInl = std::integral_constant<bool, false>;
      if constexpr (P == 1) {
        if (inl) {
          if (p.grp == 16) launch(I16{}, R2{}, std::integral_constant<bool, true>{});
          else launch(I8{}, R2{}, std::integral_constant<bool, true>{});
          return hipGetLastError();
        }
      }
      // the fixed-point forms exist where their two tile loops fit the registers (the
      // plan sends the others to the centred form)
      if (p.grp == 16) {
        if constexpr (P <= 2) {
          if (red == 2) {
            launch(I16{}, R2{}, NoInl{});
            return hipGetLastError();
          }
        }
        if (red == 1) launch(I16{}, R1{}, NoInl{});
        else launch(I16{}, R0{}, NoInl{});
      } else {
        if constexpr (P == 1) {
          if (red == 2) {
            launch(I8{}, R2{}, NoInl{});
            return hipGetLastError();
          }
        }
        if (red == 1) launch(I8{}, R1{}, NoInl{});
        else launch(I8{}, R0{}, NoInl{});
      }
      return hipGetLastError();
    }
  }
  if (red == 2) red = 0;         // the scalar-load form has no per-tile bound: centred
  if (p.grp == 16 && red == 0)
    fwd_kernel<MODE, P, FK, 16, 0><<<grid, kThreads, 0, st>>>(
        r, int(a_begin), int(a_end), int(per_split), s, p.lanes, int(p.blocks), pa, a, carry_in, direct);
  else if (p.grp == 16 && red == 1)
    fwd_kernel<MODE, P, FK, 16, 1><<<grid, kThreads, 0, st>>>(
        r, int(a_begin), int(a_end), int(per_split), s, p.lanes, int(p.blocks), pa, a, carry_in, direct);
  else if (p.grp == 32 && red == 0)
    fwd_kernel<MODE, P, FK, 32, 0><<<grid, kThreads, 0, st>>>(
        r, int(a_begin), int(a_end), int(per_split), s, p.lanes, int(p.blocks), pa, a, carry_in, direct);
  else if (p.grp == 32 && red == 1)
    fwd_kernel<MODE, P, FK, 32, 1><<<grid, kThreads, 0, st>>>(
        r, int(a_begin), int(a_end), int(per_split), s, p.lanes, int(p.blocks), pa, a, carry_in, direct);
  else if (p.grp == 8 && red == 0)
    fwd_kernel<MODE, P, FK, 8, 0><<<grid, kThreads, 0, st>>>(
        r, int(a_begin), int(a_end), int(per_split), s, p.lanes, int(p.blocks), pa, a, carry_in, direct);
  else
    fwd_kernel<MODE, P, FK, 8, 1><<<grid, kThreads, 0, st>>>(
        r, int(a_begin), int(a_end), int(per_split), s, p.lanes, int(p.blocks), pa, a, carry_in, direct);
  return hipGetLastError();
}

template <int MODE, int P>
hipError_t fwd_dispatch_fk(const Plan& p, const void* rec, int64_t a_begin, int64_t a_end,
                           int64_t per_split, const void* S, void* partial, void* A,
                           int carry_in, int direct, hipStream_t st, const float* xyz, const float* f,
                           const GridDef* gd) {
  if (p.fk)
    return fwd_dispatch_red<MODE, P, 1>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in,
                                        direct, st, p.red, xyz, f, gd);
  return fwd_dispatch_red<MODE, P, 0>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in,
                                      direct, st, p.red, xyz, f, gd);
}

template <int MODE>
hipError_t fwd_dispatch_p(const Plan& p, const void* rec, int64_t a_begin, int64_t a_end,
                          int64_t per_split, const void* S, void* partial, void* A, int carry_in,
                          int direct, hipStream_t st, const float* xyz, const float* f,
                           const GridDef* gd) {
  switch (p.per_lane) {
    case 4: return fwd_dispatch_fk<MODE, 4>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st, xyz, f, gd);
    case 2: return fwd_dispatch_fk<MODE, 2>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st, xyz, f, gd);
    default: return fwd_dispatch_fk<MODE, 1>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st, xyz, f, gd);
  }
}

template <int P, int FK>
hipError_t fwd_f64_launch(const Plan& p, const void* rec, int64_t a_begin, int64_t a_end,
                          int64_t per_split, const void* S, void* partial, void* A, int carry_in,
                          int direct, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(p.blocks * p.nsplit));
  fwd_f64_kernel<P, FK><<<grid, kThreads, 0, st>>>(
      static_cast<const AtomF64*>(rec), int(a_begin), int(a_end), int(per_split),
      static_cast<const double*>(S), p.lanes, int(p.blocks), static_cast<double2*>(partial),
      static_cast<double2*>(A), carry_in, direct);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pack_atoms(int mode, int red, int grp, const void* xyz, const void* f, int64_t n,
                             void* rec, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned g = grid_for(n);
  if (mode == kF64) pack_atoms_kernel<kF64><<<g, kThreads, 0, st>>>(xyz, f, n, rec);
  else if (mode == kPH64)
    pack_atoms_ph_kernel<<<g, kThreads, 0, st>>>(static_cast<const float*>(xyz), static_cast<const float*>(f), n,
                                                 static_cast<AtomPH*>(rec),
                                                 kPhaseShift + (red == 1 ? 0.5 : 0.0), grp,
                                                 red == 1 ? -1.f : 1.f);
  else pack_atoms_kernel<kF32><<<g, kThreads, 0, st>>>(xyz, f, n, rec);
  return hipGetLastError();
}

hipError_t launch_pack_atoms_grid(const Plan& p, const float* xyz, const float* f, int64_t n,
                                  const GridDef& g, void* rec, hipStream_t st) {
  if (p.grid != 2) return launch_pack_atoms(p.mode, p.red, p.grp, xyz, f, n, rec, st);
  if (n <= 0) return hipSuccess;
  const int steps = (p.blk_a == 2 ? 1 : 0) | (p.blk_b == 2 ? 2 : 0) | (p.blk_c == 2 ? 4 : 0);
  pack_atoms_grid_kernel<<<grid_for(n), kThreads, 0, st>>>(xyz, f, n, static_cast<AtomGrid*>(rec), g,
                                                           p.grp, steps);
  return hipGetLastError();
}

hipError_t launch_fwd_chunk(const Plan& p, const void* rec, int64_t a_begin, int64_t a_end,
                            int64_t per_split, const void* S, void* partial, void* A,
                            int carry_in, int direct, hipStream_t st, const void* xyz, const void* f,
                            const GridDef* gd) {
  if (p.mode == kPH64 && p.grid == 2 && gd) {
    const dim3 grid(static_cast<unsigned>(p.blocks * p.nsplit));
    const auto* r = static_cast<const AtomGrid*>(rec);
    auto* pa = static_cast<float4*>(partial);
    auto* a = static_cast<float2*>(A);
    // the block shape (p.blk_a, p.blk_b, p.blk_c); with 8-atom groups one point per lane
    auto launch = [&](auto fk_c, auto grp_c) {
      constexpr int FK = decltype(fk_c)::value, GRP = decltype(grp_c)::value;
      const int shape = (p.blk_a - 1) | ((p.blk_b - 1) << 1) | ((p.blk_c - 1) << 2);
#define NX_BLOCK(BA, BB, BC)                                                                         \
  fwd_block_kernel<FK, GRP, BA, BB, BC><<<grid, kThreads, 0, st>>>(r, int(a_begin), int(a_end),      \
                                                                  int(per_split), *gd, p.lanes,      \
                                                                  int(p.blocks), pa, a, carry_in, direct)
      if constexpr (GRP == 16) {
        switch (shape) {
          case 1: NX_BLOCK(2, 1, 1); return;
          case 2: NX_BLOCK(1, 2, 1); return;
          case 3: NX_BLOCK(2, 2, 1); return;
          case 6: NX_BLOCK(1, 2, 2); return;
          case 7: NX_BLOCK(2, 2, 2); return;
          default: NX_BLOCK(1, 1, 1); return;
        }
      } else {
        (void)shape;
        NX_BLOCK(1, 1, 1);
        return;
      }
#undef NX_BLOCK
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using G8 = std::integral_constant<int, 8>;
    using G16 = std::integral_constant<int, 16>;
    if (p.fk) {
      if (p.grp == 16) launch(I1{}, G16{});
      else launch(I1{}, G8{});
    } else {
      if (p.grp == 16) launch(I0{}, G16{});
      else launch(I0{}, G8{});
    }
    return hipGetLastError();
  }
  if (p.mode == kF64) {
    if (p.per_lane == 2)
      return p.fk ? fwd_f64_launch<2, 1>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st)
                  : fwd_f64_launch<2, 0>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st);
    return p.fk ? fwd_f64_launch<1, 1>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st)
                : fwd_f64_launch<1, 0>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st);
  }
  if (p.mode == kPH64)
    return fwd_dispatch_p<kPH64>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st,
                                 static_cast<const float*>(xyz), static_cast<const float*>(f),
                                 p.grid ? gd : nullptr);
  return fwd_dispatch_p<kF32>(p, rec, a_begin, a_end, per_split, S, partial, A, carry_in, direct, st,
                              nullptr, nullptr, nullptr);
}

namespace {
template <int G>
void fwd_reduce_launch(const Plan& p, const void* partial, void* A, hipStream_t st) {
  const int64_t K = p.lanes;
  const int64_t waves = (K + 64 / G - 1) / (64 / G);
  const unsigned g = static_cast<unsigned>((waves * 64 + kThreads - 1) / kThreads);
  fwd_reduce_kernel<G><<<g, kThreads, 0, st>>>(static_cast<const float4*>(partial), p.nsplit, K,
                                              static_cast<float2*>(A));
}
}  // namespace

hipError_t launch_fwd_reduce(const Plan& p, const void* partial, void* A, hipStream_t st) {
  const int64_t K = p.lanes;
  if (p.mode == kF64) {
    const unsigned g = static_cast<unsigned>((K + kThreads - 1) / kThreads);
    fwd_reduce_f64_kernel<<<g, kThreads, 0, st>>>(static_cast<const double2*>(partial), p.nsplit, K,
                                                 static_cast<double2*>(A));
    return hipGetLastError();
  }
  switch (reduce_lanes(p.nsplit, K)) {
    case 64: fwd_reduce_launch<64>(p, partial, A, st); break;
    case 32: fwd_reduce_launch<32>(p, partial, A, st); break;
    case 16: fwd_reduce_launch<16>(p, partial, A, st); break;
    case 8: fwd_reduce_launch<8>(p, partial, A, st); break;
    case 4: fwd_reduce_launch<4>(p, partial, A, st); break;
    default: fwd_reduce_launch<1>(p, partial, A, st); break;
  }
  return hipGetLastError();
}

}  // namespace nx
