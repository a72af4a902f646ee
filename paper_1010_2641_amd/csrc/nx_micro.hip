// nx_micro.hip -- VALU issue-rate microbenchmarks of gfx950 for the roofline of the sums.
//
// Each kernel repeats the per-pair instruction sequence of one of the library's sums
// (the method's own work in the formulation the kernels use: phase, reduction, sin/cos,
// multiply-adds; see the kernels in nx_fwd.hip and nx_bwd.hip) on register operands
// only: no loads, no LDS, no barriers, no compensation and no loop overhead worth
// counting.  The lane-constant operands (the lane's points or atoms) sit in VGPRs; the
// values every lane shares (the other side of the pair) change every iteration and are
// formed by the scalar unit from the loop counter, so each VALU instruction takes at
// most one of them, as the sums do.  Each mix comes in two shapes, so that latency and
// the scheduling of the half-rate transcendentals around other work cannot hold it back:
// 4 (FP64 phase) or 8 (FP32) independent pairs per lane at 8 waves per SIMD, and twice
// the pairs at 4 waves per SIMD.  The better of the two rates is the issue ceiling of
// that instruction mix on this chip at the clock it runs under load.
//
// The results are stored once per lane so that nothing is optimised away; they mean
// nothing.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nx_micro.h"

namespace {

constexpr int kThreads = 256;
// Independent pairs per lane and iteration, narrow shape: 8 for the FP32 mixes, 4 for the
// FP64-phase mixes (their lane operands are FP64; 8 would not fit 64 VGPRs and spill).
// The wide shape doubles them at 4 waves per SIMD (128 VGPRs).
constexpr int kPairs32 = 8;
constexpr int kPairs64 = 4;

// A double whose value changes with the (wave-uniform) iteration j: its high word is
// offset by j, which moves the value by j * 2^-20 of its binade (scalar integer ops).
__device__ __forceinline__ double uniform_f64(uint32_t hi, uint32_t lo, int j) {
  return __hiloint2double(static_cast<int>(hi + static_cast<uint32_t>(j)), static_cast<int>(lo));
}
__device__ __forceinline__ float uniform_f32(uint32_t bits, int j) {
  return __uint_as_float(bits + (static_cast<uint32_t>(j) << 4));
}

// Makes a lane value opaque to the compiler (an empty asm statement that "modifies" the
// register), so that it stays in its register instead of being recomputed inside the loop
// from the lane index (rematerialisation would add VALU work the sums do not do).
template <typename T>
__device__ __forceinline__ void opaque(T& v) {
  asm volatile("" : "+v"(v));
}

// The clock under load: thread 0 of every work-group reads the shader-clock counter
// (s_memtime) and the constant-rate real-time counter (s_memrealtime) when it starts and
// when it ends, and stores the two differences (vector stores) in clk[2 b], clk[2 b + 1].
struct ClockMark {
  uint64_t t0 = 0, r0 = 0;
  __device__ __forceinline__ void start() {
    if (threadIdx.x == 0) {
      t0 = __builtin_amdgcn_s_memtime();
      r0 = __builtin_amdgcn_s_memrealtime();
    }
  }
  __device__ __forceinline__ void stop(unsigned long long* clk) {
    if (clk && threadIdx.x == 0) {
      const uint64_t t1 = __builtin_amdgcn_s_memtime();
      const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
      clk[2 * blockIdx.x] = t1 - t0;
      clk[2 * blockIdx.x + 1] = r1 - r0;
    }
  }
};

// The phase shift of the FP64-phase records (1.5 * 2^20 cycles): the phase then lies in
// [2^20, 2^21), and its low word is the centred turn in 32-bit fixed point.
constexpr double kShift = 1572864.0;

// FP64-phase forward: psi = 3 FP64 fma (the shift in the addend); the fixed-point turn
// (v_cvt_f32_i32 of the low word, scaled by 2^-32); cos, sin; m (c + i s) with 2 FP32 fma
// (complex f) or 2 adds (f = 1).
template <bool CF, int kPairs, int OCC>
__global__ __launch_bounds__(kThreads, OCC) void mix_fwd_ph64(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  const double lane = static_cast<double>(threadIdx.x + blockIdx.x * kThreads);
  double sx[kPairs], sy[kPairs], sz[kPairs], a0[kPairs];
  float ar[kPairs], ai[kPairs];
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    sx[p] = 1.0 + 1e-7 * lane + 0.01 * p;
    sy[p] = 0.5 - 2e-7 * lane + 0.02 * p;
    sz[p] = 4.0 + 3e-7 * lane - 0.01 * p;
    a0[p] = kShift + 1e-8 * lane + 0.125 * p;
    ar[p] = 0.f;
    ai[p] = 0.f;
    opaque(sx[p]);
    opaque(sy[p]);
    opaque(sz[p]);
    opaque(a0[p]);
  }
  for (int j = 0; j < iters; ++j) {
    const double x = uniform_f64(0x40240000u, 0x9999999au, j);      // ~10
    const double y = uniform_f64(0x40340000u, 0x33333333u, j);      // ~20
    const double z = uniform_f64(0x403e0000u, 0xccccccccu, j);      // ~30
    const float m = uniform_f32(0x41f80000u, j);                    // ~31
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      const double ph = __builtin_fma(sz[p], z, __builtin_fma(sy[p], y, __builtin_fma(sx[p], x, a0[p])));
      const float t = static_cast<float>(__double2loint(ph)) * 0x1.0p-32f;
      const float c = __builtin_amdgcn_cosf(t);
      const float s = __builtin_amdgcn_sinf(t);
      if constexpr (CF) {
        ar[p] = __builtin_fmaf(m, c, ar[p]);
        ai[p] = __builtin_fmaf(m, s, ai[p]);
      } else {
        ar[p] += c;
        ai[p] += s;
      }
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int p = 0; p < kPairs; ++p) acc += ar[p] - ai[p];
  out[threadIdx.x + blockIdx.x * kThreads] = acc;
  cm.stop(clk);
}

// FP64-phase adjoint: psi = 3 FP64 fma (+ 1 FP64 add of the atom's angle for complex f;
// the shift in the point's addend); the fixed-point turn (v_cvt_f32_i32 of the low word,
// scaled); sin; T_d += (|G| S_d) sin with 3 FP32 fma.
template <bool CF, int kPairs, int OCC>
__global__ __launch_bounds__(kThreads, OCC) void mix_bwd_ph64(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  const double lane = static_cast<double>(threadIdx.x + blockIdx.x * kThreads);
  double x[kPairs], y[kPairs], z[kPairs], d0[kPairs], al[kPairs];
  float t0[kPairs], t1[kPairs], t2[kPairs];
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    x[p] = 10.0 + 1e-6 * lane + 0.5 * p;
    y[p] = 20.0 - 2e-6 * lane + 0.25 * p;
    z[p] = 30.0 + 3e-6 * lane - 0.5 * p;
    d0[p] = kShift + 1e-8 * lane + 0.1 * p;
    al[p] = 0.3 - 2e-8 * lane - 0.05 * p;
    t0[p] = t1[p] = t2[p] = 0.f;
    opaque(x[p]);
    opaque(y[p]);
    opaque(z[p]);
    opaque(d0[p]);
    opaque(al[p]);
  }
  for (int j = 0; j < iters; ++j) {
    const double sx = uniform_f64(0x3ff00000u, 0x9999999au, j);     // ~1
    const double sy = uniform_f64(0x3fe00000u, 0x33333333u, j);     // ~0.5
    const double sz = uniform_f64(0x40100000u, 0xccccccccu, j);     // ~4
    const float gx = uniform_f32(0x3f800000u, j), gy = uniform_f32(0x3f000000u, j),
                gz = uniform_f32(0x40800000u, j);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      double ph = __builtin_fma(sz, z[p], __builtin_fma(sy, y[p], __builtin_fma(sx, x[p], d0[p])));
      if constexpr (CF) ph += al[p];
      const float t = static_cast<float>(__double2loint(ph)) * 0x1.0p-32f;
      const float s = __builtin_amdgcn_sinf(t);
      t0[p] = __builtin_fmaf(s, gx, t0[p]);
      t1[p] = __builtin_fmaf(s, gy, t1[p]);
      t2[p] = __builtin_fmaf(s, gz, t2[p]);
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int p = 0; p < kPairs; ++p) acc += t0[p] - t1[p] + t2[p];
  out[threadIdx.x + blockIdx.x * kThreads] = acc;
  cm.stop(clk);
}

// The same FP64-phase sequences in the sums' own shape: few lane items (1 point for the
// forward, 2 atoms for the adjoint) and kTile wave-uniform stream items per iteration,
// unrolled, as the sums' inner loops walk a group of records.
constexpr int kTile = 16;

template <bool CF>
__global__ __launch_bounds__(kThreads, 8) void mix_fwd_ph64_tile(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  const double lane = static_cast<double>(threadIdx.x + blockIdx.x * kThreads);
  double sx = 1.0 + 1e-7 * lane, sy = 0.5 - 2e-7 * lane, sz = 4.0 + 3e-7 * lane;
  float ar = 0.f, ai = 0.f;
  opaque(sx);
  opaque(sy);
  opaque(sz);
  for (int j = 0; j < iters; ++j) {
#pragma unroll
    for (int t = 0; t < kTile; ++t) {
      const double x = uniform_f64(0x40240000u + t, 0x9999999au, j);      // ~10
      const double y = uniform_f64(0x40340000u + t, 0x33333333u, j);      // ~20
      const double z = uniform_f64(0x403e0000u + t, 0xccccccccu, j);      // ~30
      const double a = kShift + 0.125 * t;
      const float m = uniform_f32(0x41f80000u + (t << 8), j);              // ~31
      const double ph = __builtin_fma(sz, z, __builtin_fma(sy, y, __builtin_fma(sx, x, a)));
      const float tt = static_cast<float>(__double2loint(ph)) * 0x1.0p-32f;
      const float c = __builtin_amdgcn_cosf(tt);
      const float s = __builtin_amdgcn_sinf(tt);
      if constexpr (CF) {
        ar = __builtin_fmaf(m, c, ar);
        ai = __builtin_fmaf(m, s, ai);
      } else {
        ar += c;
        ai += s;
      }
    }
  }
  out[threadIdx.x + blockIdx.x * kThreads] = ar - ai;
  cm.stop(clk);
}

template <bool CF>
__global__ __launch_bounds__(kThreads, 8) void mix_bwd_ph64_tile(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  const double lane = static_cast<double>(threadIdx.x + blockIdx.x * kThreads);
  double x[2], y[2], z[2], al[2];
  float t0[2], t1[2], t2[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    x[q] = 10.0 + 1e-6 * lane + 0.5 * q;
    y[q] = 20.0 - 2e-6 * lane + 0.25 * q;
    z[q] = 30.0 + 3e-6 * lane - 0.5 * q;
    al[q] = 0.3 - 2e-8 * lane - 0.05 * q;
    t0[q] = t1[q] = t2[q] = 0.f;
    opaque(x[q]);
    opaque(y[q]);
    opaque(z[q]);
    opaque(al[q]);
  }
  for (int j = 0; j < iters; ++j) {
#pragma unroll
    for (int t = 0; t < kTile; ++t) {
      const double sx = uniform_f64(0x3ff00000u + t, 0x9999999au, j);     // ~1
      const double sy = uniform_f64(0x3fe00000u + t, 0x33333333u, j);     // ~0.5
      const double sz = uniform_f64(0x40100000u + t, 0xccccccccu, j);     // ~4
      const double d0 = kShift + 0.1 * t;
      const float gx = uniform_f32(0x3f800000u + (t << 8), j), gy = uniform_f32(0x3f000000u + (t << 8), j),
                  gz = uniform_f32(0x40800000u + (t << 8), j);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double ph = __builtin_fma(sz, z[q], __builtin_fma(sy, y[q], __builtin_fma(sx, x[q], d0)));
        if constexpr (CF) ph += al[q];
        const float tt = static_cast<float>(__double2loint(ph)) * 0x1.0p-32f;
        const float s = __builtin_amdgcn_sinf(tt);
        t0[q] = __builtin_fmaf(s, gx, t0[q]);
        t1[q] = __builtin_fmaf(s, gy, t1[q]);
        t2[q] = __builtin_fmaf(s, gz, t2[q]);
      }
    }
  }
  out[threadIdx.x + blockIdx.x * kThreads] = t0[0] - t1[0] + t2[0] + t0[1] - t1[1] + t2[1];
  cm.stop(clk);
}

// The grid kernels' sequences (a grid walked by rows), in their own shapes.
//
// Forward, a 2 x 2 x 2 block of points per lane: per atom, the first point's phase
// fma(i1, c1, b) (i1 the lane's index along the row, c1 = step1.r and b the atom's row
// term, both shared by the wave), the fixed-point turn, cos and sin; the other seven
// points' phase factors stepped from it with the atom's steps w - 1, v - 1 and x - 1
// (seven steps of four fma); the eight terms accumulated (two fma or adds each).  The
// shared operands come from LDS in the kernel (vector registers): here the tile's row
// terms and steps stay in vector registers and c1 is formed by the scalar unit, which
// changes it every iteration (an addend from the scalar unit would have to be copied to
// vector registers first: the accumulating form of the FP64 fma overwrites its addend).
// 2 atoms per iteration.
constexpr int kTileGrid = 2;

template <bool CF>
__global__ __launch_bounds__(kThreads, 8) void mix_fwd_grid_tile(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  double di1 = static_cast<double>((threadIdx.x + blockIdx.x * kThreads) & 127);
  double b[kTileGrid];
  float st[kTileGrid][3][2];
#pragma unroll
  for (int t = 0; t < kTileGrid; ++t) {
    b[t] = kShift + 12.5 + 0.125 * t;
    opaque(b[t]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      st[t][d][0] = -1e-3f * (t + 1) * (d + 1);
      st[t][d][1] = 4e-2f * (t + 1) + 1e-2f * d;
      opaque(st[t][d][0]);
      opaque(st[t][d][1]);
    }
  }
  opaque(di1);
  float ar[8], ai[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) ar[p] = ai[p] = 0.f;
  for (int j = 0; j < iters; ++j) {
#pragma unroll
    for (int t = 0; t < kTileGrid; ++t) {
      const double c1 = uniform_f64(0x3f340000u + (t << 8), 0x9999999au, j);   // ~3e-4
      const float m = uniform_f32(0x41f80000u + (t << 8), j);              // ~31
      const double ph = __builtin_fma(di1, c1, b[t]);
      float z[8][2];
      const float tt = static_cast<float>(__double2loint(ph)) * 0x1.0p-32f;
      z[0][0] = __builtin_amdgcn_cosf(tt);
      z[0][1] = __builtin_amdgcn_sinf(tt);
      auto step = [](const float* a, const float* s, float* c) {
        c[0] = __builtin_fmaf(a[0], s[0], __builtin_fmaf(-a[1], s[1], a[0]));
        c[1] = __builtin_fmaf(a[0], s[1], __builtin_fmaf(a[1], s[0], a[1]));
      };
      step(z[0], st[t][0], z[1]);
      step(z[0], st[t][1], z[2]);
      step(z[1], st[t][1], z[3]);
#pragma unroll
      for (int p = 0; p < 4; ++p) step(z[p], st[t][2], z[p + 4]);
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if constexpr (CF) {
          ar[p] = __builtin_fmaf(m, z[p][0], ar[p]);
          ai[p] = __builtin_fmaf(m, z[p][1], ai[p]);
        } else {
          ar[p] += z[p][0];
          ai[p] += z[p][1];
        }
      }
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int p = 0; p < 8; ++p) acc += ar[p] - ai[p];
  out[threadIdx.x + blockIdx.x * kThreads] = acc;
  cm.stop(clk);
}

// Adjoint over grid rows, one 64-point group per iteration, two atoms per lane: per atom
// the group's first phase factor E (the row term b = c0 + i2 c2 + i3 c3 and the phase
// fma(i1, c1, b), 3 FP64 fma; the fixed-point turn, cos and sin), then per point v =
// Re G Im E - Im G Re E (mul, fma), a0 += v, a1 += u v and the step E + E (w - 1) (four fma;
// none after the last point), and per group the three S0_d a0 + e1_d a1 (two each).  The
// point's values (Re G, -Im G, u) are formed by the scalar unit, as the kernel loads them;
// the same sequence for complex f and f = 1.
template <bool CF>
__global__ __launch_bounds__(kThreads, 8) void mix_bwd_grid_tile(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  const double lane = static_cast<double>(threadIdx.x + blockIdx.x * kThreads);
  double c0[2], c1[2], c2[2], c3[2];
  float wr[2], wi[2], t0[2], t1[2], t2[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    c0[q] = kShift + 12.5 - 1e-6 * lane + 0.25 * q;
    c1[q] = 3e-4 + 1e-9 * lane + 1e-5 * q;
    c2[q] = 5e-4 - 1e-9 * lane + 2e-5 * q;
    c3[q] = 7e-4 + 2e-9 * lane - 1e-5 * q;
    wr[q] = -1e-3f * (q + 1);
    wi[q] = 4e-2f * (q + 1);
    t0[q] = t1[q] = t2[q] = 0.f;
    opaque(c0[q]);
    opaque(c1[q]);
    opaque(c2[q]);
    opaque(c3[q]);
    opaque(wr[q]);
    opaque(wi[q]);
  }
  for (int j = 0; j < iters; ++j) {
    const double d1 = uniform_f64(0x40500000u, 0x00000000u, j);           // ~64
    const double d2 = uniform_f64(0x40400000u, 0x00000000u, j);           // ~32
    const double d3 = uniform_f64(0x40300000u, 0x00000000u, j);           // ~16
    const float s0x = uniform_f32(0x40800000u, j), s0y = uniform_f32(0x3d000000u, j),
                s0z = uniform_f32(0x40800001u, j), e1x = uniform_f32(0x3a500000u, j),
                e1y = uniform_f32(0x3a100000u, j), e1z = uniform_f32(0x39d00000u, j);
    float er[2], ei[2], a0[2], a1[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double b = __builtin_fma(d3, c3[q], __builtin_fma(d2, c2[q], c0[q]));
      const double ph = __builtin_fma(d1, c1[q], b);
      const float tt = static_cast<float>(__double2loint(ph)) * 0x1.0p-32f;
      er[q] = __builtin_amdgcn_cosf(tt);
      ei[q] = __builtin_amdgcn_sinf(tt);
      a0[q] = 0.f;
      a1[q] = 0.f;
    }
#pragma unroll
    for (int u = 0; u < 64; ++u) {
      const float gr = uniform_f32(0x3f800000u + (u << 8), j), ngi = uniform_f32(0xbf000000u + (u << 8), j);
      const float uf = uniform_f32(0x3f800000u + (u << 12), j);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const float v = __builtin_fmaf(gr, ei[q], ngi * er[q]);
        a0[q] += v;
        a1[q] = __builtin_fmaf(uf, v, a1[q]);
        if (u + 1 < 64) {
          const float nr = __builtin_fmaf(er[q], wr[q], __builtin_fmaf(-ei[q], wi[q], er[q]));
          const float ni = __builtin_fmaf(er[q], wi[q], __builtin_fmaf(ei[q], wr[q], ei[q]));
          er[q] = nr;
          ei[q] = ni;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      t0[q] = __builtin_fmaf(s0x, a0[q], __builtin_fmaf(e1x, a1[q], t0[q]));
      t1[q] = __builtin_fmaf(s0y, a0[q], __builtin_fmaf(e1y, a1[q], t1[q]));
      t2[q] = __builtin_fmaf(s0z, a0[q], __builtin_fmaf(e1z, a1[q], t2[q]));
    }
  }
  out[threadIdx.x + blockIdx.x * kThreads] = t0[0] - t1[0] + t2[0] + t0[1] - t1[1] + t2[1];
  cm.stop(clk);
}

// The paper's FP32 arithmetic.  Forward: 3 FP32 fma, fract, cos, sin, then f (c + i s)
// with 4 fma (complex f) or 2 adds (f = 1).
template <bool CF, int kPairs, int OCC>
__global__ __launch_bounds__(kThreads, OCC) void mix_fwd_f32(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  const float lane = static_cast<float>(threadIdx.x + blockIdx.x * kThreads);
  float sx[kPairs], sy[kPairs], sz[kPairs], ar[kPairs], ai[kPairs];
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    sx[p] = 1.0f + 1e-7f * lane + 0.01f * p;
    sy[p] = 0.5f - 2e-7f * lane + 0.02f * p;
    sz[p] = 4.0f + 3e-7f * lane - 0.01f * p;
    ar[p] = ai[p] = 0.f;
    if constexpr (kPairs > kPairs32) {     // the wide shape: keep the lane values in registers
      opaque(sx[p]);
      opaque(sy[p]);
      opaque(sz[p]);
    }
  }
  for (int j = 0; j < iters; ++j) {
    const float x = uniform_f32(0x41200000u, j), y = uniform_f32(0x41a00000u, j),
                z = uniform_f32(0x41f00000u, j);
    const float fr = uniform_f32(0x41f80000u, j), fi = uniform_f32(0x3f800000u, j);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      const float ph = __builtin_fmaf(sz[p], z, __builtin_fmaf(sy[p], y, sx[p] * x));
      const float u = __builtin_amdgcn_fractf(ph);
      const float c = __builtin_amdgcn_cosf(u);
      const float s = __builtin_amdgcn_sinf(u);
      if constexpr (CF) {
        ar[p] = __builtin_fmaf(-fi, s, __builtin_fmaf(fr, c, ar[p]));
        ai[p] = __builtin_fmaf(fi, c, __builtin_fmaf(fr, s, ai[p]));
      } else {
        ar[p] += c;
        ai[p] += s;
      }
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int p = 0; p < kPairs; ++p) acc += ar[p] - ai[p];
  out[threadIdx.x + blockIdx.x * kThreads] = acc;
  cm.stop(clk);
}

// The paper's FP32 arithmetic, adjoint: 3 fma, fract, cos, sin; Im w = gr s - gi c (2),
// Re w (2) and v = fr Im w + fi Re w (2) for complex f; T_d += S_d v (3).
template <bool CF, int kPairs, int OCC>
__global__ __launch_bounds__(kThreads, OCC) void mix_bwd_f32(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  const float lane = static_cast<float>(threadIdx.x + blockIdx.x * kThreads);
  float x[kPairs], y[kPairs], z[kPairs], fr[kPairs], fi[kPairs], t0[kPairs], t1[kPairs], t2[kPairs];
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    x[p] = 10.f + 1e-6f * lane + 0.5f * p;
    y[p] = 20.f - 2e-6f * lane + 0.25f * p;
    z[p] = 30.f + 3e-6f * lane - 0.5f * p;
    fr[p] = 31.f - p;
    fi[p] = 1.f + p;
    t0[p] = t1[p] = t2[p] = 0.f;
    if constexpr (kPairs > kPairs32) {     // the wide shape: keep the lane values in registers
      opaque(x[p]);
      opaque(y[p]);
      opaque(z[p]);
    }
  }
  for (int j = 0; j < iters; ++j) {
    const float sx = uniform_f32(0x3f800000u, j), sy = uniform_f32(0x3f000000u, j),
                sz = uniform_f32(0x40800000u, j);
    const float gr = uniform_f32(0x3f400000u, j), gi = uniform_f32(0x3e800000u, j);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      const float ph = __builtin_fmaf(sz, z[p], __builtin_fmaf(sy, y[p], sx * x[p]));
      const float u = __builtin_amdgcn_fractf(ph);
      const float c = __builtin_amdgcn_cosf(u);
      const float s = __builtin_amdgcn_sinf(u);
      const float wim = __builtin_fmaf(-gi, c, gr * s);
      float v = wim;
      if constexpr (CF) {
        const float wre = __builtin_fmaf(gi, s, gr * c);
        v = __builtin_fmaf(fi[p], wre, fr[p] * wim);
      }
      t0[p] = __builtin_fmaf(v, sx, t0[p]);
      t1[p] = __builtin_fmaf(v, sy, t1[p]);
      t2[p] = __builtin_fmaf(v, sz, t2[p]);
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int p = 0; p < kPairs; ++p) acc += t0[p] - t1[p] + t2[p];
  out[threadIdx.x + blockIdx.x * kThreads] = acc;
  cm.stop(clk);
}

// Single-instruction rates: NP independent chains per lane of one instruction kind, 4 steps
// of each chain per iteration, for the cost of each kind per wave64 instruction: OP 0 FP32
// fma with a scalar operand (the three-operand encoding, v_fma_f32), 1 FP64 fma likewise,
// 2 v_sin_f32 on a turn in [-1/2, 1/2], 3 and 4 FP32 and FP64 fma accumulating into their
// destination with vector operands only (the two-operand encodings v_fmac_f32_e32,
// v_fmac_f64_e32, which the sums' inner loops mostly use), then the other kinds of the
// sums' loops: 5 v_add_f64, 6 v_rndne_f64, 7 v_fract_f64, 8 v_cvt_f32_i32 (on the bits of
// the previous result, a chain the compiler cannot fold), 9 v_cos_f32, 10 v_mul_f32_e32,
// 11 FP32 fma with vector operands only in the three-operand encoding (v_fma_f32,
// destination not the addend), 12 v_add_f32_e32.  The roundings, whose repetition the
// compiler could fold, pass their result through opaque() at every step, which adds no
// instruction.
template <int OP, int NP>
__global__ __launch_bounds__(kThreads, 8) void op_rate(int iters, float* out, unsigned long long* clk) {
  ClockMark cm;
  cm.start();
  const float lane = static_cast<float>(threadIdx.x + blockIdx.x * kThreads);
  float v[NP];
  double w[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    v[i] = 1e-3f * lane + 0.01f * i;
    w[i] = 1e-3 * lane + 0.01 * i;
  }
  float bv = 1.0f - 1e-9f * lane, cv = 1e-7f;
  double bw = 1.0 - 1e-12 * lane, cw = 1e-7;
  opaque(bv);
  opaque(cv);
  opaque(bw);
  opaque(cw);
  for (int j = 0; j < iters; ++j) {
    const float a = uniform_f32(0x3f800000u, j & 7);      // ~1, changes with j (scalar ops)
    const double ad = uniform_f64(0x3ff00000u, 0x00000001u, j & 7);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if constexpr (OP == 0) v[i] = __builtin_fmaf(v[i], a, 1e-7f);
        else if constexpr (OP == 1) w[i] = __builtin_fma(w[i], ad, 1e-7);
        else if constexpr (OP == 2) v[i] = __builtin_amdgcn_sinf(v[i]);
        else if constexpr (OP == 3) v[i] = __builtin_fmaf(bv, cv, v[i]);
        else if constexpr (OP == 4) w[i] = __builtin_fma(bw, cw, w[i]);
        else if constexpr (OP == 5) w[i] = w[i] + cw;
        else if constexpr (OP == 6) { w[i] = __builtin_rint(w[i]); opaque(w[i]); }
        else if constexpr (OP == 7) { w[i] = __builtin_amdgcn_fract(w[i]); opaque(w[i]); }
        else if constexpr (OP == 8) v[i] = static_cast<float>(__float_as_int(v[i]));
        else if constexpr (OP == 9) v[i] = __builtin_amdgcn_cosf(v[i]);
        else if constexpr (OP == 10) v[i] = v[i] * bv;
        else if constexpr (OP == 11) v[i] = __builtin_fmaf(v[i], bv, cv);
        else v[i] = v[i] + cv;
      }
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < NP; ++i) acc += v[i] + static_cast<float>(w[i]);
  out[threadIdx.x + blockIdx.x * kThreads] = acc;
  cm.stop(clk);
}

}  // namespace

extern "C" {

int nxm_pairs_per_lane_iter(int mix, int wide) {
  if (wide < 0 || wide > 2) return 0;
  if (mix >= NXM_OP_FMA_F32 && mix <= NXM_OP_ADD_F32) return wide == 2 ? 0 : 4 * (wide ? 16 : 8);
  if (mix >= NXM_FWD_GRID_CF && mix <= NXM_BWD_GRID_F1) {    // the sums' shape only
    if (wide != 2) return 0;
    return mix >= NXM_BWD_GRID_CF ? 2 * 64 : 8 * kTileGrid;
  }
  if (mix < NXM_FWD_PH64_CF || mix > NXM_BWD_F32_F1) return 0;
  const bool ph64 = mix >= NXM_FWD_PH64_CF && mix <= NXM_BWD_PH64_F1;
  if (wide == 2) {     // the sums' shape: FP64-phase mixes only
    if (!ph64) return 0;
    return (mix == NXM_BWD_PH64_CF || mix == NXM_BWD_PH64_F1) ? 2 * kTile : kTile;
  }
  const int np = ph64 ? kPairs64 : kPairs32;
  return wide ? 2 * np : np;
}

int nxm_threads_per_block(void) { return kThreads; }

int nxm_wallclock_khz(void) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -4;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return -4;
  return khz;
}

int nxm_run(int mix, int wide, int n_blocks, int iters, float* out, unsigned long long* clk,
            void* stream) {
  if (mix < NXM_FWD_PH64_CF || mix > NXM_BWD_GRID_F1) return -2;
  if (n_blocks < 1 || iters < 1 || !out || nxm_pairs_per_lane_iter(mix, wide) <= 0) return -1;
  if (wide == 2) {
    const dim3 g(static_cast<unsigned>(n_blocks));
    const hipStream_t s2 = static_cast<hipStream_t>(stream);
    switch (mix) {
      case NXM_FWD_PH64_CF: mix_fwd_ph64_tile<true><<<g, kThreads, 0, s2>>>(iters, out, clk); break;
      case NXM_FWD_PH64_F1: mix_fwd_ph64_tile<false><<<g, kThreads, 0, s2>>>(iters, out, clk); break;
      case NXM_BWD_PH64_CF: mix_bwd_ph64_tile<true><<<g, kThreads, 0, s2>>>(iters, out, clk); break;
      case NXM_BWD_PH64_F1: mix_bwd_ph64_tile<false><<<g, kThreads, 0, s2>>>(iters, out, clk); break;
      case NXM_FWD_GRID_CF: mix_fwd_grid_tile<true><<<g, kThreads, 0, s2>>>(iters, out, clk); break;
      case NXM_FWD_GRID_F1: mix_fwd_grid_tile<false><<<g, kThreads, 0, s2>>>(iters, out, clk); break;
      case NXM_BWD_GRID_CF: mix_bwd_grid_tile<true><<<g, kThreads, 0, s2>>>(iters, out, clk); break;
      case NXM_BWD_GRID_F1: mix_bwd_grid_tile<false><<<g, kThreads, 0, s2>>>(iters, out, clk); break;
      default: return -1;      // the FP32 mixes have no such shape
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
  }
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(n_blocks));
#define NXM_CASE(ID, KERNEL, CF, NP)                                                        \
  case ID:                                                                                  \
    if (wide) KERNEL<CF, 2 * NP, 4><<<grid, kThreads, 0, st>>>(iters, out, clk);            \
    else KERNEL<CF, NP, 8><<<grid, kThreads, 0, st>>>(iters, out, clk);                     \
    break;
#define NXM_OP(ID, OP)                                                                      \
  case ID:                                                                                  \
    if (wide) op_rate<OP, 16><<<grid, kThreads, 0, st>>>(iters, out, clk);                  \
    else op_rate<OP, 8><<<grid, kThreads, 0, st>>>(iters, out, clk);                        \
    break;
  switch (mix) {
    NXM_CASE(NXM_FWD_PH64_CF, mix_fwd_ph64, true, kPairs64)
    NXM_CASE(NXM_FWD_PH64_F1, mix_fwd_ph64, false, kPairs64)
    NXM_CASE(NXM_BWD_PH64_CF, mix_bwd_ph64, true, kPairs64)
    NXM_CASE(NXM_BWD_PH64_F1, mix_bwd_ph64, false, kPairs64)
    NXM_CASE(NXM_FWD_F32_CF, mix_fwd_f32, true, kPairs32)
    NXM_CASE(NXM_FWD_F32_F1, mix_fwd_f32, false, kPairs32)
    NXM_CASE(NXM_BWD_F32_CF, mix_bwd_f32, true, kPairs32)
    NXM_CASE(NXM_BWD_F32_F1, mix_bwd_f32, false, kPairs32)
    NXM_OP(NXM_OP_FMA_F32, 0)
    NXM_OP(NXM_OP_FMA_F64, 1)
    NXM_OP(NXM_OP_SIN_F32, 2)
    NXM_OP(NXM_OP_FMAC_F32, 3)
    NXM_OP(NXM_OP_FMAC_F64, 4)
    NXM_OP(NXM_OP_ADD_F64, 5)
    NXM_OP(NXM_OP_RNDNE_F64, 6)
    NXM_OP(NXM_OP_FRACT_F64, 7)
    NXM_OP(NXM_OP_CVT_F32_I32, 8)
    NXM_OP(NXM_OP_COS_F32, 9)
    NXM_OP(NXM_OP_MUL_F32, 10)
    NXM_OP(NXM_OP_FMA_F32_V, 11)
    NXM_OP(NXM_OP_ADD_F32, 12)
    default: return -2;
  }
#undef NXM_CASE
#undef NXM_OP
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
