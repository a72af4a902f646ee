// nx_internal.h -- records, launch plans and kernel launchers shared by the libnx
// translation units.  Not part of the public ABI (that is include/nx.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace nx {

constexpr int kThreads = 256;          // work-group size of every sum kernel (4 wave64)

// ---------------------------------------------------------------------------------
// Packed records streamed through the scalar (wave-uniform) load path.  Each record
// is read by a whole wavefront at once and its fields are used directly as SGPR
// operands of the VALU instructions, so no LDS staging and no barrier is needed.

// Atom for the FP32 mode: coordinates and factor in FP32.
struct alignas(16) AtomF32 { float x, y, z, fr, fi, pad0, pad1, pad2; };            // 32 B
// Atom for the FP64-phase mode (f = 1 and complex f alike): coordinates widened (exactly)
// to FP64; a (FP64, cycles) = arg f + kPhaseShift + the reduction offset of the variant +
// the eighth turn k/8 of the atom's compensated group; m (FP32) = |f| rounded without
// bias (stochastic rounding keyed by the atom index; 1 for f = 1); (ck, sk) = the group's
// turn-back factor exp(-2 i pi k/8), negated for the fract variant; rmax = the largest
// |x|, |y| or |z| among the 256 records of the record's block of the pack (+inf if any is
// not finite), the tile bound of the fixed-point reduction.
struct alignas(16) AtomPH { double x, y, z, a; float m, ck, sk, rmax; };             // 48 B
// Atom for the all-FP64 path.
struct alignas(16) AtomF64 { double x, y, z, fr, fi, pad; };                         // 48 B
// Point for the FP32-mode adjoint: S and the seed G.
struct alignas(16) PointF32 { float sx, sy, sz, gr, gi, pad0, pad1, pad2; };         // 32 B
// Point for the FP64-phase adjoint, with the seed in polar form conj(G) =
// |G| exp(2 i pi delta): S (FP64) and delta (cycles, FP64, plus kPhaseShift and the
// reduction offset of the variant) for the phase in the first 32 bytes, |G| S and |G| (FP32) for the
// multiply-adds into the per-atom sums in the last 16.  sx and delta come first: they
// are the two point values of the phase's first fma, which the adjoint reads from an
// LDS tile (an fma takes at most one scalar operand), the rest with scalar loads.
struct alignas(16) PointPH { double sx, delta, sy, sz; float gsx, gsy, gsz, gmag; }; // 48 B
// Point for the all-FP64 adjoint.
struct alignas(16) PointF64 { double sx, sy, sz, gr, gi, pad; };                     // 48 B

// The FP64-phase reductions of the phase psi = S.r + addend to a turn in [-1/2, 1/2]:
//   0 centred: t = psi - rint(psi), exact in FP64, rounded once to FP32;
//   1 fract:   u = fract(psi + 1/2) in [0, 1), rounded once to FP32 (the terms change sign);
//   2 fixed point: every record's addend carries kPhaseShift = 1.5 * 2^20 cycles, an
//     integer, so psi modulo one is unchanged.  While |psi - kPhaseShift| < 2^19, psi lies
//     in [2^20, 2^21), where the last bit of an FP64 is worth 2^-32 cycles, and the low 32
//     bits of its encoding are psi modulo one in 32-bit fixed point; read as a signed
//     integer they are t * 2^32 with t the centred turn in [-1/2, 1/2).  One integer to
//     FP32 conversion (rounded as the FP64 to FP32 one of the centred form) and a scaling
//     by 2^-32 replace the rounding, the subtraction and the FP64 to FP32 conversion.  The
//     three fma of the phase round at 2^-33 cycles each in that range (against about 2^-26
//     for the FP32 rounding of the turn), and the terms are those of the centred form but at
//     exactly half a turn (-1/2 here, +-1/2 after rint).  Every tile of records checks
//     the range first: (|Sx| + |Sy| + |Sz|) max(|x|, |y|, |z|) < kFixedPhaseBound for every
//     lane of the wave (the addends stay below 2 cycles from kPhaseShift), and a wave whose
//     check fails reduces that tile's phases with rint and reads the low word of the reduced
//     phase plus kPhaseShift (variant 3: the centred turn rounded to 2^-32 cycles, an extra
//     error below 2^-33 cycles where the phase was finer; the same loop shape as variant 2,
//     so the fallback does not raise the kernel's register count), on the same records.
constexpr double kPhaseShift = 1572864.0;
constexpr float kFixedPhaseBound = 524224.0f;     // 2^19 - 64

// Tile bounds of the packed FP64-phase point records of the adjoint: one float per 256
// records (the largest |Sx|, |Sy| or |Sz| of those points, +inf if any is not finite; for
// grid records also of the row's part o + i2 e2 + i3 e3), stored after the records.
inline size_t point_bound_offset(int64_t n, size_t rec_size = sizeof(PointPH)) {
  return (static_cast<size_t>(n) * rec_size + 255) / 256 * 256;
}
inline size_t point_bound_bytes(int64_t n) {
  return (static_cast<size_t>((n + kThreads - 1) / kThreads) * sizeof(float) + 255) / 256 * 256;
}

// A regular grid of points given exactly: S(i1, i2, i3) = o + i1 e1 + i2 e2 + i3 e3 in
// FP64, 0 <= i_a < n_a, point k = i1 + n1 (i2 + n2 i3) (i1 fastest).  Passed to the
// kernels by value.
struct GridDef {
  double o[3], e1[3], e2[3], e3[3];
  int64_t n1, n2, n3;
};

// Forward atom record of the grid sums: with r the atom's position and a its FP64-phase
// addend (as in AtomPH), c0 = o.r + a and c_d = e_d.r, so that the phase of point
// (i1, i2, i3) is i1 c1 + (c0 + i2 c2 + i3 c3); the bracket is one value per atom and grid
// row.  m, ck, sk, rmax as in AtomPH.  (wr, wi) = exp(2 i pi c1) - 1, the step of the
// phase factor from one point of a row to the next, (vr, vi) = exp(2 i pi c2) - 1, from one
// row to the next (i2 + 1), and (xr, xi) = exp(2 i pi c3) - 1 (i3 + 1), formed in FP64 and
// rounded to FP32 without bias (stochastically, from a hash of the atom's index), so that
// the rounding errors of atoms with equal c1, c2 or c3 (a lattice plane) add up
// incoherently.  Only the steps the plan's block shape takes are formed; the others hold 0.
struct alignas(16) AtomGrid {
  double c0, c1, c2, c3;
  float m, ck, sk, rmax, wr, wi, vr, vi, xr, xi, pad0, pad1;
};  // 80 B
// Adjoint over grid rows: along a row the phase factor of atom j steps by the constant
// w_j = exp(2 i pi step1.r_j) from one point to the next, so each 64-point group (one
// row's run) forms exp(2 i pi psi) exactly (FP64 phase, hardware cos and sin) at its first
// point only and multiplies by w_j in FP32 for the others.  Per point the record holds the
// seed as (Re G, -Im G) and the point's place u in its group (FP32); per group the
// group's first point S0 (FP32).  The sums S.v are formed per group as S0 a0 + step1 a1
// with a0 = sum v and a1 = sum u v.
struct alignas(16) PointRow { float gr, ngi, u, pad; };                             // 16 B
constexpr int kRowGroup = 64;
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
// group records (float4 S0 per 64 points) after the point records, then the tile bounds
inline size_t row_group_offset(int64_t n) { return align256(static_cast<size_t>(n) * sizeof(PointRow)); }
inline size_t row_group_bytes(int64_t n) {
  return align256(static_cast<size_t>((n + kRowGroup - 1) / kRowGroup) * 16);
}
inline size_t row_bound_offset(int64_t n) { return row_group_offset(n) + row_group_bytes(n); }

// Running state of one output lane item (a point for the forward, one component of
// an atom's sum for the adjoint) kept between launches and across splits.
//   FP32 modes: (sum_re, sum_im, comp_re, comp_im) -- float4 per point;
//   FP64 path:  (sum_re, sum_im)                   -- double2 per point.

// XCD-major block order.  The dispatcher hands work-group b to XCD b % 8 (each XCD
// has its own L2), so the hardware id is remapped such that every XCD runs a
// contiguous range of logical blocks: the blocks resident on one XCD then belong to
// the same stream slice and read the same records at about the same time.
__device__ __forceinline__ int xcd_major_block(int b, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = b & 7, idx = b >> 3;
  return x * q + (x < r ? x : r) + idx;
}

// Kernel variants selected by the host.
enum Mode : int { kF32 = 0, kPH64 = 1, kF64 = 2 };

// exp(2 i pi phi) = c + i s in FP64, for the all-FP64 path (phi in cycles, finite).
// The phase is reduced to t = phi - rint(phi) in [-1/2, 1/2] and split into q quarter
// turns, q = rint(4 t) in -2..2, and r = t - q/4 with |r| <= 1/8 (both steps exact).
// sin(2 pi r) and cos(2 pi r) come from their Taylor series in r, through r^17 and r^16:
// for |2 pi r| <= pi/4 the first omitted terms are below 1e-19 and 3e-18, under FP64's
// rounding.  Then exp(2 i pi phi) = i^q exp(2 i pi r): a swap and two signs.
__device__ __forceinline__ void cis_f64(double phi, double& c, double& s) {
  const double t = phi - __builtin_rint(phi);
  const double q = __builtin_rint(4.0 * t);
  const double r = __builtin_fma(-0.25, q, t);
  const double z = r * r;
  // (-1)^m (2 pi)^(2m+1) / (2m+1)!, m = 8 .. 0
  double ps = 0x1.aaec32af93359p-4;
  ps = __builtin_fma(ps, z, -0x1.6fadb9f155744p-1);
  ps = __builtin_fma(ps, z, 0x1.e8f434d018d63p+1);
  ps = __builtin_fma(ps, z, -0x1.e3074fde8871fp+3);
  ps = __builtin_fma(ps, z, 0x1.50783487ee782p+5);
  ps = __builtin_fma(ps, z, -0x1.32d2cce62bd86p+6);
  ps = __builtin_fma(ps, z, 0x1.466bc6775aae2p+6);
  ps = __builtin_fma(ps, z, -0x1.4abbce625be53p+5);
  ps = __builtin_fma(ps, z, 0x1.921fb54442d18p+2);
  const double sr = r * ps;
  // (-1)^m (2 pi)^(2m) / (2m)!, m = 8 .. 0
  double pc = 0x1.20c62c2f2d7f5p-2;
  pc = __builtin_fma(pc, z, -0x1.b6e24f44b128fp+0);
  pc = __builtin_fma(pc, z, 0x1.f9d38a3763cc3p+2);
  pc = __builtin_fma(pc, z, -0x1.a6d1f2a204a8cp+4);
  pc = __builtin_fma(pc, z, 0x1.e1f506891babbp+5);
  pc = __builtin_fma(pc, z, -0x1.55d3c7e3cbffap+6);
  pc = __builtin_fma(pc, z, 0x1.03c1f081b5ac4p+6);
  pc = __builtin_fma(pc, z, -0x1.3bd3cc9be45dep+4);
  const double cr = __builtin_fma(pc, z, 1.0);
  const int qi = static_cast<int>(q) & 3;      // i^q: 0 -> (c, s), 1 -> (-s, c), 2 -> (-c, -s), 3 -> (s, -c)
  const double u = (qi & 1) ? sr : cr;
  const double v = (qi & 1) ? cr : sr;
  c = (qi == 1 || qi == 2) ? -u : u;
  s = (qi >= 2) ? -v : v;
}

// ---------------------------------------------------------------------------------
// Launch plan.  "Lane items" are the outputs one lane owns (points for the forward,
// atoms for the adjoint), "stream items" are what every lane loops over (atoms for
// the forward, points for the adjoint).  The stream is cut into `nsplit` contiguous
// slices processed by different work-groups when there are too few lane items to
// fill the chip, and into chunks of at most kLaunchPairs pairs per launch so that
// no single dispatch runs for long; partial sums are carried between chunks in the
// workspace and combined across splits in a fixed order.
struct Plan {
  int mode = 0;          // Mode
  int per_lane = 1;      // lane items per lane (P points or Q atoms)
  int grp = 16;          // stream items per compensated group
  int fk = 0;            // 0: f_j = 1, 1: complex f_j
  int red = 0;           // phase reduction of the FP64-phase kernels (0 centred, 1 fract, 2 fixed point)
  int gf = 0;            // adjoint also returns dL/df
  int lds = 0;           // FP64-phase sums: record tiles staged in LDS instead of scalar loads
  int inl = 0;           // small calls: records formed in the sum kernel, no pack dispatch
  int grid = 0;          // points: 0 a list, 1 a grid (general kernels, FP64 points from the
                         // grid), 2 a grid walked by rows (the grid kernels)
  int blk_a = 1, blk_b = 1, blk_c = 1;   // forward over grid rows: points per lane along
                                         // i1, i2, i3 (per_lane = their product)
  int64_t lanes = 0;     // number of lane items
  int64_t stream = 0;    // number of stream items
  int64_t blocks = 0;    // work-groups over lane items
  int nsplit = 1;        // stream slices
  int64_t chunk = 0;     // stream items per launch
  int64_t nchunks = 0;   // launches
  size_t rec_size = 0;       // bytes of one packed stream record
  size_t rec_bytes = 0;      // packed stream records
  size_t partial_bytes = 0;  // carried / split partial state
  size_t misc_bytes = 0;     // small scratch (loss partials)
  size_t total() const { return rec_bytes + partial_bytes + misc_bytes; }
};

// Work-groups wanted per launch: about 16 rounds of the 2048 that fit the chip at once
// (8 per CU), so that the last, partly filled round costs little.  Against 4096 this
// splits the streams further and made the fit step 4-7 % faster on the 200k- to
// 4M-atom workloads (the adjoint 5-10 %).
constexpr int64_t kTargetBlocks = 32768;
// Smallest stream slice per split.  Each split costs every lane a partial state written
// and read back, and the reduce reads the splits of one output in sequence, so slices
// much below a few hundred items lose more than the fuller chip gains (64 took a
// 1e5-atom, 1e4-point forward from 2.5e12 to 1.7e12 pairs/s at 820 splits).
constexpr int64_t kMinStreamPerSplit = 256;
// Small problems: when slices of kMinStreamPerSplit leave fewer than kFillBlocks
// work-groups (4 waves per SIMD on the 1024 SIMDs), slices down to kMinStreamPerSplitSmall
// items are allowed until the grid reaches kFillBlocks: with one wave per SIMD the sums
// cannot hide their latencies, and the extra partial states of a small problem cost little.
constexpr int64_t kFillBlocks = 1024;
constexpr int64_t kMinStreamPerSplitSmall = 32;
// Small calls form their packed records inside the sum kernel (no pack dispatch) when the
// records formed in all (each work-group of lane items forms the records of its slices,
// so every record is formed `blocks` times) are at most this many.
constexpr int64_t kInlineMaxRecords = int64_t(1) << 17;
constexpr int64_t kMaxSplit = 1024;
constexpr int64_t kLaunchPairs = int64_t(1) << 39;   // pairs per launch (well under 1 s)
// Forward: when one split's slice of packed atom records exceeds an XCD's 4 MiB L2, the
// resident work-groups of an XCD drift apart along it and re-read it from HBM; launches
// then take at most this many record bytes per split, so each launch's slice stays in L2.
constexpr int64_t kL2SliceBytes = int64_t(2) << 20;
constexpr int64_t kL2Bytes = int64_t(4) << 20;
constexpr int kLossBlocks = 1024;             // fixed grid of the loss reduction
constexpr int64_t kLossSmall = 16384;         // up to this many points: one work-group

enum Op : int { kOpFwd = 0, kOpBwd = 1, kOpFwdF64 = 2, kOpBwdF64 = 3, kOpLoss = 4,
                kOpBwdGf = 5, kOpBwdGfF64 = 6 };

constexpr int kMaxSpecies = 16;   // species of the factorised entry points

// Lanes that serve one output in the split reduction (a power of two, 4 to 64): about a
// quarter of the number of splits, so that each lane folds about four splits in sequence
// and the lanes' states meet in a short fixed butterfly; one lane per output (splits in
// sequence) below 8 splits.  A wave holds 64 / G outputs side by side (consecutive lanes,
// consecutive outputs), so that one load reads 64 / G consecutive entries of G split rows:
// with many outputs (kReduceWideOutputs and up, which fill the chip with 4 lanes each) G
// stays at 4, whole 64-byte lines per row, instead of over-fetching lines for a few bytes.
constexpr int64_t kReduceWideOutputs = 16384;
inline int reduce_lanes(int nsplit, int64_t outputs) {
  if (nsplit < 8) return 1;
  if (outputs >= kReduceWideOutputs) return 4;
  const int want = (nsplit + 3) / 4;
  int g = 4;
  while (g < 64 && g < want) g <<= 1;
  return g;
}

// Builds the plan of (op, mode) for the sizes; pure host code, no HIP call.  At most
// max_split stream slices (kMaxSplit when omitted).
// `grid`: 0 for a list of points; for a grid (FP64-phase mode), 1 asks for the general
// kernels and 2 + s for the grid kernels over rows of n1 points (n1 a multiple of 64), where
// the bits of s say which counts allow two points per lane in the forward's block: 1 for
// n1 a multiple of 128, 2 for n2 even, 4 for n3 even.  The plan keeps the grid kernels
// only where they exist for it (the fixed-point reduction; 64-point groups in the
// adjoint), holds the kind it chose in p.grid (2 or 1) and the forward's block shape in
// p.blk_a, p.blk_b, p.blk_c.
Plan make_plan(int op, int mode, int64_t n_atoms, int64_t n_points, int f_is_null,
               int64_t max_split = kMaxSplit, int grid = 0);

// Per-launch stream range of chunk c: [begin, end) and the slice length per split.
void chunk_range(const Plan& p, int64_t c, int64_t* begin, int64_t* end, int64_t* per_split);

// ---------------------------------------------------------------------------------
// Launchers (defined in the kernel translation units).  All return the launch error.
// FP64-phase records depend on the plan's reduction variant and group size, and their
// groups are counted from the first atom packed: pack the atoms of each plan separately.
hipError_t launch_pack_atoms(int mode, int red, int grp, const void* xyz, const void* f, int64_t n,
                             void* rec, hipStream_t st);
hipError_t launch_pack_points(int mode, int red, const void* S, const void* G, int64_t k,
                              void* rec, hipStream_t st);
// Grid records (FP64-phase mode): the atoms as AtomGrid (plan grid 2; grid 1 packs AtomPH
// with launch_pack_atoms), the points of the grid with the seed G as PointRow with the
// group records (grid 2) or PointPH (grid 1), followed by the tile bounds.
hipError_t launch_pack_atoms_grid(const Plan& p, const float* xyz, const float* f, int64_t n,
                                  const GridDef& g, void* rec, hipStream_t st);
hipError_t launch_pack_points_grid(const Plan& p, const GridDef& g, const float* G, void* rec,
                                   hipStream_t st);

// One forward chunk over points (lane items) for atoms [a_begin, a_end).  With p.inl the
// kernel forms the records itself from xyz and f (rec is then unused).
hipError_t launch_fwd_chunk(const Plan& p, const void* rec, int64_t a_begin, int64_t a_end,
                            int64_t per_split, const void* S, void* partial, void* A,
                            int carry_in, int direct, hipStream_t st, const void* xyz = nullptr,
                            const void* f = nullptr, const GridDef* grid = nullptr);
// Combine split partials into A.
hipError_t launch_fwd_reduce(const Plan& p, const void* partial, void* A, hipStream_t st);

// One adjoint chunk over atoms (lane items) for points [k_begin, k_end); grad and
// gradf (only with p.gf) receive the outputs of the last chunk when `direct`.
// With p.inl the kernel forms the point records itself from S and G (rec is then unused).
hipError_t launch_bwd_chunk(const Plan& p, const void* rec, int64_t k_begin, int64_t k_end,
                            int64_t per_split, const void* xyz, const void* f, void* partial,
                            void* grad, void* gradf, int carry_in, int direct, hipStream_t st,
                            const void* S = nullptr, const void* G = nullptr,
                            const GridDef* grid = nullptr);
// f: the atom factors (complex f in the FP64-phase mode scales and rotates the sums).
hipError_t launch_bwd_reduce(const Plan& p, const void* partial, const void* f, void* grad,
                             void* gradf, hipStream_t st);

// Species-factorised forward: A_k = sum_s fs[s][k] * sum_sp state_s[sp][k] (FP64
// combination of the per-species (sum, comp) states), optionally the per-species sums.
struct SpeciesStates {
  const void* state[kMaxSpecies];   // float4 [nsplit][K] per species
  int nsplit[kMaxSpecies];
  int n;
};
hipError_t launch_species_combine(const SpeciesStates& ss, const float* fs, int64_t k, float* A,
                                  float* A_species, hipStream_t st);
// seed_s = G * conj(fs_s) (or G when fs_s is NULL), formed in FP64, rounded once.
hipError_t launch_species_seed(const float* G, const float* fs_s, int64_t k, float* seed,
                               hipStream_t st);
// grad_fs_s = G * conj(A_s) (the gradient of L with respect to the factor fs_s).
hipError_t launch_species_gradf(const float* G, const float* A_s, int64_t k, float* grad_fs_s,
                                hipStream_t st);

hipError_t launch_loss(const float* A, const float* I, int64_t k, double* L, float* G,
                       double* partial, hipStream_t st);

}  // namespace nx
