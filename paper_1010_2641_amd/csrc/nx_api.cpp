// nx_api.cpp -- the C ABI of libnx (declared in include/nx.h): argument validation
// (pure host code, before any HIP call), launch planning, workspace layout and the
// launch sequence of each entry point.
#include "nx.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>

#include "nx_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return NX_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Tuning knobs for launch-shape sweeps and for exercising the chunked path at small
// sizes; read on every plan so that nx_workspace_bytes and the entry points agree.
//   NX_TUNE_LAUNCH_PAIRS  pairs per launch (default 2^39)
//   NX_TUNE_P             lane items per lane (1, 2, 4; the FP64 path 1, 2)
//   NX_TUNE_GRP           stream items per compensated group (8, 16, 32)
//   NX_TUNE_RED           phase reduction variant (0 centred rint, 1 fract)
//   NX_TUNE_TARGET_BLOCKS work-groups wanted per launch (stream splits up to this)
//   NX_TUNE_L2_CHUNK      0 turns off the L2-sized atom chunks of the forward
//   NX_TUNE_LDS           FP64-phase sums: 1 stages record tiles in LDS (the forward's
//                         atom records; the phase part of the adjoint's point records),
//                         0 streams them through scalar loads (default: 1)
//   NX_TUNE_FILL_BLOCKS   small problems: work-groups the slices may be shortened to reach
//                         (default 1024); NX_TUNE_MIN_SLICE their shortest slice (32)
//   NX_TUNE_INLINE        0: always pack the records in their own dispatch; 1: form them in
//                         the sum kernel wherever that form exists (default: small calls;
//                         a grid's small forward then takes the general grid form)
int64_t env_i64(const char* name, int64_t def) {
  const char* v = std::getenv(name);
  if (!v || !*v) return def;
  char* end = nullptr;
  const long long x = std::strtoll(v, &end, 10);
  return (end && *end == 0) ? int64_t(x) : def;
}

int check_counts(const char* fn, int64_t n_atoms, int64_t n_points) {
  if (n_atoms < 0 || n_points < 0)
    return fail(NX_ERR_ARG, "%s: negative count (n_atoms=%lld, n_points=%lld)", fn,
                (long long)n_atoms, (long long)n_points);
  if (n_atoms > NX_MAX_COUNT || n_points > NX_MAX_COUNT)
    return fail(NX_ERR_ARG, "%s: count above NX_MAX_COUNT (n_atoms=%lld, n_points=%lld)", fn,
                (long long)n_atoms, (long long)n_points);
  return NX_OK;
}

int check_ws(const char* fn, const nx::Plan& p, const void* ws, size_t ws_bytes) {
  const size_t need = p.total();
  if (need == 0) return NX_OK;
  if (ws == nullptr || ws_bytes < need)
    return fail(NX_ERR_WORKSPACE, "%s: workspace of %zu bytes needed, %zu given%s", fn, need,
                ws_bytes, ws ? "" : " (NULL)");
  if (!aligned(ws, 16)) return fail(NX_ERR_WORKSPACE, "%s: workspace not 16-byte aligned", fn);
  return NX_OK;
}

int device_error(const char* fn, hipError_t e) {
  return fail(NX_ERR_DEVICE, "%s: %s", fn, hipGetErrorString(e));
}

}  // namespace

namespace nx {

Plan make_plan(int op, int mode, int64_t n_atoms, int64_t n_points, int f_is_null,
               int64_t max_split, int grid) {
  Plan p;
  p.fk = f_is_null ? 0 : 1;
  const bool fwd = (op == kOpFwd || op == kOpFwdF64);
  if (op == kOpLoss) {
    p.misc_bytes = size_t(kLossBlocks) * sizeof(double);
    return p;
  }
  p.gf = (op == kOpBwdGf || op == kOpBwdGfF64) ? 1 : 0;
  p.mode = (op == kOpFwdF64 || op == kOpBwdF64 || op == kOpBwdGfF64) ? kF64
                                                                     : (mode == NX_F32_PH64 ? kPH64 : kF32);
  p.lanes = fwd ? n_points : n_atoms;
  p.stream = fwd ? n_atoms : n_points;
  // Defaults from launch-shape and accuracy sweeps on MI355X.  FP64-phase mode, both
  // sums: the fixed-point reduction (the centred turn read from the low word of the
  // shifted phase; the centred form's rounding, which decides the pointwise intensity
  // error at the weakest points, with two instructions fewer than the centred form and
  // one fewer than fract, whose rounding is twice as coarse: fract took a strained 100^3
  // cube from 2.0e-6 to 7.7e-6).  Forward: 8-atom groups for few atoms (|A| peaks at
  // N |f|, so each term weighs more), 16 above.  Adjoint (judged normwise): 64-point
  // groups (1 % faster than 32 on C2-C4, same error), two atoms per lane.
  if (fwd) {
    const bool small = p.stream < 65536;
    p.red = p.mode == kPH64 ? 2 : 0;
    // atom tiles staged in LDS: the records' phase addend would be a second scalar
    // operand of the first fma, which the scalar-load form has to copy to VGPRs
    p.lds = p.mode == kPH64 ? 1 : 0;
    p.grp = (p.mode == kPH64 && small) ? 8 : 16;
    if (p.mode == kF64) p.per_lane = p.lanes >= 262144 ? 2 : 1;
    else p.per_lane = (p.lanes >= 32768 && p.lanes < 1048576) ? 2 : 1;
  } else {
    p.red = p.mode == kPH64 ? 2 : 0;
    p.grp = p.mode == kPH64 ? 64 : 16;
    // the phase part of the point records from LDS tiles, the rest with scalar loads
    // (1.5-3 % faster than scalar loads alone, from 1e5 to 1e6 atoms)
    p.lds = p.mode == kPH64 ? 1 : 0;
    p.per_lane = (p.mode != kF64 && p.lanes >= 16384) ? 2 : 1;
  }
  {
    // unset knobs read as -1, which no knob accepts
    const int64_t tp = env_i64("NX_TUNE_P", -1);
    if (tp == 1 || tp == 2 || (tp == 4 && p.mode != kF64)) p.per_lane = int(tp);
    const int64_t tg = env_i64("NX_TUNE_GRP", -1);
    // forward: 8, 16, 32; adjoint: 16, 32, 64
    if (p.mode == kPH64 && (fwd ? (tg == 8 || tg == 16 || tg == 32) : (tg == 16 || tg == 32 || tg == 64)))
      p.grp = int(tg);
    const int64_t tr = env_i64("NX_TUNE_RED", -1);
    if (p.mode == kPH64 && (tr == 0 || tr == 1 || tr == 2)) p.red = int(tr);
    const int64_t tl = env_i64("NX_TUNE_LDS", -1);
    if (p.mode == kPH64 && (tl == 0 || tl == 1)) p.lds = int(tl);
  }
  // a grid walked by rows (its own kernels): every wave's points lie in one row; where its
  // kernels do not exist for the plan the general kernels take the grid's points
  // (NX_TUNE_GRID=1 sends every grid to the general kernels)
  const int shape_ok = grid >= 2 ? grid - 2 : 0;   // counts that allow a 2 along i1, i2, i3
  if (grid >= 2) grid = 2;
  if (grid == 2 && env_i64("NX_TUNE_GRID", -1) == 1) grid = 1;
  // a grid's forward: LDS tiles and the fixed-point reduction, the forms built to walk
  // grid rows (grid 2) or to form each lane's FP64 grid point (grid 1), whatever the knobs
  // say.  Over grid rows a block of points per lane, two along i1 where n1 is a multiple
  // of 128, two along i2 where n2 is even, two along i3 where n3 is even too (the others'
  // phase factors stepped from the first's), with 16-atom groups; calls with few atoms
  // (8-atom groups) are bound by latency, not issue, and keep one point per lane, where
  // the steps would only add their rounding (C1: forward no faster with two points, T1
  // 7.4e-6 against 6.6e-6).  NX_TUNE_P=1, 2 or 4 caps the points per lane (dropping i3,
  // then i2, then i1)
  if (grid != 0 && fwd && p.mode == kPH64) {
    p.red = 2;
    p.lds = 1;
    if (p.grp != 8) p.grp = 16;
    p.blk_a = p.blk_b = p.blk_c = 1;
    if (grid == 2) {
      p.blk_a = (shape_ok & 1) ? 2 : 1;
      p.blk_b = (shape_ok & 2) ? 2 : 1;
      p.blk_c = ((shape_ok & 4) && p.blk_b == 2) ? 2 : 1;
      const int64_t tp = env_i64("NX_TUNE_P", -1);
      const int cap = (tp == 1 || tp == 2 || tp == 4) ? int(tp) : 8;
      const int limit = std::min(cap, p.grp == 16 ? 8 : 1);
      while (p.blk_a * p.blk_b * p.blk_c > limit) {
        if (p.blk_c == 2) p.blk_c = 1;
        else if (p.blk_b == 2 && p.blk_a == 2) p.blk_b = 1;
        else if (p.blk_a == 2) p.blk_a = 1;
        else p.blk_b = 1;
      }
    }
    p.per_lane = p.blk_a * p.blk_b * p.blk_c;
  }
  // the fixed-point reduction checks its range per LDS tile: the scalar-load forms (and
  // the forward's 32-atom groups, which have no LDS form) take the centred one, and so do
  // the forward's forms whose two tile loops do not fit their registers (four points per
  // lane; two with 8-atom groups)
  // (a grid's forward has the fixed-point forms for all of its shapes)
  if (p.red == 2 && !(grid != 0 && fwd) &&
      !(p.lds && (!fwd || ((p.grp == 8 || p.grp == 16) &&
                           (p.per_lane == 1 || (p.per_lane == 2 && p.grp == 16))))))
    p.red = 0;
  if (grid == 2 && !(p.mode == kPH64 && p.red == 2 && p.lds && (fwd || p.grp == 64)))
    grid = 1;
  if (grid == 1 && fwd) {
    p.per_lane = 1;
    p.blk_a = p.blk_b = p.blk_c = 1;
  }
  p.grid = p.mode == kPH64 ? grid : 0;
  const int64_t per_block = int64_t(kThreads) * p.per_lane;
  p.blocks = p.lanes > 0 ? ceil_div(p.lanes, per_block) : 0;
  p.nsplit = 1;
  int64_t target = env_i64("NX_TUNE_TARGET_BLOCKS", kTargetBlocks);
  if (target < 1) target = kTargetBlocks;
  if (p.blocks > 0 && p.blocks < target) {
    int64_t want = ceil_div(target, p.blocks);
    int64_t maxs = p.stream / kMinStreamPerSplit;
    if (maxs < 1) maxs = 1;
    if (want > maxs) want = maxs;
    if (want > kMaxSplit) want = kMaxSplit;
    const int64_t fill_blocks = std::min<int64_t>(env_i64("NX_TUNE_FILL_BLOCKS", kFillBlocks), target);
    const int64_t min_small = std::max<int64_t>(1, env_i64("NX_TUNE_MIN_SLICE", kMinStreamPerSplitSmall));
    if (want * p.blocks < fill_blocks) {
      int64_t fill = ceil_div(fill_blocks, p.blocks);
      int64_t maxf = p.stream / min_small;
      if (fill > maxf) fill = maxf;
      if (fill > kMaxSplit) fill = kMaxSplit;
      if (fill > want) want = fill;
    }
    if (want > max_split) want = max_split < 1 ? 1 : max_split;
    p.nsplit = int(want);
  }
  // small calls: records formed in the sum kernel (the LDS forms with one lane item per
  // lane and the default reduction variant); NX_TUNE_INLINE=0 turns this off, 1 forces it
  // wherever that form exists
  // (grids: records always packed)
  if (p.mode == kPH64 && p.lds && p.per_lane == 1 && p.grid == 0 &&
      (fwd ? (p.red == 2 && (p.grp == 8 || p.grp == 16)) : (p.red == 2 && p.grp == 64))) {
    const int64_t ti = env_i64("NX_TUNE_INLINE", -1);
    p.inl = (ti == 1 || (ti != 0 && p.blocks * p.stream <= kInlineMaxRecords)) ? 1 : 0;
  }
  // chunks of at most kLaunchPairs pairs, a whole number of groups per split
  const int64_t lane_pad = p.blocks * per_block;
  const int64_t gran = int64_t(p.nsplit) * p.grp;
  int64_t launch_pairs = env_i64("NX_TUNE_LAUNCH_PAIRS", kLaunchPairs);
  if (launch_pairs < 1) launch_pairs = kLaunchPairs;
  size_t rec_size;
  if (fwd && p.grid == 2) rec_size = sizeof(AtomGrid);
  else if (fwd) rec_size = p.mode == kF64 ? sizeof(AtomF64) : (p.mode == kPH64 ? sizeof(AtomPH) : sizeof(AtomF32));
  else if (p.grid == 2) rec_size = sizeof(PointRow);
  else rec_size = p.mode == kF64 ? sizeof(PointF64) : (p.mode == kPH64 ? sizeof(PointPH) : sizeof(PointF32));
  p.rec_size = rec_size;
  int64_t chunk = lane_pad > 0 ? launch_pairs / lane_pad : p.stream;
  if (fwd && ceil_div(p.stream, p.nsplit) * int64_t(rec_size) > kL2Bytes &&
      env_i64("NX_TUNE_L2_CHUNK", 1) != 0)
    chunk = std::min<int64_t>(chunk, int64_t(p.nsplit) * (kL2SliceBytes / int64_t(rec_size)));
  chunk = chunk / gran * gran;
  if (chunk < gran) chunk = gran;
  if (chunk >= p.stream) {
    p.chunk = p.stream;
    p.nchunks = 1;
  } else {
    p.chunk = chunk;
    p.nchunks = ceil_div(p.stream, chunk);
  }
  // workspace: packed stream records (with the FP64-phase adjoint's tile bounds), then
  // the partial state
  p.rec_bytes = align_up(size_t(p.stream) * rec_size, 256);
  if (!fwd && p.mode == kPH64) p.rec_bytes += point_bound_bytes(p.stream);
  if (!fwd && p.grid == 2) p.rec_bytes += row_group_bytes(p.stream);
  const bool need_partial = p.lanes > 0 && (p.nsplit > 1 || p.nchunks > 1);
  if (need_partial) {
    size_t per_item;
    if (fwd) per_item = 16;                                  // float4 or double2 per point
    else {
      const size_t ns = p.gf ? 5 : 3;                        // 3 (+ 2 for dL/df) sums per atom
      per_item = p.mode == kF64 ? ns * 8 : ns * 2 * 4;       // (+ comps in FP32)
    }
    p.partial_bytes = align_up(size_t(p.nsplit) * size_t(p.lanes) * per_item, 256);
  }
  return p;
}

void chunk_range(const Plan& p, int64_t c, int64_t* begin, int64_t* end, int64_t* per_split) {
  const int64_t b = c * p.chunk;
  int64_t e = b + p.chunk;
  if (e > p.stream || c == p.nchunks - 1) e = p.stream;
  int64_t per = ceil_div(e - b, p.nsplit);
  per = ceil_div(per, p.grp) * p.grp;
  *begin = b;
  *end = e;
  *per_split = per;
}

}  // namespace nx

namespace {

// Chunked launch sequence shared by the sum entry points.  `out` is A (forward) or
// grad_xyz (adjoint, may be NULL when only dL/df is asked for); `outf` is dL/df.
int run_sum(const char* fn, const nx::Plan& p, bool fwd, const void* xyz, const void* f,
            const void* S, const void* G, void* out, void* outf, void* ws, hipStream_t st) {
  char* base = static_cast<char*>(ws);
  void* rec = base;
  void* partial = p.partial_bytes ? base + p.rec_bytes : nullptr;
  hipError_t e = hipSuccess;
  if (!p.inl) {          // small calls form their records in the sum kernel
    if (fwd) e = nx::launch_pack_atoms(p.mode, p.red, p.grp, xyz, f, p.stream, rec, st);
    else e = nx::launch_pack_points(p.mode, p.red, S, G, p.stream, rec, st);
  }
  if (e != hipSuccess) return device_error(fn, e);
  for (int64_t c = 0; c < p.nchunks; ++c) {
    int64_t b, en, per;
    nx::chunk_range(p, c, &b, &en, &per);
    const int carry = c > 0 ? 1 : 0;
    const int direct = (p.nsplit == 1 && c == p.nchunks - 1) ? 1 : 0;
    if (fwd) e = nx::launch_fwd_chunk(p, rec, b, en, per, S, partial, out, carry, direct, st, xyz, f);
    else e = nx::launch_bwd_chunk(p, rec, b, en, per, xyz, f, partial, out, outf, carry, direct, st, S, G);
    if (e != hipSuccess) return device_error(fn, e);
  }
  if (p.nsplit > 1) {
    if (fwd) e = nx::launch_fwd_reduce(p, partial, out, st);
    else e = nx::launch_bwd_reduce(p, partial, f, out, outf, st);
    if (e != hipSuccess) return device_error(fn, e);
  }
  return ok();
}

// Grid entry points: the grid's point count (n1 n2 n3), or -1 after setting the error for
// a NULL grid, a negative or too large count, or a value that is not finite.
int64_t grid_points(const char* fn, const nx_grid* g) {
  if (!g) {
    fail(NX_ERR_ARG, "%s: NULL grid", fn);
    return -1;
  }
  const int64_t n[3] = {g->n1, g->n2, g->n3};
  int64_t k = 1;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 0 || n[a] > NX_MAX_COUNT) {
      fail(NX_ERR_ARG, "%s: grid count n%d = %lld outside [0, %lld]", fn, a + 1, (long long)n[a],
           (long long)NX_MAX_COUNT);
      return -1;
    }
    if (n[a] == 0) k = 0;
    else if (k > NX_MAX_COUNT / n[a]) k = NX_MAX_COUNT + 1;
    else k *= n[a];
  }
  if (k > NX_MAX_COUNT) {
    fail(NX_ERR_ARG, "%s: grid of %lld x %lld x %lld points exceeds %lld", fn, (long long)g->n1,
         (long long)g->n2, (long long)g->n3, (long long)NX_MAX_COUNT);
    return -1;
  }
  const double* v[4] = {g->origin, g->step1, g->step2, g->step3};
  for (int a = 0; a < 4; ++a)
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(v[a][d])) {
        fail(NX_ERR_ARG, "%s: grid origin and steps must be finite", fn);
        return -1;
      }
  return k;
}

nx::GridDef grid_def(const nx_grid* g) {
  nx::GridDef d;
  for (int a = 0; a < 3; ++a) {
    d.o[a] = g->origin[a];
    d.e1[a] = g->step1[a];
    d.e2[a] = g->step2[a];
    d.e3[a] = g->step3[a];
  }
  d.n1 = g->n1;
  d.n2 = g->n2;
  d.n3 = g->n3;
  return d;
}

// The grid kernels walk rows of n1 points; they need n1 to be a multiple of 64.  The kind
// passed to make_plan: 1 (general kernels) or 2 + the counts that allow two points per
// lane along i1 (1: n1 a multiple of 128), i2 (2: n2 even) and i3 (4: n3 even).
int grid_kind(const nx_grid* g) {
  if (g->n1 % 64 != 0) return 1;
  return 2 + ((g->n1 % 128 == 0) ? 1 : 0) + ((g->n2 % 2 == 0) ? 2 : 0) + ((g->n3 % 2 == 0) ? 4 : 0);
}

// A grid's forward with few records to form (one point per lane, 8- or 16-atom groups,
// blocks x atoms within the inline bound of the point lists): the general grid form, each
// lane forming its FP64 grid point, with the atom records formed while staging, saves the
// pack dispatch (C1, 4,096 atoms over 64 x 64 points: the grid rows' pack, 4 us, and its
// launch, against a sum kernel 3 us slower).  The workspace stays the one the plan sized
// (its record part unused).  NX_TUNE_INLINE=0 keeps the rows and their packed records.
void inline_small_grid_fwd(nx::Plan& p) {
  if (p.mode != nx::kPH64 || p.grid != 2 || p.per_lane != 1 || p.red != 2 || !p.lds ||
      (p.grp != 8 && p.grp != 16))
    return;
  const int64_t ti = env_i64("NX_TUNE_INLINE", -1);
  if (ti == 1 || (ti != 0 && p.blocks * p.stream <= nx::kInlineMaxRecords)) {
    p.grid = 1;
    p.inl = 1;
  }
}

// The launch sequence of run_sum over the points of a grid (FP64-phase mode): grid records
// packed, the chunks, the split reduce.  `out` is A (forward) or grad_xyz (adjoint).
int run_sum_grid(const char* fn, const nx::Plan& p, bool fwd, const float* xyz, const float* f,
                 const nx::GridDef& gd, const float* G, float* out, void* ws, hipStream_t st) {
  char* base = static_cast<char*>(ws);
  void* rec = base;
  void* partial = p.partial_bytes ? base + p.rec_bytes : nullptr;
  hipError_t e = hipSuccess;
  if (fwd) {
    if (!p.inl) e = nx::launch_pack_atoms_grid(p, xyz, f, p.stream, gd, rec, st);
  } else {
    e = nx::launch_pack_points_grid(p, gd, G, rec, st);
  }
  if (e != hipSuccess) return device_error(fn, e);
  for (int64_t c = 0; c < p.nchunks; ++c) {
    int64_t b, en, per;
    nx::chunk_range(p, c, &b, &en, &per);
    const int carry = c > 0 ? 1 : 0;
    const int direct = (p.nsplit == 1 && c == p.nchunks - 1) ? 1 : 0;
    if (fwd)
      e = nx::launch_fwd_chunk(p, rec, b, en, per, nullptr, partial, out, carry, direct, st, xyz, f, &gd);
    else
      e = nx::launch_bwd_chunk(p, rec, b, en, per, xyz, f, partial, out, nullptr, carry, direct, st,
                               nullptr, nullptr, &gd);
    if (e != hipSuccess) return device_error(fn, e);
  }
  if (p.nsplit > 1) {
    if (fwd) e = nx::launch_fwd_reduce(p, partial, out, st);
    else e = nx::launch_bwd_reduce(p, partial, f, out, nullptr, st);
    if (e != hipSuccess) return device_error(fn, e);
  }
  return ok();
}

// Validates a species partition: start[0] = 0, non-decreasing, start[n] = n_atoms.
int check_species(const char* fn, int64_t n_atoms, const int64_t* start, int n_species) {
  if (n_species < 1 || n_species > nx::kMaxSpecies)
    return fail(NX_ERR_ARG, "%s: n_species %d outside [1, %d]", fn, n_species, nx::kMaxSpecies);
  if (!start) return fail(NX_ERR_ARG, "%s: NULL species_start", fn);
  if (start[0] != 0 || start[n_species] != n_atoms)
    return fail(NX_ERR_ARG, "%s: species_start must run from 0 to n_atoms (%lld .. %lld given)", fn,
                (long long)start[0], (long long)start[n_species]);
  for (int s = 0; s < n_species; ++s)
    if (start[s + 1] < start[s])
      return fail(NX_ERR_ARG, "%s: species_start decreases at %d", fn, s);
  return NX_OK;
}

// Workspace of the species-factorised calls.
//   forward: atom records for all atoms, then one (sum, comp) state per species;
//   adjoint: the per-species seed, the point records, the largest per-species partial.
size_t species_ws(int op, int mode, int64_t n_points, const int64_t* start, int n_species,
                  size_t* state_off) {
  size_t total = 0;
  if (op == 0) {
    const nx::Plan p0 = nx::make_plan(nx::kOpFwd, mode, start[n_species], n_points, 1);
    total = p0.rec_bytes;
    for (int s = 0; s < n_species; ++s) {
      const nx::Plan ps = nx::make_plan(nx::kOpFwd, mode, start[s + 1] - start[s], n_points, 1);
      if (state_off) state_off[s] = total;
      total += align_up(size_t(ps.nsplit) * size_t(n_points) * 16, 256);
    }
  } else {
    size_t part = 0, rec = 0;
    for (int s = 0; s < n_species; ++s) {
      const nx::Plan ps = nx::make_plan(nx::kOpBwd, mode, start[s + 1] - start[s], n_points, 1);
      if (ps.partial_bytes > part) part = ps.partial_bytes;
      rec = ps.rec_bytes;
    }
    total = align_up(size_t(n_points) * 8, 256) + rec + part;
  }
  return total;
}

// Workspace of the species-factorised calls over a grid of k points (grid kind g, the
// FP64-phase mode): forward, every species' grid atom records at its atoms' place, then one
// (sum, comp) state per species; adjoint, the per-species seed, then the largest of the
// species' grid adjoint workspaces (point records and partials).
size_t species_grid_ws(int op, int64_t k, int g, const int64_t* start, int n_species,
                       size_t* state_off) {
  size_t total = 0;
  if (op == 0) {
    for (int s = 0; s < n_species; ++s) {
      const nx::Plan ps = nx::make_plan(nx::kOpFwd, NX_F32_PH64, start[s + 1] - start[s], k, 1,
                                        nx::kMaxSplit, g);
      total = std::max(total, align_up(size_t(start[s + 1]) * ps.rec_size, 256));
    }
    for (int s = 0; s < n_species; ++s) {
      const nx::Plan ps = nx::make_plan(nx::kOpFwd, NX_F32_PH64, start[s + 1] - start[s], k, 1,
                                        nx::kMaxSplit, g);
      if (state_off) state_off[s] = total;
      total += align_up(size_t(ps.nsplit) * size_t(k) * 16, 256);
    }
  } else {
    size_t most = 0;
    for (int s = 0; s < n_species; ++s)
      most = std::max(most, nx::make_plan(nx::kOpBwd, NX_F32_PH64, start[s + 1] - start[s], k, 1,
                                          nx::kMaxSplit, g).total());
    total = align_up(size_t(k) * 8, 256) + most;
  }
  return total;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------------
// Scratch of nx_scatter_fwd_noalloc: the packed atom records and the split/chunk partial
// sums of one call, as a static device array that every GPU the library runs on holds
// until the process ends.  In host code `scratch` names a host-side stand-in, not device
// memory: host code never passes it to a kernel or a copy.  Its device address is taken
// with hipGetSymbolAddress once per device (with that device current, on the first call
// there) and only that address is used.
static __device__ __align__(256) unsigned char scratch[NX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch.
int scratch_of_current_device(const char* fn, void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(fn, e);
  if (dev < 0 || dev >= kMaxDevices)
    return fail(NX_ERR_DEVICE, "%s: device %d outside the %d devices served", fn, dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_error(fn, e);
    if (p == nullptr) return fail(NX_ERR_DEVICE, "%s: no device address for the scratch", fn);
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return NX_OK;
}

// nx_scatter_fwd's plan with its stream slices cut down, if need be, until its workspace
// fits the scratch (the slice count is a function of the sizes only, so a call's plan and
// result are reproducible).  False when even one slice does not fit.
bool noalloc_plan(int mode, int64_t n_atoms, int64_t n_points, int f_is_null, nx::Plan* out) {
  const size_t cap = NX_NOALLOC_SCRATCH_BYTES;
  nx::Plan p = nx::make_plan(nx::kOpFwd, mode, n_atoms, n_points, f_is_null);
  if (p.total() <= cap) {
    *out = p;
    return true;
  }
  int64_t lo = 1, hi = p.nsplit - 1, best = 0;     // workspace grows with the slice count
  while (lo <= hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (nx::make_plan(nx::kOpFwd, mode, n_atoms, n_points, f_is_null, mid).total() <= cap) {
      best = mid;
      lo = mid + 1;
    } else {
      hi = mid - 1;
    }
  }
  if (best == 0) {
    *out = nx::make_plan(nx::kOpFwd, mode, n_atoms, n_points, f_is_null, 1);
    return false;
  }
  *out = nx::make_plan(nx::kOpFwd, mode, n_atoms, n_points, f_is_null, best);
  return true;
}

}  // namespace

extern "C" {

int nx_version(void) { return 104; }

const char* nx_last_error(void) { return g_last_error.c_str(); }

size_t nx_workspace_bytes(int64_t n_atoms, int64_t n_points, int mode, int op, int f_is_null) {
  if (check_counts("nx_workspace_bytes", n_atoms, n_points) != NX_OK) return 0;
  if (op < NX_OP_FWD || op > NX_OP_FIT) {
    fail(NX_ERR_MODE, "nx_workspace_bytes: unknown op %d", op);
    return 0;
  }
  if ((op == NX_OP_FWD || op == NX_OP_BWD || op == NX_OP_BWD_GF || op == NX_OP_FIT) &&
      mode != NX_F32 && mode != NX_F32_PH64) {
    fail(NX_ERR_MODE, "nx_workspace_bytes: unknown mode %d", mode);
    return 0;
  }
  ok();
  if (op == NX_OP_FIT)   // the three stages use the workspace in turn
    return std::max({nx::make_plan(nx::kOpFwd, mode, n_atoms, n_points, f_is_null).total(),
                     nx::make_plan(nx::kOpLoss, mode, 0, n_points, 1).total(),
                     nx::make_plan(nx::kOpBwd, mode, n_atoms, n_points, f_is_null).total()});
  return nx::make_plan(op, mode, n_atoms, n_points, f_is_null).total();
}

int nx_scatter_fwd(const float* xyz, const float* f, int64_t n_atoms, const float* S,
                   int64_t n_points, float* A, int mode, void* ws, size_t ws_bytes,
                   void* stream) {
  const char* fn = "nx_scatter_fwd";
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (mode != NX_F32 && mode != NX_F32_PH64) return fail(NX_ERR_MODE, "%s: unknown mode %d", fn, mode);
  if (n_points == 0) return ok();
  if (!S || !A || (n_atoms > 0 && !xyz))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p A=%p)", fn, (const void*)xyz,
                (const void*)S, (void*)A);
  if (!aligned(A, 8) || (f && !aligned(f, 8)))
    return fail(NX_ERR_ARG, "%s: A and f must be 8-byte aligned (complex64)", fn);
  const nx::Plan p = nx::make_plan(nx::kOpFwd, mode, n_atoms, n_points, f == nullptr);
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  return run_sum(fn, p, true, xyz, f, S, nullptr, A, nullptr, ws, static_cast<hipStream_t>(stream));
}

int nx_scatter_fwd_noalloc(const float* xyz, const float* f, int64_t n_atoms, const float* S,
                           int64_t n_points, float* A, int mode, void* stream) {
  const char* fn = "nx_scatter_fwd_noalloc";
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (mode != NX_F32 && mode != NX_F32_PH64) return fail(NX_ERR_MODE, "%s: unknown mode %d", fn, mode);
  if (n_points == 0) return ok();
  if (!S || !A || (n_atoms > 0 && !xyz))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p A=%p)", fn, (const void*)xyz,
                (const void*)S, (void*)A);
  if (!aligned(A, 8) || (f && !aligned(f, 8)))
    return fail(NX_ERR_ARG, "%s: A and f must be 8-byte aligned (complex64)", fn);
  nx::Plan p;
  if (!noalloc_plan(mode, n_atoms, n_points, f == nullptr, &p))
    return fail(NX_ERR_WORKSPACE,
                "%s: %lld atoms over %lld points need %zu bytes of scratch even with one stream "
                "slice; the static scratch holds %zu (use nx_scatter_fwd with a workspace)",
                fn, (long long)n_atoms, (long long)n_points, p.total(),
                (size_t)NX_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if (p.total() > 0) {
    if (int r = scratch_of_current_device(fn, &ws)) return r;
  }
  return run_sum(fn, p, true, xyz, f, S, nullptr, A, nullptr, ws, static_cast<hipStream_t>(stream));
}

int nx_scatter_bwd(const float* xyz, const float* f, int64_t n_atoms, const float* S,
                   int64_t n_points, const float* G, float* grad_xyz, int mode, void* ws,
                   size_t ws_bytes, void* stream) {
  const char* fn = "nx_scatter_bwd";
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (mode != NX_F32 && mode != NX_F32_PH64) return fail(NX_ERR_MODE, "%s: unknown mode %d", fn, mode);
  if (n_atoms == 0) return ok();
  if (!xyz || !grad_xyz || (n_points > 0 && (!S || !G)))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p G=%p grad_xyz=%p)", fn,
                (const void*)xyz, (const void*)S, (const void*)G, (void*)grad_xyz);
  if ((G && !aligned(G, 8)) || (f && !aligned(f, 8)))
    return fail(NX_ERR_ARG, "%s: G and f must be 8-byte aligned (complex64)", fn);
  const nx::Plan p = nx::make_plan(nx::kOpBwd, mode, n_atoms, n_points, f == nullptr);
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  return run_sum(fn, p, false, xyz, f, S, G, grad_xyz, nullptr, ws, static_cast<hipStream_t>(stream));
}

int nx_scatter_fwd_f64(const double* xyz, const double* f, int64_t n_atoms, const double* S,
                       int64_t n_points, double* A, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nx_scatter_fwd_f64";
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (n_points == 0) return ok();
  if (!S || !A || (n_atoms > 0 && !xyz))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p A=%p)", fn, (const void*)xyz,
                (const void*)S, (void*)A);
  if (!aligned(A, 16) || !aligned(S, 8) || (xyz && !aligned(xyz, 8)) || (f && !aligned(f, 8)))
    return fail(NX_ERR_ARG, "%s: misaligned double array (A needs 16 bytes)", fn);
  const nx::Plan p = nx::make_plan(nx::kOpFwdF64, 0, n_atoms, n_points, f == nullptr);
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  return run_sum(fn, p, true, xyz, f, S, nullptr, A, nullptr, ws, static_cast<hipStream_t>(stream));
}

int nx_scatter_bwd_f64(const double* xyz, const double* f, int64_t n_atoms, const double* S,
                       int64_t n_points, const double* G, double* grad_xyz, void* ws,
                       size_t ws_bytes, void* stream) {
  const char* fn = "nx_scatter_bwd_f64";
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (n_atoms == 0) return ok();
  if (!xyz || !grad_xyz || (n_points > 0 && (!S || !G)))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p G=%p grad_xyz=%p)", fn,
                (const void*)xyz, (const void*)S, (const void*)G, (void*)grad_xyz);
  if (!aligned(xyz, 8) || !aligned(grad_xyz, 8) || (S && !aligned(S, 8)) ||
      (G && !aligned(G, 8)) || (f && !aligned(f, 8)))
    return fail(NX_ERR_ARG, "%s: misaligned double array", fn);
  const nx::Plan p = nx::make_plan(nx::kOpBwdF64, 0, n_atoms, n_points, f == nullptr);
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  return run_sum(fn, p, false, xyz, f, S, G, grad_xyz, nullptr, ws, static_cast<hipStream_t>(stream));
}

int nx_loss_grad(const float* A, const float* I, int64_t n_points, double* L, float* G, void* ws,
                 size_t ws_bytes, void* stream) {
  const char* fn = "nx_loss_grad";
  if (int r = check_counts(fn, 0, n_points)) return r;
  if (!L || (n_points > 0 && (!A || !I)))
    return fail(NX_ERR_ARG, "%s: NULL pointer (A=%p I=%p L=%p)", fn, (const void*)A,
                (const void*)I, (void*)L);
  if (!aligned(L, 8) || (A && !aligned(A, 8)) || (G && !aligned(G, 8)))
    return fail(NX_ERR_ARG, "%s: A, G need 8-byte and L 8-byte alignment", fn);
  const nx::Plan p = nx::make_plan(nx::kOpLoss, 0, 0, n_points, 1);
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  hipError_t e = nx::launch_loss(A, I, n_points, L, G, static_cast<double*>(ws),
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_error(fn, e);
  return ok();
}

int nx_fit_step(const float* xyz, const float* f, int64_t n_atoms, const float* S,
                int64_t n_points, const float* I, float* A, double* L, float* G,
                float* grad_xyz, int mode, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nx_fit_step";
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (mode != NX_F32 && mode != NX_F32_PH64) return fail(NX_ERR_MODE, "%s: unknown mode %d", fn, mode);
  // everything the three stages check, before any of them queues work
  if (!L || (n_points > 0 && (!S || !A || !I || !G)) || (n_atoms > 0 && (!xyz || !grad_xyz)))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p I=%p A=%p L=%p G=%p grad_xyz=%p)", fn,
                (const void*)xyz, (const void*)S, (const void*)I, (void*)A, (void*)L, (void*)G,
                (void*)grad_xyz);
  if ((A && !aligned(A, 8)) || (G && !aligned(G, 8)) || (f && !aligned(f, 8)) || !aligned(L, 8))
    return fail(NX_ERR_ARG, "%s: A, G, f and L must be 8-byte aligned", fn);
  const size_t need = nx_workspace_bytes(n_atoms, n_points, mode, NX_OP_FIT, f == nullptr);
  if (need > 0 && (ws == nullptr || ws_bytes < need || !aligned(ws, 16)))
    return fail(NX_ERR_WORKSPACE, "%s: workspace of %zu bytes (16-byte aligned) needed, %zu given",
                fn, need, ws_bytes);
  if (int r = nx_scatter_fwd(xyz, f, n_atoms, S, n_points, A, mode, ws, ws_bytes, stream)) return r;
  if (int r = nx_loss_grad(A, I, n_points, L, G, ws, ws_bytes, stream)) return r;
  if (int r = nx_scatter_bwd(xyz, f, n_atoms, S, n_points, G, grad_xyz, mode, ws, ws_bytes, stream))
    return r;
  return ok();
}

int nx_scatter_bwd_ex(const float* xyz, const float* f, int64_t n_atoms, const float* S,
                      int64_t n_points, const float* G, float* grad_xyz, float* grad_f, int mode,
                      void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nx_scatter_bwd_ex";
  if (!grad_f)
    return nx_scatter_bwd(xyz, f, n_atoms, S, n_points, G, grad_xyz, mode, ws, ws_bytes, stream);
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (mode != NX_F32 && mode != NX_F32_PH64) return fail(NX_ERR_MODE, "%s: unknown mode %d", fn, mode);
  if (n_atoms == 0) return ok();
  if (!xyz || (n_points > 0 && (!S || !G)))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p G=%p)", fn, (const void*)xyz,
                (const void*)S, (const void*)G);
  if ((G && !aligned(G, 8)) || (f && !aligned(f, 8)) || !aligned(grad_f, 8))
    return fail(NX_ERR_ARG, "%s: G, f and grad_f must be 8-byte aligned (complex64)", fn);
  const nx::Plan p = nx::make_plan(nx::kOpBwdGf, mode, n_atoms, n_points, f == nullptr);
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  return run_sum(fn, p, false, xyz, f, S, G, grad_xyz, grad_f, ws, static_cast<hipStream_t>(stream));
}

int nx_scatter_bwd_ex_f64(const double* xyz, const double* f, int64_t n_atoms, const double* S,
                          int64_t n_points, const double* G, double* grad_xyz, double* grad_f,
                          void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nx_scatter_bwd_ex_f64";
  if (!grad_f)
    return nx_scatter_bwd_f64(xyz, f, n_atoms, S, n_points, G, grad_xyz, ws, ws_bytes, stream);
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (n_atoms == 0) return ok();
  if (!xyz || (n_points > 0 && (!S || !G)))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p G=%p)", fn, (const void*)xyz,
                (const void*)S, (const void*)G);
  if (!aligned(xyz, 8) || (grad_xyz && !aligned(grad_xyz, 8)) || !aligned(grad_f, 8) ||
      (S && !aligned(S, 8)) || (G && !aligned(G, 8)) || (f && !aligned(f, 8)))
    return fail(NX_ERR_ARG, "%s: misaligned double array", fn);
  const nx::Plan p = nx::make_plan(nx::kOpBwdGfF64, 0, n_atoms, n_points, f == nullptr);
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  return run_sum(fn, p, false, xyz, f, S, G, grad_xyz, grad_f, ws, static_cast<hipStream_t>(stream));
}

size_t nx_workspace_bytes_grid(int64_t n_atoms, const nx_grid* grid, int op, int f_is_null) {
  const char* fn = "nx_workspace_bytes_grid";
  const int64_t k = grid_points(fn, grid);
  if (k < 0) return 0;
  if (check_counts(fn, n_atoms, k) != NX_OK) return 0;
  if (op != NX_OP_FWD && op != NX_OP_BWD && op != NX_OP_FIT) {
    fail(NX_ERR_MODE, "%s: op must be NX_OP_FWD, NX_OP_BWD or NX_OP_FIT, got %d", fn, op);
    return 0;
  }
  ok();
  const int g = grid_kind(grid);
  const size_t fw = nx::make_plan(nx::kOpFwd, NX_F32_PH64, n_atoms, k, f_is_null, nx::kMaxSplit, g).total();
  const size_t bw = nx::make_plan(nx::kOpBwd, NX_F32_PH64, n_atoms, k, f_is_null, nx::kMaxSplit, g).total();
  if (op == NX_OP_FWD) return fw;
  if (op == NX_OP_BWD) return bw;
  return std::max({fw, bw, nx::make_plan(nx::kOpLoss, NX_F32_PH64, 0, k, 1).total()});
}

int nx_scatter_fwd_grid(const float* xyz, const float* f, int64_t n_atoms, const nx_grid* grid,
                        float* A, int mode, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nx_scatter_fwd_grid";
  const int64_t k = grid_points(fn, grid);
  if (k < 0) return NX_ERR_ARG;
  if (int r = check_counts(fn, n_atoms, k)) return r;
  if (mode != NX_F32_PH64)
    return fail(NX_ERR_MODE, "%s: mode %d: grids take the FP64-phase mode (NX_F32_PH64)", fn, mode);
  if (k == 0) return ok();
  if (!A || (n_atoms > 0 && !xyz))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p A=%p)", fn, (const void*)xyz, (void*)A);
  if (!aligned(A, 8) || (f && !aligned(f, 8)))
    return fail(NX_ERR_ARG, "%s: A and f must be 8-byte aligned (complex64)", fn);
  nx::Plan p = nx::make_plan(nx::kOpFwd, mode, n_atoms, k, f == nullptr, nx::kMaxSplit, grid_kind(grid));
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  inline_small_grid_fwd(p);
  return run_sum_grid(fn, p, true, xyz, f, grid_def(grid), nullptr, A, ws, static_cast<hipStream_t>(stream));
}

int nx_scatter_bwd_grid(const float* xyz, const float* f, int64_t n_atoms, const nx_grid* grid,
                        const float* G, float* grad_xyz, int mode, void* ws, size_t ws_bytes,
                        void* stream) {
  const char* fn = "nx_scatter_bwd_grid";
  const int64_t k = grid_points(fn, grid);
  if (k < 0) return NX_ERR_ARG;
  if (int r = check_counts(fn, n_atoms, k)) return r;
  if (mode != NX_F32_PH64)
    return fail(NX_ERR_MODE, "%s: mode %d: grids take the FP64-phase mode (NX_F32_PH64)", fn, mode);
  if (n_atoms == 0) return ok();
  if (!xyz || !grad_xyz || (k > 0 && !G))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p G=%p grad_xyz=%p)", fn, (const void*)xyz,
                (const void*)G, (void*)grad_xyz);
  if ((G && !aligned(G, 8)) || (f && !aligned(f, 8)))
    return fail(NX_ERR_ARG, "%s: G and f must be 8-byte aligned (complex64)", fn);
  // (no points: the kernel runs over an empty range and writes a zero gradient)
  const nx::Plan p = nx::make_plan(nx::kOpBwd, mode, n_atoms, k, f == nullptr, nx::kMaxSplit, grid_kind(grid));
  if (int r = check_ws(fn, p, ws, ws_bytes)) return r;
  return run_sum_grid(fn, p, false, xyz, f, grid_def(grid), G, grad_xyz, ws, static_cast<hipStream_t>(stream));
}

int nx_fit_step_grid(const float* xyz, const float* f, int64_t n_atoms, const nx_grid* grid,
                     const float* I, float* A, double* L, float* G, float* grad_xyz, int mode,
                     void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nx_fit_step_grid";
  const int64_t k = grid_points(fn, grid);
  if (k < 0) return NX_ERR_ARG;
  if (int r = check_counts(fn, n_atoms, k)) return r;
  if (mode != NX_F32_PH64)
    return fail(NX_ERR_MODE, "%s: mode %d: grids take the FP64-phase mode (NX_F32_PH64)", fn, mode);
  if (!L || (k > 0 && (!A || !I || !G)) || (n_atoms > 0 && (!xyz || !grad_xyz)))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p I=%p A=%p L=%p G=%p grad_xyz=%p)", fn,
                (const void*)xyz, (const void*)I, (void*)A, (void*)L, (void*)G, (void*)grad_xyz);
  if ((A && !aligned(A, 8)) || (G && !aligned(G, 8)) || (f && !aligned(f, 8)) || !aligned(L, 8))
    return fail(NX_ERR_ARG, "%s: A, G, f and L must be 8-byte aligned", fn);
  const size_t need = nx_workspace_bytes_grid(n_atoms, grid, NX_OP_FIT, f == nullptr);
  if (need > 0 && (ws == nullptr || ws_bytes < need || !aligned(ws, 16)))
    return fail(NX_ERR_WORKSPACE, "%s: workspace of %zu bytes (16-byte aligned) needed, %zu given",
                fn, need, ws_bytes);
  if (int r = nx_scatter_fwd_grid(xyz, f, n_atoms, grid, A, mode, ws, ws_bytes, stream)) return r;
  if (int r = nx_loss_grad(A, I, k, L, G, ws, ws_bytes, stream)) return r;
  if (int r = nx_scatter_bwd_grid(xyz, f, n_atoms, grid, G, grad_xyz, mode, ws, ws_bytes, stream))
    return r;
  return ok();
}

size_t nx_workspace_bytes_species(const int64_t* species_start, int n_species, int64_t n_points,
                                  int mode, int op) {
  const char* fn = "nx_workspace_bytes_species";
  if (n_species < 1 || n_species > nx::kMaxSpecies || !species_start) {
    fail(NX_ERR_ARG, "%s: n_species %d outside [1, %d] or NULL species_start", fn, n_species,
         nx::kMaxSpecies);
    return 0;
  }
  const int64_t n_atoms = species_start[n_species];
  if (check_counts(fn, n_atoms, n_points) != NX_OK) return 0;
  if (check_species(fn, n_atoms, species_start, n_species) != NX_OK) return 0;
  if (mode != NX_F32 && mode != NX_F32_PH64) {
    fail(NX_ERR_MODE, "%s: unknown mode %d", fn, mode);
    return 0;
  }
  if (op != 0 && op != 1) {
    fail(NX_ERR_MODE, "%s: op must be 0 (forward) or 1 (adjoint), got %d", fn, op);
    return 0;
  }
  ok();
  return species_ws(op, mode, n_points, species_start, n_species, nullptr);
}

int nx_scatter_fwd_species(const float* xyz, int64_t n_atoms, const int64_t* species_start,
                           int n_species, const float* fs, const float* S, int64_t n_points,
                           float* A, float* A_species, int mode, void* ws, size_t ws_bytes,
                           void* stream) {
  const char* fn = "nx_scatter_fwd_species";
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (int r = check_species(fn, n_atoms, species_start, n_species)) return r;
  if (mode != NX_F32 && mode != NX_F32_PH64) return fail(NX_ERR_MODE, "%s: unknown mode %d", fn, mode);
  if (n_points == 0) return ok();
  if (!S || !A || (n_atoms > 0 && !xyz))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p S=%p A=%p)", fn, (const void*)xyz,
                (const void*)S, (void*)A);
  if (!aligned(A, 8) || (fs && !aligned(fs, 8)) || (A_species && !aligned(A_species, 8)))
    return fail(NX_ERR_ARG, "%s: A, fs and A_species must be 8-byte aligned (complex64)", fn);
  size_t off[nx::kMaxSpecies];
  const size_t need = species_ws(0, mode, n_points, species_start, n_species, off);
  if (need > 0 && (ws == nullptr || ws_bytes < need || !aligned(ws, 16)))
    return fail(NX_ERR_WORKSPACE, "%s: workspace of %zu bytes (16-byte aligned) needed, %zu given", fn,
                need, ws_bytes);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  hipError_t e;
  nx::SpeciesStates ss{};
  ss.n = n_species;
  for (int s = 0; s < n_species; ++s) {
    const int64_t a0 = species_start[s];
    nx::Plan ps = nx::make_plan(nx::kOpFwd, mode, species_start[s + 1] - a0, n_points, 1);
    // each species' records are packed with its own plan (variant, group size), their
    // groups counted from the species' first atom; they sit at the species' place in ws
    // (the kernels read them there: no records formed inside the kernel)
    ps.inl = 0;
    e = nx::launch_pack_atoms(ps.mode, ps.red, ps.grp, xyz + 3 * a0, nullptr, ps.stream,
                              base + a0 * ps.rec_size, st);
    if (e != hipSuccess) return device_error(fn, e);
    void* state = base + off[s];
    ss.state[s] = state;
    ss.nsplit[s] = ps.nsplit;
    for (int64_t c = 0; c < ps.nchunks; ++c) {
      int64_t b, en, per;
      nx::chunk_range(ps, c, &b, &en, &per);
      e = nx::launch_fwd_chunk(ps, base, a0 + b, a0 + en, per, S, state, nullptr, c > 0 ? 1 : 0, 0, st);
      if (e != hipSuccess) return device_error(fn, e);
    }
  }
  e = nx::launch_species_combine(ss, fs, n_points, A, A_species, st);
  if (e != hipSuccess) return device_error(fn, e);
  return ok();
}

int nx_scatter_bwd_species(const float* xyz, int64_t n_atoms, const int64_t* species_start,
                           int n_species, const float* fs, const float* S, int64_t n_points,
                           const float* G, const float* A_species, float* grad_xyz,
                           float* grad_fs, int mode, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nx_scatter_bwd_species";
  if (int r = check_counts(fn, n_atoms, n_points)) return r;
  if (int r = check_species(fn, n_atoms, species_start, n_species)) return r;
  if (mode != NX_F32 && mode != NX_F32_PH64) return fail(NX_ERR_MODE, "%s: unknown mode %d", fn, mode);
  if (!grad_xyz && !grad_fs) return ok();
  if (n_points > 0 && (!S || !G))
    return fail(NX_ERR_ARG, "%s: NULL pointer (S=%p G=%p)", fn, (const void*)S, (const void*)G);
  if (grad_xyz && n_atoms > 0 && !xyz) return fail(NX_ERR_ARG, "%s: NULL xyz", fn);
  if (grad_fs && n_points > 0 && !A_species)
    return fail(NX_ERR_ARG, "%s: grad_fs needs the per-species sums A_species", fn);
  if ((G && !aligned(G, 8)) || (fs && !aligned(fs, 8)) || (grad_fs && !aligned(grad_fs, 8)) ||
      (A_species && !aligned(A_species, 8)))
    return fail(NX_ERR_ARG, "%s: G, fs, A_species and grad_fs must be 8-byte aligned", fn);
  const size_t need = species_ws(1, mode, n_points, species_start, n_species, nullptr);
  if (grad_xyz && n_atoms > 0 && need > 0 && (ws == nullptr || ws_bytes < need || !aligned(ws, 16)))
    return fail(NX_ERR_WORKSPACE, "%s: workspace of %zu bytes (16-byte aligned) needed, %zu given", fn,
                need, ws_bytes);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (grad_fs) {
    for (int s = 0; s < n_species; ++s) {
      e = nx::launch_species_gradf(G, A_species + 2 * int64_t(s) * n_points, n_points,
                                   grad_fs + 2 * int64_t(s) * n_points, st);
      if (e != hipSuccess) return device_error(fn, e);
    }
  }
  if (!grad_xyz || n_atoms == 0) return ok();
  char* base = static_cast<char*>(ws);
  float* seed = reinterpret_cast<float*>(base);
  char* rest = base + align_up(size_t(n_points) * 8, 256);
  for (int s = 0; s < n_species; ++s) {
    const int64_t a0 = species_start[s], ns = species_start[s + 1] - a0;
    if (ns == 0) continue;
    e = nx::launch_species_seed(G, fs ? fs + 2 * int64_t(s) * n_points : nullptr, n_points, seed, st);
    if (e != hipSuccess) return device_error(fn, e);
    const nx::Plan ps = nx::make_plan(nx::kOpBwd, mode, ns, n_points, 1);
    const int r = run_sum(fn, ps, false, xyz + 3 * a0, nullptr, S, seed, grad_xyz + 3 * a0, nullptr,
                          rest, st);
    if (r != NX_OK) return r;
  }
  return ok();
}

size_t nx_workspace_bytes_species_grid(const int64_t* species_start, int n_species,
                                       const nx_grid* grid, int op) {
  const char* fn = "nx_workspace_bytes_species_grid";
  const int64_t k = grid_points(fn, grid);
  if (k < 0) return 0;
  if (n_species < 1 || n_species > nx::kMaxSpecies || !species_start) {
    fail(NX_ERR_ARG, "%s: n_species %d outside [1, %d] or NULL species_start", fn, n_species,
         nx::kMaxSpecies);
    return 0;
  }
  const int64_t n_atoms = species_start[n_species];
  if (check_counts(fn, n_atoms, k) != NX_OK) return 0;
  if (check_species(fn, n_atoms, species_start, n_species) != NX_OK) return 0;
  if (op != 0 && op != 1) {
    fail(NX_ERR_MODE, "%s: op must be 0 (forward) or 1 (adjoint), got %d", fn, op);
    return 0;
  }
  ok();
  return species_grid_ws(op, k, grid_kind(grid), species_start, n_species, nullptr);
}

int nx_scatter_fwd_species_grid(const float* xyz, int64_t n_atoms, const int64_t* species_start,
                                int n_species, const float* fs, const nx_grid* grid, float* A,
                                float* A_species, int mode, void* ws, size_t ws_bytes,
                                void* stream) {
  const char* fn = "nx_scatter_fwd_species_grid";
  const int64_t k = grid_points(fn, grid);
  if (k < 0) return NX_ERR_ARG;
  if (int r = check_counts(fn, n_atoms, k)) return r;
  if (int r = check_species(fn, n_atoms, species_start, n_species)) return r;
  if (mode != NX_F32_PH64)
    return fail(NX_ERR_MODE, "%s: mode %d: grids take the FP64-phase mode (NX_F32_PH64)", fn, mode);
  if (k == 0) return ok();
  if (!A || (n_atoms > 0 && !xyz))
    return fail(NX_ERR_ARG, "%s: NULL pointer (xyz=%p A=%p)", fn, (const void*)xyz, (void*)A);
  if (!aligned(A, 8) || (fs && !aligned(fs, 8)) || (A_species && !aligned(A_species, 8)))
    return fail(NX_ERR_ARG, "%s: A, fs and A_species must be 8-byte aligned (complex64)", fn);
  const int g = grid_kind(grid);
  size_t off[nx::kMaxSpecies];
  const size_t need = species_grid_ws(0, k, g, species_start, n_species, off);
  if (ws == nullptr || ws_bytes < need || !aligned(ws, 16))
    return fail(NX_ERR_WORKSPACE, "%s: workspace of %zu bytes (16-byte aligned) needed, %zu given", fn,
                need, ws_bytes);
  const nx::GridDef gd = grid_def(grid);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  hipError_t e;
  nx::SpeciesStates ss{};
  ss.n = n_species;
  for (int s = 0; s < n_species; ++s) {
    const int64_t a0 = species_start[s], ns = species_start[s + 1] - a0;
    const nx::Plan ps = nx::make_plan(nx::kOpFwd, mode, ns, k, 1, nx::kMaxSplit, g);
    // each species' grid records, packed with its own plan, at its atoms' place (its groups
    // counted from its first atom); the chunks write its (sum, comp) state, never A
    e = nx::launch_pack_atoms_grid(ps, xyz + 3 * a0, nullptr, ns, gd, base + a0 * ps.rec_size, st);
    if (e != hipSuccess) return device_error(fn, e);
    void* state = base + off[s];
    ss.state[s] = state;
    ss.nsplit[s] = ps.nsplit;
    for (int64_t c = 0; c < ps.nchunks; ++c) {
      int64_t b, en, per;
      nx::chunk_range(ps, c, &b, &en, &per);
      e = nx::launch_fwd_chunk(ps, base, a0 + b, a0 + en, per, nullptr, state, nullptr, c > 0 ? 1 : 0,
                               0, st, nullptr, nullptr, &gd);
      if (e != hipSuccess) return device_error(fn, e);
    }
  }
  e = nx::launch_species_combine(ss, fs, k, A, A_species, st);
  if (e != hipSuccess) return device_error(fn, e);
  return ok();
}

int nx_scatter_bwd_species_grid(const float* xyz, int64_t n_atoms, const int64_t* species_start,
                                int n_species, const float* fs, const nx_grid* grid, const float* G,
                                const float* A_species, float* grad_xyz, float* grad_fs, int mode,
                                void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nx_scatter_bwd_species_grid";
  const int64_t k = grid_points(fn, grid);
  if (k < 0) return NX_ERR_ARG;
  if (int r = check_counts(fn, n_atoms, k)) return r;
  if (int r = check_species(fn, n_atoms, species_start, n_species)) return r;
  if (mode != NX_F32_PH64)
    return fail(NX_ERR_MODE, "%s: mode %d: grids take the FP64-phase mode (NX_F32_PH64)", fn, mode);
  if (!grad_xyz && !grad_fs) return ok();
  if (k > 0 && !G) return fail(NX_ERR_ARG, "%s: NULL G", fn);
  if (grad_xyz && n_atoms > 0 && !xyz) return fail(NX_ERR_ARG, "%s: NULL xyz", fn);
  if (grad_fs && k > 0 && !A_species)
    return fail(NX_ERR_ARG, "%s: grad_fs needs the per-species sums A_species", fn);
  if ((G && !aligned(G, 8)) || (fs && !aligned(fs, 8)) || (grad_fs && !aligned(grad_fs, 8)) ||
      (A_species && !aligned(A_species, 8)))
    return fail(NX_ERR_ARG, "%s: G, fs, A_species and grad_fs must be 8-byte aligned", fn);
  const int g = grid_kind(grid);
  const size_t need = species_grid_ws(1, k, g, species_start, n_species, nullptr);
  if (grad_xyz && n_atoms > 0 && need > 0 && (ws == nullptr || ws_bytes < need || !aligned(ws, 16)))
    return fail(NX_ERR_WORKSPACE, "%s: workspace of %zu bytes (16-byte aligned) needed, %zu given", fn,
                need, ws_bytes);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (grad_fs) {
    for (int s = 0; s < n_species; ++s) {
      e = nx::launch_species_gradf(G, A_species + 2 * int64_t(s) * k, k, grad_fs + 2 * int64_t(s) * k, st);
      if (e != hipSuccess) return device_error(fn, e);
    }
  }
  if (!grad_xyz || n_atoms == 0) return ok();
  const nx::GridDef gd = grid_def(grid);
  char* base = static_cast<char*>(ws);
  float* seed = reinterpret_cast<float*>(base);
  char* rest = base + align_up(size_t(k) * 8, 256);
  for (int s = 0; s < n_species; ++s) {
    const int64_t a0 = species_start[s], ns = species_start[s + 1] - a0;
    if (ns == 0) continue;
    e = nx::launch_species_seed(G, fs ? fs + 2 * int64_t(s) * k : nullptr, k, seed, st);
    if (e != hipSuccess) return device_error(fn, e);
    // (no points: the grid adjoint runs over an empty range and writes a zero gradient)
    const nx::Plan ps = nx::make_plan(nx::kOpBwd, mode, ns, k, 1, nx::kMaxSplit, g);
    const int r = run_sum_grid(fn, ps, false, xyz + 3 * a0, nullptr, gd, seed, grad_xyz + 3 * a0,
                               rest, st);
    if (r != NX_OK) return r;
  }
  return ok();
}

}  // extern "C"
