// nx_api.cpp -- the C ABI of libnx (declared in include/nx.h): argument validation
// (pure host code, before any HIP call), launch planning, workspace layout and the
// launch sequence of each entry point.
#include "nx.h"

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
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

Plan make_plan(int op, int mode, int64_t n_atoms, int64_t n_points, int f_is_null) {
  Plan p;
  p.fk = f_is_null ? 0 : 1;
  const bool fwd = (op == kOpFwd || op == kOpFwdF64);
  if (op == kOpLoss) {
    p.misc_bytes = size_t(kLossBlocks) * sizeof(double);
    return p;
  }
  p.mode = (op == kOpFwdF64 || op == kOpBwdF64) ? kF64 : (mode == NX_F32_PH64 ? kPH64 : kF32);
  p.lanes = fwd ? n_points : n_atoms;
  p.stream = fwd ? n_atoms : n_points;
  // Defaults from launch-shape and accuracy sweeps on MI355X.  Forward, FP64-phase
  // mode: the centred reduction (its FP32 rounding of the reduced phase is half that of
  // fract's, which decides the pointwise intensity error at the weakest points), and
  // 8-atom groups for few atoms (|A| peaks at N |f|, so each term weighs more), 16 above.
  // Adjoint (judged normwise): fract, 32-point groups, two atoms per lane.
  if (fwd) {
    const bool small = p.stream < 65536;
    p.red = 0;
    p.grp = (p.mode == kPH64 && small) ? 8 : 16;
    if (p.mode == kF64) p.per_lane = p.lanes >= 262144 ? 2 : 1;
    else p.per_lane = (p.lanes >= 32768 && p.lanes < 1048576) ? 2 : 1;
  } else {
    p.red = p.mode == kPH64 ? 1 : 0;
    p.grp = p.mode == kPH64 ? 32 : 16;
    p.per_lane = (p.mode != kF64 && p.lanes >= 16384) ? 2 : 1;
  }
  {
    // unset knobs read as -1, which no knob accepts
    const int64_t tp = env_i64("NX_TUNE_P", -1);
    if (tp == 1 || tp == 2 || (tp == 4 && p.mode != kF64)) p.per_lane = int(tp);
    const int64_t tg = env_i64("NX_TUNE_GRP", -1);
    if (p.mode == kPH64 && (tg == 8 || tg == 16 || tg == 32) && (fwd || tg != 8)) p.grp = int(tg);
    const int64_t tr = env_i64("NX_TUNE_RED", -1);
    if (p.mode == kPH64 && (tr == 0 || tr == 1)) p.red = int(tr);
  }
  const int64_t per_block = int64_t(kThreads) * p.per_lane;
  p.blocks = p.lanes > 0 ? ceil_div(p.lanes, per_block) : 0;
  p.nsplit = 1;
  if (p.blocks > 0 && p.blocks < kTargetBlocks) {
    int64_t want = ceil_div(kTargetBlocks, p.blocks);
    int64_t maxs = p.stream / kMinStreamPerSplit;
    if (maxs < 1) maxs = 1;
    if (want > maxs) want = maxs;
    if (want > kMaxSplit) want = kMaxSplit;
    p.nsplit = int(want);
  }
  // chunks of at most kLaunchPairs pairs, a whole number of groups per split
  const int64_t lane_pad = p.blocks * per_block;
  const int64_t gran = int64_t(p.nsplit) * p.grp;
  int64_t launch_pairs = env_i64("NX_TUNE_LAUNCH_PAIRS", kLaunchPairs);
  if (launch_pairs < 1) launch_pairs = kLaunchPairs;
  int64_t chunk = lane_pad > 0 ? launch_pairs / lane_pad : p.stream;
  chunk = chunk / gran * gran;
  if (chunk < gran) chunk = gran;
  if (chunk >= p.stream) {
    p.chunk = p.stream;
    p.nchunks = 1;
  } else {
    p.chunk = chunk;
    p.nchunks = ceil_div(p.stream, chunk);
  }
  // workspace: packed stream records, then the partial state
  size_t rec_size;
  if (fwd) rec_size = p.mode == kF64 ? sizeof(AtomF64) : (p.mode == kPH64 ? sizeof(AtomPH) : sizeof(AtomF32));
  else rec_size = p.mode == kF64 ? sizeof(PointF64) : (p.mode == kPH64 ? sizeof(PointPH) : sizeof(PointF32));
  p.rec_bytes = align_up(size_t(p.stream) * rec_size, 256);
  const bool need_partial = p.lanes > 0 && (p.nsplit > 1 || p.nchunks > 1);
  if (need_partial) {
    size_t per_item;
    if (fwd) per_item = 16;                                  // float4 or double2 per point
    else per_item = p.mode == kF64 ? 3 * 8 : 3 * 2 * 4;      // 3 sums (+ comps) per atom
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

// Chunked launch sequence shared by the four sum entry points.
int run_sum(const char* fn, const nx::Plan& p, bool fwd, const void* xyz, const void* f,
            const void* S, const void* G, void* out, void* ws, hipStream_t st) {
  char* base = static_cast<char*>(ws);
  void* rec = base;
  void* partial = p.partial_bytes ? base + p.rec_bytes : nullptr;
  hipError_t e;
  if (fwd) e = nx::launch_pack_atoms(p.mode, p.red, xyz, f, p.stream, rec, st);
  else e = nx::launch_pack_points(p.mode, p.red, S, G, p.stream, rec, st);
  if (e != hipSuccess) return device_error(fn, e);
  for (int64_t c = 0; c < p.nchunks; ++c) {
    int64_t b, en, per;
    nx::chunk_range(p, c, &b, &en, &per);
    const int carry = c > 0 ? 1 : 0;
    const int direct = (p.nsplit == 1 && c == p.nchunks - 1) ? 1 : 0;
    if (fwd) e = nx::launch_fwd_chunk(p, rec, b, en, per, S, partial, out, carry, direct, st);
    else e = nx::launch_bwd_chunk(p, rec, b, en, per, xyz, f, partial, out, carry, direct, st);
    if (e != hipSuccess) return device_error(fn, e);
  }
  if (p.nsplit > 1) {
    if (fwd) e = nx::launch_fwd_reduce(p, partial, out, st);
    else e = nx::launch_bwd_reduce(p, partial, f, out, st);
    if (e != hipSuccess) return device_error(fn, e);
  }
  return ok();
}

}  // namespace

extern "C" {

int nx_version(void) { return 100; }

const char* nx_last_error(void) { return g_last_error.c_str(); }

size_t nx_workspace_bytes(int64_t n_atoms, int64_t n_points, int mode, int op, int f_is_null) {
  if (check_counts("nx_workspace_bytes", n_atoms, n_points) != NX_OK) return 0;
  if (op < NX_OP_FWD || op > NX_OP_LOSS) {
    fail(NX_ERR_MODE, "nx_workspace_bytes: unknown op %d", op);
    return 0;
  }
  if ((op == NX_OP_FWD || op == NX_OP_BWD) && mode != NX_F32 && mode != NX_F32_PH64) {
    fail(NX_ERR_MODE, "nx_workspace_bytes: unknown mode %d", mode);
    return 0;
  }
  ok();
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
  return run_sum(fn, p, true, xyz, f, S, nullptr, A, ws, static_cast<hipStream_t>(stream));
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
  return run_sum(fn, p, false, xyz, f, S, G, grad_xyz, ws, static_cast<hipStream_t>(stream));
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
  return run_sum(fn, p, true, xyz, f, S, nullptr, A, ws, static_cast<hipStream_t>(stream));
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
  return run_sum(fn, p, false, xyz, f, S, G, grad_xyz, ws, static_cast<hipStream_t>(stream));
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

}  // extern "C"
