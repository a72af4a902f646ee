"""Benchmark: one fitting step of the direct scattering sum on one MI355X.

A step is the whole hot path on one batch of synthetic input resident in HBM:
the forward sum A_k = sum_j f_j exp(2 i pi S_k . r_j) (FP64 phase reduction,
compensated FP32 sums), the intensity misfit L = sum (|A|^2 - I)^2 with its seed
G = 4 (|A|^2 - I) A, and the adjoint dL/dr_j -- all in libnx's HIP kernels.

Headline workload (default): the strained Ge-like truncated-pyramid dot on an fcc
lattice, 203,557 atoms with two complex scattering factors, on a 128^3 grid of points
around (4,0,4) (2,097,152 points); the target intensity is that of the same dot with
the strain scaled by 1.1, computed once before timing.  The grid goes to the grid entry
points exactly (FP64 origin and steps; nx_fit_step_grid, whose kernels walk it by rows);
the same step through the point-list entry points (the points rounded to FP32) is timed
beside it ("list_path"), and --points list makes that the timed step.  The largest configuration,
the 4,013,800-atom nanowire on 256^3 points (39 s per step), is measured in the same
run as one timed step (the "c5" object of the line): the requested number of timed
steps of it would not fit the run's time limit.

Printed: one JSON line with the throughput in atom.point pairs per second of the
whole step (N*K pairs per step), the forward-only and adjoint-only rates, the
all-FP64 GPU path on the same step for comparison, the roofline of the dominant
kernel (timed live with events on the launch stream): the paper's count of 8 flop per
pair against the FP32 peak, and beside it the VALU issue slots of the kernel's own
instruction mix against the ceiling a register-only microbenchmark of that mix
reaches in the same run; and the FP64 CPU oracle timed on a bounded sample of the
same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 3.93e13 full-rate VALU lane-ops/s
# (nominal VALU issue slots; the library is compiled without packed FP32 instructions).
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9

# Minimal VALU instruction count per (atom, point) pair of each kernel: the method's
# own work on gfx950 in the formulation the kernels use (compensation, loads and loop
# control excluded).  Phase S.r = 3 FP64 fma, with the records' shift of 1.5 * 2^20 cycles
# in the addend; reduction mod 1 = the low word of the phase read as a fixed-point turn:
# integer to FP32 conversion and scaling by 2^-32 = 2.  sin and cos count one issue slot
# each (at half rate they keep the VALU busy longer; the microbenchmark ceiling of the
# same mix prices that in).
#   forward, complex f: f in polar form m exp(2 i pi a), a the addend of the phase's first
#                       fma; m (cos + i sin) accumulated with 2 fma
#   forward, f = 1:     (cos, sin) accumulated with 2 add
#   adjoint, complex f: f in polar form, its angle added to the phase (1 FP64 add), then
#                       only sin is needed and T_d += (|G| S_d) sin (3); |f| scales the
#                       finished sums; the seed phase rides in the first fma of the phase
#   adjoint, f = 1:     only sin is needed, T_d += (3)
# The FP32 mode (the paper's arithmetic): FP32 phase (3), v_fract_f32 (1), sin and cos (2);
#   forward: f (cos + i sin) with 4 fma, or 2 add for f = 1;
#   adjoint: w = conj(G) exp(i theta) (2 for Im w, 4 with Re w), v = Im(f w) (2 for complex
#            f), T_d += S_d v (3); sin and cos are both needed.
# libnx_micro's kernels run exactly these sequences (tests/test_device_code.py counts them).
ALG_SLOTS = {
    ("ph64", "fwd", "complex"): 3 + 2 + 2 + 2,
    ("ph64", "fwd", "unit"): 3 + 2 + 2 + 2,
    ("ph64", "bwd", "complex"): 3 + 1 + 2 + 1 + 3,
    ("ph64", "bwd", "unit"): 3 + 2 + 1 + 3,
    ("f32", "fwd", "complex"): 3 + 1 + 2 + 4,
    ("f32", "fwd", "unit"): 3 + 1 + 2 + 2,
    ("f32", "bwd", "complex"): 3 + 1 + 2 + 4 + 2 + 3,
    ("f32", "bwd", "unit"): 3 + 1 + 2 + 2 + 3,
    # grids walked by rows (FP64-phase mode), per pair on average:
    #   forward, a 2 x 2 x 2 block of points per lane: per atom the first point's phase
    #     fma(i1, step1.r, b) (b the atom's row term, formed once per atom and row), the
    #     fixed-point turn (2), cos and sin; the seven other points' phase factors stepped
    #     from it (7 steps of 4 fma); the eight terms accumulated (2 each): 49 per 8 pairs
    #   adjoint, 64-point groups, the phase factor stepped along the row: per atom and group
    #     the first point's factor (3 FP64 fma, 2, cos, sin) and the three S0 a0 + e1 a1 (2
    #     each); per pair v = Im(conj(G) E) (2), a0 and a1 (2) and the step (4, none after
    #     the group's last point): (7 + 6 + 64 * 4 + 63 * 4) / 64 per pair
    ("grid", "fwd", "complex"): 49 / 8,
    ("grid", "fwd", "unit"): 49 / 8,
    ("grid", "bwd", "complex"): (7 + 6 + 64 * 4 + 63 * 4) / 64,
    ("grid", "bwd", "unit"): (7 + 6 + 64 * 4 + 63 * 4) / 64,
}
# The paper's count of the work per pair (Eq. 3, Section 2.2: 3 mul, 4 add, 1 sincos) and
# the published FP32 vector peak of the MI355X: the roofline's flop fraction.
PAPER_FLOP_PER_PAIR = 8
FP32_PEAK_TFLOPS = 157.3

KERNEL_SOURCES = ["nx_fwd.hip", "nx_bwd.hip", "nx_loss.hip", "nx_species.hip", "nx_api.cpp",
                  "nx_internal.h"]

WORKLOADS = {
    "c1": "16^3 simple-cubic block, disorder 0.02, f=1, 64x64 map at l=4",
    "c2": "Ge-like strained fcc truncated-pyramid dot, 203,557 atoms, 2 species "
          "complex f, 128^3 grid around (4,0,4), fit step vs strain x1.1 target",
    "c3": "100^3 simple-cubic crystal, disorder 0.01, 256^2 map near (8,8,8)",
    "c4": "29^3-cell fcc cube, sinusoidal displacement, 64^3 grid around (2,2,0)",
    "c5": "strained fcc nanowire, 4,013,800 atoms, 2 species, 256^3 grid at (0,0,4), "
          "fit step vs strain x1.1 target",
    "ewald": "the c2 dot on 2,097,152 area-detector points on Ewald's sphere "
             "(128^2 pixels x 128 rocking frames around (4,0,4)), fit step vs strain "
             "x1.1 target",
    "cube41": "Section 4.1 cube, 1e6 atoms, 200x200 map around (004)",
    "cube41s": "Section 4.1 strained cube, 1e6 atoms, 200x200 map around (004)",
}

# grid edge of the workloads whose points are a regular grid (h fastest): the oracle
# sample always takes the grid lines through the map centre, where the strongest
# intensity lies
GRID_EDGE = {"c1": (64, 2), "c2": (128, 3), "c3": (256, 2), "c4": (64, 3), "c5": (256, 3)}


def _code_only(text: str) -> str:
    """C/C++ source without comments and blank lines (string literals in these sources
    hold no comment markers), so that editing a comment keeps the hash."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def source_hash() -> str:
    """Hash of the library's kernel and launch sources (code only): the traffic and
    counter summaries under profiles/ are used only while it matches theirs."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1010_2641_amd", "csrc", name)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="c2",
                   choices=["c1", "c2", "c3", "c4", "c5", "ewald", "cube41", "cube41s"])
    p.add_argument("--mode", default="ph64", choices=["ph64", "f32"])
    p.add_argument("--points", default="grid", choices=["grid", "list"],
                   help="grid: a workload whose points are a regular grid passes that grid exactly "
                        "(FP64 origin and steps) to the grid entry points, which walk it by rows "
                        "(FP64-phase mode); list: its points rounded to FP32 go to the point-list "
                        "entry points (the default for unstructured points and the FP32 mode)")
    p.add_argument("--no-f64", action="store_true", help="skip the all-FP64 comparison")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--graph", action="store_true",
                   help="also capture the fit step in one HIP graph and time its replays (reported "
                        "beside the eager rate, which stays the headline value)")
    p.add_argument("--no-species", action="store_true",
                   help="skip the species-factorised step (workloads with several species)")
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="approximate CPU time budget of the oracle sample")
    p.add_argument("--no-c5", action="store_true",
                   help="skip the one-step measurement of the largest configuration (c5) that "
                        "the headline line carries beside the default workload")
    p.add_argument("--staged", action="store_true",
                   help="time the steps as three calls (forward, misfit, adjoint) instead of one "
                        "nx_fit_step call (for one long step: the three calls also give the sums' "
                        "own times, so the step is not run twice)")
    p.add_argument("--no-list", action="store_true",
                   help="skip the point-list step timed beside a grid step (list_path)")
    p.add_argument("--no-micro", action="store_true",
                   help="skip the issue-ceiling microbenchmarks (the valu_issue fields)")
    p.add_argument("--copy-cal", type=int, default=0, metavar="BYTES",
                   help="only run a plain copy kernel over BYTES bytes (read once, written once) three times "
                        "(the reference kernel that scales the HBM counters of a profile)")
    return p.parse_args()


def progress(msg):
    """One line per finished phase on stderr (stdout carries only the JSON result)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def make_target(w, fwd):
    """|A|^2 of the workload's target structure (fwd: the forward of the points in use)."""
    import torch
    if w.target_xyz is not None:
        tx = torch.from_numpy(w.target_xyz).cuda()
    else:                       # workloads without a target structure: a shifted copy
        tx = torch.from_numpy(w.xyz).cuda() * 1.001
    I = (fwd(tx).abs() ** 2).float()
    del tx
    return I


def central_lines(name, n_points):
    """Indices of the grid lines through the map centre (empty for unstructured points)."""
    import numpy as np
    if name not in GRID_EDGE:
        return np.zeros(0, dtype=np.int64)
    n, dims = GRID_EDGE[name]
    c = n // 2
    idx = [h + n * c + (n * n * c if dims == 3 else 0) for h in range(n)]
    idx += [c + n * k + (n * n * c if dims == 3 else 0) for k in range(n)]
    if dims == 3:
        idx += [c + n * c + n * n * l for l in range(n)]
    idx = np.unique(np.array(idx, dtype=np.int64))
    assert idx.max() < n_points
    return idx


def cpu_baseline(name, w, A_gpu, G, g_gpu, budget_s, S_eval=None):
    """The FP64 oracle on a bounded sample of the same workload: the forward on the grid
    lines through the map centre and then seeded random points (all atoms), for half the
    budget, and the adjoint on seeded random atoms (all points) fed the step's own seed G,
    for the other half; the full-step time is extrapolated linearly.  Also returns the
    GPU's errors against the oracle on the sampled outputs (A_gpu: the step's amplitudes,
    g_gpu: its gradient, both numpy).  S_eval: the points the GPU evaluated ((K, 3); the
    FP64 grid points for the grid entry points), by default the FP32 list w.S."""
    import numpy as np

    import oracle

    S_all = w.S if S_eval is None else S_eval

    cores = oracle.threads()
    rng = np.random.default_rng(2024)
    lines = central_lines(name, w.n_points)
    rest = rng.permutation(np.setdiff1d(np.arange(w.n_points), lines))
    # grid-line and random points alternate, so that any cut of the budget holds both
    nl = min(len(lines), len(rest))
    mixed = np.empty(2 * nl, dtype=np.int64)
    mixed[0::2], mixed[1::2] = lines[:nl], rest[:nl]
    order_p = np.concatenate([mixed, lines[nl:], rest[nl:]])
    order_a = rng.permutation(w.n_atoms)
    bp = max(1, min(w.n_points, int(2e8 // max(w.n_atoms, 1))))
    ba = max(1, min(w.n_atoms, int(2e8 // max(w.n_points, 1))))
    A_parts, n_pts, t_fwd = [], 0, 0.0
    while n_pts < w.n_points and t_fwd < 0.5 * budget_s:
        idx = order_p[n_pts:n_pts + bp]
        t0 = time.perf_counter()
        A_parts.append(oracle.forward(w.xyz, w.f, S_all[idx]))
        t_fwd += time.perf_counter() - t0
        n_pts += len(idx)
    g_parts, n_at, t_bwd = [], 0, 0.0
    while n_at < w.n_atoms and t_bwd < 0.5 * budget_s:
        idx = order_a[n_at:n_at + ba]
        t0 = time.perf_counter()
        g_parts.append(oracle.adjoint(w.xyz[idx], None if w.f is None else w.f[idx], S_all, G))
        t_bwd += time.perf_counter() - t0
        n_at += len(idx)
    pts = order_p[:n_pts]
    atoms = order_a[:n_at]
    A_ref = np.concatenate(A_parts)
    g_ref = np.concatenate(g_parts)
    t_full = t_fwd * w.n_points / n_pts + t_bwd * w.n_atoms / n_at
    pairs = float(w.n_atoms) * float(w.n_points)
    A_s = A_gpu[pts].astype(np.complex128)
    I, Ir = np.abs(A_s) ** 2, np.abs(A_ref) ** 2
    # T1's floor is 1e-6 of the map's strongest intensity, taken from the step's own
    # amplitudes over every point (a threshold: the FP64-phase error does not move it);
    # the sample alone may miss the strongest point (the Ewald scan's sample has no grid
    # line through the reflection), which would admit points a thousand times weaker
    Imax = max(float(Ir.max()), float(np.max(np.abs(A_gpu.astype(np.complex128)) ** 2)))
    m = Ir >= 1e-6 * Imax
    g_s = g_gpu[atoms].astype(np.float64)
    err = {
        "fwd_T1_rel_I": float(np.max(np.abs(I[m] - Ir[m]) / Ir[m])),
        "fwd_T2_rel_norm": float(np.linalg.norm(A_s - A_ref) / np.linalg.norm(A_ref)),
        "bwd_T3_rel_norm": float(np.linalg.norm(g_s - g_ref) / np.linalg.norm(g_ref)),
        "bwd_T3_rel_max": float(np.max(np.abs(g_s - g_ref)) / np.max(np.abs(g_ref))),
        "tolerances": {"T1": 1e-5, "T2": 1e-6, "T3_norm": 1e-5, "T3_max": 1e-4},
        "sample": f"{int(np.isin(pts, lines).sum())} grid-line and {int((~np.isin(pts, lines)).sum())} "
                  f"random points (forward) and {n_at} random atoms with the step's own seed G "
                  f"(adjoint)",
    }
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    base = {
        "value": pairs / t_full,
        "unit": "atom.point pairs/s",
        "cores": cores,
        "cpu_model": cpu_model,
        "affinity_cpus": len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": (f"FP64 oracle forward on {n_pts} of {w.n_points} points (all atoms, "
                   f"{t_fwd:.1f} s) and adjoint on {n_at} of {w.n_atoms} atoms (all points, "
                   f"{t_bwd:.1f} s); full fit-step time extrapolated linearly to "
                   f"{t_full:.3g} s"),
    }
    return base, err


def saved_counters(name, dom, mode):
    """Traffic (HBM bytes per call) and VALU counters of profiles/ for this kernel and
    workload, used only while the kernel sources match the hash they were taken with."""
    traffic = valu = None
    tpath = os.path.join(ROOT, "profiles", f"{dom}_{name}_{mode}_traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as fh:
            tr = json.load(fh)
        if tr.get("source_sha") == source_hash():
            traffic = tr.get("hbm_bytes_per_launch")
    vpath = os.path.join(ROOT, "profiles", f"{dom}_{name}_{mode}_valu.json")
    if os.path.exists(vpath):
        with open(vpath) as fh:
            vr = json.load(fh)
        if vr.get("source_sha") == source_hash():
            valu = {k: vr[k] for k in ("valu_issue_util", "valu_busy", "valu_insts_per_pair",
                                       "trans_insts_per_pair", "clock_ghz") if k in vr}
    return traffic, valu


def kernel_roofline(name, mode, fkind, pairs, t_fwd, t_bwd, ceilings):
    """Roofline of the dominant kernel (the longer of the two sums): the paper's 8 flop
    per pair (Eq. 3) against the published FP32 peak, and a separate VALU issue-slot
    fraction against the measured ceiling of the kernel's own instruction mix.  Both
    sums' figures are listed under "sums".  mode: "ph64", "f32" or "grid" (the FP64-phase
    sums over grid rows)."""
    sums = {}
    for dom, t in (("fwd", t_fwd), ("bwd", t_bwd)):
        slots = ALG_SLOTS[(mode, dom, fkind)]
        rate = pairs / t
        ceil, ceil_ghz = ceilings.get((mode, dom, fkind), (None, None)) if ceilings else (None, None)
        sums[dom] = {
            "launch_ms": t * 1e3,
            "pairs_per_s": rate,
            "paper_tflops": PAPER_FLOP_PER_PAIR * rate / 1e12,
            "paper_flop_frac": PAPER_FLOP_PER_PAIR * rate / 1e12 / FP32_PEAK_TFLOPS,
            "valu_issue": {
                "unit": "VALU issue slots/s",
                "alg_slots_per_pair": slots,
                "achieved": slots * rate,
                "ceiling": None if ceil is None else slots * ceil,
                "ceiling_pairs_per_s": ceil,
                "ceiling_clock_ghz": ceil_ghz,
                "frac": None if ceil is None else rate / ceil,
                "nominal": VALU_SLOTS_PER_S,
                "frac_of_nominal": slots * rate / VALU_SLOTS_PER_S,
            },
        }
    for dom in ("fwd", "bwd"):
        # per cycle: the sum's clock under load from its committed counters (GRBM_GUI_ACTIVE
        # over the kernel time), the ceiling's from the microbenchmark's own clock reading
        _, v = saved_counters(name, dom, mode)
        vi = sums[dom]["valu_issue"]
        vi["kernel_clock_ghz"] = v.get("clock_ghz") if v else None
        vi["frac_per_cycle"] = (vi["frac"] * vi["ceiling_clock_ghz"] / vi["kernel_clock_ghz"]
                                if vi["frac"] and vi["ceiling_clock_ghz"] and vi["kernel_clock_ghz"]
                                else None)
    dom = "bwd" if t_bwd >= t_fwd else "fwd"
    d = sums[dom]
    traffic, valu = saved_counters(name, dom, mode)
    return {"bound": "alu", "achieved": d["paper_tflops"], "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": d["paper_flop_frac"], "traffic": traffic,
            "kernel": (f"nx_scatter_{dom}_grid (ph64, {fkind} f, rows of the grid)" if mode == "grid"
                       else f"nx_scatter_{dom} ({mode}, {fkind} f)"),
            "launch": "one entry-point call (all of its dispatches and launch chunks)",
            "flop_per_pair": PAPER_FLOP_PER_PAIR,
            "flop_convention": "the paper's count per atom-point pair (Eq. 3, Section 2.2: "
                               "3 mul, 4 add, 1 sincos) against the published FP32 vector peak",
            "launch_ms": d["launch_ms"], "valu_issue": d["valu_issue"], "counters": valu,
            "sums": sums}


def issue_ceilings(mode, fkind):
    """(pairs per second, clock in GHz under that load) of the forward's and the adjoint's
    instruction mixes on register operands (libnx_micro), measured now on this GPU."""
    from paper_1010_2641_amd import micro
    return {(mode, dom, fkind): micro.mix_rate(mode, dom, fkind) for dom in ("fwd", "bwd")}


def op_costs():
    """Cycles per wave64 instruction of the instruction kinds of the sums' loops, each
    issued alone (FP32 fma in the three-operand form with a scalar or vector operands and
    in the two-operand accumulating form, FP32 mul and add, FP64 fma in both forms, FP64
    add, rint and fract, the integer-to-FP32 conversion, v_sin_f32, v_cos_f32), from their
    measured rate and the clock the same kernels read."""
    from paper_1010_2641_amd import micro
    out = {}
    for kind in ("fma_f32", "fma_f32_v", "fmac_f32", "mul_f32", "add_f32", "fma_f64", "fmac_f64",
                 "add_f64", "rndne_f64", "fract_f64", "cvt_f32_i32", "sin_f32", "cos_f32"):
        rate, ghz = micro.op_rate(kind)
        out[kind] = {"insts_per_s_per_simd": rate, "clock_ghz": ghz,
                     "cycles_per_inst": None if ghz is None else ghz * 1e9 / rate}
    return out


def f64_path(api, tx, tf, tS, G, n, k, pairs, stream):
    """The all-FP64 GPU path on the same step (forward + adjoint, seed from the step);
    very large steps time it on the first 1/16 of the points (its rate does not depend on
    which points it is given)."""
    import torch
    ev = lambda: torch.cuda.Event(enable_timing=True)
    k64 = k if pairs <= 2e12 else max(1, k // 16)
    x64, S64 = tx.double(), tS[:k64].double().contiguous()
    f64_ = None if tf is None else tf.to(torch.complex128)
    G64 = G[:k64].to(torch.complex128).contiguous()
    pairs64 = float(n) * float(k64)
    if k64 == k:
        api.scatter_fwd_f64(x64, f64_, S64)
        torch.cuda.synchronize()
    e = [ev() for _ in range(3)]
    e[0].record(stream)
    api.scatter_fwd_f64(x64, f64_, S64)
    e[1].record(stream)
    api.scatter_bwd_f64(x64, f64_, S64, G64)
    e[2].record(stream)
    torch.cuda.synchronize()
    tf64, tb64 = e[0].elapsed_time(e[1]) / 1e3, e[1].elapsed_time(e[2]) / 1e3
    return {"fwd_pairs_per_s": pairs64 / tf64, "bwd_pairs_per_s": pairs64 / tb64,
            "step_pairs_per_s": pairs64 / (tf64 + tb64), "points_timed": k64}


def uses_grid(args, w) -> bool:
    """Whether the workload's points go to the grid entry points (see --points)."""
    return args.points == "grid" and args.mode == "ph64" and w.grid is not None


def list_path(api, tx, tf, tS, I, mode, pairs, stream, reps=3):
    """The same step through the point-list entry points (the grid's points rounded to
    FP32): one warm-up, then `reps` steps as three calls with events between them."""
    import torch
    ev = lambda: torch.cuda.Event(enable_timing=True)
    recs = [[ev() for _ in range(4)] for _ in range(reps + 1)]
    for r in recs:
        r[0].record(stream)
        A = api.scatter_fwd(tx, tf, tS, mode)
        r[1].record(stream)
        _, G = api.loss_grad(A, I)
        r[2].record(stream)
        api.scatter_bwd(tx, tf, tS, G, mode)
        r[3].record(stream)
    torch.cuda.synchronize()
    t = [sum(r[a].elapsed_time(r[b]) for r in recs[1:]) / reps / 1e3 for a, b in ((0, 1), (2, 3), (0, 3))]
    return {"entry_points": "nx_scatter_fwd, nx_loss_grad, nx_scatter_bwd (FP32 point list)",
            "fwd_pairs_per_s": pairs / t[0], "bwd_pairs_per_s": pairs / t[1],
            "step_pairs_per_s": pairs / t[2], "ms_per_step": t[2] * 1e3, "steps": reps}


def measure(name, args, steps, warmup, ceilings, want_graph=False, want_species=True,
            cpu_seconds=None, staged_only=False, want_list=False):
    """Times `steps` fit steps of workload `name` after `warmup` untimed ones and returns
    the measured fields (rates, roofline, FP64 path, species path, oracle baseline).  The
    timed steps are one library call each (nx_fit_step, or nx_fit_step_grid for a grid);
    the same steps as three calls with events between them give the forward's and the
    adjoint's own times."""
    import numpy as np
    import torch

    from paper_1010_2641_amd import api, workloads as wl

    dev = torch.device("cuda:0")
    w = wl.named(name)
    n, k = w.n_atoms, w.n_points
    pairs = float(n) * float(k)
    fkind = "unit" if w.f is None else "complex"
    grid = w.grid if uses_grid(args, w) else None
    kind = "grid" if grid is not None else args.mode       # the sums' instruction mix
    tx = torch.from_numpy(w.xyz).to(dev)
    tf = None if w.f is None else torch.from_numpy(w.f).to(dev)
    tS = torch.from_numpy(w.S).to(dev)
    if grid is not None:
        fwd = lambda x: api.scatter_fwd_grid(x, tf, grid)
        bwd = lambda G: api.scatter_bwd_grid(tx, tf, grid, G)
        fit = lambda: api.fit_step_grid(tx, tf, grid, I, return_seed=True)
    else:
        fwd = lambda x: api.scatter_fwd(x, tf, tS, args.mode)
        bwd = lambda G: api.scatter_bwd(tx, tf, tS, G, args.mode)
        fit = lambda: api.fit_step(tx, tf, tS, I, args.mode, return_seed=True)
    I = make_target(w, fwd)
    torch.cuda.synchronize()
    progress(f"workload {name}: {n} atoms x {k} points ({'exact grid' if grid else 'point list'}), "
             "target intensity ready")

    stream = torch.cuda.current_stream(dev)      # every libnx launch goes to this stream
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step():
        """The whole step, queued by one call into the library (nx_fit_step[_grid])."""
        L, A, g, G = fit()
        return L, A, g, G

    def staged(rec):
        """The same step as three calls with events between them: the time of each sum."""
        rec[0].record(stream)
        A = fwd(tx)
        rec[1].record(stream)
        L, G = api.loss_grad(A, I)
        rec[2].record(stream)
        g = bwd(G)
        rec[3].record(stream)
        return L, A, g, G

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    progress(f"{name}: {warmup} warm-up steps done")

    if staged_only:
        # long steps (seconds): the timed steps are the three calls themselves, which also
        # give the sums' own times (the host's launch overhead is nothing against them)
        recs = [[ev() for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            out = staged(recs[i])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n_staged = steps
        progress(f"{name}: {steps} timed steps done (three calls), {wall / steps * 1e3:.1f} ms per step")
    else:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            out = step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        progress(f"{name}: {steps} timed steps done, {wall / steps * 1e3:.1f} ms per step")
        # the sums' own times: the step again as three calls, events on the launch stream
        n_staged = steps
        recs = [[ev() for _ in range(4)] for _ in range(n_staged)]
        for i in range(n_staged):
            staged_out = staged(recs[i])
        torch.cuda.synchronize()
        assert torch.equal(staged_out[1], out[1]) and torch.equal(staged_out[2], out[2]), \
            "the one-call step and the three calls must agree bitwise"
        del staged_out
        progress(f"{name}: {n_staged} staged steps timed")

    # the same step captured once in a HIP graph (the library issues kernels only: no
    # allocation, copy, memset or synchronisation), replayed for at least the timed steps
    # and at least 0.2 s; small problems are bound by launch latency, which replays cut
    graph = None
    if want_graph:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        cg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cg):
            _, gA, gg, _ = step()
        torch.cuda.synchronize()
        reps = max(steps, int(0.2 / max(wall / steps, 1e-9)) + 1)
        cg.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            cg.replay()
        torch.cuda.synchronize()
        tg = (time.perf_counter() - t0) / reps
        graph = {"ms_per_step": tg * 1e3, "pairs_per_s": pairs / tg, "replays": reps,
                 "bitwise_equal_to_eager": bool(torch.equal(gA, out[1]) and torch.equal(gg, out[2]))}
        del cg, gA, gg
        # each sum on its own, captured and replayed (the GPU time of one call without the
        # host's launch overhead, which dominates eager calls of small problems)
        G0 = out[3]
        for dom, fn in (("fwd", lambda: fwd(tx)), ("bwd", lambda: bwd(G0))):
            with torch.cuda.stream(side):
                fn()
            stream.wait_stream(side)
            torch.cuda.synchronize()
            cs = torch.cuda.CUDAGraph()
            with torch.cuda.graph(cs):
                fn()
            cs.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                cs.replay()
            torch.cuda.synchronize()
            graph[f"{dom}_pairs_per_s"] = pairs / ((time.perf_counter() - t0) / reps)
            del cs
        progress(f"{name}: graph replays timed: {tg * 1e3:.3f} ms per step")
    t_fwd = sum(r[0].elapsed_time(r[1]) for r in recs) / len(recs) / 1e3
    t_loss = sum(r[1].elapsed_time(r[2]) for r in recs) / len(recs) / 1e3
    t_bwd = sum(r[2].elapsed_time(r[3]) for r in recs) / len(recs) / 1e3
    res = {
        "config": {"workload": WORKLOADS[name], "n_atoms": n, "n_points": k, "pairs_per_step": pairs,
                   "points": ("the workload's grid given exactly (FP64 origin and steps), nx_fit_step_grid"
                              if grid is not None else "point list (FP32), nx_fit_step"),
                   "precision": {"ph64": "FP64 phase reduction, FP32 sin/cos, compensated FP32 sums",
                                 "f32": "plain FP32 (the paper's arithmetic)"}[args.mode]},
        "steps": steps, "warmup": warmup, "staged_steps": n_staged,
        "ms_per_step": wall / steps * 1e3,
        "value": pairs / (wall / steps),
        "fwd_pairs_per_s": pairs / t_fwd,
        "bwd_pairs_per_s": pairs / t_bwd,
        "loss_ms": t_loss * 1e3,
        "graph_replay": graph,
        "roofline": kernel_roofline(name, kind, fkind, pairs, t_fwd, t_bwd, ceilings),
    }

    L, A, g, G = out
    S_eval = grid.points() if grid is not None else None       # the FP64 grid points
    if want_list and grid is not None:
        res["list_path"] = list_path(api, tx, tf, tS, I, args.mode, pairs, stream)
        progress(f"{name}: the point-list step timed")
    if not args.no_f64:
        tS64 = torch.from_numpy(S_eval).to(dev) if grid is not None else tS
        res["f64_path"] = f64_path(api, tx, tf, tS64, G, n, k, pairs, stream)
        del tS64
        res["speedup_vs_f64_step"] = res["value"] / res["f64_path"]["step_pairs_per_s"]
        progress(f"{name}: all-FP64 path timed on {res['f64_path']['points_timed']} points")

    # the same step with the species factored out of the sum (Section 4.2): one
    # unit-factor sum per species, atoms regrouped by species once, outside the timing;
    # over the grid when the step takes it
    if want_species and w.f is not None:
        xs, start, vals, _ = wl.group_by_species(w.xyz, w.f)
        if len(vals) <= 16:
            txs = torch.from_numpy(xs).to(dev)
            fs = torch.from_numpy(np.repeat(vals[:, None], k, axis=1)).to(dev)

            def sstep(rec):
                rec[0].record(stream)
                if grid is not None:
                    As = api.scatter_fwd_species_grid(txs, start, fs, grid)
                else:
                    As = api.scatter_fwd_species(txs, start, fs, tS, args.mode)
                rec[1].record(stream)
                _, Gs = api.loss_grad(As, I)
                rec[2].record(stream)
                if grid is not None:
                    api.scatter_bwd_species_grid(txs, start, fs, grid, Gs)
                else:
                    api.scatter_bwd_species(txs, start, fs, tS, Gs, None, args.mode)
                rec[3].record(stream)
                return As

            sstep([ev() for _ in range(4)])
            srecs = [[ev() for _ in range(4)] for _ in range(max(1, min(steps, 3)))]
            torch.cuda.synchronize()
            for r in srecs:
                A_sp = sstep(r)
            torch.cuda.synchronize()
            ts = [sum(r[a].elapsed_time(r[b]) for r in srecs) / len(srecs) / 1e3
                  for a, b in ((0, 1), (2, 3), (0, 3))]
            Ad = A.cpu().numpy().astype(np.complex128)
            As_ = A_sp.cpu().numpy().astype(np.complex128)
            progress(f"{name}: species-factorised step timed")
            res["species_path"] = {
                "n_species": len(vals),
                "entry_points": ("nx_scatter_fwd_species_grid, nx_loss_grad, nx_scatter_bwd_species_grid"
                                 if grid is not None else
                                 "nx_scatter_fwd_species, nx_loss_grad, nx_scatter_bwd_species"),
                "fwd_pairs_per_s": pairs / ts[0],
                "bwd_pairs_per_s": pairs / ts[1], "step_pairs_per_s": pairs / ts[2],
                "t2_vs_per_atom_step": float(np.linalg.norm(As_ - Ad) / np.linalg.norm(Ad))}
            del txs, fs

    if not args.no_cpu:
        A_np = A.cpu().numpy()
        G_np = G.cpu().numpy()
        g_np = g.cpu().numpy()
        res["cpu_baseline"], res["max_rel_err"] = cpu_baseline(
            name, w, A_np, G_np, g_np, cpu_seconds or args.cpu_seconds, S_eval)
        progress(f"{name}: CPU oracle baseline done")
    del tx, tf, tS, I, out, L, A, g, G
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(the sum would shard along the points with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_cal:
        src = torch.empty(args.copy_cal // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):     # an elementwise kernel (a device-to-device memcpy is no dispatch)
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_cal}), flush=True)
        return

    from paper_1010_2641_amd import workloads as wl  # noqa: F401  (fails loudly without libnx)

    torch.cuda.set_device(torch.device("cuda:0"))
    fkind_of = {"c1": "unit", "c3": "unit", "c4": "unit", "cube41": "unit", "cube41s": "unit"}
    ceilings, costs = {}, None
    if not args.no_micro:
        kinds = {args.mode}
        if args.mode == "ph64" and args.points == "grid":
            kinds.add("grid")           # the ceilings of the grid sums' own mixes too
        for kind in sorted(kinds):
            for fk in {fkind_of.get(args.workload, "complex"), "complex"}:
                ceilings.update(issue_ceilings(kind, fk))
        costs = op_costs()
        progress("issue-ceiling microbenchmarks done: " + ", ".join(
            f"{'/'.join(key)} {v[0]:.3e} pairs/s" for key, v in sorted(ceilings.items())))

    head = measure(args.workload, args, args.steps, args.warmup, ceilings, want_graph=args.graph,
                   want_species=not args.no_species, staged_only=args.staged, want_list=not args.no_list)
    c5 = None
    if args.workload == "c2" and not args.no_c5:
        # the largest configuration, one timed step (its 39 s per step would take the
        # requested timed steps past the run's time limit)
        c5 = measure("c5", args, 1, 0, ceilings, want_species=False,
                     cpu_seconds=2 * args.cpu_seconds, staged_only=True)
        progress("c5 leg done")

    config = dict(head["config"])
    if c5 is not None:
        config["headline_choice"] = ("the 203,557-atom dot: the timed steps of the largest "
                                     "configuration (4,013,800 atoms x 16,777,216 points, one "
                                     "step per 39 s) would not fit the run's time limit; that "
                                     "configuration is measured as one timed step in 'c5'")
    res = {
        "metric": "atom.point pairs/s of the fit step (forward + misfit + adjoint)",
        "value": head["value"],
        "unit": "atom.point pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
    }
    for key in ("fwd_pairs_per_s", "bwd_pairs_per_s", "loss_ms", "list_path", "f64_path", "species_path",
                "graph_replay", "speedup_vs_f64_step", "max_rel_err", "roofline", "cpu_baseline"):
        res[key] = head.get(key)
    res["c5"] = c5
    res["valu_cycles_per_wave64_inst"] = costs
    res["source_sha"] = source_hash()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
