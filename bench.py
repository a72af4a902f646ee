"""Benchmark: one fitting step of the direct scattering sum on one MI355X.

A step is the whole hot path on one batch of synthetic input resident in HBM:
the forward sum A_k = sum_j f_j exp(2 i pi S_k . r_j) (FP64 phase reduction,
compensated FP32 sums), the intensity misfit L = sum (|A|^2 - I)^2 with its seed
G = 4 (|A|^2 - I) A, and the adjoint dL/dr_j -- all in libnx's HIP kernels.

Workload (default): the strained Ge-like truncated-pyramid dot on an fcc lattice,
203,557 atoms with two complex scattering factors, on a 128^3 grid of points around
(4,0,4) (2,097,152 points); the target intensity is that of the same dot with the
strain scaled by 1.1, computed once before timing.

Printed: one JSON line with the throughput in atom.point pairs per second of the
whole step (N*K pairs per step), the forward-only and adjoint-only rates, the
all-FP64 GPU path on the same step for comparison, the roofline of the dominant
kernel (timed live with events on the launch stream), and the FP64 CPU oracle timed
on a bounded sample of the same workload on this host's cores.
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

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 3.93e13 full-rate VALU lane-ops/s;
# counting each as one FMA (2 flop) gives 78.6 TFLOP/s (the unpacked FP32 and the
# FP64 vector rate; the library is compiled without packed FP32 instructions).
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
PEAK_TFLOPS = 2 * VALU_SLOTS_PER_S / 1e12

# Minimal VALU instruction count per (atom, point) pair of each kernel: the method's
# own work on gfx950 in the formulation the kernels use (compensation, loads and loop
# control excluded).  Phase S.r = 3 FP64 fma.  Forward: centred reduction mod 1 (rint,
# subtract) and rounding to FP32 = 3; adjoint: fract and rounding = 2.  sin and cos count
# one issue slot each, the strict bound: at half rate they keep the VALU busy for two
# slots, partly overlapped with other work (the VALU counters give ~1.75 slots each).
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
ALG_SLOTS = {
    ("ph64", "fwd", "complex"): 3 + 3 + 2 + 2,
    ("ph64", "fwd", "unit"): 3 + 3 + 2 + 2,
    ("ph64", "bwd", "complex"): 3 + 1 + 2 + 1 + 3,
    ("ph64", "bwd", "unit"): 3 + 2 + 1 + 3,
    ("f32", "fwd", "complex"): 3 + 1 + 2 + 4,
    ("f32", "fwd", "unit"): 3 + 1 + 2 + 2,
    ("f32", "bwd", "complex"): 3 + 1 + 2 + 4 + 2 + 3,
    ("f32", "bwd", "unit"): 3 + 1 + 2 + 2 + 3,
}
PAPER_FLOP_PER_PAIR = 8       # the paper's count (3 mul, 4 add, 1 sincos)
FP32_PEAK_TFLOPS = 157.3      # published FP32 vector peak (packed)

KERNEL_SOURCES = ["nx_fwd.hip", "nx_bwd.hip", "nx_loss.hip", "nx_species.hip", "nx_api.cpp",
                  "nx_internal.h"]


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
    p.add_argument("--no-f64", action="store_true", help="skip the all-FP64 comparison")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--graph", action="store_true",
                   help="also capture the fit step in one HIP graph and time its replays (reported "
                        "beside the eager rate, which stays the headline value)")
    p.add_argument("--no-species", action="store_true",
                   help="skip the species-factorised step (workloads with several species)")
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="approximate CPU time budget of the oracle sample")
    p.add_argument("--copy-cal", type=int, default=0, metavar="BYTES",
                   help="only run a plain device-to-device copy of BYTES bytes three times "
                        "(the reference kernel that scales the HBM counters of a profile)")
    return p.parse_args()


def progress(msg):
    """One line per finished phase on stderr (stdout carries only the JSON result)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def make_target(api, w, tf, tS, mode):
    import torch
    if w.target_xyz is not None:
        tx = torch.from_numpy(w.target_xyz).cuda()
    else:                       # workloads without a target structure: a shifted copy
        tx = torch.from_numpy(w.xyz).cuda() * 1.001
    return (api.scatter_fwd(tx, tf, tS, mode).abs() ** 2).float()


def cpu_baseline(w, A_gpu, g_gpu_fn, budget_s):
    """The FP64 oracle on a bounded sample of the same workload: the forward on a
    seeded sample of points (all atoms) and the adjoint on a seeded sample of atoms
    (all points); the full-step time is extrapolated linearly.  Also returns the GPU's
    error against the oracle on the sampled outputs."""
    import numpy as np

    import oracle
    from paper_1010_2641_amd import workloads as wl

    cores = oracle.threads()
    rng = np.random.default_rng(2024)
    # forward on seeded batches of points (all atoms) until half the budget is spent,
    # then the adjoint on seeded batches of atoms (all points) for the other half
    order_p = rng.permutation(w.n_points)
    order_a = rng.permutation(w.n_atoms)
    G = wl.random_seed_field(w.n_points, seed=2025, scale=1e-3)
    bp = max(1, min(w.n_points, int(2e8 // max(w.n_atoms, 1))))
    ba = max(1, min(w.n_atoms, int(2e8 // max(w.n_points, 1))))
    A_parts, n_pts, t_fwd = [], 0, 0.0
    while n_pts < w.n_points and t_fwd < 0.5 * budget_s:
        idx = order_p[n_pts:n_pts + bp]
        t0 = time.perf_counter()
        A_parts.append(oracle.forward(w.xyz, w.f, w.S[idx]))
        t_fwd += time.perf_counter() - t0
        n_pts += len(idx)
    g_parts, n_at, t_bwd = [], 0, 0.0
    while n_at < w.n_atoms and t_bwd < 0.5 * budget_s:
        idx = order_a[n_at:n_at + ba]
        t0 = time.perf_counter()
        g_parts.append(oracle.adjoint(w.xyz[idx], None if w.f is None else w.f[idx], w.S, G))
        t_bwd += time.perf_counter() - t0
        n_at += len(idx)
    pts = order_p[:n_pts]
    atoms = order_a[:n_at]
    A_ref = np.concatenate(A_parts)
    g_ref = np.concatenate(g_parts)
    t_full = t_fwd * w.n_points / n_pts + t_bwd * w.n_atoms / n_at
    pairs = float(w.n_atoms) * float(w.n_points)
    # GPU error on the same sampled outputs
    A_s = A_gpu[pts].astype(np.complex128)
    I, Ir = np.abs(A_s) ** 2, np.abs(A_ref) ** 2
    m = Ir >= 1e-6 * Ir.max()
    g_gpu = g_gpu_fn(G)[atoms]
    err = {
        "fwd_T1_rel_I": float(np.max(np.abs(I[m] - Ir[m]) / Ir[m])),
        "fwd_T2_rel_norm": float(np.linalg.norm(A_s - A_ref) / np.linalg.norm(A_ref)),
        "bwd_T3_rel_norm": float(np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)),
        "bwd_T3_rel_max": float(np.max(np.abs(g_gpu - g_ref)) / np.max(np.abs(g_ref))),
        "sample": f"{n_pts} random points (forward) and {n_at} random atoms with a seeded "
                  f"random seed G (adjoint)",
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(the sum would shard along the points with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1010_2641_amd import api, workloads as wl

    if args.copy_cal:
        src = torch.empty(args.copy_cal // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_cal}), flush=True)
        return

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = wl.named(args.workload)
    n, k = w.n_atoms, w.n_points
    pairs = float(n) * float(k)
    fkind = "unit" if w.f is None else "complex"
    tx = torch.from_numpy(w.xyz).to(dev)
    tf = None if w.f is None else torch.from_numpy(w.f).to(dev)
    tS = torch.from_numpy(w.S).to(dev)
    I = make_target(api, w, tf, tS, args.mode)
    torch.cuda.synchronize()
    progress(f"workload {args.workload}: {n} atoms x {k} points, target intensity ready")

    stream = torch.cuda.current_stream(dev)      # every libnx launch goes to this stream
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(rec=None):
        if rec is not None:
            rec[0].record(stream)
        A = api.scatter_fwd(tx, tf, tS, args.mode)
        if rec is not None:
            rec[1].record(stream)
        L, G = api.loss_grad(A, I)
        if rec is not None:
            rec[2].record(stream)
        g = api.scatter_bwd(tx, tf, tS, G, args.mode)
        if rec is not None:
            rec[3].record(stream)
        return L, A, g

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    progress(f"{args.warmup} warm-up steps done")

    recs = [[ev() for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step(recs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"{args.steps} timed steps done, {wall / args.steps * 1e3:.1f} ms per step")

    # the same step captured once in a HIP graph (the library issues kernels only: no
    # allocation, copy, memset or synchronisation), replayed for at least the timed steps
    # and at least 0.2 s; small problems are bound by launch latency, which replays cut
    graph = None
    if args.graph:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        cg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cg):
            _, gA, gg = step()
        torch.cuda.synchronize()
        reps = max(args.steps, int(0.2 / max(wall / args.steps, 1e-9)) + 1)
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
        progress(f"graph replays timed: {tg * 1e3:.3f} ms per step")
    t_fwd = sum(r[0].elapsed_time(r[1]) for r in recs) / args.steps / 1e3
    t_loss = sum(r[1].elapsed_time(r[2]) for r in recs) / args.steps / 1e3
    t_bwd = sum(r[2].elapsed_time(r[3]) for r in recs) / args.steps / 1e3
    ms_per_step = wall / args.steps * 1e3
    value = pairs / (wall / args.steps)

    # roofline of the dominant kernel (its launch sequence timed on the launch stream)
    dom, t_dom = ("bwd", t_bwd) if t_bwd >= t_fwd else ("fwd", t_fwd)
    slots = ALG_SLOTS[(args.mode, dom, fkind)]
    achieved = pairs * 2 * slots / t_dom / 1e12
    traffic = None
    tpath = os.path.join(ROOT, "profiles", f"{dom}_{args.workload}_{args.mode}_traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as fh:
            tr = json.load(fh)
        if tr.get("source_sha") == source_hash():
            traffic = tr.get("hbm_bytes_per_launch")
    valu = None
    vpath = os.path.join(ROOT, "profiles", f"{dom}_{args.workload}_{args.mode}_valu.json")
    if os.path.exists(vpath):
        with open(vpath) as fh:
            vr = json.load(fh)
        if vr.get("source_sha") == source_hash():
            valu = {k: vr[k] for k in ("valu_issue_util", "valu_busy", "valu_insts_per_pair",
                                       "trans_insts_per_pair", "clock_ghz") if k in vr}
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS, "traffic": traffic,
                "kernel": f"nx_scatter_{dom} ({args.mode}, {fkind} f)",
                "launch": "one entry-point call (all of its dispatches and launch chunks)",
                "alg_valu_slots_per_pair": slots, "launch_ms": t_dom * 1e3,
                "counters": valu}

    # all-FP64 GPU path on the same step (forward + adjoint, seed from this step)
    f64 = None
    if not args.no_f64:
        L, A, _ = out
        _, G = api.loss_grad(A, I)
        # very large steps: the FP64 path is timed on the first 1/16 of the points (its
        # rate does not depend on which points it is given)
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
        f64 = {"fwd_pairs_per_s": pairs64 / tf64, "bwd_pairs_per_s": pairs64 / tb64,
               "step_pairs_per_s": pairs64 / (tf64 + tb64), "points_timed": k64}
        del x64, S64, G64, f64_
        progress(f"all-FP64 path timed on {k64} points")

    # the same step with the species factored out of the sum (Section 4.2): one
    # unit-factor sum per species, atoms regrouped by species once, outside the timing
    species = None
    if not args.no_species and w.f is not None:
        xs, start, vals, _ = wl.group_by_species(w.xyz, w.f)
        if len(vals) <= 16:
            txs = torch.from_numpy(xs).to(dev)
            fs = torch.from_numpy(np.repeat(vals[:, None], k, axis=1)).to(dev)

            def sstep(rec):
                rec[0].record(stream)
                A = api.scatter_fwd_species(txs, start, fs, tS, args.mode)
                rec[1].record(stream)
                _, G = api.loss_grad(A, I)
                rec[2].record(stream)
                api.scatter_bwd_species(txs, start, fs, tS, G, None, args.mode)
                rec[3].record(stream)
                return A

            sstep([ev() for _ in range(4)])
            srecs = [[ev() for _ in range(4)] for _ in range(max(1, min(args.steps, 3)))]
            torch.cuda.synchronize()
            for r in srecs:
                A_sp = sstep(r)
            torch.cuda.synchronize()
            ts = [sum(r[a].elapsed_time(r[b]) for r in srecs) / len(srecs) / 1e3
                  for a, b in ((0, 1), (2, 3), (0, 3))]
            Ad = out[1].cpu().numpy().astype(np.complex128)
            As_ = A_sp.cpu().numpy().astype(np.complex128)
            progress("species-factorised step timed")
            species = {"n_species": len(vals), "fwd_pairs_per_s": pairs / ts[0],
                       "bwd_pairs_per_s": pairs / ts[1], "step_pairs_per_s": pairs / ts[2],
                       "t2_vs_per_atom_step": float(np.linalg.norm(As_ - Ad) / np.linalg.norm(Ad))}
            del txs, fs

    cpu = None
    errs = None
    if not args.no_cpu:
        A_np = out[1].cpu().numpy()

        def g_gpu_fn(G):
            return api.scatter_bwd(tx, tf, tS, torch.from_numpy(G).to(dev), args.mode).cpu().numpy()

        cpu, errs = cpu_baseline(w, A_np, g_gpu_fn, args.cpu_seconds)
        progress("CPU oracle baseline done")

    res = {
        "metric": "atom.point pairs/s of the fit step (forward + misfit + adjoint)",
        "value": value,
        "unit": "atom.point pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": {
                "c1": "16^3 simple-cubic block, disorder 0.02, f=1, 64x64 map at l=4",
                "c2": "Ge-like strained fcc truncated-pyramid dot, 203,557 atoms, 2 species "
                      "complex f, 128^3 grid around (4,0,4), fit step vs strain x1.1 target",
                "c3": "100^3 simple-cubic crystal, disorder 0.01, 256^2 map near (8,8,8)",
                "c4": "29^3-cell fcc cube, sinusoidal displacement, 64^3 grid around (2,2,0)",
                "c5": "strained fcc nanowire, 4,013,800 atoms, 2 species, 256^3 grid at (0,0,4)",
                "ewald": "the c2 dot on 2,097,152 area-detector points on Ewald's sphere "
                         "(128^2 pixels x 128 rocking frames around (4,0,4)), fit step vs strain "
                         "x1.1 target",
                "cube41": "Section 4.1 cube, 1e6 atoms, 200x200 map around (004)",
                "cube41s": "Section 4.1 strained cube, 1e6 atoms, 200x200 map around (004)",
            }[args.workload],
            "n_atoms": n, "n_points": k, "pairs_per_step": pairs,
            "precision": {"ph64": "FP64 phase reduction, FP32 sin/cos, compensated FP32 sums",
                          "f32": "plain FP32 (the paper's arithmetic)"}[args.mode],
        },
        "fwd_pairs_per_s": pairs / t_fwd,
        "bwd_pairs_per_s": pairs / t_bwd,
        "loss_ms": t_loss * 1e3,
        "f64_path": f64,
        "species_path": species,
        "graph_replay": graph,
        "speedup_vs_f64_step": (value / f64["step_pairs_per_s"]) if f64 else None,
        "max_rel_err": errs,
        "paper_flop_convention": {"tflops": value * PAPER_FLOP_PER_PAIR / 1e12,
                                  "frac_of_fp32_peak": value * PAPER_FLOP_PER_PAIR / 1e12 / FP32_PEAK_TFLOPS},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "source_sha": source_hash(),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
