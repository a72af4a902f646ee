"""Replays of the paper's own experiments on synthetic inputs, timed on the GPU.

    python -m paper_1010_2641_amd.replay fig1   [--max-pairs 1e12] [--out FILE]
    python -m paper_1010_2641_amd.replay cube   [--out FILE]
    python -m paper_1010_2641_amd.replay chain  [--out FILE]

* ``fig1``  -- Section 2.2 and Fig. 1: speed of the sum against the number of atoms and
  of points, for random atom positions and random points with f = 1, in both FP32 modes;
* ``cube``  -- Section 4.1: the 100^3 simple-cubic cube on the 200 x 200 map around
  (004), plain and strained (z += 1e-6 z (x^2 + y^2)), timed against the 0.93 s the paper
  quotes; the plain cube is checked against its closed form (a product of three
  geometric series);
* ``chain`` -- Section 2.3 and Fig. 2: the periodic chain of 1e3, 1e4 and 1e5 atoms against
  the analytic chain amplitude, and the reliable intensity range of each precision mode;
  the chain with Gaussian disorder 1e-3 gives the noise floor the paper compares with.

Every sum runs in libnx's kernels; the reference values here are the closed forms the
paper itself uses (computed in FP64 with numpy on the FP32-rounded inputs).  Output is a
markdown report (stdout, or --out).
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np
import torch

from . import api, workloads as wl


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(mode, x, f, S):
    if mode == "f64":
        return api.scatter_fwd_f64(x, f, S)
    return api.scatter_fwd(x, f, S, mode)


def time_forward(x, f, S, mode, min_seconds=0.2, max_reps=200):
    """Average time of one forward call (HIP events on the launch stream), after one
    untimed call; repeats until min_seconds of GPU time or max_reps calls."""
    _run(mode, x, f, S)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    total, reps = 0.0, 0
    while reps < max_reps and (total < min_seconds or reps < 3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _run(mode, x, f, S)
        e1.record(stream)
        e1.synchronize()
        total += e0.elapsed_time(e1) / 1e3
        reps += 1
    return total / reps


# ----------------------------------------------------------------------------- closed forms

def geometric_sum(s, start, n):
    """sum_{m=0}^{n-1} exp(2 i pi s (start + m)) in FP64, s reduced mod 1 first."""
    s = np.asarray(s, dtype=np.float64)
    t = s - np.rint(s)
    out = np.empty(t.shape, dtype=np.complex128)
    small = np.abs(t) < 1e-12
    out[small] = n
    ts = t[~small]
    out[~small] = (np.exp(2j * np.pi * ts * start) * (1 - np.exp(2j * np.pi * ts * n)) /
                   (1 - np.exp(2j * np.pi * ts)))
    return out


def laue_cube41(S):
    """Closed form of the Section 4.1 cube: x, y in [-50, 50), z in [0, 100)."""
    S = np.asarray(S, dtype=np.float64)
    return geometric_sum(S[:, 0], -50, 100) * geometric_sum(S[:, 1], -50, 100) * \
        geometric_sum(S[:, 2], 0, 100)


def chain_amplitude(h, n):
    """The paper's chain formula sin(pi N H) / sin(pi H), with the phase factor of atoms
    at 0..N-1 (the modulus is the paper's expression)."""
    return geometric_sum(h, 0, n)


def t1(A, A_ref, floor=1e-6):
    I, Ir = np.abs(A) ** 2, np.abs(A_ref) ** 2
    m = Ir >= floor * Ir.max()
    return float(np.max(np.abs(I[m] - Ir[m]) / Ir[m]))


def reliable_range(A, A_ref, rel=1e-2):
    """max I_ref over the largest I_ref at which the relative intensity error first
    exceeds rel, visiting the points from the strongest down (inf if never)."""
    I, Ir = np.abs(A) ** 2, np.abs(A_ref) ** 2
    order = np.argsort(-Ir)
    e = np.abs(I[order] - Ir[order]) / np.maximum(Ir[order], 1e-300)
    bad = np.nonzero(e > rel)[0]
    return np.inf if bad.size == 0 else float(Ir[order[0]] / max(Ir[order[bad[0]]], 1e-300))


# ----------------------------------------------------------------------------- experiments

def fig1(max_pairs=1e12, sizes=(100, 1000, 10_000, 100_000, 1_000_000, 10_000_000)):
    lines = ["## Fig. 1 replay: forward speed against atoms and points (random atoms in "
             "[0,100)^3, random S in [-4,4)^3, f = 1)", "",
             "atom.point pairs/s per call (HIP events, average of >= 3 calls and >= 0.2 s); "
             f"cases above {max_pairs:.0e} pairs are not run.", ""]
    for mode in ("ph64", "f32"):
        lines += [f"### mode {mode}", "",
                  "| atoms \\ points | " + " | ".join(f"{k:.0e}" for k in sizes) + " |",
                  "|---|" + "---:|" * len(sizes)]
        for n in sizes:
            row = []
            for k in sizes:
                if float(n) * k > max_pairs:
                    row.append("–")
                    continue
                xyz, _, S = wl.random_problem(n, k, seed=11, extent=100.0, s_range=4.0,
                                              complex_f=False)
                x, s = _dev(xyz), _dev(S)
                t = time_forward(x, None, s, mode)
                row.append(f"{float(n) * k / t:.2e}")
                del x, s
                print(f"fig1 mode={mode} N={n} K={k}: {row[-1]} pairs/s", flush=True)
            lines.append(f"| {n:.0e} | " + " | ".join(row) + " |")
        lines.append("")
    lines.append("The paper's card reached about 4.6e10 pairs/s once both counts exceed 1e4 "
                 "(Section 2.2); context only.")
    return "\n".join(lines) + "\n"


def cube():
    lines = ["## Section 4.1 replay: 100^3 simple-cubic cube, 200 x 200 map around (004)", "",
             "1e6 atoms x 40,000 points = 4e10 pairs per map.  The paper quotes 0.93 s on its "
             "card (context only).", "",
             "T1 is the largest relative intensity error over points with I >= floor * max I.", "",
             "| structure | mode | time per map (ms) | pairs/s | T1, floor 1e-6 | T1, floor 1e-4 | T2 |",
             "|---|---|---:|---:|---:|---:|---:|"]
    for strained in (False, True):
        w = wl.cube41(strained)
        x, S = _dev(w.xyz), _dev(w.S)
        x64, S64 = x.double(), S.double()
        ref = None if strained else laue_cube41(w.S)
        A64 = None
        for mode in ("ph64", "f32", "f64"):
            xx, ss = (x64, S64) if mode == "f64" else (x, S)
            t = time_forward(xx, None, ss, mode)
            A = _run(mode, xx, None, ss).cpu().numpy().astype(np.complex128)
            if mode == "f64":
                A64 = A
            r = ref
            e1 = e1b = e2 = "–"
            if r is not None:
                e1, e1b = f"{t1(A, r):.2e}", f"{t1(A, r, 1e-4):.2e}"
                e2 = f"{np.linalg.norm(A - r) / np.linalg.norm(r):.2e}"
            lines.append(f"| {'strained' if strained else 'plain (vs closed form)'} | {mode} | "
                         f"{t * 1e3:.2f} | {4e10 / t:.2e} | {e1} | {e1b} | {e2} |")
            print(lines[-1], flush=True)
        if strained:
            Aph = _run("ph64", x, None, S).cpu().numpy().astype(np.complex128)
            lines.append(f"| strained (ph64 vs f64 path) | ph64 | | | {t1(Aph, A64):.2e} | "
                         f"{t1(Aph, A64, 1e-4):.2e} | "
                         f"{np.linalg.norm(Aph - A64) / np.linalg.norm(A64):.2e} |")
        del x, S, x64, S64
    return "\n".join(lines) + "\n"


def chain():
    lines = ["## Fig. 2 replay: periodic chains against sin(pi N H)/sin(pi H)", "",
             "Atoms at 0..N-1, H from 0 to 1 every 0.001 r.l.u. (1001 points).  Every H but 0 "
             "and 1 is a zero of the chain amplitude, up to the FP32 rounding of H, so the map "
             "is almost all minima, where the paper sees single precision fail.", "",
             "- reliable range: max I over the strongest I at which the relative intensity "
             "error first exceeds 1e-2 (points visited from the strongest down);",
             "- within 1e-2: share of points whose relative intensity error is at most 1e-2;",
             "- median |dI|/max I: the typical absolute intensity error on the map's scale;",
             "- the disordered chain (Gaussian 1e-3 on each coordinate, the paper's gray curve) "
             "gives the median of I/max I it reaches: the noise level an error must stay under.",
             "", "| atoms | mode | reliable range | within 1e-2 | median \\|dI\\|/max I |",
             "|---:|---|---:|---:|---:|"]
    for n in (1000, 10_000, 100_000):
        xyz, S = wl.chain(n)
        ref = chain_amplitude(S[:, 0].astype(np.float64), n)
        Ir = np.abs(ref) ** 2
        for mode in ("f32", "ph64", "f64"):
            if mode == "f64":
                A = api.scatter_fwd_f64(_dev(xyz.astype(np.float64)), None, _dev(S.astype(np.float64)))
            else:
                A = api.scatter_fwd(_dev(xyz), None, _dev(S), mode)
            A = A.cpu().numpy().astype(np.complex128)
            I = np.abs(A) ** 2
            err = np.abs(I - Ir) / np.maximum(Ir, 1e-300)
            lines.append(f"| {n} | {mode} | {reliable_range(A, ref):.2e} | "
                         f"{np.mean(err <= 1e-2) * 100:.1f} % | "
                         f"{np.median(np.abs(I - Ir)) / Ir.max():.1e} |")
            print(lines[-1], flush=True)
        xd, _ = wl.chain(n, sigma=1e-3)
        Ad = api.scatter_fwd_f64(_dev(xd.astype(np.float64)), None, _dev(S.astype(np.float64)))
        Id = np.abs(Ad.cpu().numpy()) ** 2
        lines.append(f"| {n} | disorder 1e-3: median I/max I | | | {np.median(Id) / Ir.max():.1e} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    p = argparse.ArgumentParser(description="replays of the paper's experiments")
    p.add_argument("what", choices=["fig1", "cube", "chain"])
    p.add_argument("--max-pairs", type=float, default=1e12)
    p.add_argument("--out", default=None)
    a = p.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("replay: needs a GPU (libnx has no CPU path)")
    t0 = time.time()
    text = {"fig1": lambda: fig1(a.max_pairs), "cube": cube, "chain": chain}[a.what]()
    text += f"\n(device: {torch.cuda.get_device_name(0)}; wall {time.time() - t0:.0f} s)\n"
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    print(text, flush=True)


if __name__ == "__main__":
    main()
