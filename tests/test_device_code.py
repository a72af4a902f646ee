"""The gfx950 code the build produces, checked on the CPU (hipcc cross-compiles): no
packed-FP32 instructions anywhere (their selection is disabled at compile time), no
kernel that spills to scratch, the two hot kernels of the default FP64-phase path at
their occupancy (the forward's LDS-tiled kernel with one point per lane at 8 waves per
SIMD; the split adjoint with two atoms per lane at 6, the register cost of its per-tile
fallback loop: a build without that loop ran at 8 waves and no faster, 102.3 against
101.9 ms on the 203,557-atom, 2,097,152-point adjoint), and the issue-ceiling
microbenchmarks' loops
made of exactly the per-pair instruction counts the benchmark prices its sums with."""
import collections
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_1010_2641_amd import build

HIP_SOURCES = [s for s in build.SOURCES + build.MICRO_SOURCES if s.endswith(".hip")]
PACKED_FP32 = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")

pytestmark = pytest.mark.skipif(not os.path.exists(build._hipcc()) and shutil.which("hipcc") is None,
                                reason="hipcc not available")


@pytest.fixture(scope="module")
def device_asm():
    tmp = tempfile.mkdtemp(prefix="nx_asm_")

    def compile_one(src):
        out = os.path.join(tmp, src + ".s")
        cmd = [build._hipcc(), *build.FLAGS, "--cuda-device-only", "-S",
               os.path.join(build.CSRC, src), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return src, open(out).read()

    try:
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            yield dict(ex.map(compile_one, HIP_SOURCES))
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def kernel_notes(asm):
    """(kernel symbol, ScratchSize, Occupancy) for every kernel of one assembly file."""
    out, name = [], None
    scratch = None
    for line in asm.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            name = m.group(1)
            scratch = None
        m = re.match(r"^; ScratchSize: (\d+)", line)
        if m:
            scratch = int(m.group(1))
        m = re.match(r"^; Occupancy: (\d+)", line)
        if m and name is not None:
            out.append((name, scratch, int(m.group(1))))
            name = None
    return out


def test_no_packed_fp32(device_asm):
    for src, asm in device_asm.items():
        hits = PACKED_FP32.findall(asm)
        assert not hits, f"{src}: {len(hits)} packed-FP32 instructions"


def test_no_scratch_spills(device_asm):
    n = 0
    for src, asm in device_asm.items():
        for name, scratch, _ in kernel_notes(asm):
            n += 1
            assert scratch == 0, f"{src}: {name} uses {scratch} bytes of scratch"
    assert n > 100          # every instantiation was seen


def test_hot_kernels_occupancy(device_asm):
    occ = {name: o for asm in device_asm.values() for name, _, o in kernel_notes(asm)}
    want = {"fwd_lds_kernelILi1ELi1ELi16ELi2ELb0E": 8,      # forward, complex f, 16-atom groups
            "fwd_lds_kernelILi1ELi0ELi16ELi2ELb0E": 8,      # forward, f = 1
            "bwd_split_kernelILi2ELi1ELi64ELi2ELb0ELb0E": 6,    # adjoint, complex f
            "bwd_split_kernelILi2ELi0ELi64ELi2ELb0ELb0E": 6,    # adjoint, f = 1
            # grids walked by rows: blocks of 1, 2, 4 and 8 points per lane (forward); the
            # stepped adjoint, two atoms per lane
            "fwd_block_kernelILi1ELi16ELi1ELi1ELi1E": 8,
            "fwd_block_kernelILi1ELi16ELi2ELi1ELi1E": 8,
            "fwd_block_kernelILi1ELi16ELi1ELi2ELi1E": 8,
            "fwd_block_kernelILi1ELi16ELi2ELi2ELi1E": 5,
            "fwd_block_kernelILi1ELi16ELi1ELi2ELi2E": 5,
            "fwd_block_kernelILi1ELi16ELi2ELi2ELi2E": 3,
            "fwd_block_kernelILi0ELi16ELi2ELi2ELi2E": 3,
            "fwd_block_kernelILi1ELi8ELi1ELi1ELi1E": 7,
            "bwd_rows_kernelILi2ELi1E": 7,
            "bwd_rows_kernelILi2ELi0E": 7}
    for key, o in want.items():
        found = [v for k, v in occ.items() if key in k]
        assert found, key
        assert min(found) >= o, (key, found)


def loop_bodies(asm):
    """{kernel symbol: Counter of the instructions of its loop} for kernels with one
    loop (a label with a backward branch to it)."""
    lines = asm.splitlines()
    out, kern = {}, None
    for i, line in enumerate(lines):
        m = re.match(r"^(_Z\S+):", line)
        if m:
            kern = m.group(1)
            continue
        m = re.match(r"^(\.LBB\d+_\d+):", line)
        if not (m and kern):
            continue
        body = []
        for l in lines[i + 1:]:
            l = l.strip()
            if re.match(r"^_Z\S+:", l):
                break
            if re.match(r"s_c?branch\w* " + re.escape(m.group(1)) + "$", l):
                c = collections.Counter(t.split()[0] for t in body
                                        if t and not t.startswith((".", ";")) and not t.endswith(":"))
                out.setdefault(kern, c)
                break
            body.append(l)
    return out


def test_micro_loops_are_the_priced_instruction_mixes(device_asm):
    import bench
    loops = loop_bodies(device_asm["nx_micro.hip"])
    kinds = {"mix_fwd_ph64": ("ph64", "fwd"), "mix_bwd_ph64": ("ph64", "bwd"),
             "mix_fwd_f32": ("f32", "fwd"), "mix_bwd_f32": ("f32", "bwd")}
    seen = 0
    for name, c in loops.items():
        for key, (mode, op) in kinds.items():
            m = re.search(key + r"ILb([01])ELi(\d+)ELi\d+E", name)
            if not m:
                continue
            fkind = "complex" if m.group(1) == "1" else "unit"
            pairs = int(m.group(2))
            valu = sum(v for k, v in c.items() if k.startswith("v_"))
            trans = c["v_sin_f32_e32"] + c["v_cos_f32_e32"]
            assert valu == pairs * bench.ALG_SLOTS[(mode, op, fkind)], (name, dict(c))
            assert trans == pairs * (1 if (mode, op) == ("ph64", "bwd") else 2), (name, dict(c))
            assert not any(k.startswith(("scratch_", "global_load", "buffer_load", "ds_"))
                           for k in c), (name, dict(c))
            seen += 1
    assert seen == 16
    # the sums' own shape: 1 point (forward) or 2 atoms (adjoint) x 16 stream items
    tiles = 0
    for name, c in loops.items():
        m = re.search(r"mix_(fwd|bwd)_ph64_tileILb([01])E", name)
        if not m:
            continue
        op, fkind = m.group(1), "complex" if m.group(2) == "1" else "unit"
        pairs = 16 * (2 if op == "bwd" else 1)
        valu = sum(v for k, v in c.items() if k.startswith("v_"))
        trans = c["v_sin_f32_e32"] + c["v_cos_f32_e32"]
        assert valu == pairs * bench.ALG_SLOTS[("ph64", op, fkind)], (name, dict(c))
        assert trans == pairs * (1 if op == "bwd" else 2), (name, dict(c))
        assert not any(k.startswith(("scratch_", "global_load", "buffer_load", "ds_")) for k in c)
        tiles += 1
    assert tiles == 4
    # the sums over grid rows in their own shapes: forward, 2 atoms against a 2 x 2 x 2
    # block of points (one phase, cos and sin per atom); adjoint, one 64-point group
    # against 2 atoms (3 FP64 fma, cos and sin per atom)
    grids = 0
    for name, c in loops.items():
        m = re.search(r"mix_(fwd|bwd)_grid_tileILb([01])E", name)
        if not m:
            continue
        op, fkind = m.group(1), "complex" if m.group(2) == "1" else "unit"
        pairs, atoms, fma64 = (128, 2, 6) if op == "bwd" else (16, 2, 2)
        valu = sum(v for k, v in c.items() if k.startswith("v_"))
        trans = c["v_sin_f32_e32"] + c["v_cos_f32_e32"]
        assert valu == round(pairs * bench.ALG_SLOTS[("grid", op, fkind)]), (name, dict(c))
        assert trans == 2 * atoms, (name, dict(c))
        assert c["v_fma_f64"] + c["v_fmac_f64_e32"] == fma64, (name, dict(c))
        assert not any(k.startswith(("scratch_", "global_load", "buffer_load", "ds_", "v_mov")) for k in c)
        grids += 1
    assert grids == 4
    # the single-instruction kernels: 4 steps of NP chains of one kind per iteration
    kinds = {"0": "v_fma_f32", "1": "v_fma_f64", "2": "v_sin_f32", "3": "v_fmac_f32_e32",
             "4": "v_fmac_f64_e32", "5": "v_add_f64", "6": "v_rndne_f64", "7": "v_fract_f64",
             "8": "v_cvt_f32_i32", "9": "v_cos_f32", "10": "v_mul_f32_e32", "11": "v_fma_f32",
             "12": "v_add_f32_e32"}
    ops = 0
    for name, c in loops.items():
        m = re.search(r"op_rateILi(\d+)ELi(\d+)E", name)
        if not m:
            continue
        valu = sum(v for k, v in c.items() if k.startswith("v_"))
        want = 4 * int(m.group(2))
        kind = sum(v for k, v in c.items() if k.startswith(kinds[m.group(1)]))
        assert valu == want and kind == want, (name, dict(c))
        ops += 1
    assert ops == 26
