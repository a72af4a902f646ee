"""The gfx950 code the build produces, checked on the CPU (hipcc cross-compiles): no
packed-FP32 instructions anywhere (their selection is disabled at compile time), no
kernel that spills to scratch, and the two hot kernels of the default FP64-phase path
at 8 waves per SIMD (the forward's LDS-tiled kernel with one point per lane and the
split adjoint with two atoms per lane)."""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_1010_2641_amd import build

HIP_SOURCES = [s for s in build.SOURCES if s.endswith(".hip")]
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


def test_hot_kernels_at_eight_waves(device_asm):
    occ = {name: o for asm in device_asm.values() for name, _, o in kernel_notes(asm)}
    want = {"fwd_lds_kernelILi1ELi1ELi16ELi0E": 8,          # forward, complex f, 16-atom groups
            "fwd_lds_kernelILi1ELi0ELi16ELi0E": 8,          # forward, f = 1
            "bwd_split_kernelILi2ELi1ELi64ELi1ELb0E": 8,    # adjoint, complex f
            "bwd_split_kernelILi2ELi0ELi64ELi1ELb0E": 8}    # adjoint, f = 1
    for key, o in want.items():
        found = [v for k, v in occ.items() if key in k]
        assert found, key
        assert min(found) >= o, (key, found)
