"""Structure of the persistent kernel's machine code (host only: hipcc -S).

The ticket loop must stay one loop with a workgroup-uniform exit: a barrier
inside a loop whose exit is decided per lane (an exec-mask update, the
signature of a divergent loop exit) lets some lanes of a wave run the
barrier and the loop body again while another lane of that wave waits
outside the loop -- an endless loop on the GPU. This test compiles
k_persist.hip for gfx950 and checks every loop that contains an
s_barrier: none of its own blocks may update exec to drop exiting lanes."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_19683_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def compile_asm(src, out):
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           src, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read()


def kernels(asm):
    """{kernel symbol: list of lines} for the k_persist instantiations."""
    out = {}
    for m in re.finditer(r"^(_Z\w*k_persist\w*):.*?$(.*?)s_endpgm", asm, re.S | re.M):
        out[m.group(1)] = m.group(2).split("\n")
    return out


def barrier_loops_with_lane_exits(lines):
    block_loop = None
    loops_with_barrier, lane_exit = set(), set()
    for l in lines:
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):\s*(;\s*(.*))?$", l)
        if m:
            txt = m.group(3) or ""
            h = re.search(r"Header=(BB\d+_\d+)", txt)
            if "This Loop Header" in txt:
                h2 = re.match(r"^\.L(BB\d+_\d+):", l)
                block_loop = h2.group(1) if h2 else None
            else:
                block_loop = h.group(1) if h else None
            continue
        if block_loop is None:
            continue
        if "s_barrier" in l:
            loops_with_barrier.add(block_loop)
        if re.search(r"s_andn2_b64\s+exec,\s*exec", l):
            lane_exit.add(block_loop)
    return loops_with_barrier, loops_with_barrier & lane_exit


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_persistent_ticket_loop_has_uniform_exits(tmp_path):
    asm = compile_asm(os.path.join(CSRC, "k_persist.hip"), str(tmp_path / "k_persist.s"))
    ks = kernels(asm)
    assert ks, "no k_persist kernel in the assembly"
    for name, lines in ks.items():
        with_barrier, bad = barrier_loops_with_lane_exits(lines)
        assert with_barrier, f"{name}: no loop with a barrier found (parser out of date?)"
        assert not bad, f"{name}: loops {sorted(bad)} hold a barrier and a per-lane exit"
