"""CPU check of an invariant of the ring load-vector kernel's inline asm.

Each global-to-LDS load sets M0 (the LDS destination) in the same asm block
and names M0 as clobbered.  M0 is a reserved register, so the compiler warns
that it may not honour that clobber; the asm is then safe only while compiled
code never keeps a value of its own in M0 inside these kernels.  This test
compiles the kernels to gfx950 assembly with the library's flags and checks
that every instruction of the ring kernels that names M0 is one of the asm
blocks' own writes, each followed by its global-to-LDS load.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2105_12764_amd import build

pytestmark = pytest.mark.skipif(not os.path.exists(build.HIPCC) and shutil.which("hipcc") is None,
                                reason="hipcc not available")


def test_ring_kernels_use_m0_only_in_their_lds_loads(tmp_path):
    asm = tmp_path / "k.s"
    flags = [f for f in build.FLAGS if f != "-fPIC"]
    cmd = [build.HIPCC, *flags, "-x", "hip", "--cuda-device-only", "-S",
           os.path.join(build.CSRC, "mgr_kernels.hip"), "-o", str(asm)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    txt = asm.read_text()
    names = re.findall(r"^(_Z\S*k_loadvec_ring\S*):", txt, re.M)
    assert names, "no ring kernel in the assembly"
    for name in names:
        body = txt[txt.index("\n" + name + ":"):]
        body = body[:body.index(".Lfunc_end")]
        lines = [l.split(";")[0].strip() for l in body.split("\n")]
        lines = [l for l in lines if l]
        uses = [i for i, l in enumerate(lines) if re.search(r"\bm0\b", l)]
        assert uses, name
        for i in uses:
            assert re.fullmatch(r"s_mov_b32 m0, s\d+", lines[i]), (name, lines[i])
            follow = lines[i + 1:i + 3]
            assert follow and follow[-1].startswith("global_load_lds_dword"), (name, follow)
