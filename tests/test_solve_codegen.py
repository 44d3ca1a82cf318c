"""Generated gfx950 code of the full-row strip solve, checked on the CPU.

Every full-row tile finishes its rows at two call sites of one routine: the
rows held in registers, then the streamed rows in a loop.  Each call ends
with a wave sum (DPP moves and lane reads, which need all 64 lanes active)
and lane 0 storing the complex result as two 8-byte device-coherent stores
(real part, then imaginary part at offset 8).  When the compiler's IR-level
sinking of common code merged the imaginary-part stores of the two call
sites, the structurized loop executed the streamed rows' wave sums with
lane 0 masked off, and the solve returned non-finite values.  The build
disables that sinking; this test compiles the kernels with the build's
flags and checks that every full-row instantiation keeps one imaginary
store per real store.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asm(tmp_path, flags):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    src = os.path.join(ROOT, "paper_1603_05110_amd", "csrc", "kernels_solve.hip")
    out = os.path.join(tmp_path, "ks.s")
    dev_flags = [f for f in flags if f not in ("-fPIC",)]
    cmd = [hipcc, *dev_flags, "--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


def _kernels(asm):
    """{mangled name: body} of every full-row strip-solve instantiation."""
    out = {}
    for m in re.finditer(r"^(_Z\w*strip_solve_pf_kernel\w*):", asm, re.M):
        end = asm.find("s_endpgm", m.end())
        out[m.group(1)] = asm[m.end():end]
    return out


def test_every_full_row_tile_keeps_its_row_stores_apart(tmp_path):
    from paper_1603_05110_amd.build import FLAGS
    assert "-simplifycfg-sink-common=false" in FLAGS
    ks = _kernels(_asm(str(tmp_path), FLAGS))
    assert len(ks) == 19
    for name, body in ks.items():
        stores = re.findall(r"global_store_dwordx2 [^\n]*sc1", body)
        imag = [s for s in stores if "offset:8" in s]
        real = [s for s in stores if "offset:8" not in s]
        assert len(real) >= 2 and len(imag) == len(real), (name, len(real), len(imag))
