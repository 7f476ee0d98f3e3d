"""Register budget of the fused batched LU (CPU only: hipcc's resource report).

`k_lu_fused` runs at the 256-register limit of its 512-thread workgroups.  How
the compiler treats the helpers it shares with other kernels decides whether it
fits: inlined into it, the 16-row block substitution once made it spill 602
registers (and run 50 % slower) without any change to its own source.  The
FP64 and FP32 variants are compiled here and their spills bounded."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _report(src):
    from paper_2609_33216_amd import build as b
    hipcc = b.HIPCC if os.path.exists(b.HIPCC) else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    cmd = [hipcc, *b.FLAGS, "-Rpass-analysis=kernel-resource-usage", "--offload-device-only", "-x", "hip", "-c",
           os.path.join(b.SRC, src), "-o", os.devnull]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    # remarks per kernel: "Function Name: <mangled>" then its figures
    out = {}
    cur = None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\])?: (\d+)", line)
        if m and cur:
            out[cur][m.group(1).strip()] = int(m.group(2))
    return out


@pytest.mark.parametrize("src,name", [("dense.hip", "_ZN6symhss10k_lu_fusedEPKNS_6LuDescE"),
                                      ("dense32.hip", "_ZN6symhss3f3210k_lu_fusedEPKNS0_6LuDescE")])
def test_fused_lu_fits_its_registers(src, name):
    rep = _report(src)
    assert name in rep, sorted(rep)[:10]
    r = rep[name]
    print(src, r)
    assert r["VGPRs"] <= 256
    assert r["VGPRs Spill"] <= 8
    assert r["ScratchSize"] <= 64
