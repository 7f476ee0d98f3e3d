"""Host-side replica of the index arithmetic of the fused LU's matrix-core
trailing update (stream_update_mfma in csrc/dense_body.inc), run on the CPU.

The update stages U[0:kb, c0:c0+cw] in LDS as lds[k * kUpdCols + c] and the
matrix-core steps read lds[(4 s4 + lk) * kUpdCols + cu]; C, L and U are
addressed through row and column masks.  For every shape the fused LU can
hand it (blocks of up to 512 rows with up to 256 appended columns, any panel
depth kb <= kNB), this replica walks every thread's staging loop and every
lane's reads and checks them against the LDS array k_lu_fused declares and
against the matrix extents.  The constants are read from the source, so a
change of the chunk width or of the array is checked as it stands.

It also records the finding behind the wider chunks that were taken out:
256-column chunks need 16 * 256 staging entries, more than the array holds,
so the staging would run past it into the LDS variables declared after it
(among them the panel's row lists, which the row interchanges use as
addresses).
"""

import os
import re

import numpy as np
import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2609_33216_amd", "csrc", "dense_body.inc")


def _constants():
    text = open(SRC).read()

    def const(name):
        m = re.search(rf"constexpr int {name} = (\d+);", text)
        assert m, name
        return int(m.group(1))

    c = {k: const(k) for k in ("kUpdCols", "kKC", "kNB", "kLuThreads")}
    # the LDS array of k_lu_fused
    m = re.search(r"k_lu_fused\(const LuDesc\* __restrict__ descs\) \{\s*__shared__ cplx lds\[([^\]]+)\];", text)
    assert m, "LDS declaration of k_lu_fused"
    expr = m.group(1)
    for k, v in c.items():
        expr = expr.replace(k, str(v))
    assert re.fullmatch(r"[\d\s\*\+/]+", expr), expr
    c["lds_entries"] = int(eval(expr))  # arithmetic on integer literals only
    return c


def _replica(m, ncols, kb, kupd, nt, knb, lds_entries):
    """Largest LDS index touched and whether every global access is inside
    the C (m x ncols), L (m x kb) and U (kb x ncols) blocks."""
    lds_max = -1
    for c0 in range(0, ncols, kupd):
        cw = min(kupd, ncols - c0)
        # staging: q = tid, tid + NT, ... < kNB * cw  ->  lds[k * kUpdCols + c]
        q = np.arange(knb * cw)
        k, c = q % knb, q // knb
        idx = k * kupd + c
        lds_max = max(lds_max, int(idx.max()))
        uk, uc = k[k < kb], c0 + c[k < kb]
        assert (uk < kb).all() and (uc < ncols).all()
        # matrix-core reads: lane l of a tile, cu = ct * 16 + l % 16 < cw, k = 4 s4 + l / 16
        ct_n = (cw + 15) // 16
        lane = np.arange(64)
        lq, lk = lane % 16, lane // 16
        for ct in range(ct_n):
            cu = ct * 16 + lq
            for s4 in range(4):
                r = ((4 * s4 + lk) * kupd + cu)[cu < cw]
                if r.size:
                    lds_max = max(lds_max, int(r.max()))
        # C tiles: row = rt * 16 + lq < m, col = ct * 16 + (4 r + lk) < cw (FP64 accumulator rows)
        rt_n = (m + 15) // 16
        rows = (np.arange(rt_n)[:, None] * 16 + lq[None, :]).ravel()
        cols = (np.arange(ct_n)[:, None] * 16 + (4 * np.arange(4)[:, None] + lk[None, :]).ravel()[None, :]).ravel()
        assert rows[rows < m].max(initial=0) < m and (c0 + cols[cols < cw]).max(initial=0) < ncols
    return lds_max


SHAPES = [(m, nc, kb) for m in (1, 15, 16, 17, 100, 255, 256, 257, 496, 512)
          for nc in (1, 16, 127, 128, 129, 255, 256, 257, 300, 511, 640, 768) for kb in (1, 7, 16)]


def test_update_staging_stays_in_the_lds_array():
    c = _constants()
    worst = max(_replica(m, nc, kb, c["kUpdCols"], c["kLuThreads"], c["kNB"], c["lds_entries"])
                for m, nc, kb in SHAPES)
    print("largest staging index", worst, "array entries", c["lds_entries"])
    assert worst < c["lds_entries"]
    # the chunk width fixes the bound: (kNB - 1) kUpdCols + kUpdCols - 1
    assert worst == c["kNB"] * c["kUpdCols"] - 1


@pytest.mark.parametrize("kupd", [256])
def test_wider_chunks_would_overrun_the_array(kupd):
    """The 256-column chunks tried and taken out: with the array as declared
    the staging runs 16 * (256 - kUpdCols) entries past its end."""
    c = _constants()
    worst = max(_replica(m, nc, 16, kupd, c["kLuThreads"], c["kNB"], c["lds_entries"])
                for m, nc, _ in SHAPES)
    assert worst == c["kNB"] * kupd - 1
    assert worst >= c["lds_entries"], "a 256-column chunk fits: the recorded cause no longer applies"
