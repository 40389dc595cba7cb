"""CPU checks of the FP32 lattice coefficients the HIP kernels use (csrc/coeffs.h):
exact mass and momentum sums on the binary32 values, closeness to the textbook
weights, and that the committed header is what its generator writes."""
import os
import re
import subprocess
import sys
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import lbm as olbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_12929_amd", "csrc")


def _tables():
    txt = open(os.path.join(CSRC, "coeffs.h")).read()
    out = {}
    for m in re.finditer(r"k(\w+)_(W|A|B)\[\d+\] = \{([^}]*)\}", txt):
        out[(m.group(1), m.group(2))] = [Fr(float.fromhex(v.strip().rstrip("f"))) for v in m.group(3).split(",")]
    return out


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_exact_conservation_sums(name):
    tab = _tables()
    st = olbm.stencil(name)
    rows = st.c.tolist()
    cls = [sum(v * v for v in r) for r in rows]
    W = [tab[(name, "W")][k] for k in cls]
    A = [tab[(name, "A")][k] for k in cls]
    B = [tab[(name, "B")][k] for k in cls]
    for vals in (W, A, B):
        for v in vals:  # every value is a binary32 number
            assert Fr(float(np.float32(float(v)))) == v
    assert sum(W) == 1
    for a in range(st.D):
        for b in range(st.D):
            sA = sum(Ai * r[a] * r[b] for Ai, r in zip(A, rows))
            sB = sum(Bi * r[a] * r[b] for Bi, r in zip(B, rows))
            assert sA == (1 if a == b else 0)
            assert sB == (Fr(3, 2) if a == b else 0)
        assert sum(Ai * r[a] for Ai, r in zip(A, rows)) == 0
    # within ~1 ulp of the textbook values w, 3w, 9w/2
    for i, w in enumerate(st.w.tolist()):
        u = np.spacing(np.float32(w))
        assert abs(float(W[i]) - w) <= 1.5 * u
        if cls[i]:
            assert abs(float(A[i]) - 3 * w) <= 1.5 * np.spacing(np.float32(3 * w))
            assert abs(float(B[i]) - 4.5 * w) <= 1.5 * np.spacing(np.float32(4.5 * w))


def test_header_matches_generator():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_coeffs.py")], capture_output=True, text=True,
                         check=True).stdout
    assert out.strip() == open(os.path.join(CSRC, "coeffs.h")).read().strip()
