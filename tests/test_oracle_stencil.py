"""Pins of the oracle's lattice tables (velocity sets and weights).

The paper names w_i, c_i and c_s (Sec. 2.1) but prints no values.  The weights are
pinned by the exact isotropy conditions a lattice must satisfy to recover
Navier-Stokes with c_s^2 = 1/3 (Krueger 2016, Sec. 3.4), checked in rational
arithmetic: a wrong weight class breaks at least one of them.
"""
from fractions import Fraction
import itertools

import pytest

from oracle import lbm


def _exact(st):
    ws = [Fraction(float(w)).limit_denominator(1000) for w in st.w]
    for wf, w in zip(ws, st.w.tolist()):
        assert float(wf) == w, "weight is not the float of a small rational"
    return [tuple(r) for r in st.c.tolist()], ws


@pytest.mark.parametrize("name,D,Q", [("D2Q9", 2, 9), ("D3Q19", 3, 19), ("D3Q27", 3, 27)])
def test_isotropy_exact(name, D, Q):
    st = lbm.stencil(name)
    assert (st.D, st.Q) == (D, Q)
    c, w = _exact(st)
    assert len(set(c)) == Q and all(all(v in (-1, 0, 1) for v in r) for r in c)
    third = Fraction(1, 3)
    assert sum(w) == 1
    for a in range(D):
        assert sum(wi * ci[a] for wi, ci in zip(w, c)) == 0
    for a, b in itertools.product(range(D), repeat=2):
        assert sum(wi * ci[a] * ci[b] for wi, ci in zip(w, c)) == (third if a == b else 0)
    for a, b, e in itertools.product(range(D), repeat=3):
        assert sum(wi * ci[a] * ci[b] * ci[e] for wi, ci in zip(w, c)) == 0
    for a, b, e, d in itertools.product(range(D), repeat=4):
        expect = Fraction(0)
        expect += third * third * ((a == b) * (e == d) + (a == e) * (b == d) + (a == d) * (b == e))
        assert sum(wi * ci[a] * ci[b] * ci[e] * ci[d] for wi, ci in zip(w, c)) == expect


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_velocity_order(name):
    st = lbm.stencil(name)
    c = st.c.tolist()
    full = [sum(3 ** a * (r[a] + 1) for a in range(st.D)) for r in c]
    if name == "D3Q19":
        # the D3Q27 order without the 8 corners
        assert full == [k for k in range(27) if k not in (0, 2, 6, 8, 18, 20, 24, 26)]
    else:
        assert full == list(range(st.Q))
    assert c[st.Q // 2] == [0] * st.D
    assert st.opposite == [st.Q - 1 - i for i in range(st.Q)]


@pytest.mark.parametrize("name,table", [("D2Q9", {0: {4 / 9}, 1: {1 / 9}, 2: {1 / 36}}),
                                        ("D3Q19", {0: {1 / 3}, 1: {1 / 18}, 2: {1 / 36}})])
def test_textbook_weight_values(name, table):
    # The familiar D2Q9 and D3Q19 values (Krueger 2016, Table 3.3).
    st = lbm.stencil(name)
    by_class = {}
    for r, w in zip(st.c.tolist(), st.w.tolist()):
        by_class.setdefault(sum(v * v for v in r), set()).add(w)
    assert by_class == table
