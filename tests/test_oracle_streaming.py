"""Pins of the oracle's streaming (Eq. 1): direction, periodic wrap and the
permutation property, by brute force on tiny grids."""
import itertools

import pytest
import torch

import synthetic
from oracle import lbm, storage


@pytest.mark.parametrize("name,spatial", [("D2Q9", (4, 5)), ("D3Q19", (3, 4, 3)), ("D3Q27", (3, 4, 5))])
def test_single_population_moves_along_c(name, spatial):
    # Eq. 1: the value of f_i at x reappears at x + c_i one step later.
    st = lbm.stencil(name)
    sizes = tuple(reversed(spatial))  # (nx, ny[, nz])
    for i in range(st.Q):
        for x0 in itertools.product(*[range(n) for n in sizes]):
            f = torch.zeros((st.Q,) + spatial, dtype=torch.float64)
            f[(i,) + tuple(reversed(x0))] = 1.0
            out = lbm.stream(f, st)
            dst = tuple((x0[a] + int(st.c[i, a])) % sizes[a] for a in range(st.D))
            assert out[(i,) + tuple(reversed(dst))] == 1.0
            assert out.sum() == 1.0


def test_brute_force_loops_3d():
    st = lbm.stencil("D3Q27")
    nz, ny, nx = 3, 4, 5
    f = synthetic.random_normal((st.Q, nz, ny, nx), 0)
    out = lbm.stream(f, st)
    for i in range(st.Q):
        cx, cy, cz = (int(v) for v in st.c[i])
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    assert out[i, z, y, x] == f[i, (z - cz) % nz, (y - cy) % ny, (x - cx) % nx]


@pytest.mark.parametrize("name,spatial", [("D2Q9", (6, 6)), ("D3Q19", (4, 4, 4)), ("D3Q27", (4, 4, 4))])
def test_round_trip_identity(name, spatial):
    # n streaming steps on an n-periodic cube return every population home.
    st = lbm.stencil(name)
    f = synthetic.random_normal((st.Q,) + spatial, 1)
    out = f
    for _ in range(spatial[0]):
        out = lbm.stream(out, st)
    assert torch.equal(out, f)


@pytest.mark.parametrize("kind", storage.KINDS)
def test_streaming_is_bitwise_permutation(kind):
    st = lbm.stencil("D3Q27")
    f = lbm.equilibrium(*synthetic.random_fields((3, 5, 4), 3, 2), st)
    s = storage.quantize(f, st, kind)
    out = storage.stream_stored(s, st)
    for i in range(st.Q):
        a = torch.sort(s[i].reshape(-1).view(torch.int8 if s.element_size() == 1 else {2: torch.int16, 4: torch.int32, 8: torch.int64}[s.element_size()]))[0]
        b = torch.sort(out[i].reshape(-1).view(a.dtype))[0]
        assert torch.equal(a, b)
