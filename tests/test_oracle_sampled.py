"""Pins of the oracle's pointwise helpers, the references of every full-size sampled
parity test (the whole-grid oracle step does not fit those grids).

Each helper is checked against two independent definitions of the same quantity:
* the whole-grid oracle functions (`stream`, `step`, `step_emulated`'s FP64 step on the
  dequantised words), indexed at the sampled cells;
* a brute-force loop over the cells that applies the periodic pull rule of Eq. 1,
  h_i(x) = g_i(x - c_i) with every coordinate wrapped by hand.

Grids are non-cubic with different extents per axis (a transposed axis or a wrong sign
of the shift lands on a different cell), and the samples include every box corner
(where the wrap acts) plus random interior cells.
"""
import itertools

import pytest
import torch

import synthetic
from oracle import lbm
from oracle import storage as ost

SHAPES = {"D2Q9": (9, 4), "D3Q19": (7, 5, 3), "D3Q27": (7, 5, 3)}  # (nx, ny[, nz])
# The pointwise and whole-grid collisions sum the same terms over differently shaped
# tensors, so their FP64 results may differ in summation order: a few ulps of the
# largest population (about 3 ulps observed).  A wrong neighbour or a dropped term
# moves a population by ~1e-3.
_ROUNDING = 4 * torch.finfo(torch.float64).eps


def _cells(sizes, n_random=23, seed=3):
    """Every box corner, then random cells: [M, D] int64 coordinates (x, y[, z])."""
    corners = [list(c) for c in itertools.product(*[(0, s - 1) for s in sizes])]
    gen = torch.Generator().manual_seed(seed)
    rnd = torch.stack([torch.randint(0, s, (n_random,), generator=gen) for s in sizes], dim=1)
    return torch.cat([torch.tensor(corners, dtype=torch.int64), rnd])


def _state(lattice, seed=1):
    st = lbm.stencil(lattice)
    sizes = SHAPES[lattice]
    spatial = tuple(reversed(sizes))
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.02, umax=0.05)
    f = lbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, seed + 1, 0.02))
    F = synthetic.random_normal((st.D,) + spatial, seed + 2, 1e-4)
    return st, sizes, f, F


def _at(field, cells):
    """field[..., z, y, x] at each cell: [leading, M]."""
    idx = tuple(cells[:, a] for a in reversed(range(cells.shape[1])))
    return field[(slice(None),) + idx]


def _brute_gather(g, st, sizes, cells):
    out = torch.empty((st.Q, cells.shape[0]), dtype=torch.float64)
    for m, cell in enumerate(cells.tolist()):
        for i in range(st.Q):
            src = [(cell[a] - int(st.c[i, a])) % sizes[a] for a in range(st.D)]
            out[i, m] = float(g[(i,) + tuple(reversed(src))])
    return out


@pytest.mark.parametrize("lattice", sorted(SHAPES))
def test_gather_at_cells_equals_stream_and_brute_force(lattice):
    st, sizes, f, _ = _state(lattice)
    cells = _cells(sizes)
    h = lbm.gather_at_cells(f, st, cells)
    assert torch.equal(h, _at(lbm.stream(f, st), cells))
    assert torch.equal(h, _brute_gather(f, st, sizes, cells))


@pytest.mark.parametrize("lattice", sorted(SHAPES))
def test_gather_at_cells_reads_stored_words_exactly(lattice):
    """Stored words of every kind come out of the gather unrounded (the words are
    permuted, then converted exactly to FP64)."""
    st, sizes, f, _ = _state(lattice)
    cells = _cells(sizes)
    for kind in ost.KINDS:
        s = ost.quantize(f, st, kind)
        h = lbm.gather_at_cells(s, st, cells)
        assert torch.equal(h, _at(lbm.stream(s, st), cells).to(torch.float64)), kind


@pytest.mark.parametrize("lattice", sorted(SHAPES))
def test_force_at_cells_is_direct_indexing(lattice):
    st, sizes, _, F = _state(lattice)
    cells = _cells(sizes)
    got = lbm.force_at_cells(F, st, cells)
    assert got.shape == (st.D, cells.shape[0])
    for m, cell in enumerate(cells.tolist()):
        for a in range(st.D):
            assert float(got[a, m]) == float(F[(a,) + tuple(reversed(cell))])


@pytest.mark.parametrize("lattice", sorted(SHAPES))
@pytest.mark.parametrize("forced", [False, True])
def test_step_at_cells_equals_whole_grid_step(lattice, forced):
    st, sizes, f, F = _state(lattice)
    cells = _cells(sizes)
    force = F if forced else None
    got = lbm.step_at_cells(f, 0.53, st, cells, force)
    ref = _at(lbm.step(f, 0.53, st, force), cells)
    assert float((got - ref).abs().max()) <= _ROUNDING * float(ref.abs().max())


@pytest.mark.parametrize("lattice", sorted(SHAPES))
@pytest.mark.parametrize("kind", ost.KINDS)
@pytest.mark.parametrize("forced", [False, True])
def test_step_at_cells_emulated_equals_fp64_step_of_stored_words(lattice, kind, forced):
    """The FP64 populations before the final rounding: the whole-grid FP64 step of the
    dequantised words (shifted kinds add w_i back before the step), at the cells; and
    rounding them gives `step_emulated`'s stored words."""
    st, sizes, f, F = _state(lattice)
    cells = _cells(sizes)
    force = F if forced else None
    s = ost.quantize(f, st, kind)
    got = ost.step_at_cells_emulated(s, 0.53, st, kind, cells, force)
    ref = _at(lbm.step(ost.dequantize(s, st, kind), 0.53, st, force), cells)
    assert float((got - ref).abs().max()) <= _ROUNDING * float(ref.abs().max())
    # Rounding the returned populations the way quantize does (shifted kinds store
    # f - w) reproduces the emulated step's words: bit for bit for the narrower kinds,
    # whose rounding absorbs the FP64 summation-order difference; FP64 words keep it.
    w = st.w.reshape(st.Q, 1)
    rounded = ((got - w) if ost.is_shifted(kind) else got).to(ost.dtype_of(kind))
    words = _at(ost.step_emulated(s, 0.53, st, kind, force), cells)
    if kind == "f64":
        assert float((rounded - words).abs().max()) <= _ROUNDING * float(words.abs().max())
    else:
        assert torch.equal(rounded, words)


def test_planted_transposition_is_caught():
    """A gather that swaps the x and y shifts differs from the pull rule on the test
    grids: the shapes above are able to tell the axes apart."""
    st, sizes, f, _ = _state("D3Q27")
    cells = _cells(sizes)
    wrong = torch.empty((st.Q, cells.shape[0]), dtype=torch.float64)
    for m, cell in enumerate(cells.tolist()):
        for i in range(st.Q):
            c = [int(st.c[i, 1]), int(st.c[i, 0]), int(st.c[i, 2])]  # x and y shifts swapped
            src = [(cell[a] - c[a]) % sizes[a] for a in range(3)]
            wrong[i, m] = float(f[(i,) + tuple(reversed(src))])
    assert not torch.equal(wrong, lbm.gather_at_cells(f, st, cells))
