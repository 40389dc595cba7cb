"""CPU checks of the binding's grid helpers: population shapes with and without a row
pitch, the padded-grid constructor, and exact layout round trips."""
import pytest
import torch

from oracle import lbm as olbm


@pytest.fixture(scope="module")
def B():
    from paper_2106_12929_amd import binding

    return binding


@pytest.mark.parametrize("lat,shape", [("D2Q9", (13, 7, 1)), ("D3Q19", (10, 4, 3)), ("D3Q27", (9, 5, 2))])
@pytest.mark.parametrize("pitch", [None, 16])
def test_layout_round_trip(B, lat, shape, pitch):
    grid = B.Grid(lat, "f32", *shape, pitch)
    st = olbm.stencil(lat)
    spatial = grid.spatial
    f = torch.arange(st.Q * grid.ncells, dtype=torch.float32).reshape((st.Q,) + spatial)
    lay = grid.to_layout(f)
    assert tuple(lay.shape) == grid.population_shape()
    assert lay.numel() == grid.pop_size
    assert torch.equal(grid.from_layout(lay), f)
    # word (i, x, y, z) sits at ((z*ny + y)*Q + i)*pitch + x
    flat = lay.reshape(-1)
    p = grid.row_pitch
    for i, x, y, z in [(0, 0, 0, 0), (st.Q - 1, shape[0] - 1, shape[1] - 1, shape[2] - 1), (st.Q // 2, 2, 1, 0)]:
        idx = f[(i, y, x)] if grid.D == 2 else f[(i, z, y, x)]
        assert flat[((z * grid.ny + y) * st.Q + i) * p + x] == idx
    if pitch:
        assert bool((lay[..., shape[0]:] == 0).all())


@pytest.mark.parametrize("storage,nx,want", [("f32", 37, 64), ("f32", 64, 64), ("f16s", 255, 256),
                                             ("f64", 33, 64), ("bf16s", 129, 256)])
def test_padded_rows_are_256_bytes(B, storage, nx, want):
    grid = B.Grid.padded("D3Q27", storage, nx, 4, 3)
    assert grid.row_pitch == want
    assert grid.row_pitch * grid.word_dtype.itemsize % 256 == 0
    assert grid.population_shape() == (3, 4, 27, want)
    assert grid.slab_population_shape() == (5, 4, 27, want)


@pytest.mark.parametrize("lattice,storage,nx,want", [
    ("D3Q27", "f16s", 512, 576), ("D3Q27", "bf16s", 1024, 1088), ("D3Q27", "f16s", 500, 576),
    ("D3Q27", "f64", 512, 528), ("D3Q19", "f16s", 512, 576), ("D3Q27", "f16s", 2048, 2112),
    ("D3Q27", "f32", 512, 512), ("D3Q27", "f32", 256, 256), ("D3Q27", "f16s", 256, 256),
    ("D3Q27", "f16s", 768, 768), ("D3Q27", "f64", 128, 128), ("D3Q27", "f32", 37, 64),
    ("D2Q9", "f16s", 8192, 8192), ("D2Q9", "f64", 512, 512)])
def test_tuned_pitch(B, lattice, storage, nx, want):
    """One extra 128-byte line only on split power-of-two rows of 2- or 8-byte words
    of the 3D lattices; otherwise the 256-byte padding."""
    grid = B.Grid.tuned(lattice, storage, nx, 4, 1 if lattice == "D2Q9" else 3)
    assert grid.row_pitch == want
    assert grid.row_pitch * grid.word_dtype.itemsize % 128 == 0


def test_c_struct_carries_the_pitch(B):
    assert B.Grid("D3Q27", "f32", 8, 8, 8).c_struct().pitch == 0
    assert B.Grid("D3Q27", "f32", 8, 8, 8, 12).c_struct().pitch == 12
    with pytest.raises(ValueError):
        B.Grid("D2Q9", "f32", 8, 8).slab_population_shape()


def test_shell_table_layout(B):
    """ShellTable (the lbm_shells arrays): order sorts the wavevectors by shell, stably;
    offsets delimit the shells; shell is kept as int32."""
    shell = torch.tensor([3, 0, 1, 1, 3, 2, 0, 1])
    t = B.ShellTable.from_shells(shell)
    assert (t.n, t.nshell) == (8, 4)
    assert t.order.tolist() == [1, 6, 2, 3, 7, 5, 0, 4]
    assert t.offsets.tolist() == [0, 2, 5, 6, 8]
    assert t.shell.tolist() == shell.tolist()
    assert {t.order.dtype, t.offsets.dtype, t.shell.dtype} == {torch.int32}
