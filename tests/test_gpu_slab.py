"""GPU checks of the z-slab step (one shard of a domain decomposition along z): a
periodic grid cut into slabs with ghost planes and a halo exchange reproduces the
periodic step of the whole grid bit for bit, for every storage kind, with and without
a body force, with the exchange overlapped on a second stream or not; and so do slabs
with two ghost planes that advance two steps per launch."""
import pytest
import torch

from oracle import lbm as olbm
from oracle import storage as ost

import synthetic
from _helpers import binding, bits, need_gpu, say

pytestmark = pytest.mark.gpu

SHAPE = (37, 13, 11)  # nx (ragged against 64-wide blocks), ny, nz
PARTS = [[11], [6, 5], [4, 4, 3], [1, 9, 1], [2] * 5 + [1]]


def _state(st, spatial, seed, kind):
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.03, umax=0.06)
    f = olbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, seed + 1, 0.02))
    return ost.quantize(f, st, kind)


def _periodic(B, grid, g0, tau, F, T):
    a, b = g0.clone(), grid.empty_populations()
    for _ in range(T):
        B.lbm_step(grid, a, b, tau, F, 1)
        a, b = b, a
    return a


@pytest.mark.parametrize("parts", PARTS, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("lat,kind", [("D3Q27", "f64"), ("D3Q27", "f32"), ("D3Q27", "f32s"), ("D3Q27", "f16s"),
                                      ("D3Q27", "bf16s"), ("D3Q19", "f32"), ("D3Q19", "f16s")])
@pytest.mark.parametrize("forced", [False, True])
def test_slabs_match_periodic_step(parts, lat, kind, forced):
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    st = olbm.stencil(lat)
    nx, ny, nz = SHAPE
    spatial = (nz, ny, nx)
    grid = B.Grid(lat, kind, nx, ny, nz)
    say(f"slabs {lat} {kind} parts={parts} forced={forced}")
    g0 = grid.to_layout(_state(st, spatial, 31, kind)).cuda()
    F = synthetic.random_normal((3,) + spatial, 5, 1e-4).to(grid.real_dtype).cuda() if forced else None
    T = 4
    ref = _periodic(B, grid, g0, 0.56, F, T)
    S = SlabSet(grid, parts)
    S.scatter(g0)
    forces = S.split_field(F)
    for t in range(T):
        S.step(0.56, forces, overlap=(t % 2 == 1))
    torch.cuda.synchronize()
    assert torch.equal(bits(S.gather()), bits(ref))


@pytest.mark.parametrize("kind", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("parts", [[9], [5, 4], [3, 3, 3]], ids=lambda p: "x".join(map(str, p)))
def test_slabs_match_periodic_step_vector_halo(kind, parts):
    """nx = 64: rows are whole 16-byte units, so the exchange copies 16-byte vectors."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    st = olbm.stencil("D3Q27")
    spatial = (9, 5, 64)
    grid = B.Grid("D3Q27", kind, 64, 5, 9)
    say(f"slabs vector halo {kind} parts={parts}")
    g0 = grid.to_layout(_state(st, spatial, 41, kind)).cuda()
    ref = _periodic(B, grid, g0, 0.6, None, 3)
    S = SlabSet(grid, parts)
    S.scatter(g0)
    for t in range(3):
        S.step(0.6, overlap=True)
    torch.cuda.synchronize()
    assert torch.equal(bits(S.gather()), bits(ref))


def test_slab_plane_ranges_compose():
    """Any split of a slab's planes into launches gives the same step as one launch
    over all of them, and planes outside the range are left untouched."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    st = olbm.stencil("D3Q27")
    grid = B.Grid("D3Q27", "f32", 64, 6, 7)
    g0 = grid.to_layout(_state(st, (7, 6, 64), 3, "f32")).cuda()
    S = SlabSet(grid, 1)
    S.scatter(g0)
    S.exchange()
    slab, a = S.slabs[0], S.bufs[0][0]
    one = torch.full_like(a, float("nan"))
    B.lbm_step_slab(slab, a, one, 0.7)
    pieces = torch.full_like(a, float("nan"))
    for z0, z1 in ((3, 5), (0, 1), (5, 7), (1, 3)):
        B.lbm_step_slab(slab, a, pieces, 0.7, None, z0, z1)
    part = torch.full_like(a, float("nan"))
    B.lbm_step_slab(slab, a, part, 0.7, None, 2, 4)
    torch.cuda.synchronize()
    assert torch.equal(bits(one[1:8]), bits(pieces[1:8]))
    assert torch.equal(bits(part[3:5]), bits(one[3:5]))
    assert torch.isnan(part[1:3]).all() and torch.isnan(part[5:]).all() and torch.isnan(part[0]).all()
    # ghost planes are never written
    assert torch.isnan(one[0]).all() and torch.isnan(one[8]).all()


def test_halo_copy_moves_only_the_crossing_directions():
    """The exchange writes exactly the c_z = +1 directions of the lower ghost plane and
    the c_z = -1 directions of the upper one, with the neighbours' boundary words."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D3Q19")
    grid_a = B.Grid("D3Q19", "f16s", 70, 5, 3)
    grid_b = B.Grid("D3Q19", "f16s", 70, 5, 4)
    a = torch.randn(grid_a.slab_population_shape(), device="cuda").to(torch.float16)
    b = torch.zeros(grid_b.slab_population_shape(), device="cuda", dtype=torch.float16)
    B.lbm_slab_halo_copy(grid_a, a, grid_b, b, "high")  # a lies below b
    B.lbm_slab_halo_copy(grid_a, a, grid_b, b, "low")   # a also lies above b (two slabs, periodic)
    torch.cuda.synchronize()
    up = (st.c[:, 2] == 1).cuda()
    down = (st.c[:, 2] == -1).cuda()
    assert torch.equal(bits(b[0][:, up]), bits(a[3][:, up]))
    assert (b[0][:, ~up] == 0).all()
    assert torch.equal(bits(b[5][:, down]), bits(a[1][:, down]))
    assert (b[5][:, ~down] == 0).all()
    assert (b[1:5] == 0).all()


@pytest.mark.parametrize("parts", [1, 2])
def test_full_size_shard_matches_periodic_step(parts):
    """The 512 x 512 x 64 f16s shard the benchmark times, as one slab (its own
    neighbour) and as two: 3 steps, sequential and overlapped exchange, bit for bit the
    periodic step of the whole grid."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    nx, ny, nz = 512, 512, 64
    grid = B.Grid("D3Q27", "f16s", nx, ny, nz)
    say(f"full-size shard 512x512x64 f16s parts={parts}")
    g0 = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, synthetic.taylor_green_3d_on("cuda", nx, ny, nz, 0.05), g0)
    T = 3
    ref = _periodic(B, grid, g0, 0.51, None, T)
    S = SlabSet(grid, parts)
    S.scatter(g0)
    for t in range(T):
        S.step(0.51, None, overlap=(t % 2 == 1))
    torch.cuda.synchronize()
    assert torch.equal(bits(S.gather()), bits(ref))


PARTS2 = [[12], [6, 6], [5, 4, 3], [2] * 6, [2, 10]]


@pytest.mark.parametrize("parts", PARTS2, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("lat,kind,shape", [("D3Q27", "f32", (64, 16, 12)), ("D3Q27", "f16s", (64, 8, 12)),
                                            ("D3Q27", "bf16s", (128, 4, 12)), ("D3Q27", "f64", (32, 8, 12)),
                                            ("D3Q19", "f32", (32, 8, 12)), ("D3Q27", "f32s", (32, 16, 12))])
@pytest.mark.parametrize("forced", [False, True])
def test_slabs_two_steps_per_launch_match_periodic_step(parts, lat, kind, shape, forced):
    """Slabs with two ghost planes on each side, one two-plane-deep exchange and one
    two-step launch per slab for every two steps: bit for bit the periodic step of the
    whole grid (3 pairs, 6 steps), with and without a Guo force (the slab's force
    carries a ghost plane each side)."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    st = olbm.stencil(lat)
    nx, ny, nz = shape
    spatial = (nz, ny, nx)
    grid = B.Grid(lat, kind, nx, ny, nz)
    say(f"slabs, two steps per launch {lat} {kind} {shape} parts={parts} forced={forced}")
    g0 = grid.to_layout(_state(st, spatial, 37, kind)).cuda()
    F = synthetic.random_normal((3,) + spatial, 6, 1e-4).to(grid.real_dtype).cuda() if forced else None
    ref = _periodic(B, grid, g0, 0.56, F, 6)
    S = SlabSet(grid, parts, ghost=2)
    S.scatter(g0)
    forces = S.split_field(F)
    for t in range(3):
        S.step_pair(0.56, forces, overlap=(t % 2 == 1))
    torch.cuda.synchronize()
    assert torch.equal(bits(S.gather()), bits(ref))


@pytest.mark.parametrize("kind", ["f32", "f16s"])
def test_two_step_slab_plane_ranges_compose(kind):
    """lbm_step_slab2 over the plane ranges [0, 3), [3, 7), [7, 9), [9, 12) writes what one
    launch over [0, 12) writes, word for word (the launches read the same input)."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    lat = "D3Q27"
    shape = (64, 8, 12)
    st = olbm.stencil(lat)
    grid = B.Grid(lat, kind, *shape)
    spatial = (shape[2], shape[1], shape[0])
    S = SlabSet(grid, 1, ghost=2)
    S.scatter(grid.to_layout(_state(st, spatial, 41, kind)).cuda())
    S.exchange()
    slab, src = S.slabs[0], S.bufs[0][S.cur]
    whole = torch.zeros_like(src)
    B.lbm_step_slab2(slab, src, whole, 0.56)
    parts = torch.zeros_like(src)
    for z0, z1 in ((0, 3), (3, 7), (7, 9), (9, 12)):
        B.lbm_step_slab2(slab, src, parts, 0.56, None, z0, z1)
    torch.cuda.synchronize()
    assert torch.equal(bits(parts), bits(whole))
    assert (whole[:2] == 0).all() and (whole[-2:] == 0).all()  # ghost planes untouched


def test_two_step_slabs_reject_other_shapes():
    """Slabs off the two-step tiles, or of one plane, are refused instead of stepping
    another way."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    with pytest.raises(ValueError):
        SlabSet(B.Grid("D3Q27", "f32", 48, 8, 8), 2, ghost=2)
    with pytest.raises(ValueError):
        SlabSet(B.Grid("D3Q27", "f32", 32, 8, 8), [1, 7], ghost=2)
    S = SlabSet(B.Grid("D3Q27", "f32", 32, 8, 8), 2, ghost=2)
    with pytest.raises(ValueError):
        S.step(0.6)


@pytest.mark.parametrize("parts", [1, 2])
def test_full_size_shard_two_steps_per_launch_matches_periodic_step(parts):
    """The 512 x 512 x 64 f16s shard of the benchmark with two ghost planes, as one slab
    (its own neighbour) and as two: 2 pairs, bit for bit 4 periodic steps."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    nx, ny, nz = 512, 512, 64
    grid = B.Grid("D3Q27", "f16s", nx, ny, nz)
    say(f"full-size shard 512x512x64 f16s, two steps per launch, parts={parts}")
    g0 = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, synthetic.taylor_green_3d_on("cuda", nx, ny, nz, 0.05), g0)
    ref = _periodic(B, grid, g0, 0.51, None, 4)
    S = SlabSet(grid, parts, ghost=2)
    S.scatter(g0)
    for t in range(2):
        S.step_pair(0.51, overlap=(t == 1))
    torch.cuda.synchronize()
    assert torch.equal(bits(S.gather()), bits(ref))
