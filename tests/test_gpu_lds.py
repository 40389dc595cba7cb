"""GPU checks of the LDS-staged step kernel, which lbm_step uses for 2- and 4-byte
storage words whenever nx is a multiple of the block's row segment (64, 128 or 256
cells): one-step parity with the oracle on such shapes (including row counts that
leave the last block partly empty), and bitwise agreement with the one-word-per-lane
kernel, which handles every other shape."""
import pytest
import torch

import synthetic
from oracle import lbm as olbm
from oracle import storage as ost

from _helpers import binding, bits, need_gpu, say
from test_gpu_forward import _force, _state, _tolerance_ok

pytestmark = pytest.mark.gpu

KINDS = ["f32", "f32s", "f16s", "bf16s"]
# (nx, ny, nz): segments of 64 (nx = 64, 192), 128 (nx = 128, 384) and 256 cells; the
# row counts ny*nz are not multiples of the 4 or 2 rows a 64- or 128-cell block covers
SHAPES = {
    "D3Q27": [(64, 7, 5), (128, 5, 3), (256, 3, 2), (384, 3, 2), (192, 3, 3)],
    "D3Q19": [(64, 5, 3), (256, 3, 3)],
    "D2Q9": [(64, 13, 1), (256, 5, 1), (384, 7, 1)],
}
CASES = [(lat, s) for lat, shapes in SHAPES.items() for s in shapes]


def _spatial(lat, shape):
    nx, ny, nz = shape
    return (ny, nx) if lat == "D2Q9" else (nz, ny, nx)


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("mode", ["none", "guo", "shift"])
def test_lds_step_parity(lat, shape, kind, mode):
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = B.Grid(lat, kind, *shape)
    spatial = _spatial(lat, shape)
    tau = 0.57
    say(f"lds step {lat} {kind} {shape} {mode}")
    s = _state(st, spatial, 21, kind)
    out = grid.empty_populations()
    g_in = grid.to_layout(s).cuda()
    if mode == "shift":
        du = synthetic.random_normal((grid.D,) + spatial, 23, 1e-3).to(grid.real_dtype)
        assert B.lbm_step_shifted(grid, g_in, out, tau, du.cuda(), 1) == 0
        ref = ost.step_emulated(s, tau, st, kind, du=du.double())
    else:
        F = _force(grid, spatial, 22) if mode == "guo" else None
        assert B.lbm_step(grid, g_in, out, tau, None if F is None else F.cuda(), 1) == 0
        ref = ost.step_emulated(s, tau, st, kind, None if F is None else F.double())
    excess, ratio, same = _tolerance_ok(kind, st, grid.from_layout(out.cpu()), ref, tau)
    say(f"  max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio


@pytest.mark.parametrize("lat", ["D3Q27", "D3Q19", "D2Q9"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("forced", [False, True])
def test_lds_path_matches_word_path_bitwise(lat, kind, forced):
    """A field on nx = 96 (one-word kernel: 96 is not a multiple of the chosen 128-cell
    segment) and the same field repeated twice along x on nx = 192 (LDS kernel, 64-cell
    segments) are the same periodic problem: both halves of the wide result must equal
    the narrow result bit for bit, over three steps."""
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    ny, nz = (5, 1) if lat == "D2Q9" else (4, 3)
    narrow = B.Grid(lat, kind, 96, ny, nz)
    wide = B.Grid(lat, kind, 192, ny, nz)
    spatial = _spatial(lat, (96, ny, nz))
    say(f"lds vs word path {lat} {kind} forced={forced}")
    s = _state(st, spatial, 27, kind)
    s2 = torch.cat([s, s], dim=-1)
    F = _force(narrow, spatial, 28) if forced else None
    F2 = None if F is None else torch.cat([F, F], dim=-1).contiguous()

    def run(grid, state, force):
        a, b = grid.to_layout(state).cuda(), grid.empty_populations()
        B.lbm_step(grid, a, b, 0.55, None if force is None else force.cuda(), 3)  # odd: result in b
        return grid.from_layout(b.cpu())

    got_n = run(narrow, s, F)
    got_w = run(wide, s2, F2)
    assert torch.equal(bits(got_w[..., :96].contiguous()), bits(got_n))
    assert torch.equal(bits(got_w[..., 96:].contiguous()), bits(got_n))
