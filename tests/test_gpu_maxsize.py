"""GPU checks at the largest grids the library accepts and one MI355X holds: index
arithmetic past 2^32 words and up to the 2^31 - 1 cell limit.

  * D3Q27 FP16-shifted on 1024^3 (2^30 cells, 2.9e10 words, 58 GB per buffer);
  * D2Q9 FP16-shifted on 46340^2 (2,147,395,600 cells, just under 2^31 - 1);
  * the two-step kernel on z planes of more than 2^31 bytes (4096 x 4864 x 3 FP32,
    4096 x 9728 x 3 FP16-shifted), bit for bit against single steps.

After a few steps from a Taylor-Green start, one more step is compared with the
oracle's collision at sampled cells (and at the corners of the box, where the
periodic wrap acts), reading the pull sources out of the device buffer directly; the
moments' FP64 reductions are checked for mass and peak speed.
"""
import pytest
import torch

import synthetic
from oracle import lbm as olbm
from oracle import storage as ost

from _helpers import binding, need_gpu, say
from test_gpu_forward import _tolerance_ok

pytestmark = pytest.mark.gpu


def _word_index(grid, st, i, x, y, z):
    """Flat word index of direction i at cell (x, y, z) in the row-interleaved layout."""
    return ((z * grid.ny + y) * grid.Q + i) * grid.nx + x


def _sampled_step_check(B, grid, st, before, after, tau, cells):
    """`after` = one step of `before`: compare at `cells` ([M, 3] x, y, z on the GPU)."""
    x, y, z = cells[:, 0], cells[:, 1], cells[:, 2]
    src, dst = [], []
    for i in range(grid.Q):
        cx, cy = int(st.c[i, 0]), int(st.c[i, 1])
        cz = int(st.c[i, 2]) if grid.D == 3 else 0
        sx, sy, sz = (x - cx) % grid.nx, (y - cy) % grid.ny, (z - cz) % grid.nz
        src.append(_word_index(grid, st, i, sx, sy, sz))
        dst.append(_word_index(grid, st, i, x, y, z))
    words_in = before.view(-1)[torch.stack(src)].cpu()   # [Q, M] pull-streamed words
    got = after.view(-1)[torch.stack(dst)].cpu()
    h = ost.dequantize(words_in, st, grid.storage)
    ref = olbm.bgk_collide(h, tau, st)
    excess, ratio, same = _tolerance_ok(grid.storage, st, got, ost.quantize(ref, st, grid.storage), tau)
    say(f"  sampled step: max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio


def _reductions(B, grid, f):
    red = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
    ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device="cuda")
    B.lbm_moments(grid, f, None, None, None, red, ws)
    return dict(zip(B.RED_NAMES, red.cpu().tolist()))


def _cells(grid, m, seed):
    gen = torch.Generator().manual_seed(seed)
    dims = (grid.nx, grid.ny, grid.nz)
    rnd = torch.stack([torch.randint(0, d, (m,), generator=gen) for d in dims], dim=1)
    corners = torch.tensor([[x, y, z] for x in (0, dims[0] - 1) for y in (0, dims[1] - 1)
                            for z in sorted({0, dims[2] - 1})])
    return torch.cat([rnd, corners]).cuda()


def _run(B, grid, st, u, tau, u0):
    a = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u, a)
    del u
    torch.cuda.empty_cache()
    b = grid.empty_populations()
    B.lbm_step(grid, a, b, tau, None, 3)   # odd: result in b
    B.lbm_step(grid, b, a, tau, None, 1)   # result in a
    torch.cuda.synchronize()
    _sampled_step_check(B, grid, st, b, a, tau, _cells(grid, 4096, 11))
    red = _reductions(B, grid, a)
    say(f"  mass {red['mass']:.6e} of {grid.ncells}, max speed {red['max_speed']:.5f}")
    assert red["nonfinite_cells"] == 0
    assert abs(red["mass"] - grid.ncells) / grid.ncells < 1e-6
    assert abs(red["max_speed"] - u0) < 0.01 * u0
    del a, b
    torch.cuda.empty_cache()


def test_d3q27_f16s_1024_cubed():
    need_gpu()
    B = binding()
    st = olbm.stencil("D3Q27")
    n, u0 = 1024, 0.05
    grid = B.Grid("D3Q27", "f16s", n, n, n)
    say("max size: D3Q27 f16s 1024^3")
    _run(B, grid, st, synthetic.taylor_green_3d_on("cuda", n, n, n, u0), 0.51, u0)


def test_d2q9_f16s_at_the_cell_limit():
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    n, u0 = 46340, 0.05
    assert n * n <= 2 ** 31 - 1
    grid = B.Grid("D2Q9", "f16s", n, n)
    say(f"max size: D2Q9 f16s {n}^2 = {n * n} cells")
    _run(B, grid, st, synthetic.taylor_green_2d_on("cuda", n, n, u0), 0.6, u0)


@pytest.mark.parametrize("kind,ny", [("f32", 4864), ("f16s", 9728)])
def test_two_step_launch_on_planes_past_2_gib(kind, ny):
    """The two-step kernel addresses each z plane through 32-bit offsets from the
    plane's base: on a 4096 x ny x 3 grid whose z plane holds more than 2^31 bytes
    (27 direction rows per grid row), four steps as two two-step launches equal four
    one-step launches bit for bit."""
    need_gpu()
    B = binding()
    nx, nz, u0, tau = 4096, 3, 0.05, 0.6
    grid = B.Grid("D3Q27", kind, nx, ny, nz)
    word = torch.empty((), dtype=grid.word_dtype).element_size()
    plane = 27 * ny * nx * word
    assert 2 ** 31 < plane < 2 ** 32
    assert B.lbm_step_launches(grid, 4) == (0, 2, 0)
    say(f"two-step launch, D3Q27 {kind} {nx}x{ny}x{nz}: {plane / 2 ** 30:.2f} GiB per z plane")
    u = synthetic.taylor_green_3d_on("cuda", nx, ny, nz, u0)
    u[2] = 0.5 * u[0].flip(-1)  # a z velocity too, so every direction carries a deviation
    a = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u, a)
    del u
    ref = a.clone()
    b = grid.empty_populations()
    where = B.lbm_step(grid, a, b, tau, None, 4)
    paired = b if where == 0 else a
    tmp = b if where != 0 else a  # the other buffer: reused for the single steps
    x, y = ref, torch.empty_like(ref)
    for _ in range(4):
        B.lbm_step(grid, x, y, tau, None, 1)
        x, y = y, x
    torch.cuda.synchronize()
    del tmp, y
    same = torch.equal(paired, x)
    say(f"  two-step launches bit-identical to single steps: {same}")
    assert same
    del a, b, ref, x, paired
    torch.cuda.empty_cache()
