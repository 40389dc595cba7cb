"""Two time steps per launch.

For n_steps >= 4, lbm_step runs pairs of steps as one LDS-blocked launch on 3D grids
(FP32 and shifted-FP32 words with nx a multiple of 32 and ny of 8, shifted FP16 with nx
a multiple of 64 and ny of 4, FP64 with nx a multiple of 32 and ny of 4; the first
n_steps mod 4 steps run singly).  Each collision of that kernel is the one-step
kernel's, applied to the same rounded storage words, so the result must equal the same
number of single-step launches bit for bit; the single steps are tied to the oracle
(Eqs. 1-4) by the one-step parity tests, and the last test here ties the paired
launches to the oracle directly.

The shapes cover one tile (every neighbour wraps onto the tile itself), several tiles
in x and y, the smallest nz (3), odd nz and z chunks with a ragged last chunk, padded
rows, D3Q19, D2Q9 (segments of x marching along y; nx a multiple of 64, ny >= 3), and
shapes the kernels do not take (nx or ny off the tile grid, nz < 3), which must run as
single steps with the same results.
"""
import pytest
import torch

import synthetic
from oracle import lbm as olbm
from oracle import storage as ost

from _helpers import binding, bits, need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu

CASES = [  # lattice, (nx, ny, nz), pitch (None = nx)
    ("D3Q27", (32, 8, 3), None),
    ("D3Q27", (64, 16, 20), None),
    ("D3Q27", (96, 24, 37), None),
    ("D3Q27", (32, 40, 5), 96),
    ("D3Q19", (64, 16, 11), None),
    ("D3Q19", (32, 8, 4), 64),
    ("D3Q27", (48, 16, 6), None),  # nx off the tile grid: single steps only
    ("D3Q27", (32, 12, 6), None),  # ny off the tile grid
    ("D3Q27", (32, 8, 2), None),   # nz < 3
    ("D3Q27", (64, 4, 9), 128),    # 2-byte words: one 64 x 4 tile, padded rows
    ("D3Q27", (128, 12, 5), None),
    ("D3Q27", (64, 4, 3), None),     # 2-byte words: 5 planes per block (the three-set
    ("D3Q27", (64, 8, 6), None),     # producer loop's tails), 8 planes
    ("D3Q27", (32, 4, 7), None),     # 8-byte words: one 32 x 4 tile
    ("D3Q27", (64, 12, 4), 96),      # 8-byte words: 32 x 4 tiles, padded rows
    ("D2Q9", (256, 20, 1), None),  # 2D: one 256-cell segment per row, chunks of rows
    ("D2Q9", (64, 37, 1), None),   # 64-cell segments, odd ny
    ("D2Q9", (128, 3, 1), 192),    # ny = 3, padded rows
    ("D2Q9", (96, 8, 1), None),    # nx off the segments: single steps only
    ("D2Q9", (128, 5, 1), 192),    # four steps per launch at the smallest ny
    ("D2Q9", (64, 4, 1), None),    # ny = 4: two steps per launch only
]


def _setup(B, lat, shape, pitch, kind, mode, seed=31):
    st = olbm.stencil(lat)
    nx, ny, nz = shape
    spatial = (ny, nx) if st.D == 2 else (nz, ny, nx)
    grid = B.Grid(lat, kind, nx, ny, nz, pitch)
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.03, umax=0.06)
    f = olbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, seed + 1, 0.02))
    g = grid.to_layout(ost.quantize(f, st, kind)).cuda()
    field = None
    if mode != "none":
        scale = 1e-4 if mode == "guo" else 1e-3
        field = synthetic.random_normal((st.D,) + spatial, seed + 2, scale).to(grid.real_dtype).cuda()
    return st, grid, g, field


def _run(B, grid, g, tau, field, mode, n):
    step = B.lbm_step_shifted if mode == "shift" else B.lbm_step
    a, b = g.clone(), grid.empty_populations()
    where = step(grid, a, b, tau, field, n)
    return (b if where == 0 else a), where


def _singles(B, grid, g, tau, field, mode, n):
    step = B.lbm_step_shifted if mode == "shift" else B.lbm_step
    x, y = g.clone(), grid.empty_populations()
    for _ in range(n):
        assert step(grid, x, y, tau, field, 1) == 0
        x, y = y, x
    return x


@pytest.mark.parametrize("lat,shape,pitch", CASES)
@pytest.mark.parametrize("kind", ["f32", "f32s", "f16s", "bf16s", "f64"])
@pytest.mark.parametrize("mode", ["none", "guo", "shift"])
def test_paired_steps_equal_single_steps(lat, shape, pitch, kind, mode):
    need_gpu()
    B = binding()
    say(f"paired steps {lat} {shape} pitch {pitch} {kind} {mode}")
    st, grid, g, field = _setup(B, lat, shape, pitch, kind, mode)
    for n in (4, 7, 8, 10, 19):
        got, where = _run(B, grid, g, 0.55, field, mode, n)
        assert where == (0 if n % 2 else 1), n
        ref = _singles(B, grid, g, 0.55, field, mode, n)
        same = torch.equal(bits(grid.from_layout(got.cpu())), bits(grid.from_layout(ref.cpu())))
        assert same, f"n_steps={n}"


@pytest.mark.parametrize("kind", ["f32", "f64", "f16s", "bf16s"])
def test_paired_steps_d2q9_full_size_equal_single_steps(kind):
    """8192^2 D2Q9 (the 2D benchmark grid): eight steps as two four-step launches (64
    segments of 128 cells per row) and four
    steps as two two-step launches (32 segments of 256 cells), against single steps,
    every word compared."""
    need_gpu()
    B = binding()
    n = 8192
    grid = B.Grid("D2Q9", kind, n, n)
    say(f"paired steps D2Q9 {kind} {n}^2")
    u = synthetic.taylor_green_2d(n, n, 0.05)
    a = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u.cuda(), a)
    del u
    b = grid.empty_populations()
    assert B.lbm_step(grid, a, b, 0.6, None, 1) == 0
    start = b.clone()
    for n, plan in ((4, (0, 2, 0)), (8, (0, 0, 2))):
        x, y = start.clone(), a
        for _ in range(n):
            B.lbm_step(grid, x, y, 0.6, None, 1)
            x, y = y, x
        ref = x.clone()
        del x
        p, q = start.clone(), y
        assert B.lbm_step_launches(grid, n) == plan
        assert B.lbm_step(grid, p, q, 0.6, None, n) == 1
        torch.cuda.synchronize()
        assert torch.equal(bits(p), bits(ref)), n
        del p, ref


def test_paired_steps_leave_pad_words_alone():
    """The paired launches write live cells only: the pad words of padded rows keep
    what they held (the one-step kernel may overwrite them, the ABI allows either)."""
    need_gpu()
    B = binding()
    st, grid, g, _ = _setup(B, "D3Q27", (32, 8, 6), 64, "f32", "none")
    a, b = g.clone(), grid.empty_populations()
    b.fill_(7.0)
    # four steps = two paired launches, a -> b -> a
    assert B.lbm_step(grid, a, b, 0.6, None, 4) == 1
    rows = b.view(6 * 8, 27, 64)
    assert torch.all(rows[:, :, 32:] == 7.0)
    assert torch.all(torch.isfinite(rows[:, :, :32]))


@pytest.mark.parametrize("kind", ["f32", "f32s", "f16s", "bf16s", "f64"])
def test_paired_steps_full_size_equal_single_steps(kind):
    """256^3 in the launch shape of the benchmark (one chunk of 256 planes per tile,
    tiles of 32 x 8 columns, 64 x 4 for FP16 and BF16, 32 x 4 for FP64): four steps as two paired
    launches against four single steps, every word compared."""
    need_gpu()
    B = binding()
    n = 256
    grid = B.Grid("D3Q27", kind, n, n, n)
    say(f"paired steps full size {kind} {n}^3")
    u = synthetic.taylor_green_3d(n, n, n, 0.05)
    a = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u.cuda(), a)
    del u
    b = grid.empty_populations()
    assert B.lbm_step(grid, a, b, 0.51, None, 1) == 0  # a non-equilibrium state in b
    start = b.clone()
    x, y = b, a
    for _ in range(4):
        B.lbm_step(grid, x, y, 0.51, None, 1)
        x, y = y, x
    ref = x.clone()  # result of the singles (x is b again after 4 steps)
    p, q = start.clone(), y
    assert B.lbm_step(grid, p, q, 0.51, None, 4) == 1
    torch.cuda.synchronize()
    assert torch.equal(bits(p), bits(ref))


@pytest.mark.parametrize("kind,bound", [("f32", 1e-5), ("f32s", 1e-5), ("f16s", 1e-2), ("bf16s", 2e-2), ("f64", 1e-12)])
def test_paired_steps_vs_oracle(kind, bound):
    """A decaying Taylor-Green vortex on 64 x 32 x 24 cells, 200 steps (100 paired
    launches) against the FP64 oracle (FP16, BF16: a sanity bound on the storage noise; FP64:
    rounding order only)."""
    need_gpu()
    B = binding()
    nx, ny, nz = 64, 32, 24
    tau, steps = 0.55, 200
    say(f"paired steps vs oracle {kind} ({nx}, {ny}, {nz}) {steps} steps")
    st = olbm.stencil("D3Q27")
    u0 = synthetic.taylor_green_3d(nx, ny, nz, 0.05)
    g0 = olbm.equilibrium(torch.ones(nz, ny, nx, dtype=torch.float64), u0, st)
    _, u_ref = olbm.state_moments(olbm.run(g0, tau, st, steps), st)
    grid = B.Grid("D3Q27", kind, nx, ny, nz)
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u0.cuda(), a)
    where = B.lbm_step(grid, a, b, tau, None, steps)
    u = grid.empty_real(3)
    B.lbm_moments(grid, b if where == 0 else a, None, None, u, None,
                  torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device="cuda"))
    err = rel_l2(u.cpu().double(), u_ref)
    say(f"  u rel L2 vs oracle: {err:.2e}")
    assert err <= bound


MRT_TAUS = [1.0, 1.0, 1.0, 0.56, 0.56, 0.56, 0.9, 0.8, 0.7]


def _ghost_times(grid, seed):
    """Per-cell ghost relaxation times tau_6..8 in [0.55, 1.25] ([3, ny, nx] reals)."""
    gen = torch.Generator().manual_seed(seed)
    return (0.55 + 0.7 * torch.rand((3, grid.ny, grid.nx), generator=gen, dtype=torch.float64)).to(grid.real_dtype).cuda()


@pytest.mark.parametrize("lat,shape,pitch", [c for c in CASES if c[0] == "D2Q9"])
@pytest.mark.parametrize("kind", ["f32", "f32s", "f16s", "bf16s", "f64"])
@pytest.mark.parametrize("times", ["uniform", "per_cell"])
def test_mrt_multi_step_launches_equal_single_steps(lat, shape, pitch, kind, times):
    """lbm_step_mrt with uniform relaxation times or a per-cell ghost-time field runs
    two or four steps per launch where lbm_step would (the same D2Q9 pipeline with the
    MRT collision of Eq. 5; the field read a row ahead like a force): every word equals
    single MRT steps, for n_steps whose plans mix single, two-step and four-step
    launches."""
    need_gpu()
    B = binding()
    say(f"MRT multi-step {shape} pitch {pitch} {kind} {times}")
    st, grid, g, _ = _setup(B, lat, shape, pitch, kind, "none")
    ghost = _ghost_times(grid, 5) if times == "per_cell" else None
    for n in (4, 7, 8, 10, 19):
        a, b = g.clone(), grid.empty_populations()
        where = B.lbm_step_mrt(grid, a, b, MRT_TAUS, ghost, n)
        assert where == (0 if n % 2 else 1), n
        got = b if where == 0 else a
        x, y = g.clone(), grid.empty_populations()
        for _ in range(n):
            assert B.lbm_step_mrt(grid, x, y, MRT_TAUS, ghost, 1) == 0
            x, y = y, x
        same = torch.equal(bits(grid.from_layout(got.cpu())), bits(grid.from_layout(x.cpu())))
        assert same, f"n_steps={n}"


@pytest.mark.parametrize("kind,times", [("f32", "uniform"), ("f16s", "uniform"), ("f32", "per_cell"),
                                        ("f16s", "per_cell")])
def test_mrt_multi_step_full_size_equal_single_steps(kind, times):
    """8192^2 D2Q9 MRT (uniform or per-cell ghost times): eight steps as two four-step
    launches against single steps."""
    need_gpu()
    B = binding()
    n = 8192
    grid = B.Grid("D2Q9", kind, n, n)
    say(f"MRT multi-step D2Q9 {kind} {n}^2 {times}")
    ghost = _ghost_times(grid, 6) if times == "per_cell" else None
    u = synthetic.taylor_green_2d(n, n, 0.05)
    a = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u.cuda(), a)
    del u
    b = grid.empty_populations()
    assert B.lbm_step_mrt(grid, a, b, MRT_TAUS, ghost, 1) == 0
    start = b.clone()
    x, y = start.clone(), a
    for _ in range(8):
        B.lbm_step_mrt(grid, x, y, MRT_TAUS, ghost, 1)
        x, y = y, x
    ref = x.clone()
    del x
    p, q = start.clone(), y
    assert B.lbm_step_launches(grid, 8) == (0, 0, 2)
    assert B.lbm_step_mrt(grid, p, q, MRT_TAUS, ghost, 8) == 1
    torch.cuda.synchronize()
    assert torch.equal(bits(p), bits(ref))

