"""GPU test of lbm_moments_noalloc, the moments entry point whose reduction partials live
in the library's fixed device scratch instead of a caller workspace: its fields and its
FP64 reductions equal lbm_moments' bit for bit, on consecutive calls whose second input
is smaller than the first (the scratch keeps the first call's partials beyond the
second's range, and they must not leak into it)."""
import pytest
import torch

import synthetic
from oracle import lbm as olbm
from oracle import storage as ost
from _helpers import binding, bits, need_gpu, say

# (lattice, storage, (nx, ny, nz), forced, write_fields): each sequence runs in order
SEQUENCES = [
    [("D3Q27", "f32", (130, 37, 21), True, True), ("D3Q27", "f16s", (40, 9, 7), False, True)],
    [("D2Q9", "f64", (700, 90, 1), False, True), ("D2Q9", "bf16s", (300, 7, 1), True, False)],
    [("D3Q19", "f32s", (96, 64, 40), False, False), ("D3Q27", "f64", (17, 13, 11), True, True)],
]


def _inputs(B, lat, kind, shape, forced, seed):
    st = olbm.stencil(lat)
    nx, ny, nz = shape
    spatial = (ny, nx) if lat == "D2Q9" else (nz, ny, nx)
    grid = B.Grid(lat, kind, nx, ny, nz)
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.02, umax=0.05)
    f = olbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, seed + 1, 0.01))
    g = grid.to_layout(ost.quantize(f, st, kind)).cuda()
    F = None
    if forced:
        F = synthetic.random_normal((st.D,) + spatial, seed + 2, 1e-5).to(grid.real_dtype).cuda()
    return grid, g, F


def _moments(B, grid, g, F, fields, noalloc):
    rho = grid.empty_real(0).fill_(float("nan")) if fields else None
    u = grid.empty_real(grid.D).fill_(float("nan")) if fields else None
    red = torch.full((B.NRED,), float("nan"), dtype=torch.float64, device="cuda")
    if noalloc:
        B.lbm_moments_noalloc(grid, g, F, rho, u, red)
    else:
        ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device="cuda")
        B.lbm_moments(grid, g, F, rho, u, red, ws)
    torch.cuda.synchronize()
    return [None if t is None else t.cpu() for t in (rho, u, red)]


@pytest.mark.gpu
@pytest.mark.parametrize("seq", range(len(SEQUENCES)))
def test_noalloc_moments_equal_workspace_moments(seq):
    need_gpu()
    B = binding()
    for k, (lat, kind, shape, forced, fields) in enumerate(SEQUENCES[seq]):
        say(f"lbm_moments_noalloc {lat} {kind} {shape} forced={forced} fields={fields} (call {k + 1})")
        grid, g, F = _inputs(B, lat, kind, shape, forced, 50 + 10 * seq + k)
        got = _moments(B, grid, g, F, fields, noalloc=True)
        ref = _moments(B, grid, g, F, fields, noalloc=False)
        for name, a, b in zip(("rho", "u", "red"), got, ref):
            if b is None:
                assert a is None
                continue
            assert torch.equal(bits(a), bits(b)), (name, lat, kind, shape)
        assert torch.isfinite(got[2]).all() and float(got[2][5]) == 0.0


@pytest.mark.gpu
def test_noalloc_moments_replayed_in_a_graph():
    """The use the entry point exists for: captured once in a HIP graph (no allocation
    inside the capture), replayed several times with eager work and synchronisations in
    between (the state changes between replays); every replay equals an eager
    lbm_moments call on the same state, bit for bit."""
    need_gpu()
    B = binding()
    say("lbm_moments_noalloc under graph capture, D3Q27 f32 (40, 24, 20), 3 replays")
    grid, g, _ = _inputs(B, "D3Q27", "f32", (40, 24, 20), False, 90)
    rho, u = grid.empty_real(0), grid.empty_real(3)
    red = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.lbm_moments_noalloc(grid, g, None, rho, u, red)  # first call on the device: symbol lookup
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            B.lbm_moments_noalloc(grid, g, None, rho, u, red)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for k in range(3):
        g.mul_(1.0 + 1e-3 * (k + 1))  # eager work on the captured input
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ref = _moments(B, grid, g, None, True, noalloc=False)
        for name, a, b in zip(("rho", "u", "red"), (rho.cpu(), u.cpu(), red.cpu()), ref):
            assert torch.equal(bits(a), bits(b)), (name, k)
