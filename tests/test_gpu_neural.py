"""GPU checks of lbm_step_neural (the neural collision of Sec. 3.1: MRT with ghost
relaxation times from a 6-53-3 network evaluated per cell): one-step parity with the
oracle for every storage kind and both activations, the zero network against the
MRT kernel with ghost times 3/2, and a stable multi-step run."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import lbm as olbm
from oracle import neural as onn
from oracle import storage as ost

from _helpers import binding, bits, need_gpu, say
from test_gpu_forward import KINDS, _state, _tolerance_ok

pytestmark = pytest.mark.gpu

SHAPES = [(13, 17), (300, 7), (64, 13)]


def _params(st, s, kind, seed, w2_scale=0.3):
    """Random network whose first layer is scaled to the spread of the inputs, so that
    the pre-activations are of order one (the inputs themselves are ~1e-3)."""
    x = onn.inputs(olbm.stream(ost.dequantize(s, st, kind), st), st).reshape(6, -1)
    spread = x.std(dim=1).numpy() + 1e-30
    g = np.random.default_rng(seed)
    W1 = g.normal(0, 1, (onn.N_HIDDEN, onn.N_IN)) / spread
    b1 = g.normal(0, 0.5, onn.N_HIDDEN)
    W2 = g.normal(0, w2_scale, (onn.N_OUT, onn.N_HIDDEN))
    return torch.from_numpy(np.concatenate([W1.ravel(), b1, W2.ravel()]))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("activation", ["relu", "tanh"])
def test_neural_step_parity(shape, kind, activation):
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    nx, ny = shape
    grid = B.Grid("D2Q9", kind, nx, ny)
    say(f"neural step {kind} {shape} {activation}")
    s = _state(st, (ny, nx), 51, kind)
    p = _params(st, s, kind, 52).to(grid.real_dtype)
    out = grid.empty_populations()
    assert B.lbm_step_neural(grid, grid.to_layout(s).cuda(), out, 0.57, p.cuda(), activation, 1) == 0
    ref = ost.step_emulated(s, 0.57, st, kind, neural=(p.double(), activation))
    excess, ratio, same = _tolerance_ok(kind, st, grid.from_layout(out.cpu()), ref, 0.57)
    say(f"  max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio
    # the network moves the ghost times away from any uniform value
    taus = onn.ghost_taus(olbm.stream(ost.dequantize(s, st, kind), st), p.double(), activation, st)
    assert float(taus.std()) > 0.05


@pytest.mark.parametrize("kind", KINDS)
def test_zero_network_equals_mrt_with_ghost_times_three_halves(kind):
    """All parameters zero: t = 0, tau_6..8 = 3/2; bitwise the uniform MRT step."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    grid = B.Grid("D2Q9", kind, 70, 9)
    s = grid.to_layout(_state(st, (9, 70), 53, kind)).cuda()
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_step_neural(grid, s, a, 0.6, torch.zeros(530, dtype=grid.real_dtype, device="cuda"), "relu", 1)
    B.lbm_step_mrt(grid, s, b, [1, 1, 1, 0.6, 0.6, 0.6, 1.5, 1.5, 1.5], None, 1)
    torch.cuda.synchronize()
    assert torch.equal(bits(a), bits(b))


def _reductions(B, grid, f):
    red = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
    ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device="cuda")
    B.lbm_moments(grid, f, None, None, None, red, ws)
    return dict(zip(B.RED_NAMES, red.cpu().tolist()))


@pytest.mark.parametrize("activation", ["relu", "tanh"])
def test_neural_shear_layer_run_matches_oracle(activation):
    """500 steps of a 128^2 doubly periodic shear layer (Re 5000 at u0 = 0.05) under a
    random network with ghost times between about 1.07 and 2.2: the GPU FP64 and FP32
    velocity fields against the oracle's FP64 run (FP32 emulation drifts 1.2e-6 over
    these steps), and mass conservation."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    n, u0, steps = 128, 0.05, 500
    tau = 0.5 + 3 * u0 * n / 5000
    y = (torch.arange(n, dtype=torch.float64) + 0.5) / n
    Y, X = torch.meshgrid(y, y, indexing="ij")
    ux = torch.where(Y <= 0.5, u0 * torch.tanh(80 * (Y - 0.25)), u0 * torch.tanh(80 * (0.75 - Y)))
    uy = 0.05 * u0 * torch.sin(2 * torch.pi * (X + 0.25))
    u = torch.stack([ux, uy]).contiguous()
    g = np.random.default_rng(54)
    p = torch.from_numpy(np.concatenate([g.normal(0, 1e2, 318), g.normal(0, 0.5, 53), g.normal(0, 0.05, 159)]))
    say(f"neural shear layer {activation}: oracle run")
    f = olbm.equilibrium(torch.ones(n, n, dtype=torch.float64), u, st)
    for _ in range(steps):
        f = onn.step(f, tau, p, activation, st)
    _, u_ref = olbm.state_moments(f, st)
    for kind, bound in (("f64", 1e-11), ("f32", 1e-5)):
        grid = B.Grid("D2Q9", kind, n, n)
        say(f"  gpu {kind}")
        a, b = grid.empty_populations(), grid.empty_populations()
        B.lbm_init_equilibrium(grid, None, u.cuda(), a)
        m0 = _reductions(B, grid, a)["mass"]
        where = B.lbm_step_neural(grid, a, b, tau, p.to(grid.real_dtype).cuda(), activation, steps)
        out = b if where == 0 else a
        red = _reductions(B, grid, out)
        uu = torch.empty((2, n, n), dtype=grid.real_dtype, device="cuda")
        B.lbm_moments(grid, out, None, None, uu)
        err = float((uu.cpu().double() - u_ref).norm() / u_ref.norm())
        say(f"  {kind}: u rel L2 vs oracle {err:.3e}, mass drift {abs(red['mass'] - m0) / m0:.2e}")
        assert red["nonfinite_cells"] == 0
        assert err < bound
        assert abs(red["mass"] - m0) / m0 < (1e-13 if kind == "f64" else 1e-6)


@pytest.mark.parametrize("mode", ["mrt", "mrt_cell", "relu", "tanh"])
def test_full_size_sampled_8192(mode):
    """The MRT and neural steps on the 8192^2 FP32 grid of the benchmark, in its launch
    shape: one step from a state two BGK steps past an equilibrium of random density and
    velocity, compared with the oracle's collision of the streamed populations at 4096
    sampled cells and the four corners (the pull sources gathered from the device
    buffer).  The random start keeps the network's inputs (non-equilibrium moments)
    near 1e-2: on a smooth field they fall to ~1e-5, where the FP32 roundoff of
    h - f^eq on terms of size w_i is a percent of them and a first layer scaled to
    their spread amplifies it past any per-word bound."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    n = 8192
    grid = B.Grid("D2Q9", "f32", n, n)
    say(f"full size 8192^2 {mode}")
    a, b = grid.empty_populations(), grid.empty_populations()
    rho, u = synthetic.random_fields((n, n), 2, 74, drho=0.03, umax=0.06)
    B.lbm_init_equilibrium(grid, rho.cuda(), u.cuda(), a)
    del rho, u
    B.lbm_step(grid, a, b, 0.6, None, 2)  # result in a
    gen = torch.Generator().manual_seed(73)
    cells = torch.cat([torch.randint(0, n, (4096, 2), generator=gen),
                       torch.tensor([[0, 0], [n - 1, 0], [0, n - 1], [n - 1, n - 1]])])
    x, y = cells[:, 0].cuda(), cells[:, 1].cuda()
    src = torch.stack([(((y - int(st.c[i, 1])) % n) * 9 + i) * n + (x - int(st.c[i, 0])) % n for i in range(9)])
    dst = torch.stack([(y * 9 + i) * n + x for i in range(9)])
    h = a.view(-1)[src].cpu().double()  # [9, M]: the populations the compared step collides
    taus = [1.0, 1.0, 1.0, 0.6, 0.6, 0.6, 0.9, 0.8, 0.7]
    if mode in ("mrt", "mrt_cell"):
        tg = None
        if mode == "mrt_cell":
            tg = torch.rand((3, n, n), generator=torch.Generator().manual_seed(72)).float() * 0.6 + 0.55
            taus = taus[:6] + list(tg[:, cells[:, 1], cells[:, 0]].double())
        B.lbm_step_mrt(grid, a, b, [1.0, 1.0, 1.0, 0.6, 0.6, 0.6, 0.9, 0.8, 0.7],
                       None if tg is None else tg.cuda(), 1)
        ref = olbm.mrt_collide(h, taus, st)
        tau_min = 0.55
    else:
        spread = onn.inputs(h, st).std(dim=1).numpy() + 1e-30
        g = np.random.default_rng(71)
        W1 = g.normal(0, 1, (onn.N_HIDDEN, onn.N_IN)) / spread
        p = torch.from_numpy(np.concatenate([W1.ravel(), g.normal(0, 0.5, onn.N_HIDDEN),
                                             g.normal(0, 0.3, onn.N_OUT * onn.N_HIDDEN)])).float()
        B.lbm_step_neural(grid, a, b, 0.6, p.cuda(), mode, 1)
        ref = onn.collide(h, 0.6, p.double(), mode, st)
        tg = onn.ghost_taus(h, p.double(), mode, st)
        assert float(tg.std()) > 0.05  # the network moves the ghost times cell by cell
        tau_min = min(0.6, float(tg.min()))
    torch.cuda.synchronize()
    got = b.view(-1)[dst].cpu()
    excess, ratio, same = _tolerance_ok("f32", st, got, ost.quantize(ref, st, "f32"), tau_min)
    say(f"  max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio
