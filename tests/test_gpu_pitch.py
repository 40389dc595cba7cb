"""GPU checks of padded population rows (lbm_grid.pitch > nx): every kernel gives the
same bits as on the unpadded layout; the steps may write the pad words (unspecified
values), every other kernel leaves them untouched."""
import pytest
import torch

import synthetic
from oracle import lbm as olbm

from _helpers import binding, bits, need_gpu, say
from test_gpu_forward import _force, _state

pytestmark = pytest.mark.gpu

CASES = [("D3Q27", (37, 6, 5)), ("D3Q19", (70, 5, 3)), ("D2Q9", (255, 9, 1))]


def _spatial(lat, shape):
    nx, ny, nz = shape
    return (ny, nx) if lat == "D2Q9" else (nz, ny, nx)


def _sentinel(t):
    """The buffer filled with a recognisable bit pattern (so untouched pads show up)."""
    t.view(torch.uint8).fill_(0xA5)
    return t


def _pads_untouched(t, nx):
    return bool((t[..., nx:].contiguous().view(torch.uint8) == 0xA5).all())


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("extra", [3, "padded"])
def test_pitched_layout_matches_dense(lat, shape, kind, extra):
    need_gpu()
    B = binding()
    pitched = B.Grid.padded(lat, kind, *shape) if extra == "padded" else B.Grid(lat, kind, *shape, shape[0] + extra)
    _check_layout(B, lat, shape, kind, pitched)


@pytest.mark.parametrize("lat,kind,pitch", [("D3Q27", "f16s", 576), ("D3Q27", "f64", 528), ("D3Q19", "bf16s", 576)])
def test_tuned_layout_matches_dense(lat, kind, pitch):
    """Grid.tuned's extra line on 512-cell rows (two blocks per row): the same bits."""
    need_gpu()
    B = binding()
    shape = (512, 3, 2)
    tuned = B.Grid.tuned(lat, kind, *shape)
    assert tuned.row_pitch == pitch
    _check_layout(B, lat, shape, kind, tuned)


def _check_layout(B, lat, shape, kind, pitched):
    st = olbm.stencil(lat)
    dense = B.Grid(lat, kind, *shape)
    assert pitched.row_pitch > dense.nx
    spatial = _spatial(lat, shape)
    say(f"pitch {lat} {kind} {shape} pitch={pitched.row_pitch}")
    s = _state(st, spatial, 61, kind)
    F = _force(dense, spatial, 62).cuda()

    def both(fn):
        """Run fn(grid, input) on the dense and the pitched layout; compare outputs."""
        outs = []
        for grid in (dense, pitched):
            g_in = grid.to_layout(s).cuda()
            outs.append(fn(grid, g_in))
        return outs

    # init
    u = synthetic.random_fields(spatial, st.D, 63, umax=0.05)[1].cuda()

    def init(g, _):
        out = _sentinel(g.empty_populations())
        B.lbm_init_equilibrium(g, None, u, out)
        return out
    a0, a1 = both(init)
    assert torch.equal(bits(pitched.from_layout(a1)), bits(dense.from_layout(a0)))
    assert _pads_untouched(a1, dense.nx)
    # stream only, and 3 forced steps
    for op in ("stream", "step"):
        def run(g, g_in):
            out = _sentinel(g.empty_populations())
            if op == "stream":
                B.lbm_stream_only(g, g_in, out)
                return out
            tmp = _sentinel(g.empty_populations())
            B.lbm_step(g, g_in, out, 0.57, F, 1)
            B.lbm_step(g, out, tmp, 0.57, F, 1)
            B.lbm_step(g, tmp, out, 0.57, F, 1)
            return out
        o0, o1 = both(run)
        assert torch.equal(bits(pitched.from_layout(o1)), bits(dense.from_layout(o0))), op
        if op == "stream":
            assert _pads_untouched(o1, dense.nx)
    # moments (fields and reductions)
    def moms(g, g_in):
        rho, uu = g.empty_real(0), g.empty_real(g.D)
        red = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
        ws = torch.empty(B.lbm_moments_workspace_size(g), dtype=torch.uint8, device="cuda")
        B.lbm_moments(g, g_in, F, rho, uu, red, ws)
        return rho, uu, red
    m0, m1 = both(moms)
    for x0, x1 in zip(m0, m1):
        assert torch.equal(bits(x0), bits(x1))
    # adjoint (collision-local form with chi input, scatter form, unstream, moments adjoint)
    lam = synthetic.random_normal((st.Q,) + spatial, 64, 1.0).to(dense.real_dtype)

    def adj(g, g_in):
        """(population-layout outputs, force gradients) of every adjoint entry point."""
        lam_in = g.to_layout(lam).cuda()
        pops, grads = [], []
        for mode in ("local", "scatter"):
            out = _sentinel(torch.empty(g.population_shape(), dtype=g.real_dtype, device="cuda"))
            dF = torch.zeros_like(F)
            if mode == "local":
                B.lbm_adjoint_step_local(g, g_in, lam_in, True, out, 0.57, F, dF)
                lam0 = _sentinel(torch.empty_like(out))
                B.lbm_adjoint_unstream(g, out, lam0)
                pops.append(lam0)
            else:
                B.lbm_adjoint_step(g, g_in, lam_in, out, 0.57, F, dF)
                pops.append(out)
            grads.append(dF)
        ma = _sentinel(torch.empty(g.population_shape(), dtype=g.real_dtype, device="cuda"))
        B.lbm_moments_adjoint(g, g_in, F, torch.ones(g.spatial, dtype=g.real_dtype, device="cuda"),
                              torch.ones((g.D,) + g.spatial, dtype=g.real_dtype, device="cuda"), ma, None)
        pops.append(ma)
        return pops, grads
    (p0, d0), (p1, d1) = both(adj)
    for k, (x0, x1) in enumerate(zip(p0, p1)):
        assert torch.equal(bits(pitched.from_layout(x1)), bits(dense.from_layout(x0))), k
        assert _pads_untouched(x1, dense.nx), k
    for x0, x1 in zip(d0, d1):
        assert torch.equal(bits(x0), bits(x1))


def test_pitched_slabs_match_periodic_step():
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.slabs import SlabSet

    st = olbm.stencil("D3Q27")
    grid = B.Grid.padded("D3Q27", "f16s", 37, 5, 7)
    assert grid.row_pitch == 128
    g0 = grid.to_layout(_state(st, (7, 5, 37), 65, "f16s")).cuda()
    a, b = g0.clone(), grid.empty_populations()
    for _ in range(3):
        B.lbm_step(grid, a, b, 0.6, None, 1)
        a, b = b, a
    S = SlabSet(grid, [4, 3])
    S.scatter(g0)
    for t in range(3):
        S.step(0.6, overlap=bool(t % 2))
    torch.cuda.synchronize()
    assert torch.equal(bits(grid.from_layout(S.gather())), bits(grid.from_layout(a)))


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_pitched_rollout_gradient_matches_dense(kind):
    """The checkpointed autograd rollout and the differentiable moments on a padded
    layout: loss, force gradient and the gradient with respect to the initial state
    equal the dense layout's bit for bit (pad entries of the state gradient are zero)."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd import autograd as AG

    st = olbm.stencil("D3Q27")
    shape = (21, 6, 5)
    spatial = (5, 6, 21)
    dense = B.Grid("D3Q27", kind, *shape)
    pitched = B.Grid.padded("D3Q27", kind, *shape)
    s = _state(st, spatial, 66, kind)
    F0 = _force(dense, spatial, 67).cuda()
    out = []
    for grid in (dense, pitched):
        g0 = grid.to_layout(s).cuda().requires_grad_(kind == "f64")
        F = F0.clone().requires_grad_(True)
        gT = AG.rollout(grid, g0, F, 0.57, 7, checkpoint_every=3)
        rho, u = AG.moments(grid, gT, F)
        loss = (u.double() ** 2).sum() + (rho.double() - 1).pow(2).sum()
        loss.backward()
        out.append((loss.detach(), F.grad, g0.grad))
    (l0, f0, s0), (l1, f1, s1) = out
    assert torch.equal(bits(l0), bits(l1))
    assert torch.equal(bits(f0), bits(f1))
    if kind == "f64":
        assert torch.equal(bits(pitched.from_layout(s1)), bits(dense.from_layout(s0)))
        assert bool((s1[..., shape[0]:] == 0).all())
