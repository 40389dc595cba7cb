"""GPU parity of the forward path (stream, init, step, moments) against the FP64
oracle, through the C ABI.

Sizes span several 256-thread blocks with ragged tails in x and in the row count;
the full-size cases run the launch configuration the benchmark times and compare
sampled cells against the oracle's pointwise step.
"""
import math

import pytest
import torch

import synthetic
from oracle import lbm as olbm
from oracle import storage as ost

from _helpers import binding, bits, need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu

KINDS = ["f64", "f32", "f32s", "f16s", "bf16s"]
SHAPES = {  # (nx, ny, nz): ragged x tails and partial row blocks
    "D2Q9": [(13, 17, 1), (300, 7, 1)],
    "D3Q19": [(70, 9, 7)],
    "D3Q27": [(17, 13, 11), (130, 5, 3)],
}
CASES = [(lat, s) for lat, shapes in SHAPES.items() for s in shapes]


def _grid(B, lat, kind, shape):
    return B.Grid(lat, kind, *shape)


def _spatial(lat, shape):
    nx, ny, nz = shape
    return (ny, nx) if lat == "D2Q9" else (nz, ny, nx)


def _tgv3d_errors(B, lattice, n, tau, u0, T, kinds):
    """u relative L2 error of each storage kind against the FP64 oracle after T steps
    of the 3D Taylor-Green vortex."""
    st = olbm.stencil(lattice)
    u = synthetic.taylor_green_3d(n, n, n, u0)
    g = olbm.equilibrium(torch.ones(n, n, n, dtype=torch.float64), u, st)
    _, u_ref = olbm.state_moments(olbm.run(g, tau, st, T), st)
    errs = {}
    for kind in kinds:
        grid = B.Grid(lattice, kind, n, n, n)
        a = grid.empty_populations()
        b = grid.empty_populations()
        B.lbm_init_equilibrium(grid, None, u.cuda(), a)
        where = B.lbm_step(grid, a, b, tau, None, T)
        _, uu = _moments(B, grid, b if where == 0 else a)
        errs[kind] = rel_l2(uu, u_ref)
    return errs


def _state(st, spatial, seed, kind):
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.03, umax=0.06)
    f = olbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, seed + 1, 0.02))
    return ost.quantize(f, st, kind)


def _force(grid, spatial, seed):
    return synthetic.random_normal((grid.D,) + spatial, seed, 1e-4).to(grid.real_dtype)


def _tolerance_ok(kind, st, got, ref, tau=0.57):
    """Elementwise bound of the GPU step against the oracle's emulated step.

    f64: FP64 roundoff of the deviation-form arithmetic.
    f32: 3 ulps of the result, plus omega * 1.5 ulp(w_i): the kernels read an
      unshifted word as W_i + d with binary32 base weights W_i that lie within 1.5 ulp
      of w_i (chosen for exact conservation sums), and the relaxation carries that
      base offset through with factor omega.
    f32s: 1 ulp of the stored deviation plus FP32 roundoff of terms of size w_i.
    f16s/bf16s: 1 ulp of the storage format (the FP32 arithmetic may land on the
    other side of a rounding boundary than exact arithmetic), plus the same FP32
    roundoff floor: where the deviation itself is tiny, one bfloat16 ulp is smaller
    than the absolute error of FP32 arithmetic on terms of size w_i.
    """
    g = ost.dequantize(got.cpu(), st, kind)
    r = ost.dequantize(ref, st, kind)
    diff = (g - r).abs()
    w = st.w.reshape((st.Q,) + (1,) * (g.dim() - 1))
    if kind == "f64":
        bound = 1e-15 * torch.ones_like(r)
    elif kind == "f32":
        bound = 3 * ost.ulp(r, kind) + (1.0 / tau) * 1.5 * ost.ulp(w.expand_as(r), kind)
    else:
        dev_r = ost.quantize(r, st, kind).double()
        dev_g = got.cpu().double()
        u = torch.maximum(ost.ulp(dev_r, kind), ost.ulp(dev_g, kind))
        bound = u + 8 * 2.0 ** -24 * w
    excess = diff - bound
    same = float((bits(got.cpu()) == bits(ost.quantize(r, st, kind))).double().mean())
    return float(excess.max()), float((diff / bound.clamp(min=1e-300)).max()), same


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", KINDS)
def test_stream_only_bit_exact(lat, shape, kind):
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = _grid(B, lat, kind, shape)
    spatial = _spatial(lat, shape)
    say(f"stream_only {lat} {kind} {shape}")
    s = _state(st, spatial, 3, kind)
    out = grid.empty_populations()
    B.lbm_stream_only(grid, grid.to_layout(s).cuda(), out)
    ref = ost.stream_stored(s, st)
    assert torch.equal(bits(grid.from_layout(out.cpu())), bits(ref))


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", KINDS)
def test_init_equilibrium(lat, shape, kind):
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = _grid(B, lat, kind, shape)
    spatial = _spatial(lat, shape)
    say(f"init {lat} {kind} {shape}")
    rho, u = synthetic.random_fields(spatial, st.D, 5, drho=0.05, umax=0.08)
    out = grid.empty_populations()
    B.lbm_init_equilibrium(grid, rho.cuda(), u.cuda(), out)
    _check_init(grid.from_layout(out.cpu()), ost.quantize(olbm.equilibrium(rho, u, st), st, kind), st, kind)
    # rho = None means rho = 1
    B.lbm_init_equilibrium(grid, None, u.cuda(), out)
    ones = torch.ones(spatial, dtype=torch.float64)
    _check_init(grid.from_layout(out.cpu()), ost.quantize(olbm.equilibrium(ones, u, st), st, kind), st, kind)


def _check_init(got, ref, st, kind):
    """One rounding of an FP64 value: at most one storage ulp from the oracle's own
    rounding of its FP64 equilibrium (FP64: a few ulps of roundoff).  Unshifted FP32
    stores W_i + (f^eq_i - w_i) with the kernels' binary32 base W_i, which lies within
    1.1 ulp of w_i, so it may sit up to 2 ulps further away."""
    diff = (got.double() - ref.double()).abs()
    mag = ref.double().abs()
    if kind == "f64":
        tol = 4 * 2.0 ** -52 * mag
    elif kind == "f32":
        tol = 3 * ost.ulp(mag, kind)
    else:
        tol = ost.ulp(mag, kind)
    assert bool((diff <= tol).all()), float((diff / tol).max())


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("forced", [False, True])
def test_one_step_parity(lat, shape, kind, forced):
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = _grid(B, lat, kind, shape)
    spatial = _spatial(lat, shape)
    tau = 0.57
    say(f"step {lat} {kind} {shape} forced={forced}")
    s = _state(st, spatial, 11, kind)
    F = _force(grid, spatial, 12) if forced else None
    out = grid.empty_populations()
    rc = B.lbm_step(grid, grid.to_layout(s).cuda(), out, tau, None if F is None else F.cuda(), 1)
    assert rc == 0
    ref = ost.step_emulated(s, tau, st, kind, None if F is None else F.double())
    excess, ratio, same = _tolerance_ok(kind, st, grid.from_layout(out.cpu()), ref, tau)
    say(f"  max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", KINDS)
def test_shifted_step_parity(lat, shape, kind):
    """lbm_step_shifted (equilibrium at u + du, the flow-control forcing) against the
    oracle's shifted step."""
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = _grid(B, lat, kind, shape)
    spatial = _spatial(lat, shape)
    tau = 0.57
    say(f"shifted step {lat} {kind} {shape}")
    s = _state(st, spatial, 14, kind)
    du = synthetic.random_normal((grid.D,) + spatial, 15, 1e-3).to(grid.real_dtype)
    out = grid.empty_populations()
    assert B.lbm_step_shifted(grid, grid.to_layout(s).cuda(), out, tau, du.cuda(), 1) == 0
    ref = ost.step_emulated(s, tau, st, kind, du=du.double())
    excess, ratio, same = _tolerance_ok(kind, st, grid.from_layout(out.cpu()), ref, tau)
    say(f"  max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio


MRT_TAUS = [1.0, 1.0, 1.0, 0.57, 0.57, 0.57, 0.9, 1.3, 1.2]


@pytest.mark.parametrize("shape", SHAPES["D2Q9"])
@pytest.mark.parametrize("kind", KINDS)
def test_mrt_step_parity(shape, kind):
    """lbm_step_mrt (D2Q9, Dellar basis, Eq. 5) against the oracle's MRT step."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    grid = _grid(B, "D2Q9", kind, shape)
    spatial = _spatial("D2Q9", shape)
    say(f"mrt step {kind} {shape}")
    s = _state(st, spatial, 16, kind)
    out = grid.empty_populations()
    assert B.lbm_step_mrt(grid, grid.to_layout(s).cuda(), out, MRT_TAUS, None, 1) == 0
    ref = ost.step_emulated(s, 0.57, st, kind, mrt_taus=MRT_TAUS)
    excess, ratio, same = _tolerance_ok(kind, st, grid.from_layout(out.cpu()), ref, 0.57)
    say(f"  max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_mrt_per_cell_ghost_times(kind):
    """Per-cell tau_6..8 (the neural collision's outputs) against the oracle with the
    same fields."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    shape = (37, 11, 1)
    grid = _grid(B, "D2Q9", kind, shape)
    spatial = _spatial("D2Q9", shape)
    s = _state(st, spatial, 17, kind)
    ghost = (0.55 + torch.rand((3,) + spatial, generator=torch.Generator().manual_seed(5), dtype=torch.float64))
    ghost = ghost.to(grid.real_dtype)
    taus = MRT_TAUS[:6] + [ghost[0].double(), ghost[1].double(), ghost[2].double()]
    out = grid.empty_populations()
    B.lbm_step_mrt(grid, grid.to_layout(s).cuda(), out, MRT_TAUS, ghost.cuda(), 1)
    ref = ost.step_emulated(s, 0.57, st, kind, mrt_taus=taus)
    excess, ratio, same = _tolerance_ok(kind, st, grid.from_layout(out.cpu()), ref, 0.57)
    assert excess <= 0, ratio


def test_mrt_equal_times_match_bgk_kernel():
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    grid = B.Grid("D2Q9", "f64", 40, 23)
    s = grid.to_layout(_state(st, (23, 40), 18, "f64")).cuda()
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_step_mrt(grid, s, a, [0.61] * 9, None, 1)
    B.lbm_step(grid, s, b, 0.61, None, 1)
    assert float((a - b).abs().max()) < 1e-15


@pytest.mark.parametrize("kind", KINDS)
def test_rest_state_bit_exact(kind):
    need_gpu()
    B = binding()
    grid = B.Grid("D3Q27", kind, 19, 6, 5)
    say(f"rest {kind}")
    u = torch.zeros((3, 5, 6, 19), dtype=torch.float64, device="cuda")  # [D, nz, ny, nx]
    a = grid.empty_populations()
    b = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u, a)
    first = a.clone()
    where = B.lbm_step(grid, a, b, 0.53, None, 7)
    res = b if where == 0 else a
    assert torch.equal(bits(res), bits(first))
    if kind.endswith("s"):
        assert int(torch.count_nonzero(bits(res))) == 0


def test_ping_pong_return_value():
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    grid = B.Grid("D2Q9", "f64", 11, 9)
    s = _state(st, (9, 11), 21, "f64")
    a, b = grid.to_layout(s).cuda(), grid.empty_populations()
    assert B.lbm_step(grid, a, b, 0.8, None, 2) == 1
    ref = olbm.run(s, 0.8, st, 2)
    assert float((grid.from_layout(a.cpu()) - ref).abs().max()) < 1e-15
    assert B.lbm_step(grid, a, b, 0.8, None, 3) == 0
    ref = olbm.run(ref, 0.8, st, 3)
    assert float((grid.from_layout(b.cpu()) - ref).abs().max()) < 1e-15


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("forced", [False, True])
def test_moments_parity(lat, shape, kind, forced):
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = _grid(B, lat, kind, shape)
    spatial = _spatial(lat, shape)
    say(f"moments {lat} {kind} {shape} forced={forced}")
    s = _state(st, spatial, 31, kind)
    F = _force(grid, spatial, 32) if forced else None
    rho = grid.empty_real(0)
    u = grid.empty_real(grid.D)
    red = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
    ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device="cuda")
    f = grid.to_layout(s).cuda()
    Fd = None if F is None else F.cuda()
    B.lbm_moments(grid, f, Fd, rho, u, red, ws)
    # a call with the reductions alone walks the cells in other blocks: the same maximum,
    # minimum and count, sums equal to FP64 rounding
    red_only = torch.full((B.NRED,), float("nan"), dtype=torch.float64, device="cuda")
    B.lbm_moments(grid, f, Fd, None, None, red_only, ws)
    red_only = red_only.cpu()
    r_ref, u_ref = olbm.state_moments(ost.dequantize(s, st, kind), st, None if F is None else F.double())
    tol = 1e-14 if kind == "f64" else 2e-6
    assert float((rho.cpu().double() - r_ref).abs().max()) < tol
    assert float((u.cpu().double() - u_ref).abs().max()) < tol
    red = red.cpu()
    mass = float(r_ref.sum())
    mom = (r_ref * u_ref).sum(dim=tuple(range(1, st.D + 1)))
    ke = float(0.5 * (u_ref * u_ref).sum())
    rtol = 1e-13 if kind == "f64" else 1e-6
    assert abs(float(red[0]) - mass) <= rtol * mass
    for a in range(st.D):
        assert abs(float(red[1 + a]) - float(mom[a])) <= rtol * mass * 0.1
    assert abs(float(red[4]) - ke) <= rtol * 10 * ke
    assert float(red[5]) == 0.0
    assert abs(float(red[6]) - float(u_ref.norm(dim=0).max())) <= tol * 10
    assert abs(float(red[7]) - float(r_ref.min())) <= tol * 10
    assert torch.equal(red_only[5:], red[5:])
    assert float((red_only[:5] - red[:5]).abs().max()) <= 1e-13 * mass


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("forced", [False, True])
def test_moments_fields_only_equal_fields_with_reductions(lat, shape, kind, forced):
    """Calls without reductions take the fields-only kernel, calls with them the reducing
    one (whose blocks may walk several blocks of cells): rho and u agree bit for bit
    (both start as NaN, so a cell either kernel skipped would show), also where planted
    NaN and inf words make cells non-finite."""
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = _grid(B, lat, kind, shape)
    spatial = _spatial(lat, shape)
    say(f"moments fields-only vs reductions {lat} {kind} {shape} forced={forced}")
    s = _state(st, spatial, 33, kind)
    s.view(st.Q, -1)[3, 5] = float("nan")
    s.view(st.Q, -1)[0, -1] = float("inf")
    f = grid.to_layout(s).cuda()
    F = _force(grid, spatial, 34).cuda() if forced else None
    outs = []
    for with_red in (False, True):
        rho = grid.empty_real(0).fill_(float("nan"))
        u = grid.empty_real(grid.D).fill_(float("nan"))
        if with_red:
            red = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
            ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device="cuda")
            B.lbm_moments(grid, f, F, rho, u, red, ws)
            assert float(red[5].cpu()) == 2.0
        else:
            B.lbm_moments(grid, f, F, rho, u)
        outs.append((rho.cpu(), u.cpu()))
    assert torch.equal(bits(outs[0][0]), bits(outs[1][0]))
    assert torch.equal(bits(outs[0][1]), bits(outs[1][1]))
    finite = torch.isfinite(outs[0][0]).reshape(-1)
    assert int((~finite).sum()) == 2  # exactly the two planted cells


def test_nonfinite_cells_are_counted():
    need_gpu()
    B = binding()
    st = olbm.stencil("D3Q27")
    grid = B.Grid("D3Q27", "f32", 20, 7, 3)
    s = _state(st, (3, 7, 20), 41, "f32")
    s[5, 1, 2, 3] = float("nan")
    s[0, 2, 6, 19] = float("inf")
    red = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
    ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device="cuda")
    B.lbm_moments(grid, grid.to_layout(s).cuda(), None, None, None, red, ws)
    assert float(red[5].cpu()) == 2.0


@pytest.mark.parametrize("kind", KINDS)
def test_determinism(kind):
    need_gpu()
    B = binding()
    grid = B.Grid("D3Q27", kind, 33, 9, 7)
    u = synthetic.random_fields((7, 9, 33), 3, 51, umax=0.05)[1]
    outs = []
    for _ in range(2):
        a = grid.empty_populations()
        b = grid.empty_populations()
        B.lbm_init_equilibrium(grid, None, u.cuda(), a)
        where = B.lbm_step(grid, a, b, 0.52, None, 25)
        outs.append((b if where == 0 else a).clone())
    assert torch.equal(bits(outs[0]), bits(outs[1]))


def _tgv2d_run(B, kind, steps):
    n, tau, u0 = 64, 0.6, 0.05
    grid = B.Grid("D2Q9", kind, n, n)
    u = synthetic.taylor_green_2d(n, n, u0)
    a = grid.empty_populations()
    b = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u.cuda(), a)
    where = B.lbm_step(grid, a, b, tau, None, steps)
    res = b if where == 0 else a
    _, uu = _moments(B, grid, res)
    return uu


def _moments(B, grid, f):
    rho = grid.empty_real(0)
    u = grid.empty_real(grid.D)
    B.lbm_moments(grid, f, None, rho, u)
    return rho.cpu().double(), u.cpu().double()


def test_tgv2d_1000_steps_vs_oracle_and_closed_form():
    """64x64 D2Q9 Taylor-Green vortex, tau = 0.6, u0 = 0.05, 1000 steps."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    n, tau, u0, T = 64, 0.6, 0.05, 1000
    say("tgv2d 1000 steps")
    g = olbm.equilibrium(torch.ones(n, n, dtype=torch.float64), synthetic.taylor_green_2d(n, n, u0), st)
    _, u_ref = olbm.state_moments(olbm.run(g, tau, st, T), st)
    u64 = _tgv2d_run(B, "f64", T)
    u32 = _tgv2d_run(B, "f32", T)
    u32s = _tgv2d_run(B, "f32s", T)
    e64, e32, e32s = rel_l2(u64, u_ref), rel_l2(u32, u_ref), rel_l2(u32s, u_ref)
    say(f"  u rel L2 vs oracle: f64 {e64:.3e} f32 {e32:.3e} f32s {e32s:.3e}")
    assert e64 <= 1e-11
    assert e32 <= 1e-5
    assert e32s <= 1e-5
    b = synthetic.taylor_green_2d(n, n, 1.0)[0]
    amp = float((u64[0] * b).sum() / (b * b).sum()) / u0
    nu = (tau - 0.5) / 3
    assert abs(amp / math.exp(-2 * nu * (2 * math.pi / n) ** 2 * T) - 1) < 1e-2


def test_tgv3d_vs_oracle():
    """D3Q27 Taylor-Green vortex, 32^3, tau = 0.51, u0 = 0.05, 1000 steps."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D3Q27")
    n, tau, u0, T = 32, 0.51, 0.05, 1000
    say("tgv3d 32^3 1000 steps")
    u = synthetic.taylor_green_3d(n, n, n, u0)
    _, u_ref = olbm.state_moments(olbm.run(olbm.equilibrium(torch.ones(n, n, n, dtype=torch.float64), u, st),
                                            tau, st, T), st)
    errs = {}
    for kind in KINDS:
        grid = B.Grid("D3Q27", kind, n, n, n)
        a = grid.empty_populations()
        b = grid.empty_populations()
        B.lbm_init_equilibrium(grid, None, u.cuda(), a)
        where = B.lbm_step(grid, a, b, tau, None, T)
        _, uu = _moments(B, grid, b if where == 0 else a)
        errs[kind] = rel_l2(uu, u_ref)
    say("  u rel L2 vs oracle: " + " ".join(f"{k} {v:.3e}" for k, v in errs.items()))
    assert errs["f64"] <= 1e-11
    assert errs["f32"] <= 1e-5
    assert errs["f32s"] <= 1e-5
    assert errs["f16s"] <= 1e-2 and errs["bf16s"] <= 1e-1  # reported; loose sanity bounds


def test_tgv3d_d3q19_vs_oracle():
    """D3Q19 Taylor-Green vortex (the paper's 3D benchmark lattice), 24^3, tau = 0.51,
    u0 = 0.05, 500 steps."""
    need_gpu()
    B = binding()
    say("tgv3d D3Q19 24^3 500 steps")
    errs = _tgv3d_errors(B, "D3Q19", 24, 0.51, 0.05, 500, ["f64", "f32", "f16s"])
    say("  u rel L2 vs oracle: " + " ".join(f"{k} {v:.3e}" for k, v in errs.items()))
    assert errs["f64"] <= 1e-11
    assert errs["f32"] <= 1e-5
    assert errs["f16s"] <= 1e-2


DEGENERATE = [("D3Q27", (1, 1, 1)), ("D3Q27", (1, 5, 3)), ("D3Q27", (7, 1, 1)), ("D3Q27", (3, 1, 4)),
              ("D3Q19", (2, 1, 1)), ("D2Q9", (1, 1, 1)), ("D2Q9", (64, 1, 1)), ("D2Q9", (1, 70, 1))]


@pytest.mark.parametrize("lat,shape", DEGENERATE)
@pytest.mark.parametrize("kind", ["f64", "f32", "f16s"])
def test_degenerate_grids(lat, shape, kind):
    """Grids one cell thick in some direction (a population streams back onto its own
    cell there), including a single cell: stream-only bit-exact and one step within
    the usual bound."""
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = _grid(B, lat, kind, shape)
    spatial = _spatial(lat, shape)
    say(f"degenerate {lat} {kind} {shape}")
    s = _state(st, spatial, 19, kind)
    out = grid.empty_populations()
    B.lbm_stream_only(grid, grid.to_layout(s).cuda(), out)
    assert torch.equal(bits(grid.from_layout(out.cpu())), bits(ost.stream_stored(s, st)))
    B.lbm_step(grid, grid.to_layout(s).cuda(), out, 0.57, None, 1)
    ref = ost.step_emulated(s, 0.57, st, kind)
    excess, ratio, same = _tolerance_ok(kind, st, grid.from_layout(out.cpu()), ref, 0.57)
    assert excess <= 0, ratio


def test_tau_one_writes_the_equilibrium():
    """tau = 1 (omega = 1): one step replaces the streamed populations by their
    equilibrium, i.e. lbm_init_equilibrium of the streamed moments."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D3Q27")
    grid = B.Grid("D3Q27", "f64", 19, 7, 6)
    s = _state(st, (6, 7, 19), 20, "f64")
    out = grid.empty_populations()
    B.lbm_step(grid, grid.to_layout(s).cuda(), out, 1.0, None, 1)
    h = olbm.stream(s, st)
    feq = olbm.equilibrium(olbm.density(h), olbm.momentum(h, st) / olbm.density(h), st)
    assert float((grid.from_layout(out.cpu()) - feq).abs().max()) < 1e-15


def test_large_2d_grid_sampled():
    """A 8192 x 8192 D2Q9 FP32 grid (67M cells, 2.4 GB per buffer): one step from a
    Taylor-Green start plus 2 steps, compared at sampled cells."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D2Q9")
    n = 8192
    grid = B.Grid("D2Q9", "f32", n, n)
    say("large 2D 8192^2 f32")
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, synthetic.taylor_green_2d(n, n, 0.05).cuda(), a)
    B.lbm_step(grid, a, b, 0.6, None, 2)  # result in a
    B.lbm_step(grid, a, b, 0.6, None, 1)  # result in b
    gen = torch.Generator().manual_seed(8)
    cells = torch.cat([torch.randint(0, n, (2048, 2), generator=gen),
                       torch.tensor([[0, 0], [n - 1, 0], [0, n - 1], [n - 1, n - 1]])])
    g_in = a.cpu().permute(1, 0, 2)  # [Q, y, x] view
    ref = ost.step_at_cells_emulated(g_in, 0.6, st, "f32", cells)
    got = b.cpu()[cells[:, 1], :, cells[:, 0]].T
    excess, ratio, same = _tolerance_ok("f32", st, got, ost.quantize(ref, st, "f32"), 0.6)
    assert excess <= 0, ratio


# nx a multiple of the block's row segment (64, 128 or 256 cells) with row counts that
# leave the last block of 4 or 2 rows partly empty
ALIGNED = [("D3Q27", (64, 7, 5)), ("D3Q27", (128, 5, 3)), ("D3Q27", (256, 3, 2)), ("D3Q27", (384, 3, 2)),
           ("D3Q27", (192, 3, 3)), ("D3Q19", (64, 5, 3)), ("D3Q19", (256, 3, 3)), ("D2Q9", (64, 13, 1)),
           ("D2Q9", (256, 5, 1)), ("D2Q9", (384, 7, 1))]


@pytest.mark.parametrize("lat,shape", ALIGNED)
@pytest.mark.parametrize("kind", ["f32", "f32s", "f16s", "bf16s"])
@pytest.mark.parametrize("mode", ["none", "guo", "shift"])
def test_aligned_shapes_step_parity(lat, shape, kind, mode):
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    grid = B.Grid(lat, kind, *shape)
    spatial = _spatial(lat, shape)
    tau = 0.57
    say(f"aligned step {lat} {kind} {shape} {mode}")
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


@pytest.mark.parametrize("kind,n,tuned", [("f32", 256, False), ("f64", 256, False), ("f16s", 256, False),
                                          ("bf16s", 256, False), ("f32", 384, False), ("f16s", 384, False),
                                          ("f16s", 512, False), ("f16s", 512, True)])
def test_full_size_sampled(kind, n, tuned):
    """Full-size grids in the benchmark's launch shape: one step compared with the
    oracle's pointwise step at 4096 sampled cells (and all 8 corners of the box).  The
    tuned case takes Grid.tuned's 576-word rows, as the 512^3 workloads do (row bases
    beyond 2^32 words)."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D3Q27")
    grid = B.Grid.tuned("D3Q27", kind, n, n, n) if tuned else B.Grid("D3Q27", kind, n, n, n)
    tau = 0.51
    say(f"full size {kind} {n}^3 pitch {grid.row_pitch}")
    u = synthetic.taylor_green_3d(n, n, n, 0.05)
    a = grid.empty_populations()
    b = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u.cuda(), a)
    del u
    B.lbm_step(grid, a, b, tau, None, 3)  # non-equilibrium state in b
    B.lbm_step(grid, b, a, tau, None, 1)
    torch.cuda.synchronize()
    gen = torch.Generator().manual_seed(7)
    cells = torch.randint(0, n, (4096, 3), generator=gen)
    corners = torch.tensor([[x, y, z] for x in (0, n - 1) for y in (0, n - 1) for z in (0, n - 1)])
    cells = torch.cat([cells, corners])
    g_in = b.cpu()[..., :n].permute(2, 0, 1, 3)  # a [Q, z, y, x] view of the row-interleaved words
    ref = ost.step_at_cells_emulated(g_in, tau, st, kind, cells)
    del g_in
    out = a.cpu()
    got = out[cells[:, 2], cells[:, 1], :, cells[:, 0]].T
    excess, ratio, same = _tolerance_ok(kind, st, got, ost.quantize(ref, st, kind), tau)
    say(f"  max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio


@pytest.mark.parametrize("kind", ["f32", "f16s"])
def test_full_size_moments_sampled(kind):
    """Moments of the 256^3 D3Q27 grid the benchmark times, both kernels: rho, u at 4096
    sampled cells and the 8 corners against the oracle's Eq. 4 on the stored words;
    the FP64 reductions against FP64 sums of the returned fields (max and min exact),
    and those of a call without fields against them; the fields-only kernel bit for bit
    equal to the reduction kernel's fields."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D3Q27")
    n, Q = 256, 27
    grid = B.Grid("D3Q27", kind, n, n, n)
    say(f"full-size moments {kind}")
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, synthetic.taylor_green_3d_on("cuda", n, n, n, 0.05), a)
    B.lbm_step(grid, a, b, 0.51, None, 2)  # result in a
    del b
    rho, u = grid.empty_real(0), grid.empty_real(3)
    red = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
    ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device="cuda")
    B.lbm_moments(grid, a, None, rho, u, red, ws)
    rho2, u2 = grid.empty_real(0), grid.empty_real(3)
    B.lbm_moments(grid, a, None, rho2, u2)
    red_only = torch.zeros(B.NRED, dtype=torch.float64, device="cuda")
    B.lbm_moments(grid, a, None, None, None, red_only, ws)
    torch.cuda.synchronize()
    assert torch.equal(bits(rho), bits(rho2)) and torch.equal(bits(u), bits(u2))
    cg = torch.Generator().manual_seed(66)
    cells = torch.cat([torch.randint(0, n, (4096, 3), generator=cg),
                       torch.tensor([[x, y, z] for x in (0, n - 1) for y in (0, n - 1) for z in (0, n - 1)])])
    x, y, z = (cells[:, k].cuda() for k in range(3))
    words = torch.stack([a.view(-1)[(((z * n + y) * Q + i) * n + x)] for i in range(Q)]).cpu()
    f = ost.dequantize(words, st, kind)  # [Q, M] FP64
    flat = (z * n + y) * n + x
    r_ref, u_ref = olbm.density(f), olbm.velocity(f, st)
    assert float((rho.view(-1)[flat].cpu().double() - r_ref).abs().max()) < 2e-6
    assert float((u.view(3, -1)[:, flat].cpu().double() - u_ref).abs().max()) < 2e-6
    rd, ud = rho.double(), u.double()
    red = red.cpu()
    usq = (ud * ud).sum(0)
    mass, mom, ke = float(rd.sum()), (rd * ud).sum(dim=(1, 2, 3)).cpu(), float(0.5 * usq.sum())
    # the kernel sums N + sum(drho) in FP64; each rho field value is 1 + drho rounded to
    # FP32, off by at most 2^-24 per cell
    assert abs(float(red[0]) - mass) <= 2.0 ** -24 * n ** 3 + 1e-12 * mass
    for k in range(3):  # the same FP64 products, summed in another order
        assert abs(float(red[1 + k]) - float(mom[k])) <= 1e-12 * mass
    assert abs(float(red[4]) - ke) <= 1e-11 * ke
    assert float(red[5]) == 0.0
    umax = float(usq.max().sqrt())  # the kernel's |u|^2 may round once differently (FMA)
    assert abs(float(red[6]) - umax) <= 1e-15 * umax
    assert float(red[7]) == float(rd.min())
    red_only = red_only.cpu()  # other blocks, other order: sums to FP64 rounding, the rest exact
    assert torch.equal(red_only[5:], red[5:])
    assert float((red_only[:5] - red[:5]).abs().max()) <= 1e-12 * mass


@pytest.mark.parametrize("lat,kind,mode", [("D3Q19", "f32", "none"), ("D3Q19", "f16s", "none"), ("D3Q27", "f32", "guo"),
                                           ("D3Q27", "f16s", "guo"), ("D3Q27", "f32", "shift"), ("D3Q27", "f16s", "shift")])
def test_full_size_sampled_d3q19_and_forced(lat, kind, mode):
    """The other 256^3 steps the benchmark times, in its launch shape: D3Q19, and D3Q27
    with a Guo body force or a velocity-shift field (random, 1e-5): one step from a
    Taylor-Green state two steps old, against the oracle's collision of the gathered
    stored words at 4096 sampled cells and the 8 corners."""
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    n, Q, tau = 256, st.Q, 0.51
    grid = B.Grid(lat, kind, n, n, n)
    say(f"full size {lat} {kind} {mode}")
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, synthetic.taylor_green_3d_on("cuda", n, n, n, 0.05), a)
    B.lbm_step(grid, a, b, tau, None, 2)  # result in a
    field = None
    if mode != "none":
        gen = torch.Generator(device="cuda").manual_seed(67)
        field = 1e-5 * torch.randn((3, n, n, n), generator=gen, device="cuda")
    if mode == "shift":
        B.lbm_step_shifted(grid, a, b, tau, field, 1)
    else:
        B.lbm_step(grid, a, b, tau, field, 1)
    torch.cuda.synchronize()
    cg = torch.Generator().manual_seed(68)
    cells = torch.cat([torch.randint(0, n, (4096, 3), generator=cg),
                       torch.tensor([[x, y, z] for x in (0, n - 1) for y in (0, n - 1) for z in (0, n - 1)])])
    x, y, z = (cells[:, k].cuda() for k in range(3))
    c = st.c.to(torch.int64)

    def word(i, dx, dy, dz):
        return ((((z + dz) % n) * n + (y + dy) % n) * Q + i) * n + (x + dx) % n

    h = ost.dequantize(torch.stack([a.view(-1)[word(i, -c[i, 0], -c[i, 1], -c[i, 2])] for i in range(Q)]).cpu(),
                       st, kind)
    got = torch.stack([b.view(-1)[word(i, 0, 0, 0)] for i in range(Q)]).cpu()
    Fc = None
    if field is not None:
        flat = (z * n + y) * n + x
        Fc = torch.stack([field[k].reshape(-1)[flat] for k in range(3)]).cpu().double()
    ref = olbm.bgk_collide_shifted(h, tau, st, Fc) if mode == "shift" else olbm.bgk_collide(h, tau, st, Fc)
    excess, ratio, same = _tolerance_ok(kind, st, got, ost.quantize(ref, st, kind), tau)
    say(f"  max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio
