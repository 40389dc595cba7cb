"""CPU tests of the host-side schedules above the C ABI: the launch sequence of the
checkpointed rollout's backward pass (which adjoint steps run singly and which in
pairs), and the z-slab bookkeeping with two ghost planes.  The library calls of the
rollout are replaced by recorders, so no GPU is needed."""
import pytest
import torch


@pytest.fixture(scope="module")
def B():
    from paper_2106_12929_amd import binding

    return binding


class _Recorder:
    """Stands in for the step and adjoint entry points.  It labels every population
    buffer with the time step it holds (a step call writes label(a) + n into the output
    it leaves the result in; an unlabelled input is the initial state) and records the
    adjoint calls by those labels; no arithmetic is done."""

    def __init__(self):
        self.ids = {}
        self.calls = []

    def label(self, t):
        return self.ids.get(t.data_ptr(), 0)

    def step(self, grid, a, b, tau, F, n):
        where = 0 if n % 2 else 1  # the library's ping-pong: odd n ends in b
        self.ids[(b if where == 0 else a).data_ptr()] = self.label(a) + n
        return where

    def adjoint(self, grid, g, adj, is_chi, out, tau, F, dF):
        self.calls.append(("adj1", self.label(g), bool(is_chi)))

    def adjoint2(self, grid, g_t, g_tm1, chi, out, tau, F, dF):
        self.calls.append(("adj2", self.label(g_t), self.label(g_tm1)))

    def unstream(self, grid, chi, lam):
        self.calls.append(("unstream",))


@pytest.mark.parametrize("n,K,pair", [(11, 4, True), (11, 3, True), (12, 5, True), (10, 10, True), (7, 1, True),
                                      (9, 4, False), (1, 3, True)])
def test_rollout_backward_covers_every_step_once(B, monkeypatch, n, K, pair):
    """Every step t = n-1 .. 0 is differentiated exactly once, last to first, at the
    state of that step; the first adjoint step (the loss gradient comes in as lambda,
    not chi) runs singly; pairs (t, t-1) only within one checkpoint segment and only
    when pairing is on; a lone chi step only at a segment's first step."""
    from paper_2106_12929_amd import autograd as AG

    grid = B.Grid("D3Q27", "f32", 32, 8, 3)  # on the two-step tiles: pairing is available
    assert B.lbm_adjoint_step2_available(grid)
    rec = _Recorder()
    monkeypatch.setattr(AG.B, "lbm_step", rec.step)
    monkeypatch.setattr(AG.B, "lbm_adjoint_step_local", rec.adjoint)
    monkeypatch.setattr(AG.B, "lbm_adjoint_step2_local", rec.adjoint2)
    monkeypatch.setattr(AG.B, "lbm_adjoint_unstream", rec.unstream)
    g0 = torch.zeros(grid.population_shape(), requires_grad=True)
    out = AG.LBMRollout.apply(g0, None, grid, 0.6, n, K, pair)
    assert rec.label(out) == n
    out.sum().backward()
    adj = [c for c in rec.calls if c[0] in ("adj1", "adj2")]
    covered = []
    for c in adj:
        covered += [c[1]] if c[0] == "adj1" else [c[1], c[2]]
    assert covered == list(range(n - 1, -1, -1))
    assert adj[0][0] == "adj1" and adj[0][2] is False  # lambda in
    assert all(c[2] is True for c in adj[1:] if c[0] == "adj1")  # chi in afterwards
    for c in adj:
        if c[0] == "adj2":
            assert pair
            assert c[2] == c[1] - 1 and c[1] // K == c[2] // K  # within one segment
    if pair:
        assert all(c[1] % K == 0 for c in adj[1:] if c[0] == "adj1")
    else:
        assert all(c[0] == "adj1" for c in adj)
    assert rec.calls[-1] == ("unstream",)


def test_slab_fields_with_two_ghost_planes(B):
    """split_field of slabs with two ghost planes gives each slab its planes plus the
    plane below and above (periodic in z); interior views and scatter/gather round-trip."""
    from paper_2106_12929_amd.slabs import SlabSet

    grid = B.Grid("D3Q27", "f32", 32, 8, 12)
    S = SlabSet(grid, [5, 4, 3], device="cpu", ghost=2)
    assert [b[0].shape[0] for b in S.bufs] == [5 + 4, 4 + 4, 3 + 4]
    v = torch.arange(3 * 12 * 8 * 32, dtype=torch.float32).reshape(3, 12, 8, 32)
    parts = S.split_field(v)
    for p, (z0, n) in enumerate(zip(S.z0, S.planes)):
        want = torch.stack([v[:, (z0 + k) % 12] for k in range(-1, n + 1)], dim=1)
        assert torch.equal(parts[p], want)
    f = torch.randn(grid.population_shape())
    S.scatter(f)
    assert torch.equal(S.gather(), f)
    for p in range(S.P):
        assert S.interior(p).shape[0] == S.planes[p]
    with pytest.raises(ValueError):
        SlabSet(grid, [1, 11], device="cpu", ghost=2)   # a slab of one plane
    with pytest.raises(ValueError):
        SlabSet(grid, 2, device="cpu", ghost=3)
    with pytest.raises(ValueError):
        S.step(0.6)                                      # two ghost planes: step_pair
