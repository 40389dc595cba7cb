"""z-slab domain decomposition of a periodic 3D grid: the shape the step takes when a
grid is split over several devices.

A grid periodic in x, y and z is cut into P slabs of consecutive z planes.  Each slab
keeps its planes in a buffer with one ghost plane below and one above
(`lbm_step_slab`), and one step of the whole grid becomes, for every slab:

  1. halo exchange (`lbm_slab_halo_copy`): the populations with c_z = +1 of the
     slab's top plane go to the lower ghost plane of the slab above it, those with
     c_z = -1 of its bottom plane to the upper ghost plane of the slab below (Eq. 1's
     streaming across the cut; P = 1 exchanges with itself);
  2. the step of the inner planes [1, nz-1), which reads no ghost data and so can run
     while the exchange is in flight;
  3. the step of the two boundary planes once the exchange has landed.

`SlabSet` runs the P slabs on one device, each with its own buffers, with the
exchange on a second stream when `overlap` is set.  The result is bitwise the
periodic `lbm_step` of the whole grid: every cell runs the same kernel arithmetic on
the same words.

With `ghost=2` the slabs keep two ghost planes on each side and advance two steps per
launch (`lbm_step_slab2`, the two-step kernel with the intermediate state on chip):
`step_pair` exchanges the two-plane-deep halo (`lbm_slab2_halo_copy`) once and then
steps every slab twice.  Halving the exchanges halves the latency-bound
synchronisations between devices, for 1.5 times the exchanged bytes per two steps.  On several devices each slab would live on its own device and the
exchange would cross xGMI; the buffers, the kernels and the order of operations are
the ones used here.
"""
from __future__ import annotations

import torch

from . import binding as B


def split_planes(nz: int, parts: int) -> list[int]:
    """nz planes split into `parts` slabs as evenly as possible (larger slabs first)."""
    if not 1 <= parts <= nz:
        raise ValueError(f"cannot split {nz} planes into {parts} slabs")
    q, r = divmod(nz, parts)
    return [q + 1] * r + [q] * (parts - r)


class SlabSet:
    def __init__(self, grid: B.Grid, planes, device="cuda", ghost: int = 1):
        if grid.D != 3:
            raise ValueError("z-slabs need a 3D lattice")
        if ghost not in (1, 2):
            raise ValueError("a slab has 1 or 2 ghost planes on each side")
        planes = split_planes(grid.nz, planes) if isinstance(planes, int) else [int(p) for p in planes]
        if sum(planes) != grid.nz or min(planes) < ghost:
            raise ValueError(f"slab plane counts {planes} do not partition nz = {grid.nz} into slabs of "
                             f"at least {ghost} planes")
        self.grid = grid
        self.ghost = ghost
        self.planes = planes
        self.z0 = [sum(planes[:p]) for p in range(len(planes))]
        self.slabs = [B.Grid(grid.lattice, grid.storage, grid.nx, grid.ny, n, grid.pitch) for n in planes]
        if ghost == 2 and not all(B.lbm_step_slab2_available(s) for s in self.slabs):
            raise ValueError("two steps per launch do not take these slabs (lbm_step_slab2_available)")
        self.bufs = [[s.empty_slab_populations(device, ghost), s.empty_slab_populations(device, ghost)]
                     for s in self.slabs]
        self.cur = 0
        self._halo_stream = None

    @property
    def P(self) -> int:
        return len(self.slabs)

    def interior(self, p: int, which: int | None = None) -> torch.Tensor:
        """View of slab p's own planes (buffer planes ghost .. ghost + nz - 1) in the
        current buffer."""
        b = self.bufs[p][self.cur if which is None else which]
        return b[self.ghost:self.planes[p] + self.ghost]

    def scatter(self, f: torch.Tensor) -> None:
        """Loads a whole-grid population buffer (population layout) into the slabs."""
        for p in range(self.P):
            self.interior(p).copy_(f[self.z0[p]:self.z0[p] + self.planes[p]])

    def gather(self) -> torch.Tensor:
        """The whole-grid population buffer assembled from the slabs."""
        return torch.cat([self.interior(p) for p in range(self.P)], dim=0)

    def split_field(self, v: torch.Tensor | None):
        """A whole-grid [D, nz, ny, nx] real field cut into the slabs' own cells; with
        two ghost planes, each slab's part also holds the plane below and the plane above
        it (periodic in z), as lbm_step_slab2 takes its force."""
        if v is None:
            return [None] * self.P
        if self.ghost == 1:
            return [v[:, self.z0[p]:self.z0[p] + self.planes[p]].contiguous() for p in range(self.P)]
        nz = self.grid.nz
        out = []
        for p in range(self.P):
            idx = torch.arange(self.z0[p] - 1, self.z0[p] + self.planes[p] + 1, device=v.device) % nz
            out.append(v.index_select(1, idx).contiguous())
        return out

    def exchange(self, stream=None) -> None:
        """Fills every slab's ghost planes of the current buffer from its neighbours."""
        c = self.cur
        copy = B.lbm_slab_halo_copy if self.ghost == 1 else B.lbm_slab2_halo_copy
        for p in range(self.P):
            up, down = (p + 1) % self.P, (p - 1) % self.P
            copy(self.slabs[p], self.bufs[p][c], self.slabs[up], self.bufs[up][c], "high", stream)
            copy(self.slabs[p], self.bufs[p][c], self.slabs[down], self.bufs[down][c], "low", stream)

    def _launch2(self, p: int, tau: float, force, z_begin: int, z_end: int) -> None:
        if z_begin < z_end:
            B.lbm_step_slab2(self.slabs[p], self.bufs[p][self.cur], self.bufs[p][1 - self.cur], tau, force,
                             z_begin, z_end)

    def step_pair(self, tau: float, forces=None, overlap: bool = False) -> None:
        """Two steps of the whole grid (slabs with two ghost planes): one exchange, then
        one two-step launch per slab.  With `overlap` the exchange runs on a second
        stream concurrently with a launch of the inner planes [2, nz-2), which read no
        ghost data, and the four boundary planes follow once it has landed (slabs of
        fewer than 5 planes: one launch of all after the exchange).  forces: per slab,
        D x (nz + 2) planes of force (split_field), or None."""
        if self.ghost != 2:
            raise ValueError("step_pair needs slabs with two ghost planes (ghost=2)")
        forces = forces if forces is not None else [None] * self.P
        main = torch.cuda.current_stream()
        split = [overlap and n >= 5 for n in self.planes]
        if overlap:
            if self._halo_stream is None:
                self._halo_stream = torch.cuda.Stream()
            hs = self._halo_stream
            hs.wait_stream(main)  # the previous launch has written the planes being sent
            with torch.cuda.stream(hs):
                self.exchange(hs)
        else:
            self.exchange()
        for p in range(self.P):
            if split[p]:
                self._launch2(p, tau, forces[p], 2, self.planes[p] - 2)
        if overlap:
            main.wait_stream(hs)
        for p in range(self.P):
            n = self.planes[p]
            if split[p]:
                self._launch2(p, tau, forces[p], 0, 2)
                self._launch2(p, tau, forces[p], n - 2, n)
            else:
                self._launch2(p, tau, forces[p], 0, n)
        self.cur = 1 - self.cur

    def _launch(self, p: int, tau: float, force, z_begin: int, z_end: int) -> None:
        if z_begin < z_end:
            B.lbm_step_slab(self.slabs[p], self.bufs[p][self.cur], self.bufs[p][1 - self.cur], tau, force,
                            z_begin, z_end)

    def step(self, tau: float, forces=None, overlap: bool = False) -> None:
        """One step of the whole grid: exchange, inner planes, boundary planes.  With
        `overlap` the exchange runs on a second stream concurrently with the inner
        planes; the boundary planes wait for it."""
        if self.ghost != 1:
            raise ValueError("slabs with two ghost planes advance two steps at a time (step_pair)")
        forces = forces if forces is not None else [None] * self.P
        main = torch.cuda.current_stream()
        if overlap:
            if self._halo_stream is None:
                self._halo_stream = torch.cuda.Stream()
            hs = self._halo_stream
            hs.wait_stream(main)  # the previous step has written the planes being sent
            with torch.cuda.stream(hs):
                self.exchange(hs)
            for p in range(self.P):
                self._launch(p, tau, forces[p], 1, self.planes[p] - 1)
            main.wait_stream(hs)
        else:
            self.exchange()
            for p in range(self.P):
                self._launch(p, tau, forces[p], 1, self.planes[p] - 1)
        for p in range(self.P):
            n = self.planes[p]
            self._launch(p, tau, forces[p], 0, 1)
            if n > 1:
                self._launch(p, tau, forces[p], n - 1, n)
        self.cur = 1 - self.cur
