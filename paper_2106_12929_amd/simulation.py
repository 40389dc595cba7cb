"""A small simulation driver over the C ABI (the Simulation.step(num_steps) usage of
the paper's Listing 1): owns the two population buffers of the ping-pong scheme and
tracks which one holds the current state."""
from __future__ import annotations

import torch

from . import binding as B


_FORMAT = "lbm-simulation-1"


class Diverged(RuntimeError):
    """A run produced non-finite cells (for BGK: tau too close to 1/2 for the flow)."""

    def __init__(self, steps_done: int, reductions: dict):
        self.steps_done = steps_done
        self.reductions = reductions
        super().__init__(f"{int(reductions['nonfinite_cells'])} non-finite cells after {steps_done} steps")


class Simulation:
    """Populations of one grid on one GPU.

    grid: binding.Grid.  tau: BGK relaxation time.  force: optional [D, *spatial]
    real-typed GPU tensor, constant in time.
    """

    def __init__(self, grid: B.Grid, tau: float, force: torch.Tensor | None = None, device="cuda"):
        self.grid = grid
        self.tau = float(tau)
        self.force = force
        self.device = torch.device(device)
        self.bufs = [grid.empty_populations(self.device), grid.empty_populations(self.device)]
        self.cur = 0
        self.steps_done = 0
        self._red = torch.zeros(B.NRED, dtype=torch.float64, device=self.device)
        self._ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device=self.device)

    @property
    def f(self) -> torch.Tensor:
        """The current state g(t) (storage words)."""
        return self.bufs[self.cur]

    def init_equilibrium(self, u: torch.Tensor, rho: torch.Tensor | None = None) -> None:
        """g(0) = f^eq(rho, u) from FP64 fields (moved to the GPU if needed)."""
        u = u.to(self.device, torch.float64).contiguous()
        rho = None if rho is None else rho.to(self.device, torch.float64).contiguous()
        B.lbm_init_equilibrium(self.grid, rho, u, self.bufs[self.cur])
        self.steps_done = 0

    def load(self, f: torch.Tensor) -> None:
        """Set the state from stored words of the right dtype and shape."""
        self.bufs[self.cur].copy_(f.to(self.device))

    def save(self, path: str) -> None:
        """Writes the current state (the storage words, bit for bit), the grid, tau, the
        force and the step count to a safetensors file; Simulation.restore continues
        from it exactly as the uninterrupted run would (the steps are deterministic)."""
        from safetensors.torch import save_file

        g = self.grid
        tensors = {"populations": self.f.contiguous().view(torch.uint8).reshape(-1).cpu()}
        if self.force is not None:
            tensors["force"] = self.force.contiguous().cpu()
        meta = {"format": _FORMAT, "lattice": g.lattice, "storage": g.storage, "nx": str(g.nx), "ny": str(g.ny),
                "nz": str(g.nz), "pitch": str(g.row_pitch), "tau": repr(self.tau), "steps_done": str(self.steps_done)}
        save_file(tensors, path, metadata=meta)

    @classmethod
    def restore(cls, path: str, device="cuda") -> "Simulation":
        """A Simulation holding the state, grid, tau, force and step count of a file
        written by save (read with safetensors: nothing in the file is executed)."""
        from safetensors import safe_open

        with safe_open(path, framework="pt") as fh:
            meta = fh.metadata() or {}
            if meta.get("format") != _FORMAT:
                raise ValueError(f"{path} is not a saved simulation ({meta.get('format')!r})")
            words = fh.get_tensor("populations")
            force = fh.get_tensor("force") if "force" in fh.keys() else None
        nx, pitch = int(meta["nx"]), int(meta["pitch"])
        grid = B.Grid(meta["lattice"], meta["storage"], nx, int(meta["ny"]), int(meta["nz"]),
                      None if pitch == nx else pitch)
        if words.numel() != grid.pop_size * torch.tensor([], dtype=grid.word_dtype).element_size():
            raise ValueError(f"{path}: population bytes do not match the grid")
        sim = cls(grid, float(meta["tau"]), None if force is None else force.to(device), device)
        sim.load(words.view(grid.word_dtype).reshape(grid.population_shape()))
        sim.steps_done = int(meta["steps_done"])
        return sim

    def step(self, n_steps: int = 1) -> None:
        src, dst = self.bufs[self.cur], self.bufs[1 - self.cur]
        where = B.lbm_step(self.grid, src, dst, self.tau, self.force, n_steps)
        self.cur = (1 - self.cur) if where == 0 else self.cur
        self.steps_done += n_steps

    def moments(self):
        """(rho [*spatial], u [D, *spatial]) of the current state, real dtype."""
        rho = self.grid.empty_real(0, self.device)
        u = self.grid.empty_real(self.grid.D, self.device)
        B.lbm_moments(self.grid, self.f, self.force, rho, u)
        return rho, u

    def reductions(self) -> dict:
        """FP64 mass, momentum, kinetic energy, non-finite count, max speed, min density
        (copies 8 doubles to the host, which waits for the stream)."""
        B.lbm_moments(self.grid, self.f, self.force, None, None, self._red, self._ws)
        vals = self._red.cpu().tolist()
        return dict(zip(B.RED_NAMES, vals))

    def run(self, n_steps: int, check_every: int = 100) -> dict:
        """n_steps steps in chunks of check_every, reading the FP64 reductions after
        each chunk; raises Diverged at the first check that finds non-finite cells.
        Returns the last reductions."""
        if n_steps < 1 or check_every < 1:
            raise ValueError("n_steps and check_every must be >= 1")
        left = n_steps
        red = None
        while left > 0:
            k = min(check_every, left)
            self.step(k)
            left -= k
            red = self.reductions()
            if red["nonfinite_cells"] > 0:
                raise Diverged(self.steps_done, red)
        return red
