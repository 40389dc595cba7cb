"""CPU checks of the simulation save/restore file: the storage words come back bit for
bit with the grid, tau, force and step count, and foreign files are refused."""
import pytest
import torch

from paper_2106_12929_amd import binding as B
from paper_2106_12929_amd.simulation import Simulation


@pytest.mark.parametrize("storage,pitch", [("f16s", None), ("f64", None), ("bf16s", 48), ("f32", None)])
def test_save_restore_round_trip(tmp_path, storage, pitch):
    grid = B.Grid("D3Q27", storage, 37, 5, 4, pitch)
    force = torch.randn((3, 4, 5, 37), dtype=grid.real_dtype)
    sim = Simulation(grid, 0.5123456789, force, device="cpu")
    gen = torch.Generator().manual_seed(3)
    words = torch.randint(0, 256, (grid.pop_size * torch.tensor([], dtype=grid.word_dtype).element_size(),),
                          generator=gen, dtype=torch.uint8)
    sim.load(words.view(grid.word_dtype).reshape(grid.population_shape()))
    sim.steps_done = 1234
    path = str(tmp_path / "state.safetensors")
    sim.save(path)
    back = Simulation.restore(path, device="cpu")
    assert back.grid == grid
    assert back.tau == sim.tau and back.steps_done == 1234
    assert torch.equal(back.f.view(torch.uint8), sim.f.view(torch.uint8))
    assert torch.equal(back.force, force)


def test_restore_refuses_other_files(tmp_path):
    from safetensors.torch import save_file

    path = str(tmp_path / "other.safetensors")
    save_file({"x": torch.zeros(4)}, path, metadata={"format": "something-else"})
    with pytest.raises(ValueError):
        Simulation.restore(path, device="cpu")
