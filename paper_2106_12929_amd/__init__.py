"""MI355X (gfx950) lattice-Boltzmann stream-and-collide library.

The compute path is the HIP library liblbm.so (C ABI in include/lbm.h) built from
csrc/; `binding` is its thin ctypes binding (same entry-point names), `autograd`
wraps the hand-written adjoint in a torch.autograd.Function with checkpointing,
`spectrum` is the FFT loss head used by the forcing-optimisation workload.
PyTorch supplies device memory and streams only.

Importing the package does not load the library; `from paper_2106_12929_amd import
binding` does, and raises if liblbm.so has not been built.
"""

__all__ = ["binding", "autograd", "spectrum", "simulation", "build"]
