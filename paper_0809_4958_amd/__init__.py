"""MI355X (gfx950) fine-box lattice-Boltzmann library: D3Q19 collide+stream with
tracer-driven equilibrium boundaries and friction-coupled FENE chains.

``lbm`` binds the HIP shared library (C ABI of include/lbm.h); ``inputs``
generates the seeded synthetic inputs; ``build`` compiles the library.
"""
__all__ = ["lbm", "inputs", "build"]
