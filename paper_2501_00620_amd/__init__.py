"""MI355X (gfx950) implementation of the bump-function D3Q19 lattice Boltzmann sweep of
Afrasiabian & Denniston (arXiv:2501.00620).

Submodules: ``lbm`` (binding of the C ABI in include/lbm.h: ``Lattice`` for one lattice,
``Server`` for the continuous batching of many), ``workloads`` (seeded synthetic initial fields),
``build`` (hipcc build).
"""
__all__ = ["lbm", "workloads", "build"]
