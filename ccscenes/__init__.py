"""Seeded synthetic scene generators shared by the oracle and the GPU path.

This package only produces *inputs*: structured simplicial grids, Dirichlet
vertex sets, prescribed boundary targets, material constants and the seeded
random draws of the batched and training workloads.  It holds none of the
solver's arithmetic (no deformation gradients, energies, masses, bases or
colourings); each side computes those on its own from these arrays.
"""
from .grid import grid2d, grid3d
from .scenes import (Scene, stretch2d, tet_bar, twist_beam, rod_impulse, cantilever_bend, batch_bars, mlp_init,
                     warm_start_train_scene, warm_start_eval_scene)

__all__ = ["grid2d", "grid3d", "Scene", "stretch2d", "tet_bar", "twist_beam", "rod_impulse", "cantilever_bend",
           "batch_bars", "mlp_init", "warm_start_train_scene", "warm_start_eval_scene"]
