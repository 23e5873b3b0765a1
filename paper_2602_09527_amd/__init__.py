"""MI355X (gfx950) ProxSkip-SVRG for TV-regularised parallel-beam tomography.

The compute path is the HIP library ``libproxskip.so`` (C ABI in include/proxskip.h); this
package is its Python binding.  Submodules:

* ``api``      -- Geometry, project, backproject, tv_prox, solve, Solver, sample_sequences
* ``autograd`` -- ProjectSubset, a torch.autograd.Function over the projector
* ``serve``    -- continuous-batching reconstruction server
* ``synth``    -- seeded synthetic phantoms and their analytic sinograms (inputs only)
"""
from __future__ import annotations

import importlib

_API = {"Geometry", "project", "backproject", "tv_prox", "SolverParams", "solve", "Solver",
        "run_epochs", "sample_sequences", "lipschitz"}


def __getattr__(name):
    if name in _API:
        return getattr(importlib.import_module(".api", __name__), name)
    if name == "ProjectSubset":
        return importlib.import_module(".autograd", __name__).ProjectSubset
    raise AttributeError(name)
