"""MI355X (gfx950) implementation of the preconditioned projected nonlinear
conjugate gradient minimizer for P1 finite-element micromagnetics.

The compute path is the HIP library libmmncg.so (C ABI in include/mmncg.h);
`binding` wraps it with ctypes, `inputs` generates seeded synthetic workloads.
"""
import importlib

from . import inputs  # noqa: F401

__all__ = ["inputs", "binding", "Context"]


def __getattr__(name):
    if name in ("binding", "Context"):
        mod = importlib.import_module(__name__ + ".binding")
        return mod if name == "binding" else mod.Context
    raise AttributeError(name)
