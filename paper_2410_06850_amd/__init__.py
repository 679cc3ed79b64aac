"""MI355X multiscale-multigrid PCG for SIMP heat conduction (Q1 hexahedra).

All computation runs in the HIP library ``libmsmg.so`` (see include/msmg.h);
this package only marshals torch tensors and streams into its C ABI.
"""
from . import _lib  # noqa: F401
from . import autograd, topopt  # noqa: F401
from .solver import Solver, density_filter, prolong_element, prolong_nodal  # noqa: F401

__all__ = ["Solver", "prolong_nodal", "prolong_element", "density_filter", "autograd", "topopt"]
