"""CPU FP64 oracle for the Q1 SIMP heat-conduction solve and its multiscale
multigrid preconditioner.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
package never imports it, and this package imports nothing from the product
package: the two share no kernels, helpers, tables or constants.  Inputs come
from ``synth`` (seeded generators without solver arithmetic).

Modules
  q1      discretisation: element matrix, assembly, load, Dirichlet lifting,
          compliance, adjoint sensitivity, the design-dependent heat source
          and the mean-temperature objective (paper section 2 and its
          ``material``, ``new linear system``, ``cost function`` and
          ``adjoint`` equations).
  msmg    three-grid multiscale preconditioner and PCG (paper section 3,
          Algorithm 1, equations ``spepb`` and ``spectral cc``).
  interp  grid-to-grid interpolation of temperatures and densities (the
          interpolation technique of section 3).
  topopt  the optimisation loop's design update: hat density filter and the
          optimality-criteria update (section 2.3's sensitivities feed it).

q1 also evaluates residual and load rows node by node and the full residual
slab by slab, for grids too large to assemble.

Every function is pinned by tests in ``tests/test_oracle_*.py`` against
closed forms, invariants or brute force; none is marked "parity unpinned".
"""
