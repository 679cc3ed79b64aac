"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side bench.

This package holds no arithmetic of the solver method: it only draws design
fields and builds the Dirichlet node mask (or, for cell-centred unknowns,
the Dirichlet face flags) of the model problem.  Both the oracle (``oracle/``) and the product
package consume it; neither imports the other.
"""
from .fields import (  # noqa: F401
    uniform_noise_rho,
    grf_rho,
    grf_raw,
    threshold_field,
    block_average,
    dirichlet_patch_mask,
    dirichlet_patch_faces,
    field_sha256,
)
