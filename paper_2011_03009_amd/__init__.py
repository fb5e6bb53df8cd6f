"""nvp: nested-mesh Helmholtz volume potentials on MI355X.

The computation lives in the HIP library lib/libnvp.so (C ABI in
include/nvp.h); this package is its Python binding.
"""

from . import nvp  # noqa: F401
from .nvp import (NVP_C64, NVP_C128, NVP_QUAD_BALL, NVP_QUAD_CORRECTED, Batch, BoxNet,  # noqa: F401
                  CascadePlan, Context, NvpError, box_potential, difference_term,
                  incident_at, incident_field, radiated_power, quadrature_weights, set_quadrature,
                  cascade_constant, circulant_size, grid, grid_from_box, grid_from_counts, qbox,
                  rule_of_thumb_box, spacing, transform_lengths, vie_solve, volume_potential,
                  volume_potential_box, volume_potential_noalloc, field_lin3, field_diff_norms, wavenumber)
