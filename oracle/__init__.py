"""ORACLE — test infrastructure only.

A plain, slow FP64 CPU implementation of what the nested-mesh volume-potential
path computes, written from the paper (Groth et al., arXiv 2011.03009).  Only
the tests, the entry point's smoke check and the benchmark's CPU-baseline leg
may import it; the HIP library never does, and the two share no code.

Parity status of each function is stated in its docstring; none is
"parity unpinned" except where noted there.
"""

from .core import *  # noqa: F401,F403
from .incident import incident_at, incident_field, radiated_power  # noqa: F401
from .vie import dense_operator, vie_solve  # noqa: F401
from .quadrature import (conv_circulant_corrected, conv_direct_corrected, corrected_weights,  # noqa: F401
                         gaussian_potential, lattice_zeta, volume_potential_corrected)
from . import full_cascade  # noqa: F401
