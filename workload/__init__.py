"""Seeded synthetic inputs shared by the HIP path's callers and the oracle's tests.

This package holds no arithmetic of the volume-potential method itself: it
states the physical configurations (transducer, medium, voxel counts), places
the bowl's surface points, evaluates the incident field p1 that the method
takes as its input, and draws seeded random source fields.  Grid spacings,
origins, wavenumbers, kernels, transfers and convolutions are computed by the
library and, independently, by the oracle.
"""

from . import bowl, configs, fields  # noqa: F401
