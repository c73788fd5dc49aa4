"""Seeded synthetic inputs shared by the HIP path's tests and benchmarks and by the
CPU oracle.  This package holds input generators only: random streams, point clouds,
neighbour lists, physical fields, species tables, ray sets and frequency quadratures.
It contains none of the radiative-transfer arithmetic."""
from . import configs, directions, models, rng, species  # noqa: F401
