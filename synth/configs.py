"""The synthetic workloads, each with its seed, sizes and physics.

sphere2     1,000 points uniform in a ball of radius 1e17 cm, n_H2 = 1e4 (max(r, 1e15 cm)/1e15 cm)^-2,
            T = 20 K, static, abundance 1e-8, two-level species at 100 GHz (A = 1e-5 s^-1,
            K = 1e-10 (T/20)^1/2 cm^3 s^-1, g_u/g_l = 3), 12 HEALPix rays (Nside 1),
            31 frequencies over +-4 widths, CMB boundary at 2.725 K.
outflow5    50,000 points in the same ball, n_H2 = 1e7 (max(r, r_in)/r_in)^-2 (1e3..1e7 cm^-3),
            T = 100 (max(r, r_in)/r_in)^-1/2 (10..100 K), radial outflow of 15 km/s,
            abundance 1e-6, 5-level linear rotor (4 lines at 115.2..460.8 GHz),
            48 HEALPix rays (Nside 2).
batch256    256 models with the physics of outflow5, point counts log-uniform in
            [500, 20000], temperature and density scales log-uniform in [0.3, 3].
disc10      1,000,000 points in a flared Keplerian disc (R 10..500 AU, H/R = 0.1),
            10-level rotor (9 lines), 192 HEALPix rays (Nside 4).
discs       16 discs of the disc10 family (seeds 200..215), 8,000 points each, batched,
            12 HEALPix rays (Nside 1).

Species mass 28 amu and turbulent speed 150 m/s for all of them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import directions, species
from .models import Model, concat_models, keplerian_disc, power_law_sphere
from .rng import Stream


@dataclass
class Workload:
    name: str
    model: Model
    species: species.Species
    rays: np.ndarray
    quad_x: np.ndarray
    quad_w: np.ndarray
    offsets: Optional[np.ndarray] = None       # batched: [n_models + 1]
    t_cmb: float = 2.725
    f_sub: float = 0.25
    max_iter: int = 50
    tol: float = 1e-4
    meta: dict = field(default_factory=dict)

    @property
    def n_points(self) -> int:
        return self.model.n_points

    @property
    def n_models(self) -> int:
        return 1 if self.offsets is None else len(self.offsets) - 1

    def units(self) -> int:
        """point * ray * frequency per formal-solve sweep."""
        return self.n_points * self.rays.shape[0] * self.species.n_lines * self.quad_x.shape[0]


def sphere2(n_points: int = 1000, seed: int = 0) -> Workload:
    m = power_law_sphere(seed, n_points, radius=1e17, r_in=1e15, n_in=1e4, n_slope=-2.0,
                         T_in=20.0, T_slope=0.0, v_out=0.0, abundance=1e-8)
    x, w = directions.uniform_grid(31, 4.0)
    return Workload("sphere2", m, species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0),
                    directions.healpix_ring(1), x, w, max_iter=50)


def outflow5(n_points: int = 50000, seed: int = 1, nside: int = 2) -> Workload:
    m = power_law_sphere(seed, n_points, radius=1e17, r_in=1e15, n_in=1e7, n_slope=-2.0,
                         T_in=100.0, T_slope=-0.5, v_out=15.0e5, abundance=1e-6)
    x, w = directions.uniform_grid(31, 4.0)
    return Workload("outflow5", m, species.linear_rotor(5), directions.healpix_ring(nside), x, w,
                    max_iter=50)


def batch256(n_models: int = 256, n_min: int = 500, n_max: int = 20000, seed0: int = 1000) -> Workload:
    models: List[Model] = []
    counts = []
    for i in range(n_models):
        st = Stream(seed0 + i, "batch")
        u = st.uniform(3)
        n = int(round(np.exp(np.log(n_min) + u[0] * np.log(n_max / n_min))))
        sT = float(np.exp(np.log(0.3) + u[1] * np.log(10.0)))
        sn = float(np.exp(np.log(0.3) + u[2] * np.log(10.0)))
        m = power_law_sphere(seed0 + i, n, radius=1e17, r_in=1e15, n_in=1e7 * sn, n_slope=-2.0,
                             T_in=100.0 * sT, T_slope=-0.5, v_out=15.0e5, abundance=1e-6)
        models.append(m)
        counts.append(n)
    offs, merged = concat_models(models)
    x, w = directions.uniform_grid(31, 4.0)
    return Workload("batch256", merged, species.linear_rotor(5), directions.healpix_ring(2), x, w,
                    offsets=offs, meta={"counts": counts})


def disc10(n_points: int = 1_000_000, seed: int = 3) -> Workload:
    m = keplerian_disc(seed, n_points)
    x, w = directions.uniform_grid(31, 4.0)
    return Workload("disc10", m, species.linear_rotor(10), directions.healpix_ring(4), x, w)


def discs(n_models: int = 16, n_points: int = 8000, seed0: int = 200, nside: int = 1) -> Workload:
    models = [keplerian_disc(seed0 + i, n_points) for i in range(n_models)]
    offs, merged = concat_models(models)
    x, w = directions.uniform_grid(31, 4.0)
    return Workload("discs", merged, species.linear_rotor(10), directions.healpix_ring(nside), x, w,
                    offsets=offs)


def disc_model(seed: int, n_points: int = 8000, nside: int = 1) -> Workload:
    """One disc of the `discs` family (for training the warm start on other seeds)."""
    m = keplerian_disc(seed, n_points)
    x, w = directions.uniform_grid(31, 4.0)
    return Workload("disc", m, species.linear_rotor(10), directions.healpix_ring(nside), x, w)
