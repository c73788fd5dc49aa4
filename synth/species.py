"""Synthetic line species (levels, radiative lines, collisional de-excitation tables).

The paper's models use tabulated molecular data (level energies, statistical weights,
Einstein A coefficients and H2 collisional de-excitation rates tabulated in
temperature, Sec. 2.2.1).  Those tables are not available here, so these species stand
in for them with the same structure:

* ``table1_species``: the fictitious two-level species of the paper's Table 1
  (E2 - E1 = 6.0 cm^-1, g2/g1 = 3, A21 = 1e-4 s^-1, K21 = 2e-10 cm^3 s^-1); its mass
  is one atomic mass unit, the value that reproduces the line widths the paper quotes
  for its semi-analytic tests (Sec. 4.1).
* ``two_level``: a two-level species given by its line frequency.
* ``linear_rotor``: levels E_J = h B J (J + 1), g_J = 2J + 1, lines J -> J-1 with
  A_J = A_10 * 3 J^4 / (2J + 1), collisions between every pair of levels.

Collision rates are tabulated on a temperature grid; consumers interpolate linearly
in T and clamp at the table ends.  Energies are in erg, everything else CGS.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# CGS values of the SI-exact constants (used only to express the inputs in erg).
H_PLANCK = 6.62607015e-27
C_LIGHT = 2.99792458e10
AMU = 1.66053906660e-24


@dataclass
class Species:
    energy: np.ndarray          # [n_lev] erg
    weight: np.ndarray          # [n_lev] statistical weights g
    mass: float                 # g
    line_up: np.ndarray         # [n_lines] int32 upper level
    line_lo: np.ndarray         # [n_lines] int32 lower level
    line_A: np.ndarray          # [n_lines] s^-1
    coll_up: np.ndarray         # [n_coll] int32
    coll_lo: np.ndarray         # [n_coll] int32
    coll_T: np.ndarray          # [n_T] K, strictly increasing
    coll_K: np.ndarray          # [n_coll, n_T] cm^3 s^-1 (de-excitation, up -> lo)
    name: str = field(default="species")

    @property
    def n_lev(self) -> int:
        return int(self.energy.shape[0])

    @property
    def n_lines(self) -> int:
        return int(self.line_up.shape[0])


def _temperature_grid() -> np.ndarray:
    return np.geomspace(1.0, 5000.0, 48)


def _sqrt_law(K0: float, T: np.ndarray) -> np.ndarray:
    return K0 * np.sqrt(T / 20.0)


def two_level(nu: float = 100e9, g_ratio: float = 3.0, A: float = 1e-5,
              K0: float = 1e-10, mass_amu: float = 28.0, sqrt_law: bool = True) -> Species:
    T = _temperature_grid()
    K = _sqrt_law(K0, T) if sqrt_law else np.full_like(T, K0)
    return Species(
        energy=np.array([0.0, H_PLANCK * nu]),
        weight=np.array([1.0, g_ratio]),
        mass=mass_amu * AMU,
        line_up=np.array([1], dtype=np.int32),
        line_lo=np.array([0], dtype=np.int32),
        line_A=np.array([A]),
        coll_up=np.array([1], dtype=np.int32),
        coll_lo=np.array([0], dtype=np.int32),
        coll_T=T,
        coll_K=K[None, :].copy(),
        name=f"two_level_{nu/1e9:g}GHz",
    )


def table1_species() -> Species:
    """The paper's Table 1 species, with a temperature-independent K21."""
    nu = 6.0 * C_LIGHT
    sp = two_level(nu=nu, g_ratio=3.0, A=1.0e-4, K0=2.0e-10, mass_amu=1.0, sqrt_law=False)
    sp.name = "table1"
    return sp


def linear_rotor(n_lev: int, B_hz: float = 57.6e9, A10: float = 7e-8, K0: float = 1e-10,
                 mass_amu: float = 28.0) -> Species:
    J = np.arange(n_lev, dtype=np.float64)
    energy = H_PLANCK * B_hz * J * (J + 1.0)
    weight = 2.0 * J + 1.0
    up = np.arange(1, n_lev, dtype=np.int32)
    lo = up - 1
    Ju = up.astype(np.float64)
    A = A10 * 3.0 * Ju ** 4 / (2.0 * Ju + 1.0)
    cu, cl = [], []
    for u in range(1, n_lev):
        for l in range(u):
            cu.append(u)
            cl.append(l)
    T = _temperature_grid()
    K = np.tile(_sqrt_law(K0, T), (len(cu), 1))
    return Species(energy=energy, weight=weight, mass=mass_amu * AMU,
                   line_up=up, line_lo=lo, line_A=A,
                   coll_up=np.array(cu, dtype=np.int32), coll_lo=np.array(cl, dtype=np.int32),
                   coll_T=T, coll_K=K, name=f"rotor{n_lev}")
