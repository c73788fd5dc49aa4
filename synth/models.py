"""Seeded synthetic models: point clouds, neighbour lists and physical fields.

The paper's inputs are a point cloud with nearest-neighbour lists plus density,
temperature, velocity and turbulence fields (Sec. 3.1.1).  Its own workloads
(van Zadelhoff problem 1 spheres, a LIME-meshed Keplerian disc) are not available, so
these generators stand in with the same structure: power-law spheres like benchmark
problem 1 (Sec. 4.2.1) and a flared Keplerian disc (Sec. 5), plus the 1-D grids of the
semi-analytic tests (Sec. 4.1).

Neighbour lists are exact k-nearest neighbours (self excluded) unless a generator
builds them explicitly (1-D chains, lattices).  All quantities are CGS.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
from scipy.spatial import cKDTree

from .rng import Stream

AU = 1.495978707e13
GM_SUN = 1.32712440018e26
KM = 1.0e5


@dataclass
class Model:
    pos: np.ndarray              # [P, 3] cm
    vel: np.ndarray              # [P, 3] cm/s
    n_h2: np.ndarray             # [P] cm^-3
    temperature: np.ndarray      # [P] K
    v_turb: np.ndarray           # [P] cm/s
    abundance: np.ndarray        # [P] n_species / n_H2
    nbr: np.ndarray              # [P, k] int32, -1 = unused slot
    boundary: Optional[np.ndarray] = None   # [P] uint8 or None

    @property
    def n_points(self) -> int:
        return int(self.pos.shape[0])

    def subset_fields(self, scale_T: float = 1.0, scale_n: float = 1.0) -> "Model":
        return Model(self.pos, self.vel, self.n_h2 * scale_n, self.temperature * scale_T,
                     self.v_turb, self.abundance, self.nbr, self.boundary)


def knn(pos: np.ndarray, k: int = 12) -> np.ndarray:
    """Exact k nearest neighbours of every point, self excluded, nearest first."""
    n = pos.shape[0]
    kk = min(k + 1, n)
    tree = cKDTree(pos)
    _, idx = tree.query(pos, k=kk)
    idx = np.atleast_2d(idx)
    out = np.full((n, k), -1, dtype=np.int32)
    for row in range(n):
        cand = [int(j) for j in idx[row] if j != row and j < n][:k]
        out[row, :len(cand)] = cand
    return out


def sample_ball(stream: Stream, n: int, radius: float) -> np.ndarray:
    """Uniform points in a ball by rejection from the enclosing cube."""
    pts = []
    have = 0
    while have < n:
        m = max(64, int(1.3 * (n - have)) + 16)
        u = stream.uniform(3 * m).reshape(m, 3)
        c = (2.0 * u - 1.0) * radius
        keep = c[np.einsum("ij,ij->i", c, c) <= radius * radius]
        pts.append(keep)
        have += keep.shape[0]
    return np.concatenate(pts)[:n].copy()


def power_law_sphere(seed: int, n: int, radius: float, r_in: float, n_in: float, n_slope: float,
                     T_in: float, T_slope: float, v_out: float, abundance: float,
                     v_turb: float = 1.5e4, k: int = 12) -> Model:
    """Points uniform in a ball; n = n_in (max(r, r_in)/r_in)^n_slope, T likewise,
    radial velocity of constant magnitude v_out."""
    st = Stream(seed, "ball")
    pos = sample_ball(st, n, radius)
    r = np.sqrt(np.einsum("ij,ij->i", pos, pos))
    rr = np.maximum(r, r_in) / r_in
    n_h2 = n_in * rr ** n_slope
    T = T_in * rr ** T_slope
    rhat = pos / np.maximum(r, 1e-300)[:, None]
    vel = v_out * rhat
    return Model(pos=pos, vel=vel, n_h2=n_h2, temperature=T,
                 v_turb=np.full(n, v_turb), abundance=np.full(n, abundance),
                 nbr=knn(pos, k))


def keplerian_disc(seed: int, n: int, r_min_au: float = 10.0, r_max_au: float = 500.0,
                   h_over_r: float = 0.1, n0: float = 1.5e9, T0: float = 200.0,
                   abundance: float = 1e-6, v_turb: float = 1.5e4, k: int = 12) -> Model:
    """Flared disc: R log-uniform, phi uniform, z = H N(0,1) truncated at 3H, H = 0.1 R,
    n = n0 (R/10 AU)^-2 exp(-z^2 / 2H^2), T = T0 (R/10 AU)^-1/2, Keplerian v_phi."""
    st = Stream(seed, "disc")
    R = r_min_au * AU * np.exp(st.uniform(n) * np.log(r_max_au / r_min_au))
    phi = 2.0 * np.pi * st.uniform(n)
    H = h_over_r * R
    zeta = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        g = st.normal(todo.size)
        ok = np.abs(g) <= 3.0
        zeta[todo[ok]] = g[ok]
        todo = todo[~ok]
    z = H * zeta
    pos = np.stack([R * np.cos(phi), R * np.sin(phi), z], axis=1)
    n_h2 = n0 * (R / (10.0 * AU)) ** -2 * np.exp(-0.5 * zeta * zeta)
    T = T0 * (R / (10.0 * AU)) ** -0.5
    vphi = np.sqrt(GM_SUN / R)
    vel = np.stack([-vphi * np.sin(phi), vphi * np.cos(phi), np.zeros(n)], axis=1)
    return Model(pos=pos, vel=vel, n_h2=n_h2, temperature=T,
                 v_turb=np.full(n, v_turb), abundance=np.full(n, abundance),
                 nbr=knn(pos, k))


def shell_sphere(seed: int, radii: np.ndarray, counts: np.ndarray, k: int = 12) -> Model:
    """Points on concentric spheres (the paper maps each grid point of a 1-D model to a
    shell of points spread over a sphere, Sec. 4.1.1-4.1.2): counts[s] points on the
    sphere of radius radii[s], spread by a golden-angle spiral (equal-area rings in z)
    and turned by a seeded random rotation per shell, with exact k-NN neighbours.  The
    physical fields are left for the caller (zero velocity, unit density and
    temperature, no turbulence, unit abundance)."""
    st = Stream(seed, "shells")
    golden = np.pi * (3.0 - np.sqrt(5.0))
    pts = []
    for rad, m in zip(np.asarray(radii, dtype=np.float64), np.asarray(counts, dtype=np.int64)):
        i = np.arange(m, dtype=np.float64) + 0.5
        z = 1.0 - 2.0 * i / m
        s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        ph = golden * np.arange(m)
        p = np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)
        # rotation from a unit quaternion with Gaussian components
        q = st.normal(4)
        q = q / np.sqrt((q * q).sum())
        a, b, c, d = q
        rot = np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])
        pts.append(rad * (p @ rot.T))
    pos = np.concatenate(pts)
    n = pos.shape[0]
    return Model(pos=pos, vel=np.zeros((n, 3)), n_h2=np.ones(n), temperature=np.ones(n),
                 v_turb=np.zeros(n), abundance=np.ones(n), nbr=knn(pos, k))


def chain_1d(x: np.ndarray, vel_x: np.ndarray, n_h2, temperature, v_turb, abundance) -> Model:
    """Points on the x axis with chain neighbours (left, right)."""
    n = x.shape[0]
    pos = np.zeros((n, 3))
    pos[:, 0] = x
    vel = np.zeros((n, 3))
    vel[:, 0] = vel_x
    nbr = np.full((n, 2), -1, dtype=np.int32)
    nbr[1:, 0] = np.arange(n - 1)
    nbr[:-1, 1] = np.arange(1, n)

    def full(v):
        return np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)).copy()

    return Model(pos=pos, vel=vel, n_h2=full(n_h2), temperature=full(temperature),
                 v_turb=full(v_turb), abundance=full(abundance), nbr=nbr)


def lattice_3d(m: int, spacing: float, n_h2=1e4, temperature=20.0, v_turb=1.5e4,
               abundance=1e-8) -> Model:
    """m^3 cubic lattice centred on the origin with 6-connected (face) neighbours."""
    idx = np.arange(m)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    c = (m - 1) / 2.0
    pos = np.stack([(I - c) * spacing, (J - c) * spacing, (K - c) * spacing], axis=1)
    n = pos.shape[0]
    lin = lambda a, b, d: (a * m + b) * m + d
    nbr = np.full((n, 6), -1, dtype=np.int32)
    slot = 0
    for (di, dj, dk) in [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]:
        a, b, d = I + di, J + dj, K + dk
        ok = (a >= 0) & (a < m) & (b >= 0) & (b < m) & (d >= 0) & (d < m)
        nbr[ok, slot] = lin(a[ok], b[ok], d[ok])
        slot += 1

    def full(v):
        return np.full(n, float(v))

    return Model(pos=pos, vel=np.zeros((n, 3)), n_h2=full(n_h2), temperature=full(temperature),
                 v_turb=full(v_turb), abundance=full(abundance), nbr=nbr)


def concat_models(models):
    """Concatenate models for a batched run: returns (offsets, merged model) with
    neighbour indices kept model-local."""
    offs = [0]
    for m in models:
        offs.append(offs[-1] + m.n_points)
    k = max(m.nbr.shape[1] for m in models)
    nbr = np.full((offs[-1], k), -1, dtype=np.int32)
    for m, o in zip(models, offs[:-1]):
        nbr[o:o + m.n_points, :m.nbr.shape[1]] = m.nbr
    cat = lambda name: np.concatenate([getattr(m, name) for m in models])
    merged = Model(pos=cat("pos"), vel=cat("vel"), n_h2=cat("n_h2"), temperature=cat("temperature"),
                   v_turb=cat("v_turb"), abundance=cat("abundance"), nbr=nbr)
    return np.array(offs, dtype=np.int64), merged
