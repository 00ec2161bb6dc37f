"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module only *makes inputs*: lattices, thermal velocities, random
boxes and polycrystals.  It holds none of the pair-loop arithmetic (no
distances, forces, bond orders or neighbour analysis) so that the oracle
and the device path stay independent while consuming identical data.

All generators use numpy's PCG64 with an explicit seed.

Workload recipes (the paper's LJ benchmark parameters: density 0.8442,
cutoff 2.5 sigma, periodic cubic box; Sec. 5.1 Tab. "7.2T1"; initial state
"periodic cubic lattice, normally distributed velocities", Sec. 5.3):

* ``lj_fluid(n_side, ...)``: simple-cubic sites at (i+1/2) a with
  a = L / n_side and L = (N / rho)^(1/3); velocities N(0, 1) * sqrt(T)
  per component, mean removed, rescaled so that sum m v^2 / (3 (N-1)) = T.
* ``polycrystal(...)``: periodic Voronoi grains of FCC / HCP / BCC (grain g
  gets phase g mod 3) with Haar-random orientations and Gaussian jitter.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng",
    "sc_lattice",
    "fcc_cells",
    "bcc_cells",
    "hcp_cells",
    "gaussian_velocities",
    "lj_fluid",
    "random_box",
    "random_rotation",
    "polycrystal",
    "perturb",
    "LJ_RHO",
    "mlp_init",
    "batch_indices",
    "fcc_lj",
]

LJ_RHO = 0.8442


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sc_lattice(n_side: int, rho: float = LJ_RHO):
    """Simple-cubic lattice of n_side^3 sites filling a cube at density rho.

    Returns (pos (N,3) float64, box (3,) float64)."""
    n = n_side ** 3
    L = (n / rho) ** (1.0 / 3.0)
    a = L / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * a
    # x fastest, then y, then z
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    return np.ascontiguousarray(pos), np.array([L, L, L])


def _tile(basis: np.ndarray, cell: np.ndarray, reps) -> np.ndarray:
    nx, ny, nz = reps
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    shifts = np.stack([ii.ravel() * cell[0], jj.ravel() * cell[1], kk.ravel() * cell[2]], axis=1)
    pts = (shifts[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    return pts


def fcc_cells(reps, a: float, offset: float = 0.25):
    """FCC crystal of reps=(nx,ny,nz) conventional cubic cells of side a."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], dtype=np.float64)
    basis = (basis + offset) * a
    pts = _tile(basis, np.array([a, a, a]), reps)
    return pts, np.array(reps, dtype=np.float64) * a


def bcc_cells(reps, a: float, offset: float = 0.25):
    basis = (np.array([[0, 0, 0], [0.5, 0.5, 0.5]], dtype=np.float64) + offset) * a
    pts = _tile(basis, np.array([a, a, a]), reps)
    return pts, np.array(reps, dtype=np.float64) * a


def hcp_cells(reps, d: float, offset: float = 0.1):
    """Ideal HCP (c/a = sqrt(8/3)) in the orthohexagonal 4-atom cell.

    Cell edges (d, d*sqrt(3), c); nearest-neighbour distance d."""
    c = d * math.sqrt(8.0 / 3.0)
    s3 = math.sqrt(3.0)
    cell = np.array([d, d * s3, c])
    basis = np.array(
        [
            [0.0, 0.0, 0.0],
            [0.5 * d, 0.5 * s3 * d, 0.0],
            [0.5 * d, s3 * d / 6.0, 0.5 * c],
            [0.0, 2.0 * s3 * d / 3.0, 0.5 * c],
        ]
    )
    basis = basis + offset * cell
    pts = _tile(basis, cell, reps)
    return pts, np.array(reps, dtype=np.float64) * cell


def gaussian_velocities(n: int, temperature: float, seed: int, mass: float = 1.0):
    """Gaussian velocities with zero net momentum and exact kinetic temperature."""
    r = rng(seed)
    v = r.standard_normal((n, 3)) * math.sqrt(temperature / mass)
    v -= v.mean(axis=0, keepdims=True)
    t_now = mass * float(np.sum(v * v)) / (3.0 * (n - 1))
    v *= math.sqrt(temperature / t_now)
    return np.ascontiguousarray(v)


def lj_fluid(n_side: int, rho: float = LJ_RHO, temperature: float = 1.0, seed: int = 1):
    """Simple-cubic start of the LJ benchmark workload: dict(pos, vel, box)."""
    pos, box = sc_lattice(n_side, rho)
    vel = gaussian_velocities(pos.shape[0], temperature, seed)
    return {"pos": pos, "vel": vel, "box": box}


def random_box(n: int, box, seed: int):
    """n uniformly random positions in [0, box)."""
    r = rng(seed)
    box = np.asarray(box, dtype=np.float64)
    return np.ascontiguousarray(r.random((n, 3)) * box[None, :])


def perturb(pos: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """Gaussian jitter of every Cartesian component."""
    return np.ascontiguousarray(pos + rng(seed).standard_normal(pos.shape) * sigma)


def random_rotation(r: np.random.Generator) -> np.ndarray:
    """Haar-random rotation matrix from a normalised Gaussian quaternion."""
    q = r.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def _phase_points(phase: int, d: float, half_extent: float):
    """Lattice points of one phase covering the cube [-h, h]^3 (unrotated).

    All phases have atomic volume d^3 / sqrt(2) (number density sqrt(2)/d^3)."""
    if phase == 0:  # FCC, nearest-neighbour distance d
        a = d * math.sqrt(2.0)
        cell = np.array([a, a, a])
        basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) * a
    elif phase == 1:  # HCP, ideal c/a
        c = d * math.sqrt(8.0 / 3.0)
        s3 = math.sqrt(3.0)
        cell = np.array([d, d * s3, c])
        basis = np.array(
            [[0, 0, 0], [0.5 * d, 0.5 * s3 * d, 0], [0.5 * d, s3 * d / 6.0, 0.5 * c], [0, 2 * s3 * d / 3.0, 0.5 * c]]
        )
    else:  # BCC with the same atomic volume: a^3 / 2 = d^3 / sqrt(2)
        a = (2.0 * d ** 3 / math.sqrt(2.0)) ** (1.0 / 3.0)
        cell = np.array([a, a, a])
        basis = np.array([[0, 0, 0], [0.5, 0.5, 0.5]]) * a
    reps = [int(math.ceil(2 * half_extent / cell[k])) + 2 for k in range(3)]
    pts = _tile(basis, cell, reps)
    pts -= (np.array(reps) * cell) * 0.5
    return pts


def polycrystal(n_target: int, n_grains: int, seed: int, rho: float = 1.0, jitter: float = 0.05):
    """Periodic Voronoi polycrystal of FCC/HCP/BCC grains.

    Nearest-neighbour distance d follows from rho (rho = sqrt(2)/d^3 for all
    three phases); grain g has phase g mod 3 (0 FCC, 1 HCP, 2 BCC), a
    Haar-random orientation, and every coordinate gets N(0, (jitter*d)^2)
    noise.  Returns dict(pos, box, grain, phase, d)."""
    from scipy.spatial import cKDTree  # input generation only

    r = rng(seed)
    L = (n_target / rho) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    d = (math.sqrt(2.0) / rho) ** (1.0 / 3.0)
    seeds = r.random((n_grains, 3)) * L
    rots = [random_rotation(r) for _ in range(n_grains)]
    tree = cKDTree(seeds, boxsize=L)
    # bounding radius of every Voronoi cell from a probe grid
    ng = 48
    g = (np.arange(ng) + 0.5) * (L / ng)
    probe = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    dist, owner = tree.query(probe)
    rmax = np.zeros(n_grains)
    np.maximum.at(rmax, owner, dist)
    rmax += 2.0 * L / ng + 2.0 * d
    out_pos, out_grain = [], []
    for gi in range(n_grains):
        pts = _phase_points(gi % 3, d, rmax[gi])
        pts = pts[np.einsum("ij,ij->i", pts, pts) <= rmax[gi] ** 2]
        pts = pts @ rots[gi].T + seeds[gi]
        pts -= L * np.floor(pts / L)
        _, own = tree.query(pts)
        keep = pts[own == gi]
        out_pos.append(keep)
        out_grain.append(np.full(keep.shape[0], gi, dtype=np.int32))
    pos = np.concatenate(out_pos)
    grain = np.concatenate(out_grain)
    pos = pos + r.standard_normal(pos.shape) * (jitter * d)
    pos -= L * np.floor(pos / L)
    pos[pos >= L] -= L
    return {
        "pos": np.ascontiguousarray(pos),
        "box": box,
        "grain": grain,
        "phase": (grain % 3).astype(np.int32),
        "d": d,
    }


def mlp_init(seed: int, n_in: int = 24, n_pad: int = 32, n_hidden: int = 64):
    """Initial weights of the 24(32)-64-64-1 network: uniform in
    +-1/sqrt(fan_in) from PCG64(seed), biases zero, padding columns zero."""
    r = rng(seed)
    W1 = r.uniform(-1, 1, (n_hidden, n_pad)) / math.sqrt(n_in)
    W1[:, n_in:] = 0.0
    W2 = r.uniform(-1, 1, (n_hidden, n_hidden)) / math.sqrt(n_hidden)
    w3 = r.uniform(-1, 1, n_hidden) / math.sqrt(n_hidden)
    return {"W1": W1, "b1": np.zeros(n_hidden), "W2": W2, "b2": np.zeros(n_hidden), "w3": w3,
            "b3": np.zeros(1)}


def batch_indices(n_rows: int, batch: int, steps: int, seed: int):
    """Mini-batch row indices (steps x batch, int32), drawn uniformly with
    replacement from PCG64(seed)."""
    return rng(seed).integers(0, n_rows, size=(steps, batch), dtype=np.int32)


def fcc_lj(n_cells: int, rho: float = LJ_RHO, temperature: float = 1.0, seed: int = 1):
    """FCC start with n_cells^3 conventional cells at density rho and Gaussian
    velocities: dict(pos, vel, box)."""
    a = (4.0 / rho) ** (1.0 / 3.0)
    pos, box = fcc_cells((n_cells,) * 3, a)
    vel = gaussian_velocities(pos.shape[0], temperature, seed)
    return {"pos": np.ascontiguousarray(pos), "vel": vel, "box": box}
