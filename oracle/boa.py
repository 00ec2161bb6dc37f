"""FP64 oracle: Steinhardt bond-order parameters (Sec. 4.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For atom i with neighbour set N(i) = {j != i : |r_i - r_j| < rc} (min image,
strict, same exact predicate as ``oracle.lj``):
    q_lm = (1/|N(i)|) sum_{j in N(i)} Y_l^m(rhat_ij)          (Eq. qellm)
    Q_l  = sqrt(4 pi / (2l+1) sum_m |q_lm|^2)                   (Eq. Qell)
computed as the paper's two loops: a pair loop accumulating the moments
q~_lm = sum_j Y_l^m and the count nu (Alg. sph_I), then a particle loop
dividing by nu and forming Q_l (Alg. sph_II).

Readings: Y_l^m are the orthonormal complex spherical harmonics
(scipy.special.sph_harm_y), which reproduce Tab. Q4Q6; the direction is
rhat = (r_i - r_j)/|r_i - r_j| (its sign cannot change |q_lm|^2 for even l,
and for odd l it flips every term's sign together); an atom with no
neighbour gets nu = 0 and Q_l = 0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y

from .lj import separations, _chunk_rows


def neighbour_vectors(pos, box, rc: float, rows=None):
    """For each row i: the min-image vectors r_i - r_j of its neighbours.

    Returns (owner (P,), dr (P,3)) with owner the position in ``rows``."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    rc2 = float(rc) * float(rc)
    owners, drs = [], []
    step = _chunk_rows(n)
    for s in range(0, rows.shape[0], step):
        rr = rows[s : s + step]
        dx, dy, dz, d2 = separations(pos, box, rr)
        mask = d2 < rc2
        mask[np.arange(rr.shape[0]), rr] = False
        ii, jj = np.nonzero(mask)
        owners.append(ii + s)
        drs.append(np.stack([dx[ii, jj], dy[ii, jj], dz[ii, jj]], axis=1))
    if not owners:
        return np.zeros(0, dtype=np.int64), np.zeros((0, 3))
    return np.concatenate(owners), np.concatenate(drs)


def moments(owner, dr, nrows: int, l: int):
    """Alg. sph_I: q~_lm = sum_j Y_l^m(rhat_ij), m = -l..l, and nu = |N(i)|."""
    r = np.sqrt(np.sum(dr * dr, axis=1))
    u = dr / r[:, None]
    theta = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    phi = np.arctan2(u[:, 1], u[:, 0])
    q = np.zeros((nrows, 2 * l + 1), dtype=np.complex128)
    for k, m in enumerate(range(-l, l + 1)):
        y = sph_harm_y(l, m, theta, phi)
        q[:, k] = np.bincount(owner, weights=y.real, minlength=nrows) + 1j * np.bincount(
            owner, weights=y.imag, minlength=nrows
        )
    nu = np.bincount(owner, minlength=nrows)
    return q, nu


def order_parameter(qt, nu, l: int):
    """Alg. sph_II: q_lm = q~_lm / nu, Q_l = sqrt(4 pi/(2l+1) sum_m |q_lm|^2)."""
    out = np.zeros(qt.shape[0])
    ok = nu > 0
    q = qt[ok] / nu[ok][:, None]
    out[ok] = np.sqrt(4.0 * math.pi / (2 * l + 1) * np.sum(np.abs(q) ** 2, axis=1))
    return out


def bond_order(pos, box, rc: float, ls=(4, 6), rows=None):
    """Q_l for every l in ``ls`` and the neighbour count, per row.

    Returns dict {l: Q_l (R,)} plus key "nu"."""
    pos = np.asarray(pos, dtype=np.float64)
    nrows = pos.shape[0] if rows is None else len(rows)
    owner, dr = neighbour_vectors(pos, box, rc, rows)
    res = {}
    nu = None
    for l in ls:
        qt, nu = moments(owner, dr, nrows, l)
        res[l] = order_parameter(qt, nu, l)
    if nu is None:
        nu = np.bincount(owner, minlength=nrows)
    res["nu"] = nu
    return res


def q_from_directions(vectors, l: int) -> float:
    """Q_l of a single atom whose neighbours lie along the given vectors."""
    v = np.asarray(vectors, dtype=np.float64).reshape(-1, 3)
    qt, nu = moments(np.zeros(v.shape[0], dtype=np.int64), v, 1, l)
    return float(order_parameter(qt, nu, l)[0])
