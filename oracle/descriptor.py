"""FP64 oracle: atom-centred symmetry-function descriptors (not in the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The learned potential describes atom i by 24 features of its neighbours
j != i with r_ij < Rc = 2.5 (exact FP64 minimum-image predicate of
``oracle.lj``), cutoff function fc(r) = (cos(pi r / Rc) + 1) / 2:

  radial, k = 0..15:   G_k = sum_j exp(-eta_r (r_ij - R_k)^2) fc(r_ij),
                       R_k = 0.85 + 0.11 k, eta_r = 1 / (2 * 0.11^2)
  angular, 8 triples (zeta, lambda, eta) in {1,4} x {+1,-1} x {0.5, 2.0}:
                       G = 2^(1-zeta) sum_{j != k} (1 + lambda cos t_jik)^zeta w_j w_k,
                       w_j = exp(-eta r_ij^2) fc(r_ij),
  the sum over ordered pairs of distinct neighbours, t_jik the angle at i.

This is written as the direct double sum over neighbour pairs (an
independent route from a spherical-harmonic moment evaluation), together
with its analytic gradient, so that forces -dE/dr of any energy built on
these features can be formed by the chain rule.
"""
from __future__ import annotations

import math

import numpy as np

from .lj import separations, _chunk_rows

RC = 2.5
NRAD = 16
R_K = 0.85 + 0.11 * np.arange(NRAD)
ETA_R = 1.0 / (2.0 * 0.11 ** 2)
ANGULAR = [(z, lam, eta) for z in (1, 4) for lam in (1.0, -1.0) for eta in (0.5, 2.0)]
NFEAT = NRAD + len(ANGULAR)


def fc(r):
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < RC, 0.5 * (np.cos(math.pi * r / RC) + 1.0), 0.0)


def dfc(r):
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < RC, -0.5 * math.pi / RC * np.sin(math.pi * r / RC), 0.0)


def neighbour_table(pos, box, rows=None):
    """For each row i: (j indices, vectors u_ij = r_j - r_i (min image)).

    Returns a list of (j (n_i,), u (n_i, 3))."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    rc2 = RC * RC
    out = []
    step = _chunk_rows(n)
    for s in range(0, rows.shape[0], step):
        rr = rows[s : s + step]
        dx, dy, dz, d2 = separations(pos, box, rr)
        mask = d2 < rc2
        mask[np.arange(rr.shape[0]), rr] = False
        for a in range(rr.shape[0]):
            js = np.nonzero(mask[a])[0]
            # separations() gives r_i - r_j; the features use u = r_j - r_i
            u = -np.stack([dx[a, js], dy[a, js], dz[a, js]], axis=1)
            out.append((js, u))
    return out


def _center(u):
    """Features of one centre and their derivatives wrt each neighbour vector.

    Returns (G (24,), dG (24, n, 3)) with dG[f, j] = dG_f / du_j; the
    derivative wrt the centre's own position is -sum_j dG[f, j]."""
    n = u.shape[0]
    G = np.zeros(NFEAT)
    dG = np.zeros((NFEAT, n, 3))
    if n == 0:
        return G, dG
    r = np.sqrt(np.sum(u * u, axis=1))
    uh = u / r[:, None]
    f = fc(r)
    df = dfc(r)
    for k in range(NRAD):
        e = np.exp(-ETA_R * (r - R_K[k]) ** 2)
        phi = e * f
        dphi = e * (-2.0 * ETA_R * (r - R_K[k])) * f + e * df
        G[k] = phi.sum()
        dG[k] = dphi[:, None] * uh
    cos = uh @ uh.T  # c_jk
    off = ~np.eye(n, dtype=bool)
    for a, (zeta, lam, eta) in enumerate(ANGULAR):
        fidx = NRAD + a
        w = np.exp(-eta * r * r) * f
        dw = np.exp(-eta * r * r) * (-2.0 * eta * r) * f + np.exp(-eta * r * r) * df
        pref = 2.0 ** (1 - zeta)
        base = 1.0 + lam * cos
        t = base ** zeta * off
        ww = w[:, None] * w[None, :]
        G[fidx] = pref * np.sum(t * ww)
        # d/du_j of sum_{j != k} base^zeta w_j w_k, counting both (j,k) and (k,j)
        dbase = zeta * base ** (zeta - 1) * lam * off  # d(base^zeta)/dc
        # dc_jk/du_j = (uh_k - c_jk uh_j) / r_j
        coef = dbase * ww  # (j, k)
        term_c = (coef @ uh - (coef * cos).sum(axis=1)[:, None] * uh) / r[:, None]
        term_w = (t * w[None, :]).sum(axis=1)[:, None] * (dw / 1.0)[:, None] * uh
        dG[fidx] = pref * 2.0 * (term_c + term_w)
    return G, dG


def descriptors(pos, box, rows=None, with_grad: bool = False):
    """Features G (R, 24) for rows R; with_grad also returns the neighbour
    table and per-centre derivative blocks."""
    table = neighbour_table(pos, box, rows)
    G = np.zeros((len(table), NFEAT))
    grads = []
    for a, (js, u) in enumerate(table):
        g, dg = _center(u)
        G[a] = g
        if with_grad:
            grads.append(dg)
    if with_grad:
        return G, table, grads
    return G


def forces_from_feature_grad(n_atoms: int, rows, table, grads, dEdG):
    """F_a = -dE/dr_a for E = sum_i E_i(G_i), given dE_i/dG_i (R, 24) for
    every centre i in rows (rows must cover every atom whose features
    depend on a wanted force)."""
    F = np.zeros((n_atoms, 3))
    for a, i in enumerate(rows):
        js, _ = table[a]
        if js.shape[0] == 0:
            continue
        # dE/du_j for each neighbour j of centre i: sum_f dE/dG_f dG_f/du_j
        dEdu = np.einsum("f,fjc->jc", dEdG[a], grads[a])
        # u_j = r_j - r_i: dE/dr_j += dEdu_j, dE/dr_i -= sum_j dEdu_j
        np.add.at(F, js, -dEdu)
        F[i] += dEdu.sum(axis=0)
    return F
