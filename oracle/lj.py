"""FP64 oracle: neighbour sets, Lennard-Jones forces/energy/virial, velocity Verlet.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here is the plain all-pairs definition (the sequential pair loop
over all ordered pairs i != j of Sec. 3.4, Listing "simplest_pairloop"),
evaluated with the minimum-image convention in a periodic orthorhombic box
[0,Lx) x [0,Ly) x [0,Lz) (Sec. 3.5).  Cell and neighbour lists only reach
this result faster, so the oracle never builds them.

Exact operation order (shared contract with any implementation that claims
bit-exact neighbour sets):
    dx = xi - xj ; if dx > 0.5*L: dx -= L ; elif dx < -0.5*L: dx += L
    d2 = (dx*dx + dy*dy) + dz*dz           (each operation rounded, no FMA)
    neighbour  <=>  d2 < r2                (strict; r2 supplied by caller)
numpy evaluates every elementwise operation separately in IEEE binary64,
so this is exactly that sequence.

Readings of the paper taken here:
* Potential (Eq. LJpotential) carries a "+1/4" inside 4 eps(...), which the
  listing also adds.  Shift modes: "none" V = 4 eps[(s/r)^12 - (s/r)^6]
  (V(2^(1/6) s) = -eps); "paper" adds +eps (the printed form); "cutoff"
  subtracts V_none(rc).  Forces do not depend on the mode.
* Force (Eq. LJforce): F_i = sum_j 48 eps / s^2 [(s^2/d2)^7 - 1/2 (s^2/d2)^4] dr_ij
  with dr_ij = r_i - r_j (min image), i.e. F = -grad V.  The listing's
  constant C_F = -48 eps / s^2 with the same dr has the opposite sign; the
  equation is followed (finite differences and energy conservation pin it).
* Energy: the listing adds V once per ordered pair, which counts every pair
  twice; here PE = 1/2 sum_{i != j} V = sum_{i<j} V and e_i = 1/2 sum_j V.
* Virial W = sum_{i<j} dr_ij . f_ij.
* Cutoff comparisons are strict (d2 < rc^2) everywhere.
"""
from __future__ import annotations

import math

import numpy as np

from . import thermostat

SHIFT_MODES = ("none", "paper", "cutoff")

# rows of the all-pairs matrix processed per chunk: chunk * N <= this
_CHUNK_ELEMS = 1 << 22


def _chunk_rows(n: int) -> int:
    return max(1, _CHUNK_ELEMS // max(n, 1))


def min_image(d: np.ndarray, L: float) -> np.ndarray:
    """Minimum image of one coordinate difference, single conditional wrap."""
    d = np.array(d, dtype=np.float64, copy=True)
    h = 0.5 * L
    hi = d > h
    lo = d < -h
    d[hi] = d[hi] - L
    d[lo] = d[lo] + L
    return d


def separations(pos: np.ndarray, box, rows) -> tuple:
    """dr = r_i - r_j (min image) and d2 for rows i against all j.

    Returns (dx, dy, dz, d2), each of shape (len(rows), N)."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    rows = np.asarray(rows)
    dx = min_image(pos[rows, 0][:, None] - pos[None, :, 0], box[0])
    dy = min_image(pos[rows, 1][:, None] - pos[None, :, 1], box[1])
    dz = min_image(pos[rows, 2][:, None] - pos[None, :, 2], box[2])
    d2 = (dx * dx + dy * dy) + dz * dz
    return dx, dy, dz, d2


def neighbour_pairs(pos: np.ndarray, box, r2: float, rows=None) -> np.ndarray:
    """Directed pairs (i, j), i != j, with d2 < r2, sorted lexicographically.

    ``rows`` restricts i to a subset (all j are still scanned).
    Returns an int64 array of shape (P, 2)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    rows = np.arange(n) if rows is None else np.sort(np.asarray(rows, dtype=np.int64))
    out = []
    step = _chunk_rows(n)
    for s in range(0, rows.shape[0], step):
        rr = rows[s : s + step]
        _, _, _, d2 = separations(pos, box, rr)
        mask = d2 < r2
        mask[np.arange(rr.shape[0]), rr] = False
        ii, jj = np.nonzero(mask)
        out.append(np.stack([rr[ii], jj], axis=1))
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    p = np.concatenate(out).astype(np.int64)
    order = np.lexsort((p[:, 1], p[:, 0]))
    return p[order]


def ext_radius_sq(rc: float, skin: float) -> float:
    """Squared neighbour-list radius (rc + skin)^2, each step rounded in FP64."""
    r = float(rc) + float(skin)
    return r * r


# --------------------------------------------------------------------------
# Lennard-Jones pair functions (Eqs. LJpotential and LJforce)
# --------------------------------------------------------------------------

def lj_potential_r2(d2, eps: float = 1.0, sigma: float = 1.0, shift: str = "none", rc: float = 2.5):
    """V as a function of the squared distance."""
    d2 = np.asarray(d2, dtype=np.float64)
    s6 = (sigma * sigma / d2) ** 3
    v = 4.0 * eps * (s6 * s6 - s6)
    if shift == "none":
        return v
    if shift == "paper":
        return v + eps  # 4 eps * 1/4
    if shift == "cutoff":
        sc6 = (sigma * sigma / (rc * rc)) ** 3
        return v - 4.0 * eps * (sc6 * sc6 - sc6)
    raise ValueError(shift)


def lj_force_factor_r2(d2, eps: float = 1.0, sigma: float = 1.0):
    """g(d2) with f_ij = g * dr_ij:  48 eps / s^2 [(s^2/d2)^7 - 1/2 (s^2/d2)^4]."""
    d2 = np.asarray(d2, dtype=np.float64)
    s = sigma * sigma / d2
    return 48.0 * eps / (sigma * sigma) * (s ** 7 - 0.5 * s ** 4)


def lj_forces(pos, box, rc: float, eps: float = 1.0, sigma: float = 1.0, shift: str = "none", rows=None):
    """All-pairs LJ forces, per-atom energies, total PE and virial.

    Returns dict(F (R,3), e (R,), pe, w, nb (R,)) for rows R (default all).
    pe and w are sums over the rows given (the full system when rows=None)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    rc2 = float(rc) * float(rc)
    F = np.zeros((rows.shape[0], 3))
    e = np.zeros(rows.shape[0])
    w_i = np.zeros(rows.shape[0])
    nb = np.zeros(rows.shape[0], dtype=np.int64)
    step = _chunk_rows(n)
    for s in range(0, rows.shape[0], step):
        rr = rows[s : s + step]
        dx, dy, dz, d2 = separations(pos, box, rr)
        mask = d2 < rc2
        mask[np.arange(rr.shape[0]), rr] = False
        d2m = np.where(mask, d2, 1.0)
        g = np.where(mask, lj_force_factor_r2(d2m, eps, sigma), 0.0)
        F[s : s + rr.shape[0], 0] = np.sum(g * dx, axis=1)
        F[s : s + rr.shape[0], 1] = np.sum(g * dy, axis=1)
        F[s : s + rr.shape[0], 2] = np.sum(g * dz, axis=1)
        v = np.where(mask, lj_potential_r2(d2m, eps, sigma, shift, rc), 0.0)
        e[s : s + rr.shape[0]] = 0.5 * np.sum(v, axis=1)
        w_i[s : s + rr.shape[0]] = 0.5 * np.sum(g * d2m * mask, axis=1)
        nb[s : s + rr.shape[0]] = mask.sum(axis=1)
    return {"F": F, "e": e, "pe": float(np.sum(e)), "w": float(np.sum(w_i)), "nb": nb}


# --------------------------------------------------------------------------
# The same results for large N: scipy's k-d tree proposes candidate pairs,
# the definition above decides (the tree's own distance test is never
# trusted; its radius is padded so that it can only over-propose).
# --------------------------------------------------------------------------

def candidate_pairs(pos, box, radius: float, workers: int = -1):
    """Directed pairs (i, j), i != j, a superset of those closer than radius
    (cKDTree over the folded positions, periodic, all host threads)."""
    from scipy.spatial import cKDTree

    pos = np.asarray(pos, dtype=np.float64)
    folded = wrap(pos, box)
    tree = cKDTree(folded, boxsize=np.asarray(box, dtype=np.float64))
    pad = float(radius) * (1.0 + 1e-9) + 1e-9
    lists = tree.query_ball_point(folded, pad, workers=workers, return_sorted=False)
    cnt = np.fromiter((len(a) for a in lists), dtype=np.int64, count=len(lists))
    j = np.concatenate(lists).astype(np.int64) if cnt.sum() else np.zeros(0, dtype=np.int64)
    i = np.repeat(np.arange(len(lists), dtype=np.int64), cnt)
    keep = i != j
    return i[keep], j[keep]


def _pair_separations(pos, box, i, j):
    """dr = r_i - r_j (min image, the definition's operation order) and d2 for pairs."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    dx = min_image(pos[i, 0] - pos[j, 0], box[0])
    dy = min_image(pos[i, 1] - pos[j, 1], box[1])
    dz = min_image(pos[i, 2] - pos[j, 2], box[2])
    d2 = (dx * dx + dy * dy) + dz * dz
    return dx, dy, dz, d2


def neighbour_pairs_tree(pos, box, r2: float, workers: int = -1) -> np.ndarray:
    """neighbour_pairs for all rows, through candidate_pairs (sorted, int64 (P, 2))."""
    i, j = candidate_pairs(pos, box, math.sqrt(r2), workers)
    d2 = _pair_separations(pos, box, i, j)[3]
    m = d2 < r2
    p = np.stack([i[m], j[m]], axis=1)
    return p[np.lexsort((p[:, 1], p[:, 0]))]


def lj_forces_tree(pos, box, rc: float, eps: float = 1.0, sigma: float = 1.0, shift: str = "none",
                   workers: int = -1):
    """lj_forces for every atom, through candidate_pairs: the same pairs and
    pair terms, summed per atom in another order (so equal to rounding)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    rc2 = float(rc) * float(rc)
    i, j = candidate_pairs(pos, box, float(rc), workers)
    dx, dy, dz, d2 = _pair_separations(pos, box, i, j)
    m = d2 < rc2
    i, dx, dy, dz, d2 = i[m], dx[m], dy[m], dz[m], d2[m]
    g = lj_force_factor_r2(d2, eps, sigma)
    v = lj_potential_r2(d2, eps, sigma, shift, rc)
    F = np.stack([np.bincount(i, g * dx, n), np.bincount(i, g * dy, n), np.bincount(i, g * dz, n)], axis=1)
    e = 0.5 * np.bincount(i, v, n)
    w = 0.5 * float(np.sum(g * d2))
    return {"F": F, "e": e, "pe": float(np.sum(e)), "w": w, "nb": np.bincount(i, minlength=n)}


def kinetic_energy(vel, mass: float = 1.0) -> float:
    """K = sum_i 1/2 m |v_i|^2 (the Particle Loop example of Sec. 2)."""
    vel = np.asarray(vel, dtype=np.float64)
    return float(0.5 * mass * np.sum(vel * vel))


def wrap(pos, box):
    """Fold positions into [0, L) per axis: x - L floor(x / L), then one
    correction by L if rounding left the value at L or below 0."""
    box = np.asarray(box, dtype=np.float64)
    p = pos - box[None, :] * np.floor(pos / box[None, :])
    p = np.where(p >= box[None, :], p - box[None, :], p)
    p = np.where(p < 0.0, p + box[None, :], p)
    return p


def velocity_verlet(pos, vel, box, nsteps: int, dt: float, rc: float, eps: float = 1.0, sigma: float = 1.0,
                    mass: float = 1.0, shift: str = "none", sample_every: int = 0, force_fn=None,
                    andersen=None, record_vmax: bool = False):
    """Velocity Verlet exactly in the order of Alg. VelocityVerlet.

    force_fn(x) -> dict(F, pe, w) replaces the LJ force field when given
    (the algorithm is the same for any force field).  andersen: optional
    dict(temperature, nu, seed, step0, ids) adding the collisions of
    oracle.thermostat after each step's second half kick (and after its
    thermo sample); global step = step0 + local step, ids the particles' ids.

    F(r_0) is computed before the first step (the algorithm uses F in its
    first half kick without showing its computation).  Per step:
        v += dt/(2m) F ; r += dt v      (ParticleLoop, line "6")
        F  = sum_j f(r_i, r_j)          (PairLoop, INC_ZERO)
        v += dt/(2m) F                  (ParticleLoop)
    Positions are not folded back into the box (min image handles any
    |dx| < 1.5 L).  Thermo samples (step, KE, PE, W) are taken at step 0 and
    every ``sample_every`` steps after the second half kick.

    record_vmax: also return vmax, the largest speed |v| of each step's
    drift (the velocities after its first half kick), the input of the
    list-reuse rule (``rebuild_schedule``).

    Returns dict(pos, vel, F, thermo (S,4)[, vmax (nsteps,)])."""
    x = np.array(pos, dtype=np.float64, copy=True)
    v = np.array(vel, dtype=np.float64, copy=True)
    h = dt / (2.0 * mass)
    if force_fn is None:
        def force_fn(r):
            return lj_forces(r, box, rc, eps, sigma, shift)
    res = force_fn(x)
    F = res["F"]
    thermo = []
    if sample_every:
        thermo.append((0, kinetic_energy(v, mass), res["pe"], res["w"]))
    vmax = []
    for step in range(1, nsteps + 1):
        v = v + h * F
        if record_vmax:
            vmax.append(float(np.max(np.sqrt(np.sum(v * v, axis=1)))))
        x = x + dt * v
        res = force_fn(x)
        F = res["F"]
        v = v + h * F
        if sample_every and step % sample_every == 0:
            thermo.append((step, kinetic_energy(v, mass), res["pe"], res["w"]))
        if andersen is not None:
            v, _ = thermostat.andersen(v, andersen["ids"], andersen["step0"] + step, andersen["temperature"],
                                       andersen["nu"], dt, andersen["seed"], mass)
    out = {"pos": x, "vel": v, "F": F, "thermo": np.array(thermo, dtype=np.float64).reshape(-1, 4)}
    if record_vmax:
        out["vmax"] = np.array(vmax)
    return out


def rebuild_schedule(vmax, dt: float, skin: float, reuse_every: int, bound: float = 0.0,
                     since: int = 0):
    """Steps at which the lists are rebuilt under the reuse rule of Eq.
    extended_cutoff (Sec. 3.5): a list built with the extra shell delta =
    skin stays valid for n steps while 2 n dt v_max < delta.  Read per step:
    after the drift of step k, with B = sum over the steps since the last
    build of dt * vmax[k] (the largest speed of the velocities that moved
    the particles in that step), the list is rebuilt before the force pass
    of step k if 2 B >= skin, or if reuse_every steps have passed since the
    last build (the largest reuse count given with delta).  ``vmax[k - 1]``
    is step k's speed (k = 1 .. len(vmax)); ``bound`` and ``since`` carry a
    period over from an earlier call.  Returns (list of rebuild steps,
    bound, since) at the end."""
    steps = []
    for k, v in enumerate(vmax, start=1):
        bound += dt * float(v)
        since += 1
        if since >= reuse_every or 2.0 * bound >= skin:
            steps.append(k)
            bound = 0.0
            since = 0
    return steps, bound, since


def sc_shell_energy(a: float, rc: float, eps: float = 1.0, sigma: float = 1.0, shift: str = "none") -> float:
    """Per-atom energy of a perfect simple-cubic lattice by enumerating the
    lattice vectors n*a (n integer, 0 < |n a| < rc):  1/2 sum V(|n a|)."""
    m = int(math.ceil(rc / a)) + 1
    tot = 0.0
    for i in range(-m, m + 1):
        for j in range(-m, m + 1):
            for k in range(-m, m + 1):
                if i == 0 and j == 0 and k == 0:
                    continue
                d2 = (i * a) ** 2 + (j * a) ** 2 + (k * a) ** 2
                if d2 < rc * rc:
                    tot += float(lj_potential_r2(d2, eps, sigma, shift, rc))
    return 0.5 * tot


def local_subset(pos, box, centre: int, radius: float) -> np.ndarray:
    """Indices of atoms whose min-image separation from ``centre`` is
    <= radius in every axis (a conservative superset of the ball)."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    keep = np.ones(pos.shape[0], dtype=bool)
    for k in range(3):
        d = min_image(pos[centre, k] - pos[:, k], box[k])
        keep &= np.abs(d) <= radius
    return np.nonzero(keep)[0]
