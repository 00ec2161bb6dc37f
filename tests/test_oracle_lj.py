"""Pins of the FP64 oracle's pair-set, Lennard-Jones and velocity-Verlet parts.

Each pin is fixed by something other than the oracle itself: closed forms of
Eqs. LJpotential / LJforce, a pure-Python brute force of the sequential pair
loop, lattice-shell enumeration, finite differences, symmetry and
time-reversal of Alg. VelocityVerlet.
"""
import math

import numpy as np
import pytest

import mdinputs
from oracle import lj


# ---------------------------------------------------------------- closed forms
def test_potential_closed_forms():
    rmin2 = 2.0 ** (1.0 / 3.0)  # (2^(1/6))^2
    # (s/r)^6 = 1/2 at the minimum:  4 (1/4 - 1/2) = -1
    assert lj.lj_potential_r2(rmin2) == pytest.approx(-1.0, abs=1e-14)
    assert lj.lj_potential_r2(1.0) == 0.0
    # the printed form (+1/4 inside 4 eps) is zero at the minimum
    assert lj.lj_potential_r2(rmin2, shift="paper") == pytest.approx(0.0, abs=1e-14)
    # eps and sigma scale as expected
    assert lj.lj_potential_r2(rmin2 * 1.5 ** 2, eps=2.0, sigma=1.5) == pytest.approx(-2.0, abs=1e-13)
    # V(2.5) = 4 (2.5^-12 - 2.5^-6)
    v25 = 4.0 * (2.5 ** -12 - 2.5 ** -6)
    assert lj.lj_potential_r2(6.25) == pytest.approx(v25, rel=1e-15)
    assert v25 == pytest.approx(-0.016316891, abs=1e-9)
    # cutoff-shifted potential vanishes at rc
    assert lj.lj_potential_r2(6.25, shift="cutoff", rc=2.5) == pytest.approx(0.0, abs=1e-16)


def test_force_closed_forms():
    rmin2 = 2.0 ** (1.0 / 3.0)
    assert lj.lj_force_factor_r2(rmin2) == pytest.approx(0.0, abs=1e-13)
    # |F(2.5)| = 24 (2 * 2.5^-13 - 2.5^-7)
    g = lj.lj_force_factor_r2(6.25)
    assert abs(g * 2.5) == pytest.approx(abs(24.0 * (2.0 * 2.5 ** -13 - 2.5 ** -7)), rel=1e-14)
    assert abs(g * 2.5) == pytest.approx(0.0389995, abs=1e-7)
    # repulsive inside the minimum, attractive outside: g > 0 pushes i away from j
    assert lj.lj_force_factor_r2(1.0) > 0 and lj.lj_force_factor_r2(2.0) < 0


def test_force_is_minus_gradient_of_potential_1d():
    # f(r) = -dV/dr along the pair axis, central differences of the scalar V(r)
    for r in (0.95, 1.1, 1.5, 2.2):
        h = 1e-6
        dv = (lj.lj_potential_r2((r + h) ** 2) - lj.lj_potential_r2((r - h) ** 2)) / (2 * h)
        assert lj.lj_force_factor_r2(r * r) * r == pytest.approx(-dv, rel=1e-8)


# ---------------------------------------------------------------- pair sets
def _brute_pairs(pos, box, r2):
    """Sequential all-pairs loop in pure Python floats (Listing
    simplest_pairloop), same min-image and evaluation order."""
    out = []
    n = len(pos)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = []
            for k in range(3):
                t = pos[i][k] - pos[j][k]
                if t > 0.5 * box[k]:
                    t = t - box[k]
                elif t < -0.5 * box[k]:
                    t = t + box[k]
                d.append(t)
            d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
            if d2 < r2:
                out.append((i, j))
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_neighbour_pairs_match_brute_force(seed):
    box = np.array([4.1, 3.7, 5.3])
    pos = mdinputs.random_box(60, box, seed)
    # push a few atoms onto / across the box faces
    pos[:4, 0] = [0.0, box[0] - 1e-12, -0.3, box[0] + 0.2]
    r2 = lj.ext_radius_sq(1.0, 0.3)
    got = [tuple(p) for p in lj.neighbour_pairs(pos, box, r2)]
    want = sorted(_brute_pairs(pos.tolist(), box.tolist(), r2))
    assert got == want


def test_neighbour_pairs_boundary_exact():
    # two atoms at exactly r apart along x: strict '<' excludes them
    box = np.array([10.0, 10.0, 10.0])
    pos = np.array([[1.0, 5.0, 5.0], [3.0, 5.0, 5.0], [9.5, 5.0, 5.0]])
    assert lj.neighbour_pairs(pos, box, 4.0).tolist() == [[0, 2], [2, 0]]
    assert lj.neighbour_pairs(pos, box, np.nextafter(4.0, 5.0)).shape[0] == 4


def test_neighbour_pairs_permutation_invariant():
    box = np.array([6.0, 6.0, 6.0])
    pos = mdinputs.random_box(200, box, 11)
    perm = mdinputs.rng(5).permutation(200)
    r2 = lj.ext_radius_sq(1.2, 0.2)
    a = lj.neighbour_pairs(pos, box, r2)
    b = lj.neighbour_pairs(pos[perm], box, r2)
    b = perm[b]
    b = b[np.lexsort((b[:, 1], b[:, 0]))]
    assert np.array_equal(a, b)


def test_rows_subset_matches_full():
    box = np.array([6.0, 6.0, 6.0])
    pos = mdinputs.random_box(150, box, 12)
    r2 = 1.69
    full = lj.neighbour_pairs(pos, box, r2)
    rows = np.array([3, 17, 99, 149])
    sub = lj.neighbour_pairs(pos, box, r2, rows)
    assert np.array_equal(sub, full[np.isin(full[:, 0], rows)])


# ---------------------------------------------------------------- lattices
def test_sc_lattice_counts_forces_energy():
    pos, box = mdinputs.sc_lattice(10)  # the N=1000 benchmark start
    a = box[0] / 10
    assert a == pytest.approx(1.058079, abs=1e-6)
    res = lj.lj_forces(pos, box, 2.5)
    assert np.all(res["nb"] == 56)
    assert lj.neighbour_pairs(pos, box, lj.ext_radius_sq(2.5, 0.3)).shape[0] == 80 * 1000
    # perfect lattice: every force vanishes by symmetry
    assert np.max(np.abs(res["F"])) < 1e-11
    # per-atom energy from the shells 6,12,8,6,24 at a*{1,sqrt2,sqrt3,2,sqrt5}
    shells = [(6, 1.0), (12, 2.0), (8, 3.0), (6, 4.0), (24, 5.0)]
    e_atom = 0.5 * sum(n * 4.0 * ((a * a * k) ** -6 - (a * a * k) ** -3) for n, k in shells)
    assert e_atom == pytest.approx(-5.2202185, abs=2e-7)
    assert res["pe"] / 1000 == pytest.approx(e_atom, rel=1e-12)
    assert lj.sc_shell_energy(a, 2.5) == pytest.approx(e_atom, rel=1e-12)
    assert np.allclose(res["e"], e_atom, rtol=1e-12)


def test_fcc_lattice_forces_vanish():
    pos, box = mdinputs.fcc_cells((4, 4, 4), 1.6796)
    res = lj.lj_forces(pos, box, 2.5)
    assert np.max(np.abs(res["F"])) < 1e-11


# ---------------------------------------------------------------- gradients
def _config(seed, n=48, L=5.2):
    """Random configuration with no pair closer than 0.9 or within 1e-3 of rc."""
    box = np.array([L, L, L])
    r = mdinputs.rng(seed)
    pos = []
    while len(pos) < n:
        p = r.random(3) * L
        ok = True
        for q in pos:
            d = p - q
            d -= L * np.round(d / L)
            dd = math.sqrt(float(d @ d))
            if dd < 0.9 or abs(dd - 2.5) < 2e-3:
                ok = False
                break
        if ok:
            pos.append(p)
    return np.array(pos), box


@pytest.mark.parametrize("shift", ["none", "paper", "cutoff"])
def test_forces_are_minus_gradient_of_pe(shift):
    pos, box = _config(3)
    F = lj.lj_forces(pos, box, 2.5, shift=shift)["F"]
    h = 1e-6
    fd = np.zeros_like(pos)
    for i in range(0, pos.shape[0], 5):
        for k in range(3):
            p = pos.copy()
            p[i, k] += h
            ep = lj.lj_forces(p, box, 2.5, shift=shift)["pe"]
            p[i, k] -= 2 * h
            em = lj.lj_forces(p, box, 2.5, shift=shift)["pe"]
            fd[i, k] = -(ep - em) / (2 * h)
    sel = np.arange(0, pos.shape[0], 5)
    err = np.abs(fd[sel] - F[sel]).max()
    assert err <= 1e-7 * max(1.0, np.abs(F[sel]).max())


def test_net_force_zero_and_pe_is_half_sum():
    pos, box = _config(4)
    res = lj.lj_forces(pos, box, 2.5)
    assert np.linalg.norm(res["F"].sum(axis=0)) <= 1e-12 * np.abs(res["F"]).sum()
    # PE equals the sum over unordered pairs
    p = lj.neighbour_pairs(pos, box, 6.25)
    p = p[p[:, 0] < p[:, 1]]
    tot = 0.0
    for i, j in p:
        d = pos[i] - pos[j]
        d = lj.min_image(d, box[0])
        tot += float(lj.lj_potential_r2(float(d @ d)))
    assert res["pe"] == pytest.approx(tot, rel=1e-12)


def test_virial_is_minus_volume_derivative():
    pos, box = _config(5)
    w = lj.lj_forces(pos, box, 2.5)["w"]
    h = 1e-6
    up = lj.lj_forces(pos * (1 + h), box * (1 + h), 2.5)["pe"]
    dn = lj.lj_forces(pos * (1 - h), box * (1 - h), 2.5)["pe"]
    assert w == pytest.approx(-(up - dn) / (2 * h), rel=1e-6)


def test_rows_forces_match_full():
    pos, box = _config(6)
    full = lj.lj_forces(pos, box, 2.5)
    rows = np.array([0, 7, 13])
    sub = lj.lj_forces(pos, box, 2.5, rows=rows)
    assert np.allclose(sub["F"], full["F"][rows], rtol=0, atol=1e-13)
    assert np.allclose(sub["e"], full["e"][rows], rtol=0, atol=1e-14)


# ---------------------------------------------------------------- integrator
def test_kinetic_energy_closed_form():
    v = np.tile([1.0, 2.0, 2.0], (10, 1))
    assert lj.kinetic_energy(v, mass=2.0) == pytest.approx(10 * 0.5 * 2.0 * 9.0)


def test_velocity_verlet_time_reversible():
    d = mdinputs.lj_fluid(6, temperature=1.0, seed=3)
    fwd = lj.velocity_verlet(d["pos"], d["vel"], d["box"], 60, 0.002, 2.5)
    back = lj.velocity_verlet(fwd["pos"], -fwd["vel"], d["box"], 60, 0.002, 2.5)
    assert np.max(np.abs(back["pos"] - d["pos"])) < 1e-9
    assert np.max(np.abs(back["vel"] + d["vel"])) < 1e-9


def test_velocity_verlet_energy_bounded_and_wrong_sign_blows_up(monkeypatch):
    d = mdinputs.lj_fluid(6, temperature=1.0, seed=4)
    n = d["pos"].shape[0]

    def drift(dt=0.001, steps=100):
        res = lj.velocity_verlet(d["pos"], d["vel"], d["box"], steps, dt, 2.5, shift="cutoff", sample_every=10)
        e = res["thermo"][:, 1] + res["thermo"][:, 2]
        return np.max(np.abs(e - e[0])) / n

    d1 = drift()
    assert d1 < 2e-4
    # second-order integrator: halving dt (same physical time) cuts the
    # energy error about four times
    ratio = d1 / drift(0.0005, 200)
    assert 3.0 < ratio < 5.0
    # planted mistake: the listing's sign of C_F makes the force attractive at
    # short range; total energy is then far from conserved
    good = lj.lj_force_factor_r2
    monkeypatch.setattr(lj, "lj_force_factor_r2", lambda d2, eps=1.0, sigma=1.0: -good(d2, eps, sigma))
    assert drift() > 1e-2


def test_velocity_verlet_single_step_by_hand():
    d = mdinputs.lj_fluid(5, temperature=1.0, seed=9)
    dt = 0.003
    f0 = lj.lj_forces(d["pos"], d["box"], 2.5)["F"]
    v_half = d["vel"] + dt / 2 * f0
    x1 = d["pos"] + dt * v_half
    f1 = lj.lj_forces(x1, d["box"], 2.5)["F"]
    v1 = v_half + dt / 2 * f1
    res = lj.velocity_verlet(d["pos"], d["vel"], d["box"], 1, dt, 2.5)
    assert np.array_equal(res["pos"], x1)
    assert np.array_equal(res["vel"], v1)


# ------------------------------------------------------------ rebuild rule
def test_rebuild_schedule_constant_speed():
    """Constant speed v: 2 n dt v >= skin first at n = ceil(skin / (2 dt v))
    (Eq. extended_cutoff), so the rebuilds are equally spaced by n."""
    for v, dt, skin in ((5.0, 0.005, 0.3), (3.3, 0.004, 0.25), (7.0, 0.001, 0.3)):
        n = math.ceil(skin / (2.0 * dt * v) - 1e-12)
        steps, _, _ = lj.rebuild_schedule([v] * 200, dt, skin, reuse_every=1000)
        assert steps == list(range(n, 201, n)), (v, dt, skin, n, steps[:5])


def test_rebuild_schedule_reuse_cap_and_carry():
    # slow particles: only the reuse count rebuilds
    steps, b, since = lj.rebuild_schedule([1.0] * 35, 0.001, 0.3, reuse_every=10)
    assert steps == [10, 20, 30] and since == 5 and b == pytest.approx(5 * 0.001)
    # splitting the speeds over two calls gives the same schedule
    v = list(np.linspace(1.0, 9.0, 120))
    whole, _, _ = lj.rebuild_schedule(v, 0.004, 0.3, reuse_every=18)
    a, b, since = lj.rebuild_schedule(v[:47], 0.004, 0.3, reuse_every=18)
    c, _, _ = lj.rebuild_schedule(v[47:], 0.004, 0.3, reuse_every=18, bound=b, since=since)
    assert whole == a + [47 + k for k in c]
    # a faster stretch shortens the periods
    gaps = np.diff([0] + whole)
    assert gaps[0] == 18 and gaps[-1] < 18


@pytest.mark.parametrize("n_side,jit", [(12, 0.07), (16, 0.15)])
def test_tree_route_equals_all_pairs(n_side, jit):
    """The large-N route (k-d tree candidates, then the definition's test)
    gives the all-pairs neighbour set bit for bit and the same forces,
    energies and virial to rounding (the sums run in another order)."""
    pos, box = mdinputs.sc_lattice(n_side)
    pos = mdinputs.perturb(pos, jit, 90 + n_side)
    r2 = lj.ext_radius_sq(2.5, 0.3)
    assert np.array_equal(lj.neighbour_pairs_tree(pos, box, r2), lj.neighbour_pairs(pos, box, r2))
    a = lj.lj_forces(pos, box, 2.5, shift="cutoff")
    b = lj.lj_forces_tree(pos, box, 2.5, shift="cutoff")
    assert np.array_equal(a["nb"], b["nb"])
    scale = np.max(np.abs(a["F"]))
    assert np.max(np.abs(a["F"] - b["F"])) <= 1e-12 * scale
    assert b["pe"] == pytest.approx(a["pe"], rel=1e-12)
    assert b["w"] == pytest.approx(a["w"], rel=1e-12)
    assert np.max(np.abs(a["e"] - b["e"])) <= 1e-12 * np.max(np.abs(a["e"]))
