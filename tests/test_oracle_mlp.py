"""Pins of the descriptor / MLP oracle (the learned potential is not in the
paper; its definitions are stated in oracle/descriptor.py and oracle/mlp.py).

Pinned by: closed forms for one and two neighbours, an independent route for
the angular sums through the spherical-harmonic addition theorem, symmetry
invariances, and central finite differences for every gradient."""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

import mdinputs
from oracle import descriptor as D
from oracle import mlp as M


def _fc(r):
    return 0.5 * (math.cos(math.pi * r / D.RC) + 1.0) if r < D.RC else 0.0


def test_cutoff_function():
    assert D.fc(0.0) == pytest.approx(1.0)
    assert D.fc(D.RC) == 0.0 and D.fc(3.0) == 0.0
    assert D.fc(D.RC * (1 - 1e-9)) == pytest.approx(0.0, abs=1e-15)
    h = 1e-6
    for r in (0.7, 1.3, 2.2):
        assert D.dfc(r) == pytest.approx((D.fc(r + h) - D.fc(r - h)) / (2 * h), rel=1e-7)


def test_two_atoms_radial_closed_form_and_no_angular():
    box = np.array([10.0, 10.0, 10.0])
    pos = np.array([[2.0, 2.0, 2.0], [3.3, 2.0, 2.0]])
    G = D.descriptors(pos, box)
    r = 1.3
    want = [math.exp(-D.ETA_R * (r - rk) ** 2) * _fc(r) for rk in D.R_K]
    np.testing.assert_allclose(G[0, : D.NRAD], want, rtol=1e-12)
    np.testing.assert_allclose(G[1], G[0], rtol=1e-14)
    assert np.all(G[:, D.NRAD:] == 0.0)  # one neighbour: no pair j != k


def test_three_atoms_angular_closed_form():
    box = np.array([12.0, 12.0, 12.0])
    th = 1.1
    r1, r2 = 1.05, 1.4
    c = np.array([5.0, 5.0, 5.0])
    pos = np.array([c, c + [r1, 0, 0], c + [r2 * math.cos(th), r2 * math.sin(th), 0]])
    G = D.descriptors(pos, box, rows=[0])[0]
    for a, (zeta, lam, eta) in enumerate(D.ANGULAR):
        w1 = math.exp(-eta * r1 * r1) * _fc(r1)
        w2 = math.exp(-eta * r2 * r2) * _fc(r2)
        want = 2.0 ** (1 - zeta) * 2.0 * (1.0 + lam * math.cos(th)) ** zeta * w1 * w2
        assert G[D.NRAD + a] == pytest.approx(want, rel=1e-13)


def _angular_by_harmonics(u):
    """Angular features of one centre from the addition theorem:
    sum_{j,k} P_l(uh_j . uh_k) w_j w_k = 4 pi/(2l+1) sum_m |sum_j w_j Y_lm(uh_j)|^2,
    the diagonal j = k (P_l(1) = 1) removed; (1 + lam c)^zeta expanded in P_l."""
    r = np.sqrt(np.sum(u * u, axis=1))
    uh = u / r[:, None]
    theta = np.arccos(np.clip(uh[:, 2], -1, 1))
    phi = np.arctan2(uh[:, 1], uh[:, 0])
    out = []
    for zeta, lam, eta in D.ANGULAR:
        w = np.exp(-eta * r * r) * np.array([_fc(x) for x in r])
        # Legendre coefficients of (1 + lam c)^zeta by Gauss-Legendre quadrature
        xs, ws = np.polynomial.legendre.leggauss(16)
        f = (1.0 + lam * xs) ** zeta
        tot = 0.0
        for l in range(zeta + 1):
            a_l = (2 * l + 1) / 2.0 * np.sum(ws * f * eval_legendre(l, xs))
            s = sum(abs(np.sum(w * sph_harm_y(l, m, theta, phi))) ** 2 for m in range(-l, l + 1))
            tot += a_l * (4 * math.pi / (2 * l + 1) * s - np.sum(w * w))
        out.append(2.0 ** (1 - zeta) * tot)
    return np.array(out)


def test_angular_equals_addition_theorem_route():
    pc = mdinputs.perturb(mdinputs.fcc_cells((3, 3, 3), 1.62)[0], 0.07, 3)
    box = np.full(3, 3 * 1.62)
    table = D.neighbour_table(pc, box, rows=[0, 13, 40])
    G = D.descriptors(pc, box, rows=[0, 13, 40])
    for a, (js, u) in enumerate(table):
        np.testing.assert_allclose(G[a, D.NRAD:], _angular_by_harmonics(u), rtol=1e-10, atol=1e-12)


def test_descriptor_invariances():
    pos, box = mdinputs.sc_lattice(5, rho=0.9)
    pos = mdinputs.perturb(pos, 0.1, 4)
    G = D.descriptors(pos, box)
    perm = mdinputs.rng(1).permutation(pos.shape[0])
    np.testing.assert_allclose(D.descriptors(pos[perm], box), G[perm], rtol=1e-12, atol=1e-14)
    shifted = (pos + np.array([0.37, -1.1, 2.05])) % box
    np.testing.assert_allclose(D.descriptors(shifted, box), G, rtol=1e-10, atol=1e-12)


def test_feature_gradients_finite_difference():
    pos, box = mdinputs.sc_lattice(5, rho=0.9)
    pos = mdinputs.perturb(pos, 0.1, 5)
    G, table, grads = D.descriptors(pos, box, rows=[7], with_grad=True)
    js, u = table[0]
    h = 1e-6
    for jj in range(0, len(js), 7):
        j = js[jj]
        for k in range(3):
            p = pos.copy()
            p[j, k] += h
            gp = D.descriptors(p, box, rows=[7])[0]
            p[j, k] -= 2 * h
            gm = D.descriptors(p, box, rows=[7])[0]
            np.testing.assert_allclose(grads[0][:, jj, k], (gp - gm) / (2 * h), rtol=1e-6, atol=1e-8)


def _params():
    return mdinputs.mlp_init(11)


def test_mlp_input_gradient_fd():
    p = _params()
    g = mdinputs.rng(2).standard_normal((5, M.NPAD))
    g[:, M.NIN:] = 0
    y, cache = M.forward(p, g)
    dg = M.input_grad(p, cache)
    h = 1e-6
    for f in range(0, M.NIN, 5):
        gp = g.copy()
        gp[:, f] += h
        gm = g.copy()
        gm[:, f] -= h
        np.testing.assert_allclose(dg[:, f], (M.forward(p, gp)[0] - M.forward(p, gm)[0]) / (2 * h), rtol=1e-6,
                                   atol=1e-9)


def test_mlp_weight_gradients_fd():
    p = _params()
    r = mdinputs.rng(3)
    g = r.standard_normal((7, M.NPAD))
    t = r.standard_normal(7)
    L, grads = M.loss_and_grads(p, g, t)
    h = 1e-6
    for key, idx in (("W1", (3, 5)), ("b1", (10,)), ("W2", (7, 60)), ("b2", (1,)), ("w3", (33,)), ("b3", (0,))):
        q = {k: v.copy() for k, v in p.items()}
        q[key][idx] += h
        lp = M.loss_and_grads(q, g, t)[0]
        q[key][idx] -= 2 * h
        lm = M.loss_and_grads(q, g, t)[0]
        assert grads[key][idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-9), key


def test_adam_first_step_is_signed_lr():
    p = {"a": np.array([1.0, -2.0, 0.5])}
    g = {"a": np.array([0.3, -4.0, 1e-3])}
    new = M.adam_step(p, g, {}, lr=0.01)
    # first bias-corrected step: m/(sqrt(v)) = sign(g) up to eps
    np.testing.assert_allclose(new["a"], p["a"] - 0.01 * np.sign(g["a"]), rtol=1e-6)


def test_mlp_forces_match_energy_fd():
    pos, box = mdinputs.sc_lattice(5, rho=0.9)
    pos = mdinputs.perturb(pos, 0.08, 6)
    n = pos.shape[0]
    p = _params()
    G, table, grads = D.descriptors(pos, box, with_grad=True)
    mu, sd = G.mean(0), G.std(0) + 1e-3
    e, dEdG = M.energy_and_feature_grad(p, G, mu, sd, -4.0, 0.7)
    F = D.forces_from_feature_grad(n, np.arange(n), table, grads, dEdG)

    def etot(q):
        Gq = D.descriptors(q, box)
        return M.energy_and_feature_grad(p, Gq, mu, sd, -4.0, 0.7)[0].sum()

    h = 1e-6
    for i in (0, 31, 77):
        for k in range(3):
            q = pos.copy()
            q[i, k] += h
            ep = etot(q)
            q[i, k] -= 2 * h
            em = etot(q)
            assert F[i, k] == pytest.approx(-(ep - em) / (2 * h), rel=1e-5, abs=1e-7)
    # translation invariance of the learned energy: forces sum to zero
    assert np.linalg.norm(F.sum(0)) < 1e-10 * np.abs(F).sum()


def test_linear_fit_recovers_linear_model():
    r = mdinputs.rng(9)
    G = r.standard_normal((200, 24))
    a = r.standard_normal(24)
    e = G @ a + 0.3
    a2, c = M.linear_fit(G, e)
    np.testing.assert_allclose(a2, a, rtol=1e-10)
    assert c == pytest.approx(0.3)


def test_adam_bias_correction_over_several_steps():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2 at every step t (1 - b^t cancels the geometric sum), so each step
    moves by lr g / (|g| + eps): after t steps p0 - t lr g / (|g| + eps).
    A correction with the wrong power of beta (or none) misses this from
    t = 2 on.  With a gradient that flips sign at t = 2, the second step has
    the closed form m2 = (1-b1)(b1 g1 + g2) / (1-b1^2) and
    v2 = (1-b2)(b2 g1^2 + g2^2) / (1-b2^2)."""
    p0 = np.array([1.0, -2.0, 0.25])
    g = np.array([0.5, -0.1, 3.0])
    st = {}
    p = {"a": p0.copy()}
    for t in range(1, 7):
        p = M.adam_step(p, {"a": g}, st, lr=0.01, b1=0.9, b2=0.999, eps=1e-8)
        want = p0 - t * 0.01 * g / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(p["a"], want, rtol=0, atol=1e-12)
    g1, g2 = np.array([0.5, 0.2]), np.array([-0.3, 0.2])
    st = {}
    p = M.adam_step({"a": np.zeros(2)}, {"a": g1}, st, lr=0.01)
    p = M.adam_step(p, {"a": g2}, st, lr=0.01)
    b1, b2 = 0.9, 0.999
    m2 = (b1 * g1 + g2) / (1 + b1)          # (1-b1)(b1 g1 + g2) / (1 - b1^2)
    v2 = (b2 * g1 * g1 + g2 * g2) / (1 + b2)
    step1 = 0.01 * g1 / (np.abs(g1) + 1e-8)
    want = -step1 - 0.01 * m2 / (np.sqrt(v2) + 1e-8)
    np.testing.assert_allclose(p["a"], want, rtol=1e-12, atol=1e-15)
