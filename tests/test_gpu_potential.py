"""GPU parity of the learned potential (descriptor, BF16-MFMA network,
gradients, Adam, training) against the FP64 oracle.

Bars: descriptors FP32 vs FP64 relative L2 <= 1e-5; network outputs and
forces with the same bf16-rounded weights (activations are bf16 on the
matrix cores) relative L2 <= 2e-2; the descriptor backward alone (fed the
device's own dE/dG) relative L2 <= 1e-4."""
import numpy as np
import pytest
import torch

import mdinputs
from conftest import gpu_device
from oracle import descriptor as OD
from oracle import mlp as OM

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def config():
    """Jittered FCC, 6^3 cells (864 atoms) at rho 0.8442."""
    d = mdinputs.fcc_lj(6, temperature=1.0, seed=5)
    pos = mdinputs.perturb(d["pos"], 0.08, 6)
    return pos, d["box"]


def _sim(n, box):
    from paper_1704_03329_amd.sim import LJSim

    gpu_device()
    return LJSim(n, box, rc=2.5, skin=0.3, precision="fp64")


def test_descriptors_match_oracle(config):
    from paper_1704_03329_amd.potential import descriptors

    pos, box = config
    sim = _sim(pos.shape[0], box)
    G = descriptors(sim, torch.from_numpy(pos).cuda()).cpu().numpy()
    ref = OD.descriptors(pos, box)
    assert _rel(G, ref) <= 1e-5
    for f in range(OD.NFEAT):
        assert _rel(G[:, f], ref[:, f]) <= 1e-5, f


def test_descriptors_match_oracle_brick_tiles():
    """The 1e-5 descriptor bar where the tiles are 3^3-cell bricks that do
    not wrap onto themselves: every atom of a jittered 4000-atom FCC box (the
    training configuration, 6 cells per axis), and sampled rows of the
    262,144-atom evaluation configuration (a jittered 64^3 lattice)."""
    from paper_1704_03329_amd.potential import descriptors

    d = mdinputs.fcc_lj(10, temperature=1.0, seed=40)
    pos = mdinputs.perturb(d["pos"], 0.1, 7)
    box = d["box"]
    sim = _sim(pos.shape[0], box)
    G = descriptors(sim, torch.from_numpy(pos).cuda()).cpu().numpy()
    ref = OD.descriptors(pos, box)
    for f in range(OD.NFEAT):
        assert _rel(G[:, f], ref[:, f]) <= 1e-5, f
    pos, box = mdinputs.sc_lattice(64)
    pos = mdinputs.perturb(pos, 0.08, 43)
    n = pos.shape[0]
    sim = _sim(n, box)
    G = descriptors(sim, torch.from_numpy(pos).cuda()).cpu().numpy()
    rows = np.sort(mdinputs.rng(44).choice(n, 600, replace=False))
    ref = OD.descriptors(pos, box, rows=rows)
    for f in range(OD.NFEAT):
        assert _rel(G[rows, f], ref[:, f]) <= 1e-5, f


def _model(G, e, seed=3):
    from paper_1704_03329_amd.potential import MLPPotential

    m = MLPPotential(seed=seed)
    m.set_standardisation(G, e)
    return m


def _oracle_eval(m, G):
    p = m.host_params()
    mu = m.mu.double().cpu().numpy()
    sd = m.sd.double().cpu().numpy()
    return OM.energy_and_feature_grad(p, G, mu, sd, m.e_mean, m.e_sd)


def test_mlp_forward_and_input_grad_match_oracle(config):
    from paper_1704_03329_amd.potential import descriptors

    pos, box = config
    sim = _sim(pos.shape[0], box)
    Gd = descriptors(sim, torch.from_numpy(pos).cuda())
    e_lj = torch.from_numpy(np.linspace(-6, -3, pos.shape[0])).cuda()
    m = _model(Gd, e_lj)
    e, dG = m.energy(Gd, with_grad=True)
    re, rdG = _oracle_eval(m, Gd.double().cpu().numpy())
    assert _rel(e.cpu().numpy(), re) <= 2e-2
    assert _rel(dG.cpu().numpy(), rdG) <= 2e-2
    # the energies carry the network's variation, not just the mean
    assert _rel(e.cpu().numpy() - m.e_mean, re - m.e_mean) <= 5e-2


def test_mlp_forces_match_oracle(config):
    from paper_1704_03329_amd.sim import soa

    pos, box = config
    n = pos.shape[0]
    sim = _sim(n, box)
    p = torch.from_numpy(pos).cuda()
    x, y, z = soa(p)
    sim.build(x, y, z)
    from paper_1704_03329_amd.potential import mdpl_desc_fwd

    Gd = torch.empty((n, 24), dtype=torch.float32, device="cuda")
    mdpl_desc_fwd(sim, x, y, z, Gd, None)
    m = _model(Gd, torch.from_numpy(np.linspace(-6, -3, n)).cuda())
    e, fx, fy, fz = m.forces(sim, x, y, z)
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    G, table, grads = OD.descriptors(pos, box, with_grad=True)
    _, dEdG = _oracle_eval(m, G)
    Fref = OD.forces_from_feature_grad(n, np.arange(n), table, grads, dEdG)
    assert _rel(F, Fref) <= 2e-2
    # the descriptor backward alone: feed the device's dE/dG to the oracle chain rule
    _, dGd = m.energy(Gd, with_grad=True)
    Fchain = OD.forces_from_feature_grad(n, np.arange(n), table, grads, dGd.double().cpu().numpy())
    assert _rel(F, Fchain) <= 1e-4
    assert np.linalg.norm(F.sum(0)) <= 1e-4 * np.abs(F).sum()


def test_fused_forces_match_three_calls(config):
    """mdpl_mlp_forces (one call: positions gathered once, outputs cleared
    inside the descriptor pass) against mdpl_desc_fwd + mdpl_mlp_fwd +
    mdpl_desc_bwd on the same positions: identical energies (the same
    kernels on the same inputs), forces equal up to the order of the FP32
    device atomics; outputs that held garbage are overwritten; a workspace
    below mdpl_mlp_run_floats(n) is refused."""
    from paper_1704_03329_amd.mdpl import MdplError
    from paper_1704_03329_amd.sim import soa
    from paper_1704_03329_amd import potential as P

    pos, box = config
    n = pos.shape[0]
    sim = _sim(n, box)
    x, y, z = soa(torch.from_numpy(pos).cuda())
    sim.build(x, y, z)
    m = _model(P.descriptors(sim, torch.from_numpy(pos).cuda()),
               torch.from_numpy(np.linspace(-6, -3, n)).cuda())
    sim.build(x, y, z)
    b3 = m.buffers(n)
    e3, f3x, f3y, f3z = [t.clone() for t in m.forces_three_calls(sim, x, y, z, b3)]
    b1 = m.buffers(n)
    for k in ("fx", "fy", "fz"):
        b1[k].fill_(1e30)
    for _ in range(2):  # twice: the second call starts from the first's outputs
        e1, f1x, f1y, f1z = m.forces(sim, x, y, z, b1)
        assert torch.equal(e1, e3)
        F1 = torch.stack([f1x, f1y, f1z], 1).double().cpu().numpy()
        F3 = torch.stack([f3x, f3y, f3z], 1).double().cpu().numpy()
        assert _rel(F1, F3) <= 1e-6
    small = torch.empty(P.mdpl_mlp_run_floats(n) - 1, dtype=torch.float32, device="cuda")
    with pytest.raises(MdplError):
        P.mdpl_mlp_forces(sim, m.weights(), x, y, z, small, b1["e"], b1["fx"], b1["fy"], b1["fz"])


def test_backward_terms_beyond_the_fixed_point_range(config):
    """With e_sd scaled by 2^27 every pair term of the descriptor backward is
    above 2^19 and bypasses the 64-bit fixed-point LDS sums (direct device
    atomics); the forces are the unscaled ones times 2^27 (the scaling is
    exact in FP32, so only the summation differs)."""
    from paper_1704_03329_amd.sim import soa
    from paper_1704_03329_amd import potential as P

    pos, box = config
    n = pos.shape[0]
    sim = _sim(n, box)
    x, y, z = soa(torch.from_numpy(pos).cuda())
    m = _model(P.descriptors(sim, torch.from_numpy(pos).cuda()),
               torch.from_numpy(np.linspace(-6, -3, n)).cuda())
    sim.build(x, y, z)
    F0 = torch.stack(m.forces(sim, x, y, z)[1:], 1).double().cpu().numpy()
    scale = 2.0 ** 27
    m.e_sd = m.e_sd * scale
    F1 = torch.stack(m.forces(sim, x, y, z)[1:], 1).double().cpu().numpy()
    assert np.median(np.abs(F1)) > 2.0 ** 19
    # the bar of the backward (its pair terms now summed by FP32 atomics throughout)
    assert _rel(F1 / scale, F0) <= 1e-4


def test_train_gradient_and_adam_match_oracle(config):
    from paper_1704_03329_amd import potential as P

    pos, box = config
    n = pos.shape[0]
    sim = _sim(n, box)
    Gd = P.descriptors(sim, torch.from_numpy(pos).cuda())
    e = torch.from_numpy(np.sin(np.arange(n) * 0.37) - 4.0).cuda()
    m = _model(Gd, e, seed=4)
    # the kernel standardises the energies with the network's (FP32) e_mean, e_sd
    em, es = float(np.float32(m.e_mean)), float(np.float32(m.e_sd))
    target = (e.double() - em) / es
    batch = 500
    idx = torch.from_numpy(mdinputs.batch_indices(n, batch, 1, 12)[0]).cuda()
    scratch = torch.empty(P.mdpl_mlp_train_floats(batch), dtype=torch.float32, device="cuda")
    grad = torch.empty(P.NPARAM + 1, dtype=torch.float32, device="cuda")
    P.mdpl_mlp_train_grad(m.weights(), Gd, idx, batch, e.double().contiguous(), scratch, grad)
    g = grad.cpu().numpy()
    # oracle on the same rows, same bf16-rounded weights
    p = m.host_params()
    rows = idx.cpu().numpy()
    gstd = OM.standardise(Gd.double().cpu().numpy()[rows], m.mu.double().cpu().numpy(),
                          m.sd.double().cpu().numpy())
    L, ref = OM.loss_and_grads(p, gstd, target.cpu().numpy()[rows])
    assert g[P.NPARAM] == pytest.approx(L, rel=2e-2)
    refv = P.pack(ref).astype(np.float64)
    assert _rel(g[: P.NPARAM], refv) <= 3e-2
    for k, (off, shape) in P.OFF.items():
        sz = int(np.prod(shape))
        assert _rel(g[off:off + sz], refv[off:off + sz]) <= 5e-2, k
    # one Adam step equals the oracle's on the device gradient
    before = m.params.double().cpu().numpy()
    m.step = 0
    P.mdpl_adam_step(m.params, grad, m.m, m.v, 1e-3, 0.9, 0.999, 1e-8, 1, m.w1, m.w2, m.w3)
    after = m.params.double().cpu().numpy()
    want = OM.adam_step({"a": before}, {"a": g[: P.NPARAM].astype(np.float64)}, {}, lr=1e-3)["a"]
    want[:2048].reshape(64, 32)[:, 24:] = 0.0
    np.testing.assert_allclose(after, want, rtol=1e-5, atol=1e-7)


def test_standardisation_and_bf16_cast_in_the_library():
    """mdpl_mlp_standardise: FP64 means and population spreads of the
    features and energies (the definition, written out in numpy here);
    mdpl_mlp_bf16: the bf16 copies round to nearest even, bit for bit as
    torch's conversion."""
    from paper_1704_03329_amd import potential as P

    r = mdinputs.rng(21)
    n = 70_001
    G = torch.from_numpy((r.normal(size=(n, 24)) * np.linspace(0.1, 30.0, 24) + 5.0).astype(np.float32)).cuda()
    e = torch.from_numpy(r.normal(-4.2, 0.8, size=n)).cuda()
    mu = torch.empty(24, dtype=torch.float32, device="cuda")
    sd = torch.empty_like(mu)
    st = torch.empty(2, dtype=torch.float64, device="cuda")
    scratch = torch.empty(P.MDPL_MLP_STD_SCRATCH, dtype=torch.float64, device="cuda")
    P.mdpl_mlp_standardise(G, e, mu, sd, st, scratch)
    g = G.double().cpu().numpy()
    ee = e.cpu().numpy()
    np.testing.assert_allclose(mu.cpu().numpy(), g.mean(0), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(sd.cpu().numpy(), np.sqrt(((g - g.mean(0)) ** 2).mean(0)) + 1e-6, rtol=1e-6)
    assert st[0].item() == pytest.approx(ee.mean(), rel=1e-12)
    assert st[1].item() == pytest.approx(np.sqrt(((ee - ee.mean()) ** 2).mean()) + 1e-12, rel=1e-12)
    params = torch.from_numpy(r.normal(0.0, 0.3, size=P.NPARAM).astype(np.float32)).cuda()
    w1 = torch.empty(2048, dtype=torch.int16, device="cuda")
    w2 = torch.empty(4096, dtype=torch.int16, device="cuda")
    w3 = torch.empty(64, dtype=torch.int16, device="cuda")
    P.mdpl_mlp_bf16(params, w1, w2, w3)
    bf = lambda a: a.to(torch.bfloat16).view(torch.int16)  # noqa: E731
    assert torch.equal(w1, bf(params[0:2048]))
    assert torch.equal(w2, bf(params[2112:6208]))
    assert torch.equal(w3, bf(params[6272:6336]))


@pytest.fixture(scope="module")
def small_training_set():
    from paper_1704_03329_amd import potential as P

    gpu_device()
    return P.generate_training_set(temperatures=(1.0,), counts=(12,), n_cells=10, equil_steps=1000,
                                   every=100, seeds=(40,))


def test_training_beats_linear_and_untrained(small_training_set):
    from paper_1704_03329_amd import potential as P

    data = small_training_set
    G, e = data["G"], data["e"]
    snap = data["snap"].cpu().numpy()
    tr = np.nonzero(snap < 10)[0]
    va = np.nonzero(snap >= 10)[0]
    tr_t = torch.from_numpy(tr).cuda()
    va_t = torch.from_numpy(va).cuda()
    Gtr, etr = G[tr_t].contiguous(), e[tr_t].contiguous()
    Gva, eva = G[va_t].contiguous(), e[va_t].contiguous()
    m = P.MLPPotential(seed=7)
    m.set_standardisation(Gtr, etr)
    e0, _ = m.energy(Gva)
    mae0 = float(torch.mean(torch.abs(e0.double() - eva)).item())
    losses = m.train(Gtr, etr, steps=1500, batch=4096, lr=3e-3, lr_final=3e-4, log_every=500)
    e1, _ = m.energy(Gva)
    mae1 = float(torch.mean(torch.abs(e1.double() - eva)).item())
    a, c = OM.linear_fit(Gtr.double().cpu().numpy(), etr.cpu().numpy())
    elin = Gva.double().cpu().numpy() @ a + c
    mae_lin = float(np.mean(np.abs(elin - eva.cpu().numpy())))
    print(f"validation MAE: untrained {mae0:.4f}, linear {mae_lin:.4f}, trained {mae1:.4f}; losses {losses}")
    assert losses[-1][1] < losses[0][1]
    assert mae1 < mae_lin and mae1 < mae0


def test_run_mlp_matches_oracle_velocity_verlet():
    """mdpl_run_mlp (list reuse, reordering, the network as force field)
    against the oracle's velocity Verlet (Alg. VelocityVerlet) with oracle
    network forces and the same bf16-rounded weights: 864 atoms, 5 steps.
    The device's activations are bf16 on the matrix cores (forces within
    2e-2), so positions agree to dt^2 x that over the run."""
    from oracle import lj as olj
    from paper_1704_03329_amd import potential as P
    from paper_1704_03329_amd.sim import LJSim

    gpu_device()
    d = mdinputs.fcc_lj(6, temperature=1.0, seed=8)
    pos = mdinputs.perturb(d["pos"], 0.05, 9)
    box = d["box"]
    n = pos.shape[0]
    sim = LJSim(n, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=2, precision="fp32")
    G0 = P.descriptors(LJSim(n, box, rc=2.5, skin=0.3, precision="fp64"), torch.from_numpy(pos).cuda())
    m = _model(G0, torch.from_numpy(np.linspace(-6, -3, n)).cuda(), seed=5)
    st = sim.new_state(torch.from_numpy(pos), torch.from_numpy(d["vel"]))
    ws = torch.empty(P.mdpl_mlp_run_floats(n), dtype=torch.float32, device="cuda")
    th = torch.empty((6, 4), dtype=torch.float64, device="cuda")
    P.mdpl_run_mlp(sim, m.weights(), ws, st, 5, 1, th)
    assert sim.check(raise_on_error=False)[0] == 0
    p = m.host_params()
    mu, sd = m.mu.double().cpu().numpy(), m.sd.double().cpu().numpy()

    def force_fn(x):
        G, table, grads = OD.descriptors(x, box, with_grad=True)
        E, dEdG = OM.energy_and_feature_grad(p, G, mu, sd, m.e_mean, m.e_sd)
        return {"F": OD.forces_from_feature_grad(n, np.arange(n), table, grads, dEdG), "pe": float(E.sum()),
                "w": 0.0}

    ref = olj.velocity_verlet(pos, d["vel"], box, 5, 0.001, 2.5, sample_every=1, force_fn=force_fn)
    ids = st["ids"].cpu().numpy()
    got_x = np.zeros((n, 3))
    got_v = np.zeros((n, 3))
    got_x[ids] = torch.stack([st["x"], st["y"], st["z"]], 1).cpu().numpy()
    got_v[ids] = torch.stack([st["vx"], st["vy"], st["vz"]], 1).cpu().numpy()
    dx = got_x - ref["pos"]
    dx -= box * np.round(dx / box)  # the device folds positions into the box at rebuilds
    assert np.max(np.abs(dx)) <= 1e-6
    assert np.linalg.norm(got_v - ref["vel"]) <= 2e-3 * np.linalg.norm(ref["vel"])
    t = th.cpu().numpy()
    np.testing.assert_allclose(t[:, 0], ref["thermo"][:, 1], rtol=1e-4)  # KE
    np.testing.assert_allclose(t[:, 1], ref["thermo"][:, 2], rtol=2e-2)  # sum of network energies
