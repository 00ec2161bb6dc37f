"""GPU parity of the LJ path (binning, neighbour list, forces, energy,
virial, velocity Verlet) against the FP64 oracle on identical seeded inputs.

Bars: neighbour lists bit-exact as sorted directed pair sets; forces
||dF||/||F|| <= 1e-5 and max_i |dF_i| <= 1e-5 max_i |F_i|; energies and
virial 1e-9 relative (FP64 per-pair energy in both precisions)."""
import math

import numpy as np
import pytest
import torch

import mdinputs
from conftest import force_errors, gpu_device, split_dev, to_dev
from oracle import lj as olj

pytestmark = pytest.mark.gpu


def _sim(n, box, **kw):
    from paper_1704_03329_amd.sim import LJSim

    gpu_device()
    return LJSim(n, box, **kw)


def _pairs_gpu(sim, n=None):
    p = sim.pairs().numpy()
    n = int(p.max()) + 1 if (n is None and p.size) else (n or 1)
    key = np.sort(p[:, 0] * n + p[:, 1])
    return np.stack([key // n, key % n], 1)


def _jittered_grid(reps, spacing, jitter, seed):
    g = [np.arange(r) * spacing + 0.5 * spacing for r in reps]
    zz, yy, xx = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
    return mdinputs.perturb(pos, jitter, seed), np.array(reps, dtype=float) * spacing


def _cases():
    out = {}
    pos, box = mdinputs.sc_lattice(10)
    out["sc1000"] = (pos, box)
    out["sc1000_jitter"] = (mdinputs.perturb(pos, 0.08, 5), box)
    # non-cubic box, atoms on and across the faces (inputs need not be folded)
    b = np.array([8.5, 9.1, 11.7])
    p = mdinputs.random_box(900, b, 21)
    p[:6, 0] = [0.0, b[0] - 1e-13, -0.4, b[0] + 0.3, 1e-300, -1e-17]
    p[6:9, 2] = [b[2], -b[2] * 0.2, b[2] * 1.2]
    out["random_noncubic_faces"] = (p, b)
    L = (5000 / 0.8) ** (1 / 3)
    out["random5000"] = (mdinputs.random_box(5000, [L, L, L], 22), np.array([L, L, L]))
    out["sparse37"] = (mdinputs.random_box(37, [9.0, 9.0, 9.0], 23), np.array([9.0, 9.0, 9.0]))
    out["single"] = (np.array([[1.0, 2.0, 3.0]]), np.array([9.0, 9.0, 9.0]))
    # force cases: physical separations
    out["grid_noncubic_4913"] = _jittered_grid((17, 17, 17), 1.07, 0.07, 24)
    g, gb = _jittered_grid((13, 9, 21), 1.1, 0.06, 25)  # 2457 atoms, ragged vs 256
    g = g.copy()
    lo = g[:, 0] < 0.2 * gb[0]
    g[lo, 0] += gb[0]  # unfolded images just above the face
    out["grid_unfolded_2457"] = (g, gb)
    out["grid_sparse_36"] = _jittered_grid((3, 3, 4), 2.9, 0.2, 26)
    # cells within 1e-9 of the list radius (three of 2.8 (1 + 5e-10); the grid
    # takes cells of at least 1 + 1e-10 radii): the build scans whole stencil
    # rows instead of skipping half-cells along x
    p, b = _jittered_grid((6, 6, 6), 1.4, 0.2, 27)
    out["grid_cell_at_radius_216"] = (p, b * (1.0 + 5e-10))
    # particles on the cell and half-cell boundaries along x (cells 2.9 wide)
    k = np.arange(6) * 1.45
    zz, yy, xx = np.meshgrid(k + 0.3, k + 0.1, k, indexing="ij")
    out["half_cell_boundaries_216"] = (np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1),
                                       np.array([8.7, 8.7, 8.7]))
    return out


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_nlist_bit_exact(name):
    pos, box = CASES[name]
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3, max_nb=256)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    st, flags, maxc = sim.check(raise_on_error=False)
    assert st == 0, (st, flags)
    got = _pairs_gpu(sim)
    # the list is defined on positions folded into the box
    want = olj.neighbour_pairs(olj.wrap(pos, box), box, olj.ext_radius_sq(2.5, 0.3))
    assert got.shape == want.shape
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", ["sc1000_jitter", "grid_noncubic_4913", "grid_unfolded_2457", "grid_sparse_36"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shift", ["none", "paper", "cutoff"])
def test_forces_energy_virial(name, precision, shift):
    pos, box = CASES[name]
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3, precision=precision, shift=shift, max_nb=256)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    fx, fy, fz, pe_w, e = sim.forces(x, y, z, energy=True, per_atom=True)
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    ref = olj.lj_forces(pos, box, 2.5, shift=shift)
    g, m = force_errors(F, ref["F"])
    assert g <= 1e-5 and m <= 1e-5, (g, m)
    pe, w = pe_w.cpu().numpy()
    assert abs(pe - ref["pe"]) <= 1e-9 * abs(ref["pe"]) + 1e-12
    assert abs(w - ref["w"]) <= 1e-9 * abs(ref["w"]) + 1e-12
    ea = e.cpu().numpy()
    assert np.max(np.abs(ea - ref["e"])) <= 1e-9 * max(np.max(np.abs(ref["e"])), 1e-300) + 1e-13
    # forces without energy take the other kernel; same values
    fx2, fy2, fz2, _, _ = sim.forces(x, y, z)
    F2 = torch.stack([fx2, fy2, fz2], 1).double().cpu().numpy()
    g2, m2 = force_errors(F2, ref["F"])
    assert g2 <= 1e-5 and m2 <= 1e-5, (g2, m2)


def test_forces_after_motion_within_skin():
    pos, box = CASES["sc1000_jitter"]
    sim = _sim(1000, box, rc=2.5, skin=0.3, precision="fp64")
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    moved = mdinputs.perturb(pos, 0.025, 77)  # |dr| < skin/2
    assert np.max(np.linalg.norm(moved - pos, axis=1)) < 0.15
    x2, y2, z2 = split_dev(moved)
    fx, fy, fz, pe_w, _ = sim.forces(x2, y2, z2, energy=True)
    F = torch.stack([fx, fy, fz], 1).cpu().numpy()
    ref = olj.lj_forces(moved, box, 2.5)
    g, m = force_errors(F, ref["F"])
    assert g <= 1e-12 and m <= 1e-12
    assert abs(pe_w[0].item() - ref["pe"]) <= 1e-12 * abs(ref["pe"])


def test_fp32_cutoff_band_classified_exactly():
    """FP32 mode: pairs whose FP32 squared distance lands within the band
    around rc^2 are classified by the FP64 test.  Isolated pairs planted at
    rc (1 +/- d), d down to 1e-8, carry the force at the cutoff (0.039) or
    nothing, exactly as the oracle's FP64 test decides; the energy pass
    gives the same forces bit for bit."""
    r = mdinputs.rng(31)
    base = (np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) * 6.0
    base = base + r.normal(0.0, 0.3, base.shape)
    u = r.normal(size=base.shape)
    u /= np.linalg.norm(u, axis=1)[:, None]
    deltas = np.array([-1e-8, 1e-8, -1e-7, 1e-7, -5e-7, 5e-7, -2e-6, 2e-6, -1e-5, 1e-5, -1e-3, 1e-3])
    dist = 2.5 * (1.0 + deltas[np.arange(base.shape[0]) % deltas.size])
    pos = np.concatenate([base, base + dist[:, None] * u])
    box = np.array([24.0, 24.0, 24.0])
    pos = olj.wrap(pos, box)
    ref = olj.lj_forces(pos, box, 2.5)
    inside = np.linalg.norm(ref["F"], axis=1) > 0
    assert 0 < inside.sum() < pos.shape[0]  # both sides of the cutoff are planted
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3, precision="fp32", max_nb=64)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    fx, fy, fz, _, _ = sim.forces(x, y, z)
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    err = np.linalg.norm(F - ref["F"], axis=1)
    assert np.max(err) <= 1e-5 * np.max(np.linalg.norm(ref["F"], axis=1)), np.max(err)
    ex, ey, ez, _, _ = sim.forces(x, y, z, energy=True)
    for a, b in ((fx, ex), (fy, ey), (fz, ez)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_sampling_leaves_trajectory_unchanged(precision):
    """The energy pass of a sampled step computes its forces with the plain
    pass's arithmetic: runs that sample every 5 steps and never give the
    same state bit for bit."""
    d = mdinputs.lj_fluid(10, temperature=1.0, seed=5)
    box = d["box"]
    mk = lambda: _sim(1000, box, rc=2.5, skin=0.3, reuse_every=10, precision=precision)
    a, _ = _run(mk(), d["pos"], d["vel"], 30, 5)
    b, _ = _run(mk(), d["pos"], d["vel"], 30, 0)
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_fp32_forces_melted_fluid_every_atom():
    """FP32 forces on every atom of a melted fluid (8000 atoms at rho 0.8442,
    1500 FP64 steps at T* = 1 from the lattice) against the FP64 oracle."""
    d = mdinputs.lj_fluid(20, temperature=1.0, seed=12)
    box = d["box"]
    n = d["pos"].shape[0]
    md = _sim(n, box, rc=2.5, skin=0.3, dt=0.004, reuse_every=5, precision="fp64", shift="cutoff")
    state, _ = _run(md, d["pos"], d["vel"], 1500, 0)
    assert md.check(raise_on_error=False)[0] == 0
    pos, _, _ = _unpermute(state)
    sim = _sim(n, box, rc=2.5, skin=0.3, precision="fp32", max_nb=128)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    fx, fy, fz, pe_w, _ = sim.forces(x, y, z, energy=True)
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    ref = olj.lj_forces(pos, box, 2.5)
    g, m = force_errors(F, ref["F"])
    from paper_1704_03329_amd import mdpl as C

    print(f"melted fluid: {C.mdpl_nlist_entries(sim.handle) / n:.2f} entries per atom, global {g:.2e}, "
          f"per-atom {m:.2e}")
    assert g <= 1e-5 and m <= 1e-5, (g, m)
    assert abs(pe_w[0].item() - ref["pe"]) <= 1e-9 * abs(ref["pe"])
    assert abs(pe_w[1].item() - ref["w"]) <= 1e-9 * abs(ref["w"])


def test_capacity_overflow_flagged():
    from paper_1704_03329_amd import mdpl as C

    pos, box = CASES["sc1000"]
    sim = _sim(1000, box, rc=2.5, skin=0.3, max_nb=40)
    sim.build(*split_dev(pos))
    st, flags, maxc = sim.check(raise_on_error=False)
    assert st == C.MDPL_ECAPACITY and flags & C.FLAG_NL_OVERFLOW and maxc == 80


def test_dense_brick_overflow_flagged():
    """1100 atoms packed inside one cell of a dilute box: the brick that holds
    them has more particles than the list builder counts per brick.  The
    build must flag it (and the per-particle overflow), give every slot a
    count within the capacity, and the force pass must still run."""
    from paper_1704_03329_amd import mdpl as C

    L = 20.0  # 7 cells of 2.857 per axis; 3100 atoms -> bricks of 3^3 cells
    box = np.array([L, L, L])
    cluster = 9.0 + 1.6 * mdinputs.random_box(1100, [1.0, 1.0, 1.0], 41)  # inside cell (3, 3, 3)
    pos = np.concatenate([mdinputs.random_box(2000, box, 42), cluster])
    n = pos.shape[0]
    sim = _sim(n, box, rc=2.5, skin=0.3, max_nb=128)
    cols = split_dev(pos)
    sim.build(*cols)
    st, flags, _ = sim.check(raise_on_error=False)
    assert st == C.MDPL_ECAPACITY and flags & C.FLAG_NL_OVERFLOW
    assert 0 < C.mdpl_nlist_entries(sim.handle) <= n * 128
    sim.forces(*cols, energy=True)
    torch.cuda.synchronize()


def _run(sim, pos, vel, nsteps, every):
    state = sim.new_state(torch.from_numpy(pos), torch.from_numpy(vel))
    thermo = sim.run(state, nsteps, every)
    torch.cuda.synchronize()
    return state, thermo


def _unpermute(state):
    ids = state["ids"].long().cpu().numpy()
    inv = np.empty_like(ids)
    inv[ids] = np.arange(ids.shape[0])
    get = lambda a, b, c: np.stack([state[a].cpu().numpy(), state[b].cpu().numpy(), state[c].cpu().numpy()], 1)[inv]
    return get("x", "y", "z"), get("vx", "vy", "vz"), get("fx", "fy", "fz").astype(np.float64)


def _wrapdiff(a, b, box):
    d = a - b
    return d - box[None, :] * np.round(d / box[None, :])


def test_run_c1_fp64_matches_oracle():
    """The small benchmark case: N=1000 sc lattice at rho 0.8442, T*=1, rc 2.5,
    skin 0.3, dt 0.001, 100 velocity-Verlet steps in FP64, rebuild every 10."""
    d = mdinputs.lj_fluid(10, temperature=1.0, seed=1)
    box = d["box"]
    sim = _sim(1000, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision="fp64", shift="cutoff")
    state, thermo = _run(sim, d["pos"], d["vel"], 100, 10)
    assert sim.check(raise_on_error=False)[0] == 0
    ref = olj.velocity_verlet(d["pos"], d["vel"], box, 100, 0.001, 2.5, shift="cutoff", sample_every=10)
    th = thermo.cpu().numpy()
    assert th.shape == (11, 4)
    for col in (0, 1, 2):  # KE, PE, W
        np.testing.assert_allclose(th[:, col], ref["thermo"][:, col + 1], rtol=1e-9, atol=1e-10)
    assert np.all(th[:, 3] < 0.15)  # largest displacement between rebuilds < skin/2
    x, v, f = _unpermute(state)
    assert np.max(np.abs(_wrapdiff(x, ref["pos"], box))) < 1e-9
    assert np.max(np.abs(v - ref["vel"])) < 1e-9
    g, m = force_errors(f, ref["F"])
    assert g < 1e-9 and m < 1e-9
    # ids remain a permutation
    assert sorted(state["ids"].cpu().tolist()) == list(range(1000))


def test_run_c1_fp32_forces_close_to_oracle():
    d = mdinputs.lj_fluid(10, temperature=1.0, seed=1)
    box = d["box"]
    sim = _sim(1000, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision="fp32", shift="cutoff")
    state, thermo = _run(sim, d["pos"], d["vel"], 100, 10)
    assert sim.check(raise_on_error=False)[0] == 0
    ref = olj.velocity_verlet(d["pos"], d["vel"], box, 100, 0.001, 2.5, shift="cutoff", sample_every=10)
    th = thermo.cpu().numpy()
    # the FP32 trajectory departs from the FP64 one only by force rounding
    np.testing.assert_allclose(th[:, 1], ref["thermo"][:, 2], rtol=1e-6)
    np.testing.assert_allclose(th[:, 0], ref["thermo"][:, 1], rtol=1e-5)
    x, v, f = _unpermute(state)
    assert np.max(np.abs(_wrapdiff(x, ref["pos"], box))) < 1e-7
    # energies of the final FP32 state evaluated by the oracle match the sample
    e = ref["thermo"][:, 1] + ref["thermo"][:, 2]
    eg = th[:, 0] + th[:, 1]
    assert np.max(np.abs(eg - eg[0])) / 1000 < 2e-4
    assert np.max(np.abs(e - e[0])) / 1000 < 2e-4


def test_run_deterministic_and_resumable():
    d = mdinputs.lj_fluid(10, temperature=1.0, seed=2)
    box = d["box"]
    mk = lambda: _sim(1000, box, rc=2.5, skin=0.3, reuse_every=10, precision="fp64")
    s1, t1 = _run(mk(), d["pos"], d["vel"], 40, 10)
    s2, t2 = _run(mk(), d["pos"], d["vel"], 40, 10)
    for k in s1:
        assert torch.equal(s1[k], s2[k]), k
    assert torch.equal(t1, t2)
    # 20 + 20 steps from the saved state equals 40 steps (rebuild at 20 in both)
    sim = mk()
    state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    sim.run(state, 20, 10)
    sim.run(state, 20, 10)
    torch.cuda.synchronize()
    for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "ids"):
        assert torch.equal(state[k], s1[k]), k


def test_launch_timing_stride():
    """mdpl_set_timing(on, every): launches 0, every, 2 every, ... of each
    force kernel are timed; timing does not change the trajectory."""
    from paper_1704_03329_amd import mdpl as C

    d = mdinputs.lj_fluid(10, temperature=1.0, seed=2)
    box = d["box"]
    mk = lambda: _sim(1000, box, rc=2.5, skin=0.3, reuse_every=10, precision="fp32")
    ref, _ = _run(mk(), d["pos"], d["vel"], 20, 10)
    sim = mk()
    state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    counts = None
    for every in (1, 8, 30):
        C.mdpl_set_timing(sim.handle, True, reserve=32, every=every)
        sim.run(state, 20, 10)
        ms0, n0 = C.mdpl_kernel_time(sim.handle, 0)
        ms1, n1 = C.mdpl_kernel_time(sim.handle, 1)
        if counts is None:  # every launch of each kind
            counts = (n0, n1)
            assert n0 >= 17 and n1 >= 2, counts
        assert (n0, n1) == tuple(-(-c // every) for c in counts), (every, n0, n1, counts)
        assert ms0 > 0.0 and ms1 > 0.0
        state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    C.mdpl_set_timing(sim.handle, False)
    sim.run(state, 20, 10)
    C.mdpl_set_timing(sim.handle, True, every=3)
    state2 = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    sim.run(state2, 20, 10)
    torch.cuda.synchronize()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert torch.equal(state2[k], ref[k]), k
    with pytest.raises(C.MdplError):
        C.mdpl_set_timing(sim.handle, True, every=0)


def test_run_continue_bitwise():
    """MDPL_RUN_CONTINUE: runs that go on from the last run's state (no
    rebinning, no F(r0) pass, the rebuild schedule carried over) give the
    state of one longer run bit for bit, also when a call ends inside a
    reuse period."""
    from paper_1704_03329_amd import mdpl as C

    d = mdinputs.lj_fluid(10, temperature=1.0, seed=2)
    box = d["box"]
    mk = lambda: _sim(1000, box, rc=2.5, skin=0.3, reuse_every=10, precision="fp64")
    s1, t1 = _run(mk(), d["pos"], d["vel"], 40, 10)
    keys = ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "ids")
    sim = mk()
    state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    sim.run(state, 20, 10)
    t2 = sim.run(state, 20, 10, cont=True)
    torch.cuda.synchronize()
    for k in keys:
        assert torch.equal(state[k], s1[k]), k
    # rows of steps 30 and 40 come from the same passes as in the long run
    assert torch.equal(t2[1:], t1[3:])
    assert t2.shape == (3, 4)
    # blocks that end inside reuse periods, against one run with the same
    # (absent) energy sampling
    s0, _ = _run(mk(), d["pos"], d["vel"], 40, 0)
    sim = mk()
    state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    for block in (13, 1, 19, 7):
        sim.run(state, block, 0, cont=block != 13)
    torch.cuda.synchronize()
    for k in keys:
        assert torch.equal(state[k], s0[k]), k
    assert sim.rebuild_stats()[0] == 1 + 4  # the initial build and steps 10, 20, 30, 40
    # other arrays, or a standalone build in between: no state to continue
    other = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    with pytest.raises(C.MdplError) as e:
        sim.run(other, 5, 0, cont=True)
    assert e.value.status == C.MDPL_ESTATE
    sim.build(state["x"], state["y"], state["z"])
    with pytest.raises(C.MdplError) as e:
        sim.run(state, 5, 0, cont=True)
    assert e.value.status == C.MDPL_ESTATE


def test_rule_rebuilds_early_and_matches_oracle():
    """The reuse rule of Eq. extended_cutoff at dt 0.005 (the crystallisation
    step): the lists are rebuilt whenever 2 sum dt v_max reaches the skin,
    well before reuse_every = 18 steps.  The FP64 run matches the oracle to
    1e-9 with no skin flag, and the rebuilds are those of the rule applied
    to the oracle's own trajectory.  With the fixed schedule the same run
    moves particles past skin/2 and is flagged."""
    from paper_1704_03329_amd import mdpl as C

    d = mdinputs.lj_fluid(10, temperature=1.0, seed=1)
    box = d["box"]
    nsteps, dt = 60, 0.005
    sim = _sim(1000, box, rc=2.5, skin=0.3, dt=dt, reuse_every=18, precision="fp64", shift="cutoff",
               rebuild="vmax")
    state, thermo = _run(sim, d["pos"], d["vel"], nsteps, 10)
    assert sim.check(raise_on_error=False)[0] == 0
    ref = olj.velocity_verlet(d["pos"], d["vel"], box, nsteps, dt, 2.5, shift="cutoff", sample_every=10,
                              record_vmax=True)
    th = thermo.cpu().numpy()
    for col in (0, 1, 2):
        np.testing.assert_allclose(th[:, col], ref["thermo"][:, col + 1], rtol=1e-9, atol=1e-10)
    assert np.all(th[:, 3] < 0.15)
    x, v, f = _unpermute(state)
    assert np.max(np.abs(_wrapdiff(x, ref["pos"], box))) < 1e-9
    assert np.max(np.abs(v - ref["vel"])) < 1e-9
    g, m = force_errors(f, ref["F"])
    assert g < 1e-9 and m < 1e-9
    steps, _, _ = olj.rebuild_schedule(ref["vmax"], dt, 0.3, 18)
    gaps = np.diff([0] + steps)
    rebuilds, early, _ = sim.rebuild_stats()
    print(f"rebuild steps {steps}, device: {rebuilds} rebuilds, {early} early", flush=True)
    assert np.all(gaps < 18)
    assert rebuilds == 1 + len(steps) and early == int(np.sum(gaps < 18))
    fixed = _sim(1000, box, rc=2.5, skin=0.3, dt=dt, reuse_every=18, precision="fp64", shift="cutoff",
                 rebuild="fixed")
    _run(fixed, d["pos"], d["vel"], nsteps, 0)
    st, flags, _ = fixed.check(raise_on_error=False)
    assert st == C.MDPL_ESKIN and flags & C.FLAG_SKIN


def test_skin_violation_flagged():
    """The displacement check that backs every rebuild: with the fixed
    schedule one fast particle outruns the skin and is flagged; the VMAX rule
    rebuilds in time for it."""
    from paper_1704_03329_amd import mdpl as C

    d = mdinputs.lj_fluid(10, temperature=0.5, seed=3)
    vel = d["vel"].copy()
    vel[123] = [25.0, 0.0, 0.0]  # moves 0.25 in 10 steps > skin/2 = 0.15
    sim = _sim(1000, d["box"], rc=2.5, skin=0.3, reuse_every=10, precision="fp64", rebuild="fixed")
    _run(sim, d["pos"], vel, 20, 0)
    st, flags, _ = sim.check(raise_on_error=False)
    assert st == C.MDPL_ESKIN and flags & C.FLAG_SKIN
    rule = _sim(1000, d["box"], rc=2.5, skin=0.3, reuse_every=10, precision="fp64", rebuild="vmax")
    _run(rule, d["pos"], vel, 20, 0)
    assert rule.check(raise_on_error=False)[0] == 0
    assert rule.rebuild_stats()[1] > 0
    # a calm run raises nothing
    sim2 = _sim(1000, d["box"], rc=2.5, skin=0.3, reuse_every=10, precision="fp64", rebuild="fixed")
    _run(sim2, d["pos"], d["vel"], 20, 0)
    assert sim2.check(raise_on_error=False)[0] == 0


def test_nonfinite_flagged():
    from paper_1704_03329_amd import mdpl as C

    d = mdinputs.lj_fluid(10, temperature=1.0, seed=4)
    vel = d["vel"].copy()
    vel[5, 1] = np.nan
    sim = _sim(1000, d["box"], rc=2.5, skin=0.3, reuse_every=10, precision="fp64")
    _run(sim, d["pos"], vel, 3, 0)
    st, flags, _ = sim.check(raise_on_error=False)
    assert flags & C.FLAG_NONFINITE


def test_argument_errors_before_device_work():
    from paper_1704_03329_amd import mdpl as C

    gpu_device()
    with pytest.raises(C.MdplError) as e:
        _sim(100, [5.0, 5.0, 5.0])  # 5 < 3 * 2.8
    assert e.value.status == C.MDPL_EBOX
    sim = _sim(1000, [10.58] * 3)
    x = torch.zeros(1000, dtype=torch.float64, device="cuda")
    f = torch.zeros(1000, dtype=torch.float32, device="cuda")
    with pytest.raises(C.MdplError) as e:
        C.mdpl_forces(sim.handle, x, x, x, f, f, f)
    assert e.value.status == C.MDPL_ESTATE


# ------------------------------------------------------------------ full size
@pytest.fixture(scope="module")
def c2_state():
    """The 10^6-atom benchmark lattice (100^3 sc at rho 0.8442) with Gaussian
    jitter standing in for a melted configuration."""
    pos, box = mdinputs.sc_lattice(100)
    pos = mdinputs.perturb(pos, 0.06, 202)
    return pos, box


def test_c2_full_size_sampled(c2_state):
    pos, box = c2_state
    n = pos.shape[0]
    sim = _sim(n, box, rc=2.5, skin=0.3, precision="fp32", max_nb=128)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    assert sim.check(raise_on_error=False)[0] == 0
    fx, fy, fz, pe_w, e = sim.forces(x, y, z, energy=True, per_atom=True)
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    rows = np.sort(mdinputs.rng(9).choice(n, 126, replace=False))
    rows = np.concatenate([rows, [0, n - 1]])
    ref = olj.lj_forces(pos, box, 2.5, rows=rows)
    g, m = force_errors(F[rows], ref["F"])
    assert g <= 1e-5 and m <= 1e-5, (g, m)
    ea = e.cpu().numpy()[rows]
    assert np.max(np.abs(ea - ref["e"])) <= 1e-9 * np.max(np.abs(ref["e"]))
    # neighbour rows bit-exact for the sampled atoms
    pairs = _pairs_gpu(sim, n)
    got = pairs[np.isin(pairs[:, 0], rows)]
    want = olj.neighbour_pairs(pos, box, olj.ext_radius_sq(2.5, 0.3), rows=rows)
    assert np.array_equal(got, want)
    # properties at full size: every list is symmetric, net force ~ 0
    fwd = pairs[:, 0] * n + pairs[:, 1]
    bwd = np.sort(pairs[:, 1] * n + pairs[:, 0])
    assert np.array_equal(np.sort(fwd), bwd)
    assert np.linalg.norm(F.sum(0)) <= 1e-6 * np.abs(F).sum()
    pe, w = pe_w.cpu().numpy()
    assert abs(pe - e.sum().item()) <= 1e-9 * abs(pe)


def test_c2_run_steps_and_thermo():
    d = mdinputs.lj_fluid(100, temperature=1.0, seed=2)  # the benchmark start
    pos, box, vel = d["pos"], d["box"], d["vel"]
    n = pos.shape[0]
    sim = _sim(n, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision="fp32", max_nb=128,
               shift="cutoff")
    state = sim.new_state(torch.from_numpy(pos), torch.from_numpy(vel))
    thermo = sim.run(state, 30, 10).cpu().numpy()
    assert sim.check(raise_on_error=False)[0] == 0
    # sampled check of the final state: forces at the final positions
    x, v, f = _unpermute(state)
    rows = np.sort(mdinputs.rng(10).choice(n, 128, replace=False))
    ref = olj.lj_forces(x, box, 2.5, rows=rows)
    g, m = force_errors(f[rows], ref["F"])
    assert g <= 1e-5 and m <= 1e-5, (g, m)
    ke = 0.5 * np.sum(v * v)
    assert thermo[-1, 0] == pytest.approx(ke, rel=1e-12)
    e = thermo[:, 0] + thermo[:, 1]
    assert np.max(np.abs(e - e[0])) / n < 1e-4
