"""GPU parity of the half-list LJ path (Newton's third law: each pair once,
the reaction applied to the second particle; Sec. 2, the comment on
Newton's third law) against the same FP64 oracle as the full lists.

Bars: every pair of the all-pairs definition within rc+skin appears exactly
once (in one direction, no self pairs); forces, energies and virial meet
the bars of the full-list tests (||dF||/||F|| <= 1e-5 and max_i |dF_i| <=
1e-5 max_i |F_i| in FP32, PE, W and per-atom energies 1e-9 relative); the
FP64 velocity-Verlet run matches the oracle to 1e-9 like the full-list one
(the atomics only reorder FP64 additions)."""
import numpy as np
import pytest
import torch

import mdinputs
from conftest import force_errors, gpu_device, split_dev
from oracle import lj as olj
from test_gpu_lj import CASES

pytestmark = pytest.mark.gpu


def _sim(n, box, **kw):
    from paper_1704_03329_amd.sim import LJSim

    gpu_device()
    return LJSim(n, box, pairs="half", **kw)


def _undirected(p, n):
    lo, hi = np.minimum(p[:, 0], p[:, 1]), np.maximum(p[:, 0], p[:, 1])
    return np.sort(lo.astype(np.int64) * n + hi)


@pytest.mark.parametrize("name", list(CASES))
def test_half_list_each_pair_once(name):
    pos, box = CASES[name]
    n = pos.shape[0]
    sim = _sim(n, box, rc=2.5, skin=0.3, max_nb=256)
    sim.build(*split_dev(pos))
    st, flags, _ = sim.check(raise_on_error=False)
    assert st == 0, (st, flags)
    got = sim.pairs().numpy()
    assert not np.any(got[:, 0] == got[:, 1])
    want = olj.neighbour_pairs(olj.wrap(pos, box), box, olj.ext_radius_sq(2.5, 0.3))
    want = want[want[:, 0] < want[:, 1]]
    g = _undirected(got, n)
    assert g.shape[0] == want.shape[0]
    assert np.array_equal(g, want[:, 0] * n + want[:, 1])  # each once: no duplicates, none missing


@pytest.mark.parametrize("name", ["sc1000_jitter", "grid_noncubic_4913", "grid_unfolded_2457", "grid_sparse_36"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shift", ["none", "cutoff"])
def test_half_forces_energy_virial(name, precision, shift):
    pos, box = CASES[name]
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3, precision=precision, shift=shift, max_nb=256)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    ref = olj.lj_forces(pos, box, 2.5, shift=shift)
    fx, fy, fz, pe_w, e = sim.forces(x, y, z, energy=True, per_atom=True)
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    g, m = force_errors(F, ref["F"])
    assert g <= 1e-5 and m <= 1e-5, (g, m)
    pe, w = pe_w.cpu().numpy()
    assert abs(pe - ref["pe"]) <= 1e-9 * abs(ref["pe"]) + 1e-12
    assert abs(w - ref["w"]) <= 1e-9 * abs(ref["w"]) + 1e-12
    ea = e.cpu().numpy()
    assert np.max(np.abs(ea - ref["e"])) <= 1e-9 * max(np.max(np.abs(ref["e"])), 1e-300) + 1e-13
    # the plain pass and the pass with energy but without per-atom energies
    for energy in (False, True):
        f2 = sim.forces(x, y, z, energy=energy)
        F2 = torch.stack(f2[:3], 1).double().cpu().numpy()
        g2, m2 = force_errors(F2, ref["F"])
        assert g2 <= 1e-5 and m2 <= 1e-5, (energy, g2, m2)
        if energy:
            assert abs(f2[3][0].item() - ref["pe"]) <= 1e-9 * abs(ref["pe"]) + 1e-12


def test_half_reaction_beyond_the_fixed_point_range():
    """A pair 0.47 sigma apart has a force component above 2^19, which the FP32
    half pass adds to the output directly instead of through its 64-bit
    fixed-point LDS sums: the forces still meet the oracle's bars."""
    pos, box = CASES["sc1000_jitter"]
    pos = pos.copy()
    pos[1] = pos[0] + np.array([0.47, 0.0, 0.0])  # the whole force on one component
    ref = olj.lj_forces(pos, box, 2.5, shift="none")
    assert np.max(np.abs(ref["F"])) > 2.0 ** 19
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3, precision="fp32", max_nb=256)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    fx, fy, fz = sim.forces(x, y, z)[:3]
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    g, m = force_errors(F, ref["F"])
    assert g <= 1e-5 and m <= 1e-5, (g, m)
    # every other atom (forces of order one) within the bar on its own scale
    rest = np.arange(2, pos.shape[0])
    gr, mr = force_errors(F[rest], ref["F"][rest])
    assert gr <= 1e-5 and mr <= 1e-5, (gr, mr)


def test_half_backward_is_minus_force():
    pos, box = CASES["grid_noncubic_4913"]
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3, precision="fp64")
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    gx, gy, gz = sim.backward(x, y, z, torch.tensor([2.0], dtype=torch.float64, device="cuda"))
    G = torch.stack([gx, gy, gz], 1).cpu().numpy()
    ref = olj.lj_forces(pos, box, 2.5)
    g, m = force_errors(G, -2.0 * ref["F"])
    assert g <= 1e-12 and m <= 1e-12, (g, m)


def test_half_run_c1_fp64_matches_oracle():
    d = mdinputs.lj_fluid(10, temperature=1.0, seed=1)
    box = d["box"]
    sim = _sim(1000, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision="fp64", shift="cutoff")
    state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    thermo = sim.run(state, 100, 10).cpu().numpy()
    assert sim.check(raise_on_error=False)[0] == 0
    ref = olj.velocity_verlet(d["pos"], d["vel"], box, 100, 0.001, 2.5, shift="cutoff", sample_every=10)
    for col in (0, 1, 2):  # KE, PE, W
        np.testing.assert_allclose(thermo[:, col], ref["thermo"][:, col + 1], rtol=1e-9, atol=1e-10)
    ids = state["ids"].long().cpu().numpy()
    inv = np.empty_like(ids)
    inv[ids] = np.arange(ids.shape[0])
    x = np.stack([state[k].cpu().numpy() for k in ("x", "y", "z")], 1)[inv]
    d_ = x - ref["pos"]
    d_ -= box[None, :] * np.round(d_ / box[None, :])
    assert np.max(np.abs(d_)) < 1e-9


def test_half_c2_full_size_sampled():
    """The 10^6-atom benchmark lattice with jitter: sampled forces against the
    oracle, each pair once over the whole list, net force ~ 0."""
    pos, box = mdinputs.sc_lattice(100)
    pos = mdinputs.perturb(pos, 0.06, 202)
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
    assert np.max(np.abs(e.cpu().numpy()[rows] - ref["e"])) <= 1e-9 * np.max(np.abs(ref["e"]))
    pairs = sim.pairs().numpy()
    und = _undirected(pairs, n)
    assert np.all(np.diff(und) > 0)  # no pair twice
    # the sampled rows see every neighbour of the definition exactly once
    want = olj.neighbour_pairs(pos, box, olj.ext_radius_sq(2.5, 0.3), rows=rows)
    touch = pairs[np.isin(pairs[:, 0], rows) | np.isin(pairs[:, 1], rows)]
    both = np.concatenate([touch, touch[:, ::-1]])
    both = both[np.isin(both[:, 0], rows)]
    both = both[np.lexsort((both[:, 1], both[:, 0]))]
    assert np.array_equal(both, want)
    assert np.linalg.norm(F.sum(0)) <= 1e-6 * np.abs(F).sum()
    pe = pe_w[0].item()
    assert abs(pe - e.sum().item()) <= 1e-9 * abs(pe)


def test_half_list_rejected_by_learned_potential():
    from paper_1704_03329_amd import mdpl as C

    pos, box = CASES["sc1000"]
    sim = _sim(1000, box, rc=2.5, skin=0.3)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    G = torch.empty(1000 * 24, dtype=torch.float32, device="cuda")
    with pytest.raises(C.MdplError) as e:
        C.mdpl_desc_fwd(sim.handle, x, y, z, G, None)
    assert e.value.status == C.MDPL_EINVAL
