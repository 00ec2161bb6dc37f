"""GPU parity of the list-free LJ pair loop (every pass scans the 27-cell
stencil of the cell list, Sec. 3.5, with no neighbour list) against the
same FP64 oracle as the lists.

Bars as for the full lists: ||dF||/||F|| <= 1e-5 and max_i |dF_i| <= 1e-5
max_i |F_i| in FP32, PE, W and per-atom energies 1e-9 relative, the FP64
velocity-Verlet run to 1e-9; forces bit-identical from run to run (fixed
summation order, no atomics)."""
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
    return LJSim(n, box, pairs="cells", **kw)


@pytest.mark.parametrize("name", ["sc1000_jitter", "grid_noncubic_4913", "grid_unfolded_2457", "grid_sparse_36",
                                  "single"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shift", ["none", "cutoff"])
def test_cells_forces_energy_virial(name, precision, shift):
    pos, box = CASES[name]
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3, precision=precision, shift=shift)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    fx, fy, fz, pe_w, e = sim.forces(x, y, z, energy=True, per_atom=True)
    assert sim.check(raise_on_error=False)[0] == 0
    ref = olj.lj_forces(pos, box, 2.5, shift=shift)
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    if np.abs(ref["F"]).max() > 0:
        g, m = force_errors(F, ref["F"])
        assert g <= 1e-5 and m <= 1e-5, (g, m)
    else:
        assert np.all(F == 0)
    pe, w = pe_w.cpu().numpy()
    assert abs(pe - ref["pe"]) <= 1e-9 * abs(ref["pe"]) + 1e-12
    assert abs(w - ref["w"]) <= 1e-9 * abs(ref["w"]) + 1e-12
    ea = e.cpu().numpy()
    assert np.max(np.abs(ea - ref["e"])) <= 1e-9 * max(np.max(np.abs(ref["e"])), 1e-300) + 1e-13
    # the plain pass: same forces, and bit-identical on a second call
    f1 = sim.forces(x, y, z)
    f2 = sim.forces(x, y, z)
    for a, b in zip(f1[:3], f2[:3]):
        assert torch.equal(a, b)
    F1 = torch.stack(f1[:3], 1).double().cpu().numpy()
    if np.abs(ref["F"]).max() > 0:
        g1, m1 = force_errors(F1, ref["F"])
        assert g1 <= 1e-5 and m1 <= 1e-5, (g1, m1)


def test_cells_backward_is_minus_force():
    pos, box = CASES["grid_noncubic_4913"]
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3, precision="fp64")
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    gx, gy, gz = sim.backward(x, y, z, torch.tensor([-0.5], dtype=torch.float64, device="cuda"))
    G = torch.stack([gx, gy, gz], 1).cpu().numpy()
    ref = olj.lj_forces(pos, box, 2.5)
    g, m = force_errors(G, 0.5 * ref["F"])
    assert g <= 1e-12 and m <= 1e-12, (g, m)


def test_cells_run_c1_fp64_matches_oracle_and_repeats():
    d = mdinputs.lj_fluid(10, temperature=1.0, seed=1)
    box = d["box"]
    mk = lambda: _sim(1000, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision="fp64", shift="cutoff")
    sim = mk()
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
    sim2 = mk()
    state2 = sim2.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    sim2.run(state2, 100, 10)
    torch.cuda.synchronize()
    for k in state:
        assert torch.equal(state[k], state2[k]), k


def test_cells_c2_full_size_sampled():
    pos, box = mdinputs.sc_lattice(100)
    pos = mdinputs.perturb(pos, 0.06, 202)
    n = pos.shape[0]
    sim = _sim(n, box, rc=2.5, skin=0.3, precision="fp32")
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    fx, fy, fz, pe_w, e = sim.forces(x, y, z, energy=True, per_atom=True)
    assert sim.check(raise_on_error=False)[0] == 0
    F = torch.stack([fx, fy, fz], 1).double().cpu().numpy()
    rows = np.sort(mdinputs.rng(9).choice(n, 126, replace=False))
    rows = np.concatenate([rows, [0, n - 1]])
    ref = olj.lj_forces(pos, box, 2.5, rows=rows)
    g, m = force_errors(F[rows], ref["F"])
    assert g <= 1e-5 and m <= 1e-5, (g, m)
    assert np.max(np.abs(e.cpu().numpy()[rows] - ref["e"])) <= 1e-9 * np.max(np.abs(ref["e"]))
    assert np.linalg.norm(F.sum(0)) <= 1e-6 * np.abs(F).sum()
    assert abs(pe_w[0].item() - e.sum().item()) <= 1e-9 * abs(pe_w[0].item())


def test_cells_no_list_and_no_learned_potential():
    from paper_1704_03329_amd import mdpl as C

    pos, box = CASES["sc1000"]
    sim = _sim(1000, box, rc=2.5, skin=0.3)
    x, y, z = split_dev(pos)
    sim.build(x, y, z)
    with pytest.raises(C.MdplError) as e:
        C.mdpl_nlist_export(sim.handle, None, None, 0)
    assert e.value.status == C.MDPL_ESTATE
    with pytest.raises(C.MdplError) as e:
        C.mdpl_nlist_entries(sim.handle)
    assert e.value.status == C.MDPL_ESTATE
    G = torch.empty(1000 * 24, dtype=torch.float32, device="cuda")
    with pytest.raises(C.MdplError) as e:
        C.mdpl_desc_fwd(sim.handle, x, y, z, G, None)
    assert e.value.status == C.MDPL_EINVAL


def test_cells_tile_overflow_flagged():
    """3300 atoms packed inside one cell of a dilute box: the tiles that hold
    that cell exceed their capacity; the pass flags it and still runs."""
    from paper_1704_03329_amd import mdpl as C

    L = 20.0
    box = np.array([L, L, L])
    cluster = 9.0 + 1.6 * mdinputs.random_box(3300, [1.0, 1.0, 1.0], 51)
    pos = np.concatenate([mdinputs.random_box(2000, box, 52), cluster])
    sim = _sim(pos.shape[0], box, rc=2.5, skin=0.3)
    cols = split_dev(pos)
    sim.build(*cols)
    sim.forces(*cols, energy=True)
    torch.cuda.synchronize()
    st, flags, _ = sim.check(raise_on_error=False)
    assert st == C.MDPL_ECAPACITY and flags & C.FLAG_NL_OVERFLOW
