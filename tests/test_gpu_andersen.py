"""GPU parity of the Andersen thermostat run (the crystallisation run of
Sec. 5.2) against the FP64 oracle with the same Philox4x64-10 draws.

Bars: thermo (KE, PE, W), positions and velocities of the FP64 run to 1e-9
relative (the collision decisions are exact: the same 53-bit uniforms on
both sides; the Box-Muller normals use the device's and the host's log,
sqrt, cos and sin, within an ulp of each other); a zero collision rate is
bit-identical to mdpl_run; a run split in two with step0 is bit-identical
to one run; at a fixed bath temperature the kinetic temperature settles at
it."""
import numpy as np
import pytest
import torch

import mdinputs
from conftest import gpu_device
from oracle import lj as olj

pytestmark = pytest.mark.gpu


def _sim(n, box, **kw):
    from paper_1704_03329_amd.sim import LJSim

    gpu_device()
    return LJSim(n, box, **kw)


def _state_np(state):
    ids = state["ids"].long().cpu().numpy()
    inv = np.empty_like(ids)
    inv[ids] = np.arange(ids.shape[0])
    get = lambda *k: np.stack([state[c].cpu().numpy() for c in k], 1)[inv]
    return get("x", "y", "z"), get("vx", "vy", "vz")


def test_andersen_run_matches_oracle():
    d = mdinputs.lj_fluid(10, temperature=1.0, seed=1)
    box = d["box"]
    th = dict(temperature=0.5, collision_rate=50.0, seed=2024, step0=7)
    sim = _sim(1000, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision="fp64", shift="cutoff")
    state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    thermo = sim.run(state, 60, 10, andersen=th).cpu().numpy()
    assert sim.check(raise_on_error=False)[0] == 0
    ref = olj.velocity_verlet(d["pos"], d["vel"], box, 60, 0.001, 2.5, shift="cutoff", sample_every=10,
                              andersen=dict(temperature=0.5, nu=50.0, seed=2024, step0=7, ids=np.arange(1000)))
    for col in (0, 1, 2):
        np.testing.assert_allclose(thermo[:, col], ref["thermo"][:, col + 1], rtol=1e-9, atol=1e-10)
    x, v = _state_np(state)
    dx = x - ref["pos"]
    dx -= box[None, :] * np.round(dx / box[None, :])
    assert np.max(np.abs(dx)) < 1e-9
    assert np.max(np.abs(v - ref["vel"])) < 1e-9
    # the collisions did happen: about p = 0.05 of the particles per step
    moved = np.mean(np.abs(v - olj.velocity_verlet(d["pos"], d["vel"], box, 60, 0.001, 2.5, shift="cutoff")["vel"]))
    assert moved > 0.1


def test_zero_rate_is_plain_run_and_split_runs_continue():
    d = mdinputs.lj_fluid(10, temperature=1.0, seed=3)
    box = d["box"]
    mk = lambda: _sim(1000, box, rc=2.5, skin=0.3, reuse_every=10, precision="fp64")
    s0 = mk()
    a = s0.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    s0.run(a, 40, 10)
    s1 = mk()
    b = s1.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    s1.run(b, 40, 10, andersen=dict(temperature=1.0, collision_rate=0.0, seed=1))
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k
    th = dict(temperature=0.8, collision_rate=20.0, seed=77)
    s2 = mk()
    c = s2.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    s2.run(c, 40, 10, andersen=dict(th, step0=0))
    s3 = mk()
    e = s3.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    s3.run(e, 20, 10, andersen=dict(th, step0=0))
    s3.run(e, 20, 10, andersen=dict(th, step0=20))
    torch.cuda.synchronize()
    for k in c:
        assert torch.equal(c[k], e[k]), k
    # continued runs (no rebinning or F(r0) pass between them), split inside a
    # reuse period, against one run with the same (absent) energy sampling
    s5 = mk()
    g = s5.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    s5.run(g, 40, 0, andersen=dict(th, step0=0))
    s4 = mk()
    f = s4.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    s4.run(f, 17, 0, andersen=dict(th, step0=0))
    s4.run(f, 23, 0, andersen=dict(th, step0=17), cont=True)
    torch.cuda.synchronize()
    for k in g:
        assert torch.equal(g[k], f[k]), k


def test_bath_temperature_reached():
    d = mdinputs.lj_fluid(16, temperature=0.1, seed=4)  # N = 4096, cold start
    box = d["box"]
    n = d["pos"].shape[0]
    sim = _sim(n, box, rc=2.5, skin=0.3, reuse_every=10, precision="fp32")
    state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    thermo = sim.run(state, 3000, 50, andersen=dict(temperature=1.2, collision_rate=10.0, seed=5)).cpu().numpy()
    assert sim.check(raise_on_error=False)[0] == 0
    t_kin = thermo[:, 0] / (1.5 * n)
    late = t_kin[-20:].mean()
    assert abs(late - 1.2) < 0.05, t_kin.tolist()


def test_andersen_argument_errors():
    from paper_1704_03329_amd import mdpl as C

    d = mdinputs.lj_fluid(10, temperature=1.0, seed=1)
    sim = _sim(1000, d["box"], dt=0.001)
    st = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    for bad in (dict(temperature=-1.0, collision_rate=1.0, seed=1),
                dict(temperature=1.0, collision_rate=-1.0, seed=1),
                dict(temperature=1.0, collision_rate=2000.0, seed=1),   # nu dt > 1
                dict(temperature=1.0, collision_rate=1.0, seed=1, step0=-3)):
        with pytest.raises(C.MdplError) as e:
            sim.run(st, 5, 0, andersen=bad)
        assert e.value.status == C.MDPL_EINVAL
