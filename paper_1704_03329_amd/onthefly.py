"""On-the-fly bond-order analysis during crystallisation (the structure
analysis run of Sec. 5.2): particles start on a periodic cubic lattice
with velocities drawn from a normal distribution, run in the
microcanonical ensemble, then are coupled to an Andersen thermostat at a
temperature near zero; Q4, Q5 and Q6 (Sec. 4.1) are evaluated every
`boa_every` steps while the run proceeds.

Only orchestration happens here: the steps run in mdpl_run /
mdpl_run_andersen and the analysis in mdpl_boa, all on the device; the
per-step means are torch reductions of the device outputs.

Readings (the paper states the protocol, not these numbers): the LJ
parameters of its bond-order scaling runs (Tab. order_scaling: rho 0.8442,
rc 3.0, rc + delta 3.3, list rebuilt every 18 steps) with dt 0.001, the
step that keeps 18 steps of motion within delta / 2; initial temperature
1.0, bath temperature 0.01, collision rate 10 per unit time, Q_l bonds
within 1.5 sigma (the first minimum of the liquid's g(r)).
"""
from __future__ import annotations

import time

import torch

from . import mdpl as C
from .sim import LJSim, boa


def crystallise(pos, vel, box, nve_steps=50_000, nvt_steps=500_000, boa_every=1000, dt=0.001,
                rc=3.0, skin=0.3, reuse_every=18, t_bath=0.01, collision_rate=10.0, seed=1,
                boa_rc=1.5, precision="fp32", log=None):
    """Run the protocol; returns dict(trace, state, sim, md_seconds,
    boa_seconds, steps).  trace rows: (step, mean Q4, mean Q5, mean Q6,
    KE/N, PE/N) after each block of boa_every steps (and at step 0)."""
    n = pos.shape[0]
    sim = LJSim(n, box, rc=rc, skin=skin, dt=dt, reuse_every=reuse_every, shift="cutoff",
                precision=precision, max_nb=256)
    state = sim.new_state(torch.as_tensor(pos), torch.as_tensor(vel))
    trace = []
    md_s = boa_s = 0.0

    def analyse(step, thermo_row):
        nonlocal boa_s
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q = boa(state["x"], state["y"], state["z"], box, boa_rc, q5=True)
        means = [float(q[k].double().mean()) for k in ("q4", "q5", "q6")]
        torch.cuda.synchronize()
        boa_s += time.perf_counter() - t0
        ke, pe = (float(thermo_row[0]) / n, float(thermo_row[1]) / n) if thermo_row is not None else (None, None)
        trace.append((step, *means, ke, pe))
        if log:
            log(f"step {step}: Q4 {means[0]:.4f} Q5 {means[1]:.4f} Q6 {means[2]:.4f} KE/N {ke} PE/N {pe}")

    step = 0
    analyse(0, None)
    total = nve_steps + nvt_steps
    while step < total:
        nvt = step >= nve_steps
        block = min(boa_every, (nve_steps if not nvt else total) - step)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = dict(temperature=t_bath, collision_rate=collision_rate, seed=seed, step0=step) if nvt else None
        thermo = sim.run(state, block, block, andersen=th, cont=step > 0)
        torch.cuda.synchronize()
        md_s += time.perf_counter() - t0
        st, flags, _ = C.mdpl_check(sim.handle, False)
        if st != 0:
            raise C.MdplError(st, f"crystallisation run flagged {flags} at step {step + block}")
        step += block
        analyse(step, thermo[-1].cpu().numpy())
    return {"trace": trace, "state": state, "sim": sim, "md_seconds": md_s, "boa_seconds": boa_s,
            "steps": total}
