"""The hand-written backward behind torch.autograd: dE/dr = -F (Eq. LJforce),
checked against the oracle's analytic forces and against finite
differences of the device energy."""
import numpy as np
import pytest
import torch

import mdinputs
from conftest import force_errors, gpu_device
from oracle import lj as olj

pytestmark = pytest.mark.gpu


def _setup(n_side=8, jitter=0.07, seed=41, precision="fp64"):
    from paper_1704_03329_amd.sim import LJSim

    dev = gpu_device()
    pos, box = mdinputs.sc_lattice(n_side)
    pos = mdinputs.perturb(pos, jitter, seed)
    # 8 sites of 1.058 give a box of 8.46 >= 3 cells of rc + skin = 2.6
    sim = LJSim(pos.shape[0], box, rc=2.5, skin=0.1, precision=precision, shift="cutoff")
    return pos, box, sim, dev


def test_backward_is_minus_analytic_force():
    from paper_1704_03329_amd.autograd import lj_energy

    pos, box, sim, dev = _setup()
    p = torch.tensor(pos, dtype=torch.float64, device=dev, requires_grad=True)
    e = lj_energy(p, sim)
    (3.0 * e).backward()
    ref = olj.lj_forces(pos, box, 2.5, shift="cutoff")
    assert e.item() == pytest.approx(ref["pe"], rel=1e-12)
    g = p.grad.cpu().numpy()
    gerr, merr = force_errors(-g / 3.0, ref["F"])
    assert gerr < 1e-12 and merr < 1e-12


def test_backward_matches_finite_differences():
    from paper_1704_03329_amd.autograd import lj_energy

    pos, box, sim, dev = _setup(seed=42)
    p = torch.tensor(pos, dtype=torch.float64, device=dev, requires_grad=True)
    lj_energy(p, sim).backward()
    g = p.grad.cpu().numpy()
    h = 1e-6
    for i in (0, 17, 263, 511):
        for k in range(3):
            q = pos.copy()
            q[i, k] += h
            ep = lj_energy(torch.tensor(q, device=dev), sim).item()
            q[i, k] -= 2 * h
            em = lj_energy(torch.tensor(q, device=dev), sim).item()
            assert g[i, k] == pytest.approx((ep - em) / (2 * h), rel=1e-6, abs=1e-7)


def test_gradcheck_small():
    from paper_1704_03329_amd.autograd import LJEnergy

    pos, box, sim, dev = _setup(seed=43)
    p = torch.tensor(pos, dtype=torch.float64, device=dev, requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: LJEnergy.apply(t, sim), (p,), eps=1e-6, atol=1e-5, rtol=1e-5)


def test_backward_fp32_context_close():
    from paper_1704_03329_amd.autograd import lj_energy

    pos, box, sim, dev = _setup(precision="fp32", seed=44)
    p = torch.tensor(pos, dtype=torch.float64, device=dev, requires_grad=True)
    lj_energy(p, sim).backward()
    ref = olj.lj_forces(pos, box, 2.5, shift="cutoff")
    gerr, merr = force_errors(-p.grad.cpu().numpy(), ref["F"])
    assert gerr < 1e-5 and merr < 1e-5
