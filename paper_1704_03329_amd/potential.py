"""The descriptor-MLP potential on the device: training-data generation by
the LJ engine, training with the library's kernels, and force evaluation.

Every numerical step runs in libmdpl (descriptors, BF16-MFMA network,
gradients, Adam, MD); this module allocates tensors, sequences the C calls
and does host-side bookkeeping (standardisation statistics of the training
set, batch index tables from the seeded input module)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

import mdinputs

from . import mdpl as C
from .sim import LJSim, boa, soa

NPARAM = 6337
OFF = {"W1": (0, (64, 32)), "b1": (2048, (64,)), "W2": (2112, (64, 64)), "b2": (6208, (64,)),
       "w3": (6272, (64,)), "b3": (6336, (1,))}


from .mdpl import (  # noqa: E402  (re-exported names of the C entry points)
    mdpl_adam_step,
    mdpl_desc_bwd,
    mdpl_desc_fwd,
    mdpl_force_error,
    MDPL_MLP_STD_SCRATCH,
    mdpl_mlp_bf16,
    mdpl_mlp_forces,
    mdpl_mlp_fwd,
    mdpl_mlp_run_floats,
    mdpl_mlp_standardise,
    mdpl_run_mlp,
    mdpl_mlp_train_floats,
    mdpl_mlp_train_grad,
    mdpl_mlp_weights,
    mdpl_scale_velocities,
)


# ------------------------------------------------------------ model
def pack(d) -> np.ndarray:
    v = np.zeros(NPARAM, dtype=np.float32)
    for k, (off, shape) in OFF.items():
        v[off:off + int(np.prod(shape))] = np.asarray(d[k], dtype=np.float32).ravel()
    return v


def unpack(v) -> dict:
    v = np.asarray(v, dtype=np.float64)
    return {k: v[off:off + int(np.prod(shape))].reshape(shape) for k, (off, shape) in OFF.items()}


class MLPPotential:
    """Parameters on the device: FP32 master vector, Adam moments, BF16 copies
    of the weight matrices, biases (views of the master vector), feature and
    energy standardisation."""

    def __init__(self, seed: int = 0, device="cuda"):
        self.device = torch.device(device)
        self.params = torch.from_numpy(pack(mdinputs.mlp_init(seed))).to(self.device)
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.w1 = torch.empty(2048, dtype=torch.int16, device=self.device)
        self.w2 = torch.empty(4096, dtype=torch.int16, device=self.device)
        self.w3 = torch.empty(64, dtype=torch.int16, device=self.device)
        mdpl_mlp_bf16(self.params, self.w1, self.w2, self.w3)
        self.mu = torch.zeros(24, dtype=torch.float32, device=self.device)
        self.sd = torch.ones(24, dtype=torch.float32, device=self.device)
        self.e_mean = 0.0
        self.e_sd = 1.0
        self.step = 0

    def weights(self) -> mdpl_mlp_weights:
        w = mdpl_mlp_weights()
        w.w1, w.w2, w.w3 = self.w1.data_ptr(), self.w2.data_ptr(), self.w3.data_ptr()
        w.b1 = self.params.data_ptr() + 4 * 2048
        w.b2 = self.params.data_ptr() + 4 * 6208
        w.b3 = self.params.data_ptr() + 4 * 6336
        w.mu, w.sd = self.mu.data_ptr(), self.sd.data_ptr()
        w.e_mean, w.e_sd = float(self.e_mean), float(self.e_sd)
        return w

    def host_params(self) -> dict:
        """Parameters as used by the kernels: bf16-rounded weights, FP32 biases (FP64 arrays)."""
        d = unpack(self.params.cpu().numpy())
        d["W1"] = self.w1.view(torch.bfloat16).float().cpu().numpy().reshape(64, 32).astype(np.float64)
        d["W2"] = self.w2.view(torch.bfloat16).float().cpu().numpy().reshape(64, 64).astype(np.float64)
        d["w3"] = self.w3.view(torch.bfloat16).float().cpu().numpy().astype(np.float64)
        return d

    def set_standardisation(self, G: torch.Tensor, e: torch.Tensor):
        """Feature and energy statistics of the training set (mdpl_mlp_standardise)."""
        stats = torch.empty(2, dtype=torch.float64, device=self.device)
        scratch = torch.empty(MDPL_MLP_STD_SCRATCH, dtype=torch.float64, device=self.device)
        mdpl_mlp_standardise(G.contiguous(), e.contiguous(), self.mu, self.sd, stats, scratch)
        self.e_mean, self.e_sd = (float(v) for v in stats.cpu())

    def train(self, G: torch.Tensor, e: torch.Tensor, steps: int, batch: int = 4096, lr: float = 1e-3,
              seed: int = 99, log_every: int = 0, lr_final: float | None = None):
        """Adam on L = mean (y - (e - e_mean)/e_sd)^2 over random batches."""
        n = G.shape[0]
        energy = e.to(torch.float64).contiguous()
        idx = torch.from_numpy(mdinputs.batch_indices(n, batch, steps, seed)).to(self.device)
        scratch = torch.empty(mdpl_mlp_train_floats(batch), dtype=torch.float32, device=self.device)
        grad = torch.empty(NPARAM + 1, dtype=torch.float32, device=self.device)
        losses = []
        w = self.weights()
        for k in range(steps):
            mdpl_mlp_train_grad(w, G, idx[k], batch, energy, scratch, grad)
            self.step += 1
            rate = lr if lr_final is None else lr * (lr_final / lr) ** (k / max(steps - 1, 1))
            mdpl_adam_step(self.params, grad, self.m, self.v, rate, 0.9, 0.999, 1e-8, self.step, self.w1, self.w2,
                           self.w3)
            if log_every and (k % log_every == 0 or k == steps - 1):
                losses.append((k, float(grad[NPARAM].item())))
        return losses

    def energy(self, G: torch.Tensor, with_grad: bool = False):
        n = G.shape[0]
        e = torch.empty(n, dtype=torch.float32, device=self.device)
        dG = torch.empty((n, 24), dtype=torch.float32, device=self.device) if with_grad else None
        mdpl_mlp_fwd(self.weights(), G, n, e, dG)
        return e, dG

    def buffers(self, n: int) -> dict:
        """Device buffers of one force evaluation for n atoms: the library's
        workspace (features, moments, energies, dE/dG, in that order, with
        views of each) and the forces."""
        def f32(*shape):
            return torch.empty(shape, dtype=torch.float32, device=self.device)

        ws = f32(mdpl_mlp_run_floats(n))
        return {"ws": ws, "G": ws[:24 * n].view(n, 24), "mom": ws[24 * n:74 * n].view(n, 50),
                "e": ws[74 * n:75 * n], "dG": ws[75 * n:99 * n].view(n, 24),
                "fx": f32(n), "fy": f32(n), "fz": f32(n)}

    def forces(self, sim: LJSim, x, y, z, buf: dict | None = None):
        """(per-atom energies, fx, fy, fz) for positions already built in sim:
        descriptors and their moments, network energies and dE/dG, then the
        descriptor backward (a scatter of the pair terms), in one library
        call."""
        n = sim.n
        b = buf if buf is not None else self.buffers(n)
        mdpl_mlp_forces(sim, self.weights(), x, y, z, b["ws"], b["e"], b["fx"], b["fy"], b["fz"])
        return b["e"], b["fx"], b["fy"], b["fz"]

    def forces_three_calls(self, sim: LJSim, x, y, z, buf: dict | None = None):
        """forces() through the three separate entry points (descriptors,
        network, backward)."""
        n = sim.n
        b = buf if buf is not None else self.buffers(n)
        mdpl_desc_fwd(sim, x, y, z, b["G"], b["mom"])
        mdpl_mlp_fwd(self.weights(), b["G"], n, b["e"], b["dG"])
        mdpl_desc_bwd(sim, x, y, z, b["dG"], b["mom"], b["fx"], b["fy"], b["fz"])
        return b["e"], b["fx"], b["fy"], b["fz"]


# ------------------------------------------------------------ data
def descriptors(sim: LJSim, pos: torch.Tensor):
    """Build lists for pos (N,3 float64 device) and return G (N,24)."""
    x, y, z = soa(pos)
    sim.build(x, y, z)
    G = torch.empty((sim.n, 24), dtype=torch.float32, device=pos.device)
    mdpl_desc_fwd(sim, x, y, z, G, None)
    return G


def lj_snapshot_targets(sim: LJSim, pos: torch.Tensor):
    """Per-atom LJ energies (plain potential) and forces (FP64) for pos."""
    x, y, z = soa(pos)
    sim.build(x, y, z)
    fx, fy, fz, pe_w, e = sim.forces(x, y, z, energy=True, per_atom=True)
    return e, torch.stack([fx, fy, fz], 1)


def generate_training_set(temperatures=(0.7, 1.0, 1.5), counts=(67, 67, 66), n_cells: int = 10,
                          equil_steps: int = 5000, every: int = 200, rescale_every: int = 10,
                          seeds=(40, 41, 42), device="cuda"):
    """Snapshots of the FCC start (n_cells^3 cells, rho 0.8442) melted and held
    at each temperature by velocity rescaling every `rescale_every` steps for
    `equil_steps`, then sampled every `every` NVE steps.  Returns
    dict(G (M,24), e (M,), F (M,3), temp (M,), snap (M,)) on the device."""
    dev = torch.device(device)
    out_G, out_e, out_F, out_T, out_s = [], [], [], [], []
    snap = 0
    for T, cnt, seed in zip(temperatures, counts, seeds):
        d = mdinputs.fcc_lj(n_cells, temperature=T, seed=seed)
        n = d["pos"].shape[0]
        box = d["box"]
        run = LJSim(n, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision="fp64", shift="none")
        ref = LJSim(n, box, rc=2.5, skin=0.3, precision="fp64", shift="none")
        st = run.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
        # each run continues the last one (list, forces, rebuild schedule);
        # rescaling the velocities in between is allowed
        for r in range(equil_steps // rescale_every):
            th = run.run(st, rescale_every, rescale_every, cont=r > 0)
            ke = float(th[-1, 0].item())
            t_now = 2.0 * ke / (3.0 * (n - 1))
            mdpl_scale_velocities(st["vx"], st["vy"], st["vz"], (T / t_now) ** 0.5)
        for k in range(cnt):
            run.run(st, every, 0, cont=True)
            pos = torch.stack([st["x"], st["y"], st["z"]], 1)
            e, F = lj_snapshot_targets(ref, pos)
            G = descriptors(ref, pos)
            out_G.append(G)
            out_e.append(e)
            out_F.append(F)
            out_T.append(torch.full((n,), T, device=dev))
            out_s.append(torch.full((n,), snap, device=dev, dtype=torch.int32))
            snap += 1
        status = run.check(raise_on_error=False)[0]
        if status != 0:
            raise RuntimeError(f"training MD at T={T} flagged status {status}")
    return {"G": torch.cat(out_G), "e": torch.cat(out_e), "F": torch.cat(out_F), "temp": torch.cat(out_T),
            "snap": torch.cat(out_s)}


# ------------------------------------------------------------ MD with the network
def mlp_md(model: MLPPotential, pos, vel, box, nsteps: int = 500, check_every: int = 50,
           boa_every: int = 100, boa_rc: float = 1.5, sample_every: int = 10, dt: float = 0.001,
           reuse_every: int = 10, log=None):
    """Velocity-Verlet MD with the network as the force field (mdpl_run_mlp),
    in segments of check_every steps.  After each segment the network's
    forces are compared with FP64 LJ forces at the same positions
    (mdpl_force_error); every boa_every steps Q4/Q6 are evaluated with
    cutoff boa_rc.  Returns dict(state, thermo (rows KE, PE, 0, max disp),
    checks [(step, rmse, rel)], boa [(step, mean Q4, mean Q6, mean nnb)],
    force_ms (average network force pass), sim)."""
    n = int(pos.shape[0])
    sim = LJSim(n, box, rc=2.5, skin=0.3, dt=dt, reuse_every=reuse_every, precision="fp32", shift="none")
    ref = LJSim(n, box, rc=2.5, skin=0.3, precision="fp64", shift="none")
    st = sim.new_state(pos, vel)
    ws = torch.empty(mdpl_mlp_run_floats(n), dtype=torch.float32, device=sim.device)
    err = torch.empty(2, dtype=torch.float64, device=sim.device)
    w = model.weights()
    rows_per = check_every // sample_every + 1
    thermo, checks, boas = [], [], []
    from . import mdpl as C

    C.mdpl_set_timing(sim.handle, True)
    C.mdpl_kernel_time(sim.handle, 0)
    C.mdpl_kernel_time(sim.handle, 1)
    for seg in range(nsteps // check_every):
        th = torch.empty((rows_per, 4), dtype=torch.float64, device=sim.device)
        mdpl_run_mlp(sim, w, ws, st, check_every, sample_every, th, start=1 if seg else 0)
        step = (seg + 1) * check_every
        thermo.append(th if seg == 0 else th[1:])
        ref.build(st["x"], st["y"], st["z"])
        gx, gy, gz, _, _ = ref.forces(st["x"], st["y"], st["z"])
        mdpl_force_error(ref, st["fx"], st["fy"], st["fz"], gx, gy, gz, err)
        e = err.cpu().numpy()
        checks.append((step, float(np.sqrt(e[0] / (3 * n))), float(np.sqrt(e[0] / e[1]))))
        if boa_every and step % boa_every == 0:
            q = boa(st["x"], st["y"], st["z"], box, boa_rc)
            boas.append((step, float(q["q4"].double().mean().item()), float(q["q6"].double().mean().item()),
                         float(q["nnb"].double().mean().item())))
        if log:
            log(f"step {step}: force RMSE vs LJ {checks[-1][1]:.4f} (rel {checks[-1][2]:.4f})")
    p_ms, p_n = C.mdpl_kernel_time(sim.handle, 0)
    e_ms, e_n = C.mdpl_kernel_time(sim.handle, 1)
    C.mdpl_set_timing(sim.handle, False)
    return {"state": st, "thermo": torch.cat(thermo), "checks": checks, "boa": boas,
            "force_ms": (p_ms + e_ms) / max(p_n + e_n, 1), "sim": sim}
