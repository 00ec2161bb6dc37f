"""Benchmark: Lennard-Jones MD with neighbour lists, N = 10^6, one MI355X.

Workload (the paper's LJ benchmark parameters, Tab. 7.2T1, with a 0.3 skin
and a list rebuild every 10 steps): 100^3 simple-cubic lattice at density
0.8442, Gaussian velocities at T* = 1 (seed 2), eps = sigma = m = 1,
rc = 2.5 (energy shifted to zero at rc, so the reported drift measures the
integration), skin 0.3, dt = 0.001, FP32 pair forces with FP64 positions,
energies and virial; PE and virial every 10 steps.  The lattice melts in
--premelt untimed steps (default 1000) of the same run, ahead of the warmup,
so that a short timed run measures the fluid, as a long one does.

A step is one full velocity-Verlet step of the whole path: the force pass
(with energy/virial on every 10th step) followed in the same kernel by the
next step's kick-kick-drift, and on every 10th step the skin check, cell
binning, reordering and neighbour-list build; KE reductions on sampled steps.
Inputs are resident in HBM before timing starts.

Prints one JSON line (see the keys below).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s LJ N=1M + HBM GB/s; MLP vs LJ time at stated force RMSE"
HBM_PEAK_GBS = 8000.0
# the force-kernel launches timed with HIP events: one in TIME_EVERY of each kernel
TIME_EVERY = 8
# every source the force kernel is compiled from (counter summaries name their hash)
FORCE_SRC = [os.path.join(ROOT, "paper_1704_03329_amd", "csrc", f)
             for f in ("lj.hip", "tile.h", "device_util.h", "internal.h")] + \
    [os.path.join(ROOT, "include", "mdpl.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lj_force_f32_n1m_traffic.txt")
FLOPS_FILE = os.path.join(ROOT, "profiles", "lj_force_f32_n1m_flops.txt")
# vector (non-matrix) peaks: 256 CUs x 2.4 GHz x 64 lanes x 2 (fused multiply-add) for FP64 and
# for unpacked FP32; the FP32 figure doubles with packed two-wide instructions
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def force_src_hash() -> str:
    h = hashlib.sha256()
    for path in FORCE_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_summary(path):
    """The key: value lines of a committed counter summary, or None if it is
    absent or was taken on a different version of the force kernel."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("force_source_sha256_16") != force_src_hash():
        return None
    return kv


def measured_traffic():
    """HBM bytes per force launch from the committed counter summary."""
    kv = counter_summary(TRAFFIC_FILE)
    try:
        return float(kv["hbm_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def measured_flops(avg_s, entries):
    """FP32 and FP64 vector FLOP rates of the plain force kernel: the counted
    FLOPs per launch from the committed counter summary over the launch time
    measured in this run (None if the summary does not match the kernel)."""
    kv = counter_summary(FLOPS_FILE)
    if not kv:
        return None
    try:
        f32 = float(kv["fp32_flops_per_launch"]) + float(kv["fp32_trans_per_launch"])
        f64 = float(kv["fp64_flops_per_launch"]) + float(kv["fp64_trans_per_launch"])
        valu = float(kv["valu_insts_per_entry"])
        ent = float(kv["entries_per_launch"])
    except (KeyError, ValueError):
        return None
    # the summary's launches may hold another entry count than this run's
    # (the summary is taken on the melted fluid); scale the counted work to
    # this run's entry count
    k = entries / ent if ent > 0 else 1.0
    t32, t64 = f32 * k / avg_s / 1e12, f64 * k / avg_s / 1e12
    # vector issue: 256 CUs x 4 SIMDs x 16 lanes per clock at 2.4 GHz
    issue = valu * entries / avg_s / (256 * 64 * 2.4e9)
    return {"fp32_tflops": t32, "fp64_tflops": t64, "unit": "TFLOP/s",
            "peak_fp32": FP32_PEAK_TFLOPS, "peak_fp64": FP64_PEAK_TFLOPS,
            "frac_fp32": t32 / FP32_PEAK_TFLOPS, "frac_fp64": t64 / FP64_PEAK_TFLOPS,
            "fp32_flops_per_entry": f32 / ent, "fp64_flops_per_entry": f64 / ent,
            "valu_insts_per_entry": valu, "valu_issue_frac": issue,
            "source": "rocprofv3 SQ_INSTS_VALU_FLOPS_* counters (profiles/lj_force_f32_n1m_flops.txt)"}


def cpu_baseline(pos, vel, box):
    """The FP64 oracle on the same workload: one velocity-Verlet step of the
    whole N = 10^6 system (oracle.lj.velocity_verlet with the k-d tree route
    of lj_forces_tree: candidate pairs on all host threads, then the
    definition's minimum-image test and pair terms in numpy).  The run also
    computes F(r0), so a step is taken as half of the elapsed time."""
    from oracle import lj as olj

    n = pos.shape[0]
    threads = os.cpu_count()
    t0 = time.perf_counter()
    olj.velocity_verlet(pos, vel, box, 1, 0.001, 2.5, shift="cutoff",
                        force_fn=lambda r: olj.lj_forces_tree(r, box, 2.5, shift="cutoff"))
    dt = time.perf_counter() - t0
    return {
        "value": n / (dt / 2.0),
        "unit": "atom-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one FP64 velocity-Verlet step of all {n} atoms (the oracle's k-d tree route: scipy cKDTree "
                  f"candidates with workers=-1 on {threads} host threads, then numpy on one thread for the "
                  f"exact minimum-image test, forces and updates); F(r0) + 1 step took {dt:.1f} s, "
                  "a step = half of it; no neighbour-list reuse",
    }


def oracle_analysis_rate():
    """The analysis oracles (all-pairs neighbour sets; scipy spherical
    harmonics for Q4/Q6; CNA with Python sets) on a bounded sample: every
    atom of a 5,000-atom polycrystal of the same recipe (their cost grows as
    N^2, so this rate is an upper bound of theirs at N = 4e6)."""
    import mdinputs
    from oracle import boa as ob
    from oracle import cna as oc

    pc = mdinputs.polycrystal(5_000, 4, seed=3)
    pos, box, rc = pc["pos"], pc["box"], 1.2684 * pc["d"]
    n = pos.shape[0]
    t0 = time.perf_counter()
    ob.bond_order(pos, box, rc, ls=(4, 6))
    t_boa = time.perf_counter() - t0
    t0 = time.perf_counter()
    oc.cna(pos, box, rc)
    t_cna = time.perf_counter() - t0
    return {"boa_atoms_per_s": n / t_boa, "cna_atoms_per_s": n / t_cna, "cores": 1, "kind": "oracle",
            "sample": f"all {n} atoms of a 4-grain polycrystal (rho 1, jitter 0.05 d, seed 3); numpy/scipy on "
                      f"one thread; BOA {t_boa:.1f} s, CNA {t_cna:.1f} s"}


def oracle_mlp_rate(pos, box, model):
    """The learned potential's FP64 oracle (direct descriptor triple sums,
    the network, the chain rule for forces) on 200 sampled centres of the
    evaluation configuration, with the same bf16-rounded weights."""
    import numpy as np

    from oracle import descriptor as OD
    from oracle import mlp as OM

    rows = np.sort(np.random.Generator(np.random.PCG64(45)).choice(pos.shape[0], 200, replace=False))
    p = model.host_params()
    mu = model.mu.double().cpu().numpy()
    sd = model.sd.double().cpu().numpy()
    t0 = time.perf_counter()
    G, table, grads = OD.descriptors(pos, box, rows=rows, with_grad=True)
    _, dEdG = OM.energy_and_feature_grad(p, G, mu, sd, model.e_mean, model.e_sd)
    OD.forces_from_feature_grad(pos.shape[0], rows, table, grads, dEdG)
    dt = time.perf_counter() - t0
    return {"atoms_per_s": rows.shape[0] / dt, "cores": 1, "kind": "oracle",
            "sample": f"{rows.shape[0]} centres of the N={pos.shape[0]} evaluation configuration: descriptors, "
                      f"energies, dE/dG and their force terms in FP64 numpy on one thread, {dt:.1f} s"}


def event_time(fn, reps: int) -> float:
    """Average seconds of fn() over reps calls, timed with events on the
    current stream (every call of the path enqueues on it)."""
    import torch

    fn()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def mlp_report(args):
    """The learned potential beside plain LJ: train on engine-generated
    snapshots, then time one force evaluation of each on the evaluation
    configuration and state the MLP's force error against FP64 LJ."""
    import numpy as np
    import torch

    import mdinputs
    from paper_1704_03329_amd import potential as P
    from paper_1704_03329_amd.sim import LJSim, soa

    t0 = time.perf_counter()
    log("MLP: generating 200 training snapshots (FCC 10^3, N=4000, T* 0.7/1.0/1.5)")
    data = P.generate_training_set()
    snap = data["snap"].cpu().numpy()
    temp = data["temp"].cpu().numpy()
    # 20 validation snapshots, stratified by temperature: the last ones of each T*
    val_snaps = []
    for T in (0.7, 1.0, 1.5):
        s_t = np.unique(snap[np.isclose(temp, T)])
        val_snaps.extend(s_t[-(7 if T < 1.4 else 6):].tolist())
    is_val = np.isin(snap, val_snaps)
    tr = torch.from_numpy(np.nonzero(~is_val)[0]).cuda()
    va = torch.from_numpy(np.nonzero(is_val)[0]).cuda()
    Gtr, etr = data["G"][tr].contiguous(), data["e"][tr].contiguous()
    Gva, eva = data["G"][va].contiguous(), data["e"][va].contiguous()
    model = P.MLPPotential(seed=11)
    model.set_standardisation(Gtr, etr)
    e0, _ = model.energy(Gva)
    mae_untrained = float(torch.mean(torch.abs(e0.double() - eva)).item())
    log(f"MLP: training {args.mlp_steps} Adam steps, batch 4096, on {tr.numel()} atoms")
    t_train = time.perf_counter()
    losses = model.train(Gtr, etr, steps=args.mlp_steps, batch=4096, lr=3e-3, lr_final=1e-4,
                         log_every=max(args.mlp_steps // 4, 1))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    e1, _ = model.energy(Gva)
    mae_val = float(torch.mean(torch.abs(e1.double() - eva)).item())

    log("MLP: evaluation configuration (64^3 sc, rho 0.8442, melted 2000 steps at T*=1, seed 43)")
    d = mdinputs.lj_fluid(64, temperature=1.0, seed=43)
    n = d["pos"].shape[0]
    box = d["box"]
    md = LJSim(n, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision="fp64", shift="cutoff")
    st = md.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
    md.run(st, 2000, 0)
    md.check()
    pos = torch.stack([st["x"], st["y"], st["z"]], 1)
    x, y, z = soa(pos)
    ref = LJSim(n, box, rc=2.5, skin=0.3, precision="fp64", shift="none")
    ref.build(x, y, z)
    fx, fy, fz, _, e_lj = ref.forces(x, y, z, energy=True, per_atom=True)
    F_lj = torch.stack([fx, fy, fz], 1)
    lj32 = LJSim(n, box, rc=2.5, skin=0.3, precision="fp32", shift="none")
    lj32.build(x, y, z)
    f32 = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3)]

    def lj_force():
        lj32_forces(lj32, x, y, z, f32)

    lj_force()
    buf = model.buffers(n)
    model.forces(ref, x, y, z, buf)
    F_mlp = torch.stack([buf["fx"], buf["fy"], buf["fz"]], 1).double()
    e_mlp = buf["e"].double()
    F32 = torch.stack(f32, 1).double()
    rms = lambda t: float(torch.sqrt(torch.mean(t * t)).item())  # noqa: E731
    reps = 50
    t_lj = event_time(lj_force, reps)
    t_mlp = event_time(lambda: model.forces(ref, x, y, z, buf), reps)
    t_build = event_time(lambda: ref.build(x, y, z), 10)
    oracle = oracle_mlp_rate(pos.cpu().numpy(), box, model) if not args.no_cpu_baseline else None
    log(f"MLP: LJ force {t_lj * 1e6:.1f} us, MLP energy+forces {t_mlp * 1e6:.1f} us, build {t_build * 1e6:.1f} us")
    return {
        "workload": f"MLP 24-64-64-1 (16 radial + 8 angular features within 2.5, BF16 weights, FP32 "
                    f"accumulation) vs LJ forces on N={n} (64^3 sc melted 2000 steps at T*=1, seed 43); "
                    "trained on 180 + 20 validation snapshots of N=4000 at T* 0.7/1.0/1.5",
        "n_atoms": n,
        "mlp_us_per_eval": t_mlp * 1e6,
        "mlp_atoms_per_s": n / t_mlp,
        "oracle": oracle,
        "lj_fp32_us_per_eval": t_lj * 1e6,
        "nlist_build_us": t_build * 1e6,
        "time_ratio_mlp_over_lj": t_mlp / t_lj,
        "mlp_force_rmse": rms(F_mlp - F_lj),
        "lj_fp32_force_rmse": rms(F32 - F_lj),
        "lj_force_rms": rms(F_lj),
        "mlp_energy_mae_per_atom": float(torch.mean(torch.abs(e_mlp - e_lj)).item()),
        "validation_energy_mae": {"trained": mae_val, "untrained": mae_untrained},
        "train_steps": args.mlp_steps,
        "train_seconds": t_train,
        "train_loss_first_last": [losses[0][1], losses[-1][1]],
        "seconds_total": time.perf_counter() - t0,
    }


def analysis_report(with_oracle: bool = True):
    """Bond order (Q4, Q6) and CNA on the structure-analysis workload: 50
    FCC/HCP/BCC grains, N ~ 4e6, rho 1, jitter 0.05 d, seed 3, cutoff 1.2684 d."""
    import numpy as np
    import torch

    import mdinputs
    from paper_1704_03329_amd import mdpl as C
    from paper_1704_03329_amd.sim import soa

    log("analysis: generating the 4e6-atom polycrystal")
    pc = mdinputs.polycrystal(4_000_000, 50, seed=3)
    box, rc = pc["box"], 1.2684 * pc["d"]
    x, y, z = soa(torch.from_numpy(pc["pos"]).cuda())
    n = x.numel()
    dev = x.device
    ws_b = torch.empty(C.mdpl_analysis_workspace_bytes(n, box, rc, 1), dtype=torch.uint8, device=dev)
    # CNA bond-list capacity: triplets are computed for every particle with at
    # most this many bonds (labels are exact at any capacity >= 14)
    cap = 32
    ws_c = torch.empty(C.mdpl_analysis_workspace_bytes(n, box, rc, cap), dtype=torch.uint8, device=dev)
    q4 = torch.empty(n, dtype=torch.float32, device=dev)
    q6 = torch.empty_like(q4)
    nnb = torch.empty(n, dtype=torch.int32, device=dev)
    trip = torch.empty((n, cap), dtype=torch.int32, device=dev)
    label = torch.empty(n, dtype=torch.uint8, device=dev)
    most = torch.zeros(1, dtype=torch.int32, device=dev)
    t_boa = event_time(lambda: C.mdpl_boa(x, y, z, box, rc, q4, None, q6, nnb, ws_b), 5)
    t_cna = event_time(lambda: C.mdpl_cna(x, y, z, box, rc, cap, trip, nnb, label, ws_c, most), 5)
    frac = np.bincount(label.cpu().numpy(), minlength=4) / n
    max_bonds = int(most.item())
    log(f"analysis: BOA {t_boa * 1e3:.2f} ms, CNA {t_cna * 1e3:.2f} ms (capacity {cap}, "
        f"largest bond count {max_bonds})")
    oracle = oracle_analysis_rate() if with_oracle else None
    return {
        "oracle": oracle,
        "workload": f"50 FCC/HCP/BCC grains, N={n}, rho 1.0, jitter 0.05 d, seed 3, cutoff {rc:.4f} "
                    "(neighbour list, bond order and CNA each included)",
        "n_atoms": n,
        "boa_ms": t_boa * 1e3,
        "cna_ms": t_cna * 1e3,
        "boa_atoms_per_s": n / t_boa,
        "cna_atoms_per_s": n / t_cna,
        "label_fractions": {k: float(v) for k, v in zip(("other", "fcc", "hcp", "bcc"), frac)},
        "cna_capacity": cap,
        "max_bond_count": max_bonds,
        "cna_all_triplets_computed": max_bonds <= cap,
    }


def onthefly_report(args):
    """The crystallisation run of Sec. 5.2 with Q4/Q5/Q6 every 1000 steps,
    shortened (defaults 5000 + 45000 steps instead of 50,000 + 500,000):
    125,000 particles on a cubic lattice at rho 0.8442."""
    import mdinputs
    from paper_1704_03329_amd.onthefly import crystallise

    d = mdinputs.lj_fluid(50, temperature=1.0, seed=7)
    n = d["pos"].shape[0]
    nve, nvt = args.otf_steps
    log(f"crystallisation run: N={n}, {nve} + {nvt} steps")
    out = crystallise(d["pos"], d["vel"], d["box"], nve_steps=nve, nvt_steps=nvt, boa_every=1000)
    tr = out["trace"]
    after_nve = [r for r in tr if r[0] == nve][0]
    steps = nve + nvt
    return {
        "workload": f"N={n} (50^3 cubic lattice, rho 0.8442, T*=1, seed 7), LJ rc 3.0, rc+delta 3.3, "
                    f"rebuild every 18 steps, dt 0.001; {nve} NVE steps then {nvt} steps with an Andersen "
                    "bath at T*=0.01 (10 collisions per unit time); Q4/Q5/Q6 (bonds within 1.5) every 1000 steps",
        "n_atoms": n,
        "atom_steps_per_s": n * steps / out["md_seconds"],
        "md_seconds": out["md_seconds"],
        "boa_ms_per_call": out["boa_seconds"] / len(tr) * 1e3,
        "with_analysis_atom_steps_per_s": n * steps / (out["md_seconds"] + out["boa_seconds"]),
        "mean_q4_q5_q6": {"start": list(tr[0][1:4]), "after_nve": list(after_nve[1:4]), "end": list(tr[-1][1:4])},
        "ke_per_atom_end": tr[-1][4],
    }


def lj32_forces(sim, x, y, z, out):
    from paper_1704_03329_amd import mdpl as C

    C.mdpl_forces(sim.handle, x, y, z, out[0], out[1], out[2], None, None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n-side", type=int, default=100)
    ap.add_argument("--premelt", type=int, default=1000,
                    help="untimed steps that melt the lattice before the warmup (0: start from the lattice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--no-analysis", action="store_true")
    ap.add_argument("--mlp-steps", type=int, default=6000)
    ap.add_argument("--no-onthefly", action="store_true",
                    help="skip the crystallisation run with on-the-fly bond order")
    ap.add_argument("--otf-steps", type=int, nargs=2, default=[5000, 45000], metavar=("NVE", "NVT"),
                    help="steps of the crystallisation run without and with the thermostat")
    ap.add_argument("--pairs", choices=["full", "half", "cells"], default="full",
                    help="pair loop of the timed run: full lists, half lists (Newton's third law) "
                         "or no list (the cell stencil every pass)")
    ap.add_argument("--rebuild", choices=["vmax", "fixed"], default="vmax",
                    help="list reuse: every 10 steps or earlier by the rule of Eq. extended_cutoff "
                         "(vmax), or every 10 steps only (fixed)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the run without per-launch events (no roofline line)")
    ap.add_argument("--no-pairs-compare", action="store_true",
                    help="skip the short runs of the other pair loops reported beside the main one")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one elementwise copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--flop-probe-m", type=int, default=0,
                    help="first run one elementwise FP32 and one FP64 product over this many "
                         "Mi elements (FLOP counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "domain decomposition is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import mdinputs
    from paper_1704_03329_amd import mdpl as C
    from paper_1704_03329_amd.sim import LJSim

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy probe: one elementwise kernel reading and writing {args.copy_probe_mib} MiB each")
        del src, dst
    if args.flop_probe_m:
        for dt in (torch.float32, torch.float64):
            a = torch.full((args.flop_probe_m << 20,), 1.5, dtype=dt, device=dev)
            b = torch.full_like(a, 0.75)
            torch.mul(a, b, out=a)
            torch.cuda.synchronize()
            del a, b
        log(f"flop probe: one FP32 and one FP64 product over {args.flop_probe_m} Mi elements each")
    n_side = args.n_side
    d = mdinputs.lj_fluid(n_side, temperature=1.0, seed=2)
    n = d["pos"].shape[0]
    box = d["box"]
    log(f"N={n} box={box[0]:.4f} building context")
    melted = {}  # the headline run's configuration after its timed steps (the CPU baseline's input)
    def timed_run(pairs, warmup, steps, precision="fp32"):
        sim = LJSim(n, box, rc=2.5, skin=0.3, dt=0.001, reuse_every=10, precision=precision, shift="cutoff",
                    max_nb=128, pairs=pairs, rebuild=args.rebuild)
        state = sim.new_state(torch.from_numpy(d["pos"]), torch.from_numpy(d["vel"]))
        torch.cuda.synchronize()
        pre = warmup + args.premelt
        log(f"pairs={pairs}: melting the lattice and warmup, {args.premelt} + {warmup} steps")
        # the lattice melts in the first premelt steps of the same run, which
        # then goes on with the warmup; its last step is sampled, so that the
        # timed run, which continues from its state (list, forces, rebuild
        # schedule), starts from its row
        sim.run(state, pre, max(pre, 1))
        torch.cuda.synchronize()
        st, flags, _ = sim.check(raise_on_error=False)
        if st != 0:
            raise SystemExit(f"warmup flagged status {st} flags {flags}")
        # events for the timed launches are created here, not in the run; an
        # event pair makes the stream wait for the kernel before it (about 7
        # us of step time per launch at this size), so one launch in
        # TIME_EVERY of each force kernel is timed
        C.mdpl_set_timing(sim.handle, not args.no_kernel_timing, reserve=steps // TIME_EVERY + 8,
                          every=TIME_EVERY)
        C.mdpl_kernel_time(sim.handle, 0)  # reset
        C.mdpl_kernel_time(sim.handle, 1)
        rb0 = sim.rebuild_stats()
        log(f"timing {steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        thermo = sim.run(state, steps, 10, cont=pre > 0)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        rb = [a - b for a, b in zip(sim.rebuild_stats(), rb0)]
        st, flags, _ = sim.check(raise_on_error=False)
        if st != 0:
            raise SystemExit(f"timed run flagged status {st} flags {flags}")
        f_ms, f_n = C.mdpl_kernel_time(sim.handle, 0)
        fe_ms, fe_n = C.mdpl_kernel_time(sim.handle, 1)
        C.mdpl_set_timing(sim.handle, False)
        entries = C.mdpl_nlist_entries(sim.handle) if pairs != "cells" else 0
        if not melted and not args.no_cpu_baseline:
            melted["pos"] = torch.stack([state["x"], state["y"], state["z"]], 1).cpu().numpy()
            melted["vel"] = torch.stack([state["vx"], state["vy"], state["vz"]], 1).cpu().numpy()
        log(f"elapsed {elapsed:.4f} s; force {f_ms / max(f_n, 1) * 1e3:.1f} us x {f_n}; "
            f"force+energy {fe_ms / max(fe_n, 1) * 1e3:.1f} us x {fe_n}; entries/atom {entries / n:.2f}; "
            f"rebuilds {rb[0]} (early {rb[1]}, host waits {rb[2]})")
        return dict(elapsed=elapsed, thermo=thermo.cpu().numpy(), f_ms=f_ms, f_n=f_n, fe_ms=fe_ms, fe_n=fe_n,
                    entries=entries, rebuilds=rb)

    r = timed_run(args.pairs, args.warmup, args.steps)
    elapsed, th, entries = r["elapsed"], r["thermo"], r["entries"]
    f_ms, f_n, fe_ms, fe_n = r["f_ms"], r["f_n"], r["fe_ms"], r["fe_n"]
    etot = th[:, 0] + th[:, 1]

    if args.pairs == "half":
        # the half-list force pass (timed with the clearing of the outputs): per
        # atom cnt (4) + own position (24, also the neighbour positions) + its
        # force (12, added by atomics); per list entry its 16-bit tile offset (2)
        alg_bytes = n * (4 + 24 + 12) + 2 * entries
    elif args.pairs == "cells":
        # the list-free pass: per atom its position (24, also the neighbour
        # positions) and its force (12)
        alg_bytes = n * (24 + 12)
    else:
        # algorithmic bytes of one plain force launch, which in the run also
        # applies the velocity-Verlet kick-kick-drift of the next step: per atom
        # cnt (4) + own position (24, also the neighbour positions, each read
        # once) + velocity read and written (48) + new position written (24);
        # per list entry its 16-bit tile offset (2)
        alg_bytes = n * (4 + 24 + 48 + 24) + 2 * entries
    avg_s = (f_ms / 1e3) / max(f_n, 1)
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else None
    traffic = measured_traffic() if args.pairs == "full" else None
    flops = measured_flops(avg_s, entries) if args.pairs == "full" and avg_s > 0 else None

    out = {
        "metric": METRIC,
        "value": n * args.steps / elapsed,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"LJ fluid N={n} ({n_side}^3 sc lattice, rho 0.8442, T*=1, seed 2, melted by "
                        f"{args.premelt} untimed steps), rc 2.5, "
                        "skin 0.3, rebuild every 10 steps, dt 0.001, FP32 pair forces, FP64 "
                        "positions/energy/virial, PE+virial every 10 steps",
            "neighbour_lists": {"full": "full (every ordered pair)",
                                "half": "half (each pair once, reactions by atomics)",
                                "cells": "none (each pass scans the 27-cell stencil)"}[args.pairs],
            "n_atoms": n,
            "nlist_entries_per_atom": entries / n,
            "precision": {
                "full": "FP32 separations from tile-centred FP32 coordinates, FP32 pair force and per-particle "
                        "sums, forces stored as FP32; the cutoff decided by the exact FP64 test within a band "
                        "around rc^2 (the definition's pair set); FP64 positions, velocities, and FP64 "
                        "separations, pair energies and virial on sampled steps",
                "half": "FP32 pair force factor, forces stored as FP32; FP64 positions, velocities, "
                        "separations, cutoff test, per-particle force sums, energy, virial",
                "cells": "FP32 pair force factor, forces stored as FP32; FP64 positions, velocities, "
                         "separations, cutoff test, per-particle force sums, energy, virial"}[args.pairs],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": {"full": "k_lj_force32_plain<float> (with the fused kick-kick-drift)",
                       "half": "k_lj_force_half<float,float,false,false> (with the clearing of the forces)",
                       "cells": "k_lj_force_cells<float,float,false>"}[args.pairs],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_us": avg_s * 1e6,
            "timed_launches": f_n,
            "timed_every": TIME_EVERY,
        },
        "flops": flops,
        # context only, another machine and precision: the paper's framework on
        # its N=10^6 LJ benchmark (FP64, skin 0.25, list rebuilt every 20
        # steps), 10^4 steps in 385 s on one GPU and 501 s on one CPU node
        # (Sec. 5.1, Tab. strong_table); atom-steps/s = N x steps / time
        "paper_context": [
            {"value": 1e6 * 1e4 / 385.0, "unit": "atom-steps/s", "hardware": "1x NVIDIA Tesla K20X",
             "dtype": "f64"},
            {"value": 1e6 * 1e4 / 501.0, "unit": "atom-steps/s",
             "hardware": "2x Intel Xeon E5-2650v2 (16 cores)", "dtype": "f64"},
        ],
        "kernels_us": {
            "force": avg_s * 1e6,
            "force_energy_virial": (fe_ms / max(fe_n, 1)) * 1e3,
        },
        "rebuilds": {"total": r["rebuilds"][0], "early_by_vmax_rule": r["rebuilds"][1],
                     "host_waits": r["rebuilds"][2],
                     "rule": "every 10 steps, or earlier once 2 sum dt v_max >= skin (Eq. extended_cutoff)"},
        "energy_drift_per_atom": float(np.max(np.abs(etot - etot[0])) / n),
        "hbm_gbs_force": achieved,
    }
    if args.pairs == "full" and not args.no_pairs_compare:
        # the same workload with the other pair loops, shorter runs
        hs = min(args.steps, 200)
        for pairs, key, note in (
                ("half", "half_lists", "force pass timed with the clearing of the outputs; the kicks run "
                                       "as their own pass"),
                ("cells", "cell_pair_loop", "no neighbour list: each force pass scans the 27-cell stencil; "
                                            "the kicks run as their own pass")):
            h = timed_run(pairs, min(args.warmup, 20), hs)
            out[key] = {
                "value": n * hs / h["elapsed"],
                "unit": "atom-steps/s",
                "steps": hs,
                "ms_per_step": h["elapsed"] / hs * 1e3,
                "force_us": h["f_ms"] / max(h["f_n"], 1) * 1e3,
                "force_energy_virial_us": h["fe_ms"] / max(h["fe_n"], 1) * 1e3,
                "nlist_entries_per_atom": h["entries"] / n,
                "note": note,
            }
    if args.pairs == "full" and not args.no_pairs_compare:
        # the paper's precision (FP64 pair forces), same workload, as context
        hs = min(args.steps, 200)
        h = timed_run("full", min(args.warmup, 20), hs, precision="fp64")
        out["fp64_forces"] = {
            "value": n * hs / h["elapsed"],
            "unit": "atom-steps/s",
            "steps": hs,
            "ms_per_step": h["elapsed"] / hs * 1e3,
            "force_us": h["f_ms"] / max(h["f_n"], 1) * 1e3,
            "force_energy_virial_us": h["fe_ms"] / max(h["fe_n"], 1) * 1e3,
            "note": "FP64 pair forces and sums (the paper's precision); everything else as the headline run",
        }
    if not args.no_mlp:
        out["mlp_vs_lj"] = mlp_report(args)
    if not args.no_analysis:
        out["analysis"] = analysis_report(not args.no_cpu_baseline)
    if not args.no_onthefly:
        out["on_the_fly"] = onthefly_report(args)
    if not args.no_cpu_baseline:
        log("oracle CPU baseline: one FP64 step of the whole system")
        out["cpu_baseline"] = cpu_baseline(melted["pos"], melted["vel"], box)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
