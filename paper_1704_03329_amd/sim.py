"""Convenience wrappers over the C ABI: they allocate the caller-owned
device tensors (workspace, SoA arrays, outputs) with torch and call the
entry points of ``mdpl``.  No arithmetic of the method happens here."""
from __future__ import annotations

import torch

from . import mdpl as C


def soa(pos: torch.Tensor):
    """Split an (N,3) float64 CUDA tensor into three contiguous columns."""
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("positions must have shape (N, 3)")
    pos = pos.to(torch.float64)
    return pos[:, 0].contiguous(), pos[:, 1].contiguous(), pos[:, 2].contiguous()


class LJSim:
    """A Lennard-Jones simulation context (mdpl_sim) with its workspace."""

    def __init__(self, n, box, rc=2.5, skin=0.3, eps=1.0, sigma=1.0, mass=1.0, dt=0.001, reuse_every=10,
                 shift="none", precision="fp32", max_nb=128, pairs="full", rebuild="vmax", device="cuda",
                 stream=None):
        self.params = C.make_params(n, box, rc, skin, eps, sigma, mass, dt, reuse_every, shift, precision,
                                    max_nb, pairs, rebuild)
        self.n = int(n)
        self.box = [float(b) for b in box]
        self.device = torch.device(device)
        self.fdtype = torch.float32 if self.params.precision == 1 else torch.float64
        nbytes = C.mdpl_workspace_bytes(self.params)
        # 256-byte alignment: torch's caching allocator returns such blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream
        self.handle = C.mdpl_sim_create(self.params, self.workspace, stream)

    def close(self):
        if self.handle:
            C.mdpl_sim_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- pair loops
    def build(self, x, y, z):
        C.mdpl_build(self.handle, x, y, z)

    def forces(self, x, y, z, energy=False, per_atom=False):
        """Returns (fx, fy, fz, pe_w or None, e_atom or None)."""
        n = self.n
        f = [torch.empty(n, dtype=self.fdtype, device=self.device) for _ in range(3)]
        pe_w = torch.empty(2, dtype=torch.float64, device=self.device) if energy else None
        e = torch.empty(n, dtype=torch.float64, device=self.device) if per_atom else None
        C.mdpl_forces(self.handle, x, y, z, f[0], f[1], f[2], pe_w, e)
        return f[0], f[1], f[2], pe_w, e

    def backward(self, x, y, z, grad_e):
        g = [torch.empty(self.n, dtype=torch.float64, device=self.device) for _ in range(3)]
        C.mdpl_lj_backward(self.handle, x, y, z, grad_e, g[0], g[1], g[2])
        return g

    def pairs(self):
        """Directed pairs of the last build in caller indices, as an (P,2) int64 CPU tensor."""
        total = C.mdpl_nlist_export(self.handle, None, None, 0)
        i = torch.empty(max(total, 1), dtype=torch.int32, device=self.device)
        j = torch.empty(max(total, 1), dtype=torch.int32, device=self.device)
        C.mdpl_nlist_export(self.handle, i, j, total)
        return torch.stack([i[:total].long(), j[:total].long()], dim=1).cpu()

    def new_state(self, pos, vel):
        """Allocate the ten SoA state arrays from (N,3) position/velocity tensors."""
        x, y, z = soa(pos.to(self.device))
        vx, vy, vz = soa(vel.to(self.device))
        f = [torch.zeros(self.n, dtype=self.fdtype, device=self.device) for _ in range(3)]
        ids = torch.arange(self.n, dtype=torch.int32, device=self.device)
        return {"x": x, "y": y, "z": z, "vx": vx, "vy": vy, "vz": vz, "fx": f[0], "fy": f[1], "fz": f[2],
                "ids": ids}

    def run(self, state, nsteps, sample_every=0, andersen=None, cont=False):
        """nsteps of velocity Verlet; andersen: optional dict(temperature,
        collision_rate, seed, step0) for mdpl_run_andersen; cont: continue
        from the state the last run left in these arrays (MDPL_RUN_CONTINUE)."""
        thermo = None
        if sample_every:
            thermo = torch.zeros((nsteps // sample_every + 1, 4), dtype=torch.float64, device=self.device)
        s = state
        args = (self.handle, s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["fx"], s["fy"], s["fz"],
                s["ids"], nsteps, sample_every, thermo)
        start = C.RUN_CONTINUE if cont else C.RUN_SETUP
        if andersen is None:
            C.mdpl_run(*args, start=start)
        else:
            C.mdpl_run_andersen(*args, andersen["temperature"], andersen["collision_rate"], andersen["seed"],
                                andersen.get("step0", 0), start=start)
        return thermo

    def rebuild_stats(self):
        """(rebuilds, early rebuilds of the VMAX rule, host waits for the stream)."""
        return C.mdpl_rebuild_stats(self.handle)

    def check(self, raise_on_error=True):
        return C.mdpl_check(self.handle, raise_on_error)


def boa(x, y, z, box, rc, q5=False):
    """Bond-order parameters: dict(q4, q5?, q6, nnb) as CUDA tensors."""
    n = x.numel()
    dev = x.device
    ws = torch.empty(C.mdpl_analysis_workspace_bytes(n, box, rc, 1), dtype=torch.uint8, device=dev)
    out = {
        "q4": torch.empty(n, dtype=torch.float32, device=dev),
        "q6": torch.empty(n, dtype=torch.float32, device=dev),
        "nnb": torch.empty(n, dtype=torch.int32, device=dev),
    }
    out["q5"] = torch.empty(n, dtype=torch.float32, device=dev) if q5 else None
    C.mdpl_boa(x, y, z, box, rc, out["q4"], out["q5"], out["q6"], out["nnb"], ws)
    return out


def cna(x, y, z, box, rc, max_nb=32):
    """Common-neighbour analysis: dict(trip (N,max_nb) int32 codes, nnb, label,
    max_count (device int32 scalar: the largest bond count; particles with
    more than max_nb bonds have no triplets))."""
    n = x.numel()
    dev = x.device
    ws = torch.empty(C.mdpl_analysis_workspace_bytes(n, box, rc, max_nb), dtype=torch.uint8, device=dev)
    trip = torch.zeros((n, max_nb), dtype=torch.int32, device=dev)
    nnb = torch.empty(n, dtype=torch.int32, device=dev)
    label = torch.empty(n, dtype=torch.uint8, device=dev)
    most = torch.zeros(1, dtype=torch.int32, device=dev)
    C.mdpl_cna(x, y, z, box, rc, max_nb, trip, nnb, label, ws, most)
    return {"trip": trip, "nnb": nnb, "label": label, "max_count": most}


def unpack_triplets(codes):
    """Packed codes -> (n_cn, n_b, n_lcb) tuples (host side decoding)."""
    out = []
    for c in codes:
        c = int(c)
        out.append(((c >> 20) & 1023, (c >> 10) & 1023, c & 1023))
    return out
