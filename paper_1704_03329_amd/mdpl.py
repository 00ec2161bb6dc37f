"""ctypes binding of libmdpl (include/mdpl.h): argument marshalling only.

Every function here has the name of the C entry point it calls, takes torch
tensors (device memory) or plain Python values, checks shapes/dtypes,
passes raw pointers and the current HIP stream, and raises MdplError on a
non-zero status.  All computation happens in the HIP library; if it is not
built, importing works but the first call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdpl.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "mdpl.h")

MDPL_OK, MDPL_EINVAL, MDPL_EBOX, MDPL_ECAPACITY, MDPL_ESKIN = 0, 1, 2, 3, 4
MDPL_ENONFINITE, MDPL_EHIP, MDPL_ESTATE, MDPL_EWORKSPACE = 5, 6, 7, 8
MDPL_ESCRATCH = 9
MDPL_SCRATCH_BYTES = 64 << 20
FLAG_NL_OVERFLOW, FLAG_SKIN, FLAG_NONFINITE = 1, 2, 4
SHIFTS = {"none": 0, "paper": 1, "cutoff": 2}
PRECISIONS = {"fp64": 0, "fp32": 1}
PAIRS = {"full": 0, "half": 1, "cells": 2}
REBUILD = {"fixed": 0, "vmax": 1}
RUN_SETUP, RUN_CONTINUE = 0, 1


class MdplError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().mdpl_status_string(status).decode() if _lib is not None else str(status)
        extra = ""
        if status == MDPL_EHIP and _lib is not None:
            extra = f" (hipError {_lib.mdpl_last_hip_error()})"
        super().__init__(f"{where}: {msg}{extra} [status {status}]")


class mdpl_lj_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("box", ctypes.c_double * 3),
        ("rc", ctypes.c_double),
        ("skin", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("reuse_every", ctypes.c_int32),
        ("shift", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_nb", ctypes.c_int32),
        ("pairs", ctypes.c_int32),
        ("rebuild", ctypes.c_int32),
    ]


_lib = None
_P = ctypes.c_void_p
_I32, _I64, _D, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t

_SIGS = {
    "mdpl_status_string": ([_I32], ctypes.c_char_p),
    "mdpl_last_hip_error": ([], _I32),
    "mdpl_workspace_bytes": ([ctypes.POINTER(mdpl_lj_params), ctypes.POINTER(_SZ)], _I32),
    "mdpl_sim_create": ([ctypes.POINTER(mdpl_lj_params), _P, _SZ, _P, ctypes.POINTER(_P)], _I32),
    "mdpl_sim_destroy": ([_P], _I32),
    "mdpl_build": ([_P, _P, _P, _P], _I32),
    "mdpl_nlist_export": ([_P, _P, _P, _I64, ctypes.POINTER(_I64)], _I32),
    "mdpl_nlist_entries": ([_P, ctypes.POINTER(_I64)], _I32),
    "mdpl_forces": ([_P, _P, _P, _P, _P, _P, _P, _P, _P], _I32),
    "mdpl_lj_backward": ([_P, _P, _P, _P, _P, _P, _P, _P], _I32),
    "mdpl_run": ([_P] + [_P] * 10 + [_I64, _I32, _P, _I32], _I32),
    "mdpl_run_andersen": ([_P] + [_P] * 10 + [_I64, _I32, _P, _D, _D, ctypes.c_uint64, _I64, _I32], _I32),
    "mdpl_rebuild_stats": ([_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)], _I32),
    "mdpl_check": ([_P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_I32)], _I32),
    "mdpl_clear_flags": ([_P], _I32),
    "mdpl_set_timing": ([_P, _I32, _I32], _I32),
    "mdpl_kernel_time": ([_P, _I32, ctypes.POINTER(_D), ctypes.POINTER(_I64)], _I32),
    "mdpl_analysis_workspace_bytes": ([_I64, ctypes.POINTER(_D), _D, _I32, ctypes.POINTER(_SZ)], _I32),
    "mdpl_boa": ([_P, _P, _P, _I64, ctypes.POINTER(_D), _D, _P, _P, _P, _P, _P, _SZ, _P], _I32),
    "mdpl_boa_noalloc": ([_P, _P, _P, _I64, ctypes.POINTER(_D), _D, _P, _P, _P, _P, _P], _I32),
    "mdpl_cna": ([_P, _P, _P, _I64, ctypes.POINTER(_D), _D, _I32, _P, _P, _P, _P, _P, _SZ, _P], _I32),
}


def lib():
    """Load libmdpl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_1704_03329_amd.build` "
                "(there is no fallback implementation)"
            )
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def header_symbols() -> list:
    """Names of the entry points declared in include/mdpl.h."""
    with open(HEADER_PATH) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(mdpl_[a-z0-9_]+)\s*\(", txt)))


def _check(status: int, where: str):
    if status != MDPL_OK:
        raise MdplError(status, where)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _dev(t: torch.Tensor, dtype, n=None, name="array"):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor of dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, need {n}")
    return t.data_ptr()


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def make_params(n, box, rc=2.5, skin=0.3, eps=1.0, sigma=1.0, mass=1.0, dt=0.001, reuse_every=10,
                shift="none", precision="fp32", max_nb=128, pairs="full", rebuild="vmax") -> mdpl_lj_params:
    p = mdpl_lj_params()
    p.n = int(n)
    for k in range(3):
        p.box[k] = float(box[k])
    p.rc, p.skin, p.eps, p.sigma, p.mass, p.dt = map(float, (rc, skin, eps, sigma, mass, dt))
    p.reuse_every = int(reuse_every)
    p.shift = SHIFTS[shift] if isinstance(shift, str) else int(shift)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.max_nb = int(max_nb)
    p.pairs = PAIRS[pairs] if isinstance(pairs, str) else int(pairs)
    p.rebuild = REBUILD[rebuild] if isinstance(rebuild, str) else int(rebuild)
    return p


# ------------------------------------------------------------ entry points
def mdpl_workspace_bytes(params: mdpl_lj_params) -> int:
    out = _SZ(0)
    _check(lib().mdpl_workspace_bytes(ctypes.byref(params), ctypes.byref(out)), "mdpl_workspace_bytes")
    return int(out.value)


def mdpl_sim_create(params: mdpl_lj_params, workspace: torch.Tensor, stream=None) -> int:
    h = _P(0)
    _check(
        lib().mdpl_sim_create(ctypes.byref(params), _dev(workspace, torch.uint8), workspace.numel(),
                              _stream(stream), ctypes.byref(h)),
        "mdpl_sim_create",
    )
    return h.value


def mdpl_sim_destroy(sim: int):
    _check(lib().mdpl_sim_destroy(sim), "mdpl_sim_destroy")


def mdpl_build(sim: int, x, y, z):
    _check(lib().mdpl_build(sim, _ptr(x), _ptr(y), _ptr(z)), "mdpl_build")


def mdpl_nlist_export(sim: int, i_out, j_out, cap: int) -> int:
    cnt = _I64(0)
    _check(lib().mdpl_nlist_export(sim, _ptr(i_out), _ptr(j_out), int(cap), ctypes.byref(cnt)),
           "mdpl_nlist_export")
    return int(cnt.value)


def mdpl_nlist_entries(sim: int) -> int:
    cnt = _I64(0)
    _check(lib().mdpl_nlist_entries(sim, ctypes.byref(cnt)), "mdpl_nlist_entries")
    return int(cnt.value)


def mdpl_forces(sim: int, x, y, z, fx, fy, fz, pe_w=None, e_atom=None):
    _check(lib().mdpl_forces(sim, _ptr(x), _ptr(y), _ptr(z), _ptr(fx), _ptr(fy), _ptr(fz), _ptr(pe_w),
                             _ptr(e_atom)), "mdpl_forces")


def mdpl_lj_backward(sim: int, x, y, z, grad_e, gx, gy, gz):
    _check(lib().mdpl_lj_backward(sim, _ptr(x), _ptr(y), _ptr(z), _ptr(grad_e), _ptr(gx), _ptr(gy),
                                  _ptr(gz)), "mdpl_lj_backward")


def mdpl_run(sim: int, x, y, z, vx, vy, vz, fx, fy, fz, ids, nsteps: int, sample_every: int = 0,
             thermo=None, start: int = RUN_SETUP):
    _check(lib().mdpl_run(sim, _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(fx),
                          _ptr(fy), _ptr(fz), _ptr(ids), int(nsteps), int(sample_every), _ptr(thermo),
                          int(start)),
           "mdpl_run")


def mdpl_run_andersen(sim: int, x, y, z, vx, vy, vz, fx, fy, fz, ids, nsteps: int, sample_every: int,
                      thermo, temperature: float, collision_rate: float, seed: int, step0: int = 0,
                      start: int = RUN_SETUP):
    _check(lib().mdpl_run_andersen(sim, _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(fx),
                                   _ptr(fy), _ptr(fz), _ptr(ids), int(nsteps), int(sample_every),
                                   _ptr(thermo), float(temperature), float(collision_rate),
                                   int(seed) & ((1 << 64) - 1), int(step0), int(start)), "mdpl_run_andersen")


def mdpl_rebuild_stats(sim: int):
    """Returns (rebuilds, early rebuilds of the VMAX rule, host waits for the stream)."""
    a, b, c = _I64(0), _I64(0), _I64(0)
    _check(lib().mdpl_rebuild_stats(sim, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "mdpl_rebuild_stats")
    return int(a.value), int(b.value), int(c.value)


def mdpl_check(sim: int, raise_on_error: bool = False):
    """Returns (status, flags, max_count)."""
    f = ctypes.c_uint32(0)
    m = _I32(0)
    st = lib().mdpl_check(sim, ctypes.byref(f), ctypes.byref(m))
    if raise_on_error:
        _check(st, "mdpl_check")
    return int(st), int(f.value), int(m.value)


def mdpl_clear_flags(sim: int):
    _check(lib().mdpl_clear_flags(sim), "mdpl_clear_flags")


def mdpl_set_timing(sim: int, on, reserve: int = 0, every: int = 1):
    """on: bool; reserve: launches to create events for up front (none are
    then created while a timed run is enqueued); every: time launches 0,
    every, 2 every, ... of each force kernel."""
    _check(lib().mdpl_set_timing(sim, (max(int(reserve), 2) if reserve else 1) if on else 0, int(every)),
           "mdpl_set_timing")


def mdpl_kernel_time(sim: int, which: int):
    ms = _D(0.0)
    k = _I64(0)
    _check(lib().mdpl_kernel_time(sim, int(which), ctypes.byref(ms), ctypes.byref(k)), "mdpl_kernel_time")
    return float(ms.value), int(k.value)


def mdpl_analysis_workspace_bytes(n: int, box, rc: float, max_nb: int) -> int:
    b = (_D * 3)(*[float(v) for v in box])
    out = _SZ(0)
    _check(lib().mdpl_analysis_workspace_bytes(int(n), b, float(rc), int(max_nb), ctypes.byref(out)),
           "mdpl_analysis_workspace_bytes")
    return int(out.value)


def mdpl_boa(x, y, z, box, rc, q4, q5, q6, nnb, workspace, stream=None):
    n = x.numel()
    b = (_D * 3)(*[float(v) for v in box])
    _check(lib().mdpl_boa(_ptr(x), _ptr(y), _ptr(z), n, b, float(rc), _ptr(q4), _ptr(q5), _ptr(q6),
                          _ptr(nnb), _dev(workspace, torch.uint8), workspace.numel(), _stream(stream)),
           "mdpl_boa")


def mdpl_boa_noalloc(x, y, z, box, rc, q4, q5, q6, nnb, stream=None):
    n = x.numel()
    b = (_D * 3)(*[float(v) for v in box])
    _check(lib().mdpl_boa_noalloc(_ptr(x), _ptr(y), _ptr(z), n, b, float(rc), _ptr(q4), _ptr(q5), _ptr(q6),
                                  _ptr(nnb), _stream(stream)), "mdpl_boa_noalloc")


def mdpl_cna(x, y, z, box, rc, max_nb, trip, nnb, label, workspace, max_count=None, stream=None):
    n = x.numel()
    b = (_D * 3)(*[float(v) for v in box])
    _check(lib().mdpl_cna(_ptr(x), _ptr(y), _ptr(z), n, b, float(rc), int(max_nb), _ptr(trip), _ptr(nnb),
                          _ptr(label), _ptr(max_count), _dev(workspace, torch.uint8), workspace.numel(),
                          _stream(stream)),
           "mdpl_cna")


# ------------------------------------------------------- learned potential
def _handle(sim):
    return sim.handle if hasattr(sim, "handle") else sim


class mdpl_mlp_weights(ctypes.Structure):
    _fields_ = [("w1", ctypes.c_void_p), ("b1", ctypes.c_void_p), ("w2", ctypes.c_void_p),
                ("b2", ctypes.c_void_p), ("w3", ctypes.c_void_p), ("b3", ctypes.c_void_p),
                ("mu", ctypes.c_void_p), ("sd", ctypes.c_void_p), ("e_mean", ctypes.c_float),
                ("e_sd", ctypes.c_float)]


_SIGS_MLP = {
    "mdpl_desc_fwd": ([ctypes.c_void_p] * 6, ctypes.c_int32),
    "mdpl_desc_bwd": ([ctypes.c_void_p] * 9, ctypes.c_int32),
    "mdpl_mlp_fwd": ([ctypes.POINTER(mdpl_mlp_weights), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int32),
    "mdpl_mlp_train_floats": ([ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mdpl_mlp_train_grad": ([ctypes.POINTER(mdpl_mlp_weights), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
                            ctypes.c_int32),
    "mdpl_adam_step": ([ctypes.c_void_p] * 4 + [ctypes.c_float] * 4 + [ctypes.c_int32] + [ctypes.c_void_p] * 4,
                       ctypes.c_int32),
    "mdpl_mlp_standardise": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64] + [ctypes.c_void_p] * 5,
                             ctypes.c_int32),
    "mdpl_mlp_bf16": ([ctypes.c_void_p] * 5, ctypes.c_int32),
    "mdpl_scale_velocities": ([ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_double, ctypes.c_void_p],
                              ctypes.c_int32),
    "mdpl_mlp_run_floats": ([ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mdpl_mlp_forces": ([ctypes.c_void_p, ctypes.POINTER(mdpl_mlp_weights)] + [ctypes.c_void_p] * 4
                        + [ctypes.c_int64] + [ctypes.c_void_p] * 4, ctypes.c_int32),
    "mdpl_run_mlp": ([ctypes.c_void_p, ctypes.POINTER(mdpl_mlp_weights), ctypes.c_void_p, ctypes.c_int64]
                     + [ctypes.c_void_p] * 10 + [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32],
                     ctypes.c_int32),
    "mdpl_force_error": ([ctypes.c_void_p] * 8, ctypes.c_int32),
}
_SIGS.update(_SIGS_MLP)


# ------------------------------------------------------------ entry points
def mdpl_desc_fwd(sim, x, y, z, G, mom=None):
    _check(lib().mdpl_desc_fwd(_handle(sim), _ptr(x), _ptr(y), _ptr(z), _ptr(G), _ptr(mom)), "mdpl_desc_fwd")


def mdpl_desc_bwd(sim, x, y, z, dEdG, mom, fx, fy, fz):
    _check(lib().mdpl_desc_bwd(_handle(sim), _ptr(x), _ptr(y), _ptr(z), _ptr(dEdG), _ptr(mom), _ptr(fx), _ptr(fy),
                               _ptr(fz)), "mdpl_desc_bwd")


def mdpl_mlp_fwd(w: mdpl_mlp_weights, G, n, energy=None, dEdG=None):
    _check(lib().mdpl_mlp_fwd(ctypes.byref(w), _ptr(G), int(n), _ptr(energy), _ptr(dEdG), _stream()), "mdpl_mlp_fwd")


def mdpl_mlp_train_floats(batch: int) -> int:
    out = ctypes.c_int64(0)
    _check(lib().mdpl_mlp_train_floats(int(batch), ctypes.byref(out)), "mdpl_mlp_train_floats")
    return int(out.value)


def mdpl_mlp_train_grad(w, G, index, batch, energy, scratch, grad):
    """energy: per-atom FP64 energies (the library standardises them)."""
    if energy.dtype != torch.float64:
        raise TypeError("energy must be float64")
    _check(lib().mdpl_mlp_train_grad(ctypes.byref(w), _ptr(G), _ptr(index), int(batch), _ptr(energy), _ptr(scratch),
                                        scratch.numel(), _ptr(grad), _stream()), "mdpl_mlp_train_grad")


MDPL_MLP_STD_SCRATCH = 256 * 25 + 50


def mdpl_mlp_standardise(G, e, mu, sd, e_stats, scratch):
    if e.dtype != torch.float64 or e_stats.dtype != torch.float64 or scratch.dtype != torch.float64:
        raise TypeError("e, e_stats and scratch must be float64")
    if scratch.numel() < MDPL_MLP_STD_SCRATCH:
        raise ValueError("scratch needs MDPL_MLP_STD_SCRATCH doubles")
    _check(lib().mdpl_mlp_standardise(_ptr(G), _ptr(e), int(G.shape[0]), _ptr(mu), _ptr(sd), _ptr(e_stats),
                                      _ptr(scratch), _stream()), "mdpl_mlp_standardise")


def mdpl_mlp_bf16(params, w1, w2, w3):
    _check(lib().mdpl_mlp_bf16(_ptr(params), _ptr(w1), _ptr(w2), _ptr(w3), _stream()), "mdpl_mlp_bf16")


def mdpl_adam_step(params, grad, m, v, lr, b1, b2, eps, step, w1, w2, w3):
    _check(lib().mdpl_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), float(lr), float(b1), float(b2), float(eps),
                                   int(step), _ptr(w1), _ptr(w2), _ptr(w3), _stream()), "mdpl_adam_step")


def mdpl_scale_velocities(vx, vy, vz, factor):
    _check(lib().mdpl_scale_velocities(_ptr(vx), _ptr(vy), _ptr(vz), vx.numel(), float(factor), _stream()),
             "mdpl_scale_velocities")


def mdpl_mlp_run_floats(n: int) -> int:
    out = ctypes.c_int64(0)
    _check(lib().mdpl_mlp_run_floats(int(n), ctypes.byref(out)), "mdpl_mlp_run_floats")
    return int(out.value)


def mdpl_mlp_forces(sim, w: mdpl_mlp_weights, x, y, z, ws, energy, fx, fy, fz):
    _check(lib().mdpl_mlp_forces(_handle(sim), ctypes.byref(w), _ptr(x), _ptr(y), _ptr(z), _ptr(ws), ws.numel(),
                                 _ptr(energy), _ptr(fx), _ptr(fy), _ptr(fz)), "mdpl_mlp_forces")


def mdpl_run_mlp(sim, w: mdpl_mlp_weights, ws, state: dict, nsteps: int, sample_every: int, thermo=None,
                 start: int = RUN_SETUP):
    _check(lib().mdpl_run_mlp(_handle(sim), ctypes.byref(w), _ptr(ws), ws.numel(),
                              *[_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "ids")],
                              int(nsteps), int(sample_every), _ptr(thermo), int(start)), "mdpl_run_mlp")


def mdpl_force_error(sim, fx, fy, fz, gx, gy, gz, out):
    _check(lib().mdpl_force_error(_handle(sim), _ptr(fx), _ptr(fy), _ptr(fz), _ptr(gx), _ptr(gy), _ptr(gz),
                                  _ptr(out)), "mdpl_force_error")
