"""CPU-only checks of the C ABI: the library loads, exports every entry point
declared in include/mdpl.h, and rejects bad arguments on the host before any
device work (no GPU is touched here)."""
import ctypes
import os

import pytest

from paper_1704_03329_amd import mdpl as C


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(C.LIB_PATH):
        from paper_1704_03329_amd.build import build

        build()
    return C.lib()


def test_exports_every_declared_symbol(lib):
    names = C.header_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # the binding covers the same entry points
    assert set(C._SIGS) == set(names)


def test_status_strings(lib):
    for s in range(0, 9):
        assert lib.mdpl_status_string(s)
    assert b"invalid" in lib.mdpl_status_string(C.MDPL_EINVAL)


def _params(**kw):
    base = dict(n=1000, box=[10.58] * 3)
    base.update(kw)
    n, box = base.pop("n"), base.pop("box")
    return C.make_params(n, box, **base)


@pytest.mark.parametrize(
    "kw,status",
    [
        (dict(n=0), C.MDPL_EINVAL),
        (dict(n=-5), C.MDPL_EINVAL),
        (dict(n=(1 << 26) + 1), C.MDPL_EINVAL),
        (dict(box=[10.58, 0.0, 10.58]), C.MDPL_EINVAL),
        (dict(box=[10.58, float("nan"), 10.58]), C.MDPL_EINVAL),
        (dict(rc=0.0), C.MDPL_EINVAL),
        (dict(skin=-0.1), C.MDPL_EINVAL),
        (dict(dt=0.0), C.MDPL_EINVAL),
        (dict(mass=-1.0), C.MDPL_EINVAL),
        (dict(reuse_every=0), C.MDPL_EINVAL),
        (dict(shift=3), C.MDPL_EINVAL),
        (dict(precision=2), C.MDPL_EINVAL),
        (dict(max_nb=0), C.MDPL_EINVAL),
        (dict(box=[8.3, 10.58, 10.58]), C.MDPL_EBOX),   # 8.3 < 3 * 2.8
        (dict(rc=3.4), C.MDPL_EBOX),
    ],
)
def test_workspace_bytes_validation(lib, kw, status):
    p = _params(**kw)
    out = ctypes.c_size_t(0)
    assert lib.mdpl_workspace_bytes(ctypes.byref(p), ctypes.byref(out)) == status
    # creation validates the same way before touching the device
    h = ctypes.c_void_p(0)
    assert lib.mdpl_sim_create(ctypes.byref(p), ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(h)) == status
    assert not h.value


def test_pairs_mode_validated(lib):
    out = ctypes.c_size_t(0)
    for v, status in ((0, C.MDPL_OK), (1, C.MDPL_OK), (2, C.MDPL_OK), (3, C.MDPL_EINVAL), (-1, C.MDPL_EINVAL)):
        p = _params()
        p.pairs = v
        assert lib.mdpl_workspace_bytes(ctypes.byref(p), ctypes.byref(out)) == status
    # the other pair modes need no more workspace than full lists
    full = C.mdpl_workspace_bytes(_params())
    assert C.mdpl_workspace_bytes(_params(pairs="half")) == full
    assert C.mdpl_workspace_bytes(_params(pairs="cells")) == full


def test_workspace_bytes_size(lib):
    p = _params(max_nb=128)
    b = C.mdpl_workspace_bytes(p)
    npad = 1024
    # 16-bit neighbour entries plus ~15 doubles of per-particle state
    assert b >= 2 * 128 * npad + 8 * 1000 * 15
    assert b < 2 * 128 * npad + 8 * 1000 * 40 + (1 << 16)
    assert C.mdpl_workspace_bytes(_params(max_nb=256)) - b == 2 * 128 * npad


def test_misaligned_workspace_rejected(lib):
    p = _params()
    h = ctypes.c_void_p(0)
    assert lib.mdpl_sim_create(ctypes.byref(p), ctypes.c_void_p(4096 + 8), 1 << 40, None,
                               ctypes.byref(h)) == C.MDPL_EWORKSPACE


def test_null_handles_rejected(lib):
    assert lib.mdpl_sim_destroy(None) == C.MDPL_EINVAL
    assert lib.mdpl_build(None, None, None, None) == C.MDPL_EINVAL
    assert lib.mdpl_run(None, *([None] * 10), 10, 0, None, 0) == C.MDPL_EINVAL
    assert lib.mdpl_rebuild_stats(None, None, None, None) == C.MDPL_EINVAL
    assert lib.mdpl_check(None, None, None) == C.MDPL_EINVAL
    assert lib.mdpl_forces(None, *([None] * 8)) == C.MDPL_EINVAL


def test_analysis_validation(lib):
    box = (ctypes.c_double * 3)(20.0, 20.0, 20.0)
    out = ctypes.c_size_t(0)
    assert lib.mdpl_analysis_workspace_bytes(1000, box, 1.5, 32, ctypes.byref(out)) == 0
    assert out.value > 1000 * 32 * 4
    assert lib.mdpl_analysis_workspace_bytes(1000, box, 7.0, 32, ctypes.byref(out)) == C.MDPL_EBOX
    assert lib.mdpl_analysis_workspace_bytes(0, box, 1.5, 32, ctypes.byref(out)) == C.MDPL_EINVAL
    assert lib.mdpl_analysis_workspace_bytes(1000, box, -1.0, 32, ctypes.byref(out)) == C.MDPL_EINVAL
    # CNA capacity limit is checked before any device work
    assert lib.mdpl_cna(None, None, None, 10, box, 1.5, 65, None, None, None, None, None, 0, None) == C.MDPL_EINVAL
