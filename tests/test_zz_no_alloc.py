"""mdpl_boa_noalloc (no caller workspace; the library's static scratch)
against mdpl_boa with a caller workspace, through the C ABI: identical
outputs on two calls in a row, the second with a smaller input, and the
scratch limit reported as MDPL_ESCRATCH before any device work."""
import numpy as np
import pytest
import torch

import mdinputs
from conftest import gpu_device, split_dev

pytestmark = pytest.mark.gpu


def _boa_both(pos, box, rc):
    from paper_1704_03329_amd import mdpl as C

    dev = gpu_device()
    x, y, z = split_dev(pos)
    n = pos.shape[0]
    out = {}
    for kind in ("ws", "noalloc"):
        q4 = torch.full((n,), -1.0, dtype=torch.float32, device=dev)
        q5 = torch.full_like(q4, -1.0)
        q6 = torch.full_like(q4, -1.0)
        nnb = torch.full((n,), -1, dtype=torch.int32, device=dev)
        if kind == "ws":
            ws = torch.empty(C.mdpl_analysis_workspace_bytes(n, box, rc, 1), dtype=torch.uint8, device=dev)
            C.mdpl_boa(x, y, z, box, rc, q4, q5, q6, nnb, ws)
        else:
            C.mdpl_boa_noalloc(x, y, z, box, rc, q4, q5, q6, nnb)
        torch.cuda.synchronize()
        out[kind] = (q4.cpu().numpy(), q5.cpu().numpy(), q6.cpu().numpy(), nnb.cpu().numpy())
    return out


def test_noalloc_matches_workspace_entry_point():
    print("no-alloc BOA: 20k-atom polycrystal, then 2k-atom jittered FCC", flush=True)
    pc = mdinputs.polycrystal(20_000, 6, seed=13)
    big = (pc["pos"], pc["box"], 1.2684 * pc["d"])
    d = 2.0 ** (1.0 / 6.0)
    a = d * np.sqrt(2.0)
    fpos, fbox = mdinputs.fcc_cells((8, 8, 8), a)
    small = (mdinputs.perturb(fpos, 0.03, 5), fbox, 1.2684 * d)
    assert small[0].shape[0] < big[0].shape[0]
    for pos, box, rc in (big, small):
        r = _boa_both(pos, box, rc)
        for k in range(4):
            assert np.array_equal(r["ws"][k], r["noalloc"][k]), k
        assert np.all(r["noalloc"][3] >= 0)


def test_noalloc_rejects_inputs_beyond_the_scratch():
    from paper_1704_03329_amd import mdpl as C

    dev = gpu_device()
    n = 4_000_000  # ~54 bytes per particle: beyond 64 MiB
    box = [160.0, 160.0, 160.0]
    assert C.mdpl_analysis_workspace_bytes(n, box, 1.42, 1) > C.MDPL_SCRATCH_BYTES
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    q = torch.empty(n, dtype=torch.float32, device=dev)
    nnb = torch.empty(n, dtype=torch.int32, device=dev)
    with pytest.raises(C.MdplError) as e:
        C.mdpl_boa_noalloc(x, x, x, box, 1.42, q, None, q, nnb)
    assert e.value.status == C.MDPL_ESCRATCH
