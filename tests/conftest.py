import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


def gpu_device():
    """The CUDA device for -m gpu tests; fails loudly if absent."""
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import numpy as np
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(gpu_device())


def split_dev(pos):
    """(N,3) numpy float64 -> three contiguous float64 device columns."""
    return tuple(to_dev(pos[:, k].copy()) for k in range(3))


def force_errors(f_got, f_ref):
    """(global relative L2 error, max per-atom error / max per-atom norm)."""
    import numpy as np

    d = np.asarray(f_got, dtype=np.float64) - np.asarray(f_ref, dtype=np.float64)
    g = np.linalg.norm(d) / max(np.linalg.norm(f_ref), 1e-300)
    m = np.max(np.linalg.norm(d, axis=1)) / max(np.max(np.linalg.norm(f_ref, axis=1)), 1e-300)
    return g, m
