"""Helpers shared by the GPU tests: run the library on numpy inputs."""
from __future__ import annotations

import sys

import numpy as np


def announce(msg: str) -> None:
    """Print a progress line that reaches the terminal while the test runs,
    also under pytest's output capture (long GPU cases stay visibly alive)."""
    line = f"[gpu-case] {msg}"
    capman = None
    try:
        from tests import conftest
        if conftest.CONFIG is not None:
            capman = conftest.CONFIG.pluginmanager.getplugin("capturemanager")
    except Exception:
        capman = None
    if capman is not None:
        with capman.global_and_fixture_disabled():
            print(line, flush=True)
    else:
        print(line, flush=True)
    sys.stdout.flush()


def run_all(mats, prec="fp64"):
    """Library results for a list of numpy matrices: per-matrix (lam, mu, W, flag)."""
    import torch
    from paper_2002_04989_amd import eeid
    dev = [torch.from_numpy(np.ascontiguousarray(m)).to("cuda:0") for m in mats]
    lam, mu, V2, flags = eeid.all_components(dev, prec)
    torch.cuda.synchronize()
    n = [m.shape[0] for m in mats]
    lam = eeid.split(lam.cpu().numpy(), n, "lambda")
    mu = eeid.split(mu.cpu().numpy(), n, "mu")
    W = eeid.split(V2.cpu().numpy(), n, "V2")
    flags = flags.cpu().numpy()
    assert not np.any(flags & eeid.FLAG_WAIT_TIMEOUT), "a bounded wait gave up"
    return [(lam[b], mu[b], W[b], int(flags[b])) for b in range(len(mats))]


def norm2(a) -> float:
    return float(np.max(np.abs(np.linalg.eigvalsh(a))))
