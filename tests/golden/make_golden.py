"""Write the oracle's reference values for the large workloads (calls oracle/ only).

For each workload the oracle computes lambda(A), the spectra of a seeded
sample of minors M_j and the corresponding columns W[:, j] of Eq. (2).  The
full-size GPU tests compare the library against these on the same seeded
inputs (regenerated from paper_2002_04989_amd.inputs, which is deterministic).

    python tests/golden/make_golden.py goe2048 clustered2048 [gue4096]

Output: tests/golden/<name>.npz (arrays js, lam, mu, W) and <name>.json
(method, wall seconds, threads, host CPU).  Nothing here touches the GPU.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2002_04989_amd import inputs  # noqa: E402


def sample_js(n: int, seed: int, extra: int) -> list:
    base = [0, 1, n // 2, n - 1]
    rest = np.random.default_rng(seed).choice(np.arange(2, n - 1), size=extra, replace=False)
    return sorted(set(base) | set(int(j) for j in rest))


WORKLOADS = {
    "goe2048": lambda: (inputs.goe(2048, 4), sample_js(2048, 4040, 4), "jacobi"),
    "clustered2048": lambda: (inputs.clustered(2048, 16, 1e-6, 40)[0], sample_js(2048, 4041, 4), "jacobi"),
    "gue4096": lambda: (inputs.gue(4096, 5), [0, 4095], "jacobi"),
}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def make(name: str) -> None:
    A, js, method = WORKLOADS[name]()
    threads = oracle.default_threads()
    t0 = time.time()
    # lambda(A) and the sampled minors run concurrently (one eigenvalue problem per thread)
    Ah = oracle.hermitian_from_lower(A)
    with ThreadPoolExecutor(min(threads, len(js) + 1)) as ex:
        f_lam = ex.submit(oracle.eigvalsh, Ah, method)
        f_mu = [ex.submit(oracle.eigvalsh, oracle.minor(Ah, j), method) for j in js]
        lam = f_lam.result()
        mu = np.array([f.result() for f in f_mu])
    W, flags = oracle.identity_from_spectra(lam, mu)
    dt = time.time() - t0
    np.savez(os.path.join(HERE, f"{name}.npz"), js=np.array(js, dtype=np.int64), lam=lam, mu=mu, W=W,
             flags=np.array([flags], dtype=np.int32))
    meta = dict(workload=name, n=int(A.shape[0]), js=js, method=method, seconds=round(dt, 1),
                threads=threads, cpu=cpu_model(), note="lambda(A) and len(js) minors, computed concurrently")
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(f"{name}: {dt:.1f} s with {threads} threads, js={js}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["goe2048", "clustered2048"]:
        make(name)
