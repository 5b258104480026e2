"""Write the oracle's reference values for the large workloads (calls oracle/ only).

For each workload the oracle computes lambda(A), the spectra of a seeded
sample of minors M_j and the corresponding columns W[:, j] of Eq. (2).  The
full-size GPU tests compare the library against these on the same seeded
inputs (regenerated from paper_2002_04989_amd.inputs, which is deterministic).

    python tests/golden/make_golden.py [--threads T] [goe2048] [clustered2048] [gue4096]

The n = 2048 workloads use the extended-precision Jacobi (the default
oracle; about 25 min per eigenvalue problem on one core): its eigenvalue
error on 1e-6-gap clusters is far below what Eq. (2) turns into a 1e-9 error
of |v_ij|^2.  The complex n = 4096 workload uses the same Jacobi in double
precision (about 55 min per problem instead of about 5 h; its spectrum has no
tiny gaps).  All eigenvalue problems of all requested workloads share one
thread pool, longest first.

Output: tests/golden/<name>.npz (arrays js, lam, mu, W, flags) and
<name>.json (method, wall seconds, threads, host CPU, and per problem the
Jacobi sweeps, rotations and seconds).  Nothing here touches
the GPU.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time
from concurrent.futures import ThreadPoolExecutor, as_completed

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2002_04989_amd import inputs  # noqa: E402


def sample_js(n: int, seed: int, extra: int) -> list:
    """The first two, middle and last minors plus ``extra`` seeded random ones."""
    base = [0, 1, n // 2, n - 1]
    rest = np.random.default_rng(seed).choice(np.arange(2, n - 1), size=extra, replace=False)
    return sorted(set(base) | set(int(j) for j in rest))


# name -> (matrix, sampled minors, EigenValues method, relative cost of one problem)
WORKLOADS = {
    "goe2048": lambda: (inputs.goe(2048, 4), sample_js(2048, 4040, 12), "jacobi", 1.0),
    "clustered2048": lambda: (inputs.clustered(2048, 16, 1e-6, 40)[0], sample_js(2048, 4041, 12), "jacobi", 1.0),
    "gue4096": lambda: (inputs.gue(4096, 5), sample_js(4096, 5050, 0), "jacobi64", 2.2),
}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def make(names, threads: int = 0) -> None:
    threads = threads or oracle.default_threads()
    jobs = {}
    tasks = []   # (cost, name, slot): slot -1 = lambda(A), else the index into js
    for name in names:
        A, js, method, cost = WORKLOADS[name]()
        Ah = oracle.hermitian_from_lower(A)
        jobs[name] = dict(A=Ah, js=js, method=method, lam=None, mu=[None] * len(js), t0=time.time(), left=len(js) + 1,
                          stats={})
        tasks += [(cost, name, s) for s in range(-1, len(js))]
    tasks.sort(key=lambda t: -t[0])   # longest first

    def run(task):
        _, name, s = task
        job = jobs[name]
        M = job["A"] if s < 0 else oracle.minor(job["A"], job["js"][s])
        st = {}
        t0 = time.perf_counter()
        w = oracle.eigvalsh(M, job["method"], stats=st)
        st["seconds"] = round(time.perf_counter() - t0, 2)
        return task, w, st

    with ThreadPoolExecutor(threads) as ex:
        for fut in as_completed([ex.submit(run, t) for t in tasks]):
            (_, name, s), w, st = fut.result()
            job = jobs[name]
            job["stats"]["A" if s < 0 else str(job["js"][s])] = st
            if s < 0:
                job["lam"] = w
            else:
                job["mu"][s] = w
            job["left"] -= 1
            print(f"{name}: problem {'A' if s < 0 else 'M_%d' % job['js'][s]} done, {job['left']} left", flush=True)
            if job["left"] == 0:
                write(name, job, threads)


def write(name, job, threads) -> None:
    lam, mu, js = job["lam"], np.array(job["mu"]), job["js"]
    W, flags = oracle.identity_from_spectra(lam, mu)
    dt = time.time() - job["t0"]
    np.savez(os.path.join(HERE, f"{name}.npz"), js=np.array(js, dtype=np.int64), lam=lam, mu=mu, W=W,
             flags=np.array([flags], dtype=np.int32))
    meta = dict(workload=name, n=int(job["A"].shape[0]), js=js, method=job["method"], seconds=round(dt, 1),
                threads=threads, cpu=cpu_model(), problems=job["stats"],
                note="lambda(A) and len(js) minors; the problems of all workloads generated together share the threads")
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(f"{name}: written after {dt:.1f} s with {threads} threads, js={js}", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    nthreads = 0
    if "--threads" in args:
        k = args.index("--threads")
        nthreads = int(args[k + 1])
        del args[k:k + 2]
    make(args or ["goe2048", "clustered2048", "gue4096"], nthreads)
