"""Write the oracle's reference values for the large workloads (calls oracle/ only).

For each workload the oracle computes lambda(A), the spectra of a seeded
sample of minors M_j and the corresponding columns W[:, j] of Eq. (2).  The
full-size GPU tests compare the library against these on the same seeded
inputs (regenerated from paper_2002_04989_amd.inputs, which is deterministic).

    python tests/golden/make_golden.py [--threads T] [goe2048] [clustered2048] [gue4096]
                                       [goe64] [goe512] [uneven256] [goe4700]

The n = 2048 workloads use the extended-precision Jacobi (the default
oracle; about 25 min per eigenvalue problem on one core): its eigenvalue
error on 1e-6-gap clusters is far below what Eq. (2) turns into a 1e-9 error
of |v_ij|^2.  The complex n = 4096 workload uses the same Jacobi in double
precision (about 55 min per problem instead of about 5 h; its spectrum has no
tiny gaps).  All eigenvalue problems of all requested workloads share one
thread pool, longest first.

The smaller workloads (GOE n = 64 with all of its minors, GOE n = 512 with
six, and six members of the uneven batch of 256 with three minors each)
take seconds to a minute and let the benchmark state every configuration's
error against the oracle without running it.  goe4700 (the largest real
order in the GPU tests: lambda(A) and minors 0 and 2351) uses the double
precision Jacobi, about half an hour per problem.

Output: tests/golden/<name>.npz (arrays js, lam, mu, W, flags; for a batch
workload the same arrays suffixed _<member> plus ``members``) and
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


def uneven_members():
    """Members of the uneven batch checked against the oracle: the two
    smallest, the median, the largest and the first (GOE) and second
    (Wishart) member, each on minors 0, n // 3 and n - 1."""
    mats = inputs.make_workload("uneven256")
    order = np.argsort([m.shape[0] for m in mats], kind="stable")
    picks = sorted(set(int(b) for b in (order[0], order[1], order[len(order) // 2], order[-1], 0, 1)))
    return [(b, mats[b], [0, mats[b].shape[0] // 3, mats[b].shape[0] - 1]) for b in picks]


# name -> (matrix, sampled minors, EigenValues method, relative cost of one problem);
# a batch workload gives a list of (member, matrix, sampled minors) instead of one matrix
WORKLOADS = {
    "goe2048": lambda: (inputs.goe(2048, 4), sample_js(2048, 4040, 12), "jacobi", 1.0),
    "clustered2048": lambda: (inputs.clustered(2048, 16, 1e-6, 40)[0], sample_js(2048, 4041, 12), "jacobi", 1.0),
    "gue4096": lambda: (inputs.gue(4096, 5), sample_js(4096, 5050, 0), "jacobi64", 2.2),
    "goe64": lambda: (inputs.make_workload("goe64")[0], list(range(64)), "jacobi", 3e-5),
    "goe512": lambda: (inputs.make_workload("goe512")[0], [0, 1, 100, 255, 256, 511], "jacobi", 1.6e-2),
    "uneven256": lambda: (uneven_members(), None, "jacobi", 5e-3),
    "goe4700": lambda: (inputs.goe(4700, 47), [0, 2351], "jacobi64", 1.5),
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
    parts = {}   # workload -> its jobs (one per member)
    for name in names:
        A, js, method, cost = WORKLOADS[name]()
        members = A if isinstance(A, list) else [(None, A, js)]
        parts[name] = []
        for b, Ab, jsb in members:
            key = name if b is None else f"{name}[{b}]"
            Ah = oracle.hermitian_from_lower(Ab)
            jobs[key] = dict(A=Ah, js=jsb, method=method, lam=None, mu=[None] * len(jsb), t0=time.time(),
                             left=len(jsb) + 1, stats={}, member=b, workload=name)
            parts[name].append(key)
            c = cost * (Ah.shape[0] / 512.0) ** 3 if b is not None else cost
            tasks += [(c, key, s) for s in range(-1, len(jsb))]
    tasks.sort(key=lambda t: -t[0])   # longest first

    def run(task):
        _, key, s = task
        job = jobs[key]
        M = job["A"] if s < 0 else oracle.minor(job["A"], job["js"][s])
        st = {}
        t0 = time.perf_counter()
        w = oracle.eigvalsh(M, job["method"], stats=st)
        st["seconds"] = round(time.perf_counter() - t0, 2)
        return task, w, st

    with ThreadPoolExecutor(threads) as ex:
        for fut in as_completed([ex.submit(run, t) for t in tasks]):
            (_, key, s), w, st = fut.result()
            job = jobs[key]
            job["stats"]["A" if s < 0 else str(job["js"][s])] = st
            if s < 0:
                job["lam"] = w
            else:
                job["mu"][s] = w
            job["left"] -= 1
            if len(job["js"]) <= 16:
                print(f"{key}: problem {'A' if s < 0 else 'M_%d' % job['js'][s]} done, {job['left']} left",
                      flush=True)
            name = job["workload"]
            if all(jobs[k]["left"] == 0 for k in parts[name]) and not jobs[parts[name][0]].get("written"):
                write(name, [jobs[k] for k in parts[name]], threads)
                jobs[parts[name][0]]["written"] = True


def write(name, parts, threads) -> None:
    arrays, metas = {}, []
    for job in parts:
        lam, mu, js = job["lam"], np.array(job["mu"]), job["js"]
        W, flags = oracle.identity_from_spectra(lam, mu)
        sfx = "" if job["member"] is None else f"_{job['member']}"
        arrays.update({f"js{sfx}": np.array(js, dtype=np.int64), f"lam{sfx}": lam, f"mu{sfx}": mu, f"W{sfx}": W,
                       f"flags{sfx}": np.array([flags], dtype=np.int32)})
        metas.append(dict(member=job["member"], n=int(job["A"].shape[0]), js=js, problems=job["stats"]))
    if parts[0]["member"] is not None:
        arrays["members"] = np.array([job["member"] for job in parts], dtype=np.int64)
    dt = time.time() - min(job["t0"] for job in parts)
    np.savez(os.path.join(HERE, f"{name}.npz"), **arrays)
    job = parts[0]
    meta = dict(workload=name, method=job["method"], seconds=round(dt, 1), threads=threads, cpu=cpu_model(),
                note="lambda(A) and len(js) minors; the problems of all workloads generated together share the threads")
    if job["member"] is None:
        meta.update(n=metas[0]["n"], js=metas[0]["js"], problems=metas[0]["problems"])
    else:
        meta["members"] = metas
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(f"{name}: written after {dt:.1f} s with {threads} threads", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    nthreads = 0
    if "--threads" in args:
        k = args.index("--threads")
        nthreads = int(args[k + 1])
        del args[k:k + 2]
    make(args or ["goe2048", "clustered2048", "gue4096"], nthreads)
