"""Benchmark: every |v_ij|^2 of the n=2048 workload on one MI355X.

Workload (one step): a batch of two real symmetric 2048 x 2048 matrices -- a
symmetrised Gaussian (seed 4) and Q diag(lambda) Q^T with 16 clusters of 128
eigenvalues 1e-6 apart (seed 40) -- through the whole path: eigenvalues of
each matrix and of all 2048 of its minors (one persistent launch over 4098
problems), then Eq. (2) for all 2 x 2048^2 components.  Inputs are resident
in HBM before timing starts; outputs stay there.

Prints ONE JSON line.  ``value`` is components/s of the FP64 form, each
step two hipGraph replays (the eigenvalue launch, then the identity launch);
the FP32 trailing-update form is timed the same way and reported in
``fp32_form``; each form's error against the FP64 oracle (sampled minors)
and, for the clustered matrix, against the exact answer (Q**2)^T is
reported.  ``other_workloads`` times the n=64, n=512 and uneven-batch
workloads (whole path, errors against stored oracle values) and one wave of
the complex n=4096 job; ``single_component_latency`` the paper's Table 1
regime; ``cpu_baseline`` the oracle on this host.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-fp32] [--no-paired]
                    [--no-latency] [--no-others] [--no-tune | --variant V] [--copy-ref]
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

METRIC = "|v_ij|^2 components/s at n=2048 (FP64 vs FP32-MFMA form, stated error)"
HBM_PEAK_GBS = 8000.0
N = 2048


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def symv_bytes(m: int, s: int) -> int:
    """Algorithmic bytes of the SYMV half of one tridiagonalisation of order m:
    the stale lower triangle (s bytes/element) streamed once per column."""
    return s * m * (m + 1) * (m + 2) // 6


def kernel_sources_hash() -> str:
    """Hash of the library's code (comments and blank lines left out): a stored
    profile is used only while the code it measured is unchanged."""
    h = hashlib.sha256()
    for f in ("eeid.hip", "eeid_tridiag.hpp", "eeid_tridiag_c.hpp", "eeid_band.hpp", "eeid_identity.hpp",
              "eeid_latency.hpp"):
        for line in open(os.path.join(ROOT, "paper_2002_04989_amd", "csrc", f), encoding="utf-8"):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


# compiled configurations of the eigenvalue kernel (eeid.VARIANTS): panel width NB, threads per block NT
VARIANT_SHAPE = {"nb32_nt512": (32, 512), "nb32_nt256x2": (32, 256), "nb16_nt512": (16, 512), "band32_nt512": (32, 512),
                 "band32_nt256x2": (32, 256)}


def kernel_name(form: str, variant: str) -> str:
    nb, nt = VARIANT_SHAPE[variant]
    s = "double" if form == "fp64" else "float"
    if variant.startswith("band"):
        return f"void eeid::band_bisect_kernel<{s}, {nt}>(eeid::TriArgs)"
    return f"void eeid::tridiag_bisect_kernel<{s}, {nb}, {nt}, 32, true, 2>(eeid::TriArgs)"


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it matches these sources."""
    path = os.path.join(ROOT, "profiles", "band_bisect_n2048x2_counters.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_sources_hash") != kernel_sources_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def tridiag_flops(m: int) -> float:
    """Algorithmic flops of one Householder tridiagonalisation of order m (4/3 m^3)."""
    return 4.0 / 3.0 * m ** 3


# dense peaks of MI355X: FP64 matrix 78.6 TFLOP/s, FP32 matrix 157.3 TFLOP/s
MFMA_F64_TFLOPS = 78.6
MFMA_F32_TFLOPS = 157.3


def roofline_for(form: str, variant: str, kernel_ms: float, kname: str) -> dict:
    """Roofline of the eigenvalue kernel for the configuration the autotuner chose.

    One-stage reduction: HBM-bound by its SYMV, which streams the stale trailing
    triangle once per column (symv_bytes per problem).  Two-stage reduction: the
    dense-to-band stage is matrix-core work, 4/3 m^3 flops per problem (half in the
    symmetric product, half in the rank-2k update); its HBM stream is three
    triangle passes per panel of 32 columns, far below the bandwidth, so the
    bound is the FP64 matrix peak (FP32 form: symmetric product FP64, update
    FP32, harmonic mean of the two peaks)."""
    per_launch_problems = [(N - 1, N), (N, 1)]  # (order, count) per matrix: minors and A itself
    if variant.startswith("band"):
        flops = 2 * sum(c * tridiag_flops(m) for m, c in per_launch_problems)
        peak = MFMA_F64_TFLOPS if form == "fp64" else 2.0 / (1.0 / MFMA_F64_TFLOPS + 1.0 / MFMA_F32_TFLOPS)
        achieved = flops / (kernel_ms * 1e-3) / 1e12
        traffic = measured_traffic(kname)
        out = {"bound": "mfma", "achieved": round(achieved, 2), "peak": round(peak, 1), "unit": "TFLOP/s",
               "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": kname,
               "kernel_ms_per_launch": round(kernel_ms, 2), "algorithmic_flops_per_launch": flops}
        if traffic is not None:
            # the same launch against the other roof: measured HBM bytes / kernel time vs 8 TB/s
            gbs = traffic / (kernel_ms * 1e-3) / 1e9
            out["hbm_achieved_GBs"] = round(gbs, 1)
            out["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        return out
    s = 8 if form == "fp64" else 4
    nbytes = 2 * sum(c * symv_bytes(m, s) for m, c in per_launch_problems)
    achieved = nbytes / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kname), "kernel": kname,
            "kernel_ms_per_launch": round(kernel_ms, 2), "algorithmic_bytes_per_launch": nbytes}


def make_inputs():
    from paper_2002_04989_amd import inputs
    A_goe = inputs.goe(N, 4)
    A_clu, lam_true, Q = inputs.clustered(N, 16, 1e-6, 40)
    return [A_goe, A_clu], (lam_true, Q)


def load_golden(name):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def errors(mats, truth, lam, mu, V2, n):
    """Per-result error of one form against the oracle's sampled minors and the exact clustered answer."""
    import numpy as np
    from paper_2002_04989_amd import eeid
    lam = eeid.split(lam, n, "lambda")
    mu = eeid.split(mu, n, "mu")
    W = eeid.split(V2, n, "V2")
    out = {}
    for b, name in enumerate(("goe2048", "clustered2048")):
        A = mats[b]
        s = float(np.max(np.abs(np.linalg.eigvalsh(A)))) if b == 0 else 1.0
        e = {}
        g = load_golden(name)
        if g is not None:
            js = g["js"]
            e["oracle_minors"] = [int(j) for j in js]
            e["max_abs_dlam_rel"] = float(np.max(np.abs(lam[b] - g["lam"])) / s)
            e["max_abs_dmu_rel"] = float(np.max(np.abs(mu[b][js] - g["mu"])) / s)
            e["max_abs_dW_sampled"] = float(np.max(np.abs(W[b][:, js] - g["W"])))
        rows = np.abs(W[b].sum(axis=1) - 1.0)
        cols = np.abs(W[b].sum(axis=0) - 1.0)
        e["row_sum_residual"] = float(np.max(rows))
        e["col_sum_residual"] = float(np.max(cols))
        if b == 1:
            lam_true, Q = truth
            d = np.abs(W[b] - (Q ** 2).T)
            e["max_abs_dW_vs_exact"] = float(d.max())
            e["median_abs_dW_vs_exact"] = float(np.median(d))
            e["p99_abs_dW_vs_exact"] = float(np.quantile(d, 0.99))
            cl = (W[b].reshape(16, 128, N).sum(axis=1) - (Q ** 2).T.reshape(16, 128, N).sum(axis=1))
            e["cluster_projector_err"] = float(np.max(np.abs(cl)))
            e["max_abs_dlam_vs_exact"] = float(np.max(np.abs(lam[b] - lam_true)))
        out[name] = e
    return out


def run_form(mats_dev, n, form, steps, warmup, tune=True, graph=True):
    """Recording of the graphs (untimed, like the autotuning), `warmup`
    untimed steps, then `steps` timed steps: the eigenvalue launch and the
    identity launch, each a hipGraph replay in graph mode (the batch packed and
    the outputs allocated once, so every step replays the same recording), with
    HIP events on the stream around each."""
    import torch
    from paper_2002_04989_amd import eeid
    stream = torch.cuda.current_stream()
    tuned = None
    if isinstance(tune, str):  # a configuration given on the command line
        eeid.set_variant(tune)
        tuned = (tune, float("nan"))
    elif tune:  # untimed: pick the fastest kernel configuration for this batch
        tuned = eeid.autotune(mats_dev, form)
        log(f"{form}: autotune chose {tuned[0]} ({tuned[1]:.0f} ms)")
    packed = eeid.pack(mats_dev)
    nl, nm, nv = eeid.sizes(n)
    dev = packed.flat.device
    lam = torch.empty(nl, dtype=torch.float64, device=dev)
    mu = torch.empty(max(nm, 1), dtype=torch.float64, device=dev)
    flags = torch.empty(len(n), dtype=torch.int32, device=dev)
    V2 = torch.empty(nv, dtype=torch.float64, device=dev)

    def step():
        eeid.minor_eigvals(packed, form, out=(lam, mu, flags))
        eeid.components(lam, mu[:nm], n, flags, out=V2)

    eeid.set_graph_mode(graph)
    try:
        if graph:
            # recording, before the warm-up: the identity's first call uploads its
            # tables, which invalidates the eigenvalue launch recorded just before
            # (recordings are keyed on the handle's buffers); the second call pair
            # records both for good
            step()
            step()
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            e0, e1, e2 = ev[k]
            e0.record(stream)
            eeid.minor_eigvals(packed, form, out=(lam, mu, flags))     # the dominant (persistent) kernel
            e1.record(stream)
            eeid.components(lam, mu[:nm], n, flags, out=V2)
            e2.record(stream)
            log(f"{form}: step {k + 1}/{steps} enqueued")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        eeid.set_graph_mode(False)
    res = (lam, mu[:nm], V2, flags)
    tri_ms = sum(e0.elapsed_time(e1) for e0, e1, _ in ev) / steps
    id_ms = sum(e1.elapsed_time(e2) for _, e1, e2 in ev) / steps
    step_ms = sorted(e0.elapsed_time(e2) for e0, _, e2 in ev)
    spread = {"median": round(step_ms[len(step_ms) // 2] if len(step_ms) % 2 else
                              0.5 * (step_ms[len(step_ms) // 2 - 1] + step_ms[len(step_ms) // 2]), 2),
              "min": round(step_ms[0], 2), "max": round(step_ms[-1], 2)}
    return res, wall, tri_ms, id_ms, tuned, spread


def end_to_end_ms(mats_host, n, form):
    """One step from host-resident A to host-resident |v_ij|^2 (H2D + kernels + D2H)."""
    import torch
    from paper_2002_04989_amd import eeid
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = [torch.from_numpy(m).to("cuda:0") for m in mats_host]
    lam, mu, flags = eeid.minor_eigvals(dev, form)
    V2 = eeid.components(lam, mu, n, flags)
    _ = (V2.cpu(), lam.cpu(), mu.cpu())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def golden_rotations(name: str):
    """Median Jacobi rotations per problem of the stored oracle run of `name` (None if not recorded)."""
    try:
        meta = json.load(open(os.path.join(ROOT, "tests", "golden", f"{name}.json")))
        rots = sorted(int(p["rotations"]) for p in meta["problems"].values())
        return rots[len(rots) // 2], meta
    except (OSError, ValueError, KeyError, TypeError):
        return None, None


def cpu_baseline(mats, rounds=128, max_threads=16):
    """The oracle (extended-precision Jacobi EigenValues + log-sum identity)
    timed on this host's cores on a bounded sample of the same workload.

    One eigenvalue problem of order 2047 takes the oracle tens of minutes, so
    the sample is the first `rounds` Jacobi rounds of one minor per thread, all
    threads at once; a problem's full time is extrapolated by the rotations a
    complete oracle run of the same matrix needed (recorded with the stored
    oracle results), and the job's by its 2 x (n + 1) problems spread over the
    threads, plus the identity measured on a few columns."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    A = mats[0]
    n = A.shape[0]
    try:
        threads = min(max_threads, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        threads = min(max_threads, os.cpu_count() or 1)
    js = [int(j) for j in np.random.default_rng(1).choice(n, size=threads, replace=False)]
    minors = [oracle.minor(A, j) for j in js]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        samples = list(ex.map(lambda M: oracle.jacobi_rounds_sample(M, rounds), minors))
    wall = time.perf_counter() - t0
    rot_sample = sum(s["rotations"] for s in samples) / len(samples)
    rot_full, meta = golden_rotations("goe2048")
    if rot_full is None:
        # no recorded full run: a complete cyclic sweep rotates every pair; ~10 sweeps
        rot_full, basis = 10 * n * (n - 1) // 2, "10 full sweeps (no recorded oracle run)"
    else:
        basis = (f"median rotations of the stored oracle run of this matrix ({meta.get('cpu', '?')}, "
                 f"{meta.get('threads', '?')} threads)")
    t_problem = wall * rot_full / rot_sample          # wall time of one problem on one of `threads` busy cores
    # the identity's cost does not depend on the values: interlacing stand-in spectra
    lam = np.sort(np.random.default_rng(2).uniform(-90.0, 90.0, n))
    mus = np.tile(0.5 * (lam[:-1] + lam[1:]), (4, 1))
    t1 = time.perf_counter()
    oracle.denominators(lam)
    oracle.numerators(lam, mus)
    t_id = time.perf_counter() - t1                   # denominators + 4 columns
    total = 2 * ((n + 1) * t_problem / threads + t_id / 4 * n)
    return {
        "value": 2 * n * n / total, "unit": "components/s", "cores": threads, "kind": "oracle",
        "cpu": cpu_model(),
        "sample": (f"the oracle's extended-precision Jacobi EigenValues step: the first {rounds} rounds on "
                   f"{threads} minors of the GOE n={n} matrix at once ({threads} threads, {wall:.1f} s wall, "
                   f"{rot_sample:.0f} rotations each), extrapolated to a whole problem by {basis} "
                   f"({rot_full} rotations: {t_problem:.0f} s per problem) and to 2 x ({n}+1) problems over "
                   f"{threads} threads; the identity (numpy Neumaier log sums) timed on the denominators and "
                   f"4 columns, scaled to 2 x {n} columns"),
        "extrapolated_seconds_per_step": round(total, 1),
        "seconds_measured": round(time.perf_counter() - t0, 2),
    }


def oracle_single_component(n=502):
    """The oracle on the single-component query (part of the CPU baseline):
    lambda(A) and M_j of the GOE (seed 11) of order n by the extended-precision
    Jacobi, both problems on two threads at once, then the log-sum column of
    Eq. (2).  Returns (n, seconds)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    from paper_2002_04989_amd import inputs
    A = inputs.goe(n, 11)
    j = n // 2
    t0 = time.perf_counter()
    with ThreadPoolExecutor(2) as ex:
        lam, mu = ex.map(lambda M: oracle.eigvalsh(M), [A, oracle.minor(A, j)])
    oracle.identity_from_spectra(lam, mu[None, :])
    return n, time.perf_counter() - t0


def host_library(mats, budget_s=8.0):
    """Context, not the oracle: numpy/LAPACK eigvalsh for the EigenValues step on this host."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas_threads = 1
    A = mats[0]
    n = A.shape[0]
    t0 = time.perf_counter()
    np.linalg.eigvalsh(A, UPLO="L")
    t_lam = time.perf_counter() - t0
    rng = np.random.default_rng(2)
    k, t_min = 0, 0.0
    while t_min < budget_s and k < n:
        j = int(rng.integers(0, n))
        M = np.delete(np.delete(A, j, axis=0), j, axis=1)
        t1 = time.perf_counter()
        np.linalg.eigvalsh(M, UPLO="L")
        t_min += time.perf_counter() - t1
        k += 1
    total = 2 * (t_lam + t_min / k * n)
    return {"value": 2 * n * n / total, "unit": "components/s", "blas_threads": int(blas_threads),
            "kind": "host library (numpy/LAPACK eigvalsh), not the oracle", "cpu": cpu_model(),
            "sample": f"lambda(A) + {k} random minors of the GOE n={n} matrix, extrapolated to 2 x ({n}+1) "
                      f"problems (EigenValues step only)"}


def golden_errors(name, lam, mu, W, member=None):
    """Errors of one matrix's results against the stored oracle values of `name`."""
    import numpy as np
    g = load_golden(name)
    if g is None:
        return None
    sfx = "" if member is None else f"_{member}"
    js = g["js" + sfx]
    s = float(np.max(np.abs(g["lam" + sfx])))
    return {"oracle_minors": len(js), "max_abs_dlam_rel": float(np.max(np.abs(lam - g["lam" + sfx])) / s),
            "max_abs_dmu_rel": float(np.max(np.abs(mu[js] - g["mu" + sfx])) / s),
            "max_abs_dW": float(np.max(np.abs(W[:, js] - g["W" + sfx]))),
            "row_sum_residual": float(np.max(np.abs(W.sum(axis=1) - 1.0))),
            "col_sum_residual": float(np.max(np.abs(W.sum(axis=0) - 1.0)))}


def other_workloads(steps=(20, 3, 2)):
    """The three smaller workloads, each as one call over its whole batch
    (eigenvalues of every matrix and minor, then Eq. (2)), inputs resident in
    HBM: GOE n=64 (median of 20 steps), GOE n=512 (3 steps) and the uneven
    batch of 256 (2 steps of a hipGraph-captured launch, kernel configuration
    autotuned), with errors against the stored oracle values."""
    import numpy as np
    import torch
    from paper_2002_04989_amd import eeid, inputs
    out = {}
    for (name, nsteps) in (("goe64", steps[0]), ("goe512", steps[1]), ("uneven256", steps[2])):
        mats = inputs.make_workload(name)
        n = [m.shape[0] for m in mats]
        dev = [torch.from_numpy(m).to("cuda:0") for m in mats]
        torch.cuda.synchronize()
        autotuned = name == "uneven256"
        try:
            res, wall, tri, idn, tuned, spread = run_form(dev, n, "fp64", nsteps, 1, tune=autotuned)
            # the same steps launched eagerly, for comparison (launch overhead matters at n = 64)
            _, _, _, _, _, spread_eager = run_form(dev, n, "fp64", nsteps, 0, tune=False, graph=False)
        finally:
            if autotuned:
                eeid.set_variant(None)
        lam = eeid.split(res[0].cpu().numpy(), n, "lambda")
        mu = eeid.split(res[1].cpu().numpy(), n, "mu")
        W = eeid.split(res[2].cpu().numpy(), n, "V2")
        flags = [int(x) for x in res[3].cpu().numpy()]
        comps = sum(m * m for m in n)
        row = {"matrices": len(n), "problems": sum(m + 1 for m in n), "components": comps,
               "ms_per_step": round(spread["median"], 3), "step_ms": spread,
               "value": comps / (spread["median"] * 1e-3), "unit": "components/s",
               "eigenvalue_kernel_ms": round(tri, 3), "identity_ms": round(idn, 3),
               "flags_nonzero": int(sum(1 for f in flags if f))}
        row["launch"] = "hipGraph replay"
        row["eager_ms_per_step"] = round(spread_eager["median"], 3)
        if autotuned:
            row["variant"] = tuned[0] if tuned else None
        if name == "uneven256":
            g = load_golden(name)
            errs = {}
            if g is not None:
                for b in (int(x) for x in g["members"]):
                    errs[f"member{b}_n{n[b]}"] = golden_errors(name, lam[b], mu[b], W[b], b)
            row["errors_vs_oracle"] = errs
        else:
            row["errors_vs_oracle"] = golden_errors(name, lam[0], mu[0], W[0])
        log(f"{name}: {row['ms_per_step']} ms per step")
        out[name] = row
    return out


def complex4096(reps=2, extra=251):
    """Complex Hermitian n = 4096 (GUE seed 5), both forms: one launch of
    lambda(A) and 255 minors (the four with stored oracle values and 251
    seeded others) -- one problem per resident workgroup slot (256, one per
    CU), i.e. one wave of the 4097-problem job -- timed with HIP events (best
    of `reps`), errors against the stored oracle values, and the time scaled
    by the 17 waves the full job needs on the same slots (16 full ones and
    one problem).  The full job is run in the GPU tests, not here: it takes
    minutes."""
    import numpy as np
    import torch
    from paper_2002_04989_amd import eeid, inputs
    g = load_golden("gue4096")
    A = inputs.gue(4096, 5)
    n = A.shape[0]
    stored = [int(j) for j in g["js"]] if g is not None else []
    rng = np.random.default_rng(4096)
    rest = [int(j) for j in rng.choice(np.setdiff1d(np.arange(n), stored), size=extra, replace=False)]
    js = sorted(stored + rest)
    dA = torch.from_numpy(A).to("cuda:0")
    out = {"workload": "GUE n=4096 (seed 5): lambda(A) + 255 minors in one launch", "problems": len(js) + 1}
    waves = -(-(n + 1) // (len(js) + 1))
    for form in ("fp64", "fp32"):
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream())
            lam, mu, flag = eeid.minor_eigvals_subset(dA, js, prec=form)
            e1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = min(times)
        row = {"dtype": "c128" if form == "fp64" else "c64 trailing / f64 rest", "ms_per_launch": round(ms, 1),
               "scaled_s_all_4097_problems": round(ms * waves / 1e3, 1),
               "scaled_components_per_s": n * n / (ms * waves / 1e3), "flag": int(flag.cpu()[0])}
        if g is not None:
            lam_h, mu_h = lam.cpu().numpy(), mu.cpu().numpy()
            s = float(np.max(np.abs(g["lam"])))
            sel = [js.index(j) for j in stored]
            row["max_abs_dlam_rel"] = float(np.max(np.abs(lam_h - g["lam"])) / s)
            row["max_abs_dmu_rel_stored_minors"] = float(np.max(np.abs(mu_h[sel] - g["mu"])) / s)
        log(f"complex n=4096 {form}: {row['ms_per_launch']} ms for {len(js) + 1} problems")
        out[form] = row
    return out


# Table 1 of the paper (Section 4): one component of one eigenvector on a 4-core
# Xeon E3-1270 v6 (NumPy eigh / Algorithm 2, seconds, mean of 10 runs).  Context only.
PAPER_TABLE1 = {502: (0.170962, 0.119722), 1002: (1.100800, 0.595935), 2002: (9.522480, 3.212001),
                3002: (30.342656, 9.522745), 4002: (69.955400, 16.775200), 5002: (134.324200, 30.547200),
                6002: (229.338600, 50.682400)}


def single_component_latency(sizes=(502, 1002, 2002, 3002, 4002, 5002, 6002), reps=3, oracle_time=None):
    """The single-component query of Table 1 (lambda(A) + the spectrum of one minor
    M_j + Eq. (2), here for every i of column j at once) on one GOE matrix per
    size: the latency path (each problem over many workgroups) against the
    batched path (one workgroup per problem), wall time from device-resident A
    to device-resident column.  oracle_time: (n, seconds) of the oracle on the
    same query (timed in the CPU-baseline leg), scaled by n^3 to every size."""
    import numpy as np
    import torch
    from paper_2002_04989_amd import eeid, inputs
    rows = []
    for n in sizes:
        A = torch.from_numpy(inputs.goe(n, 11)).to("cuda:0")
        j = n // 2
        res = {}
        for path in ("latency", "batched"):
            ts = []
            for _ in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if path == "latency":
                    lam, mu, flag = eeid.minor_eigvals_latency(A, [j])
                else:
                    lam, mu, flag = eeid.minor_eigvals_subset(A, [j])
                W = eeid.components_subset(lam, mu, flag)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            res[path] = (sorted(ts[1:])[len(ts[1:]) // 2] * 1e3, W.cpu().numpy()[:, 0], int(flag.cpu()[0]))
        row = {"n": n, "latency_path_ms": round(res["latency"][0], 2), "batched_path_ms": round(res["batched"][0], 2),
               "max_abs_dW_latency_vs_batched": float(np.max(np.abs(res["latency"][1] - res["batched"][1]))),
               "flags": [res["latency"][2], res["batched"][2]]}
        if n in PAPER_TABLE1:
            row["paper_table1_s"] = {"numpy_eigh": PAPER_TABLE1[n][0], "algorithm2": PAPER_TABLE1[n][1]}
        rows.append(row)
        log(f"single component n={n}: latency path {row['latency_path_ms']} ms, batched {row['batched_path_ms']} ms")
        del A
    out = {"workload": "GOE (seed 11) of each order n, one minor j = n // 2; lambda(A) + mu(M_j) + column j of W",
           "rows": rows, "paper_hardware": "Intel Xeon E3-1270 v6, 4 cores / 8 threads (context only)"}
    if oracle_time is None:
        return out
    oracle_n, t_or = oracle_time
    for row in rows:
        row["oracle_s"] = round(t_or * (row["n"] / oracle_n) ** 3, 2)
        row["oracle_kind"] = "measured" if row["n"] == oracle_n else f"n^3-scaled from the measured n={oracle_n}"
    out["oracle"] = f"extended-precision Jacobi, 2 threads ({cpu_model()}), {t_or:.1f} s at n={oracle_n}"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 trailing-update form")
    ap.add_argument("--no-tune", action="store_true", help="skip the (untimed) autotuning of kernel configurations")
    ap.add_argument("--no-paired", action="store_true", help="skip timing the paired form of the identity")
    ap.add_argument("--no-latency", action="store_true", help="skip the single-component latency table")
    ap.add_argument("--no-others", action="store_true", help="skip the smaller workloads (n=64, n=512, uneven batch)")
    ap.add_argument("--variant", default=None, help="use this kernel configuration (eeid.VARIANTS) instead of autotuning")
    ap.add_argument("--copy-ref", action="store_true",
                    help="run a 1 GiB device copy first (reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "the minors shard across GPUs without communication, but no multi-GPU path is built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2002_04989_amd import eeid
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    eeid.load_library()
    log("generating inputs")
    mats, truth = make_inputs()
    n = [N, N]
    mats_dev = [torch.from_numpy(m).to("cuda:0") for m in mats]
    torch.cuda.synchronize()
    if args.copy_ref:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy reference: 1 GiB read + 1 GiB write done")

    log(f"fp64 form: warmup {args.warmup}, steps {args.steps}")
    tune = args.variant if args.variant else not args.no_tune
    res64, wall64, tri64, id64, tuned64, spread64 = run_form(mats_dev, n, "fp64", args.steps, args.warmup, tune)
    e2e64 = end_to_end_ms(mats, n, "fp64")
    comps = 2 * N * N
    ms_step = wall64 / args.steps * 1e3
    value = comps / (wall64 / args.steps)
    host = [t.cpu().numpy() for t in res64]
    err64 = errors(mats, truth, host[0], host[1], host[2], n)
    flags64 = [int(x) for x in host[3]]

    # Algorithm 2's paired form of the identity on the same spectra (timed alone, HIP events)
    paired = None
    if not args.no_paired:
        lam_d, mu_d, V2_d, fl_d = res64
        eeid.set_identity_form("paired")
        try:
            times = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                fl2 = fl_d.clone()
                e0.record(torch.cuda.current_stream())
                V2p = eeid.components(lam_d, mu_d, n, fl2)
                e1.record(torch.cuda.current_stream())
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
        finally:
            eeid.set_identity_form("products")
        d = np.abs(V2p.cpu().numpy() - host[2])
        paired = {"ms_per_launch": round(sorted(times)[1], 3), "products_ms_per_launch": round(id64, 3),
                  "max_abs_dW_vs_products": float(np.max(d)),
                  "errors_vs_oracle": errors(mats, truth, host[0], host[1], V2p.cpu().numpy(), n)}
        log(f"paired identity: {paired['ms_per_launch']} ms, max|dW| vs products {paired['max_abs_dW_vs_products']:.2e}")

    variant64 = tuned64[0] if tuned64 else "nb32_nt512"
    kname64 = kernel_name("fp64", variant64)
    roofline = roofline_for("fp64", variant64, tri64, kname64)
    roofline["identity_ms_per_launch"] = round(id64, 2)

    fp32 = None
    if not args.no_fp32:
        log(f"fp32 form: warmup {args.warmup}, steps {args.steps}")
        res32, wall32, tri32, id32, tuned32, spread32 = run_form(mats_dev, n, "fp32", args.steps, args.warmup, tune)
        h32 = [t.cpu().numpy() for t in res32]
        variant32 = tuned32[0] if tuned32 else "nb32_nt512"
        kname32 = kernel_name("fp32", variant32)
        fp32 = {"value": comps / (wall32 / args.steps), "unit": "components/s",
                "ms_per_step": round(wall32 / args.steps * 1e3, 2), "step_ms": spread32,
                "dtype": "f32 trailing matrix / f64 rest",
                "speedup_vs_fp64": round((wall64 / wall32), 3),
                "roofline": roofline_for("fp32", variant32, tri32, kname32),
                "errors_vs_oracle": errors(mats, truth, h32[0], h32[1], h32[2], n),
                "flags": [int(x) for x in h32[3]]}

    others = None
    if not args.no_others:
        log("smaller workloads")
        others = other_workloads()
        log("complex n=4096 (one wave of its problems)")
        others["complex4096"] = complex4096()
    cpu = hostlib = oracle_sc = None
    if not args.no_cpu:
        log("cpu baseline (oracle) on a bounded sample")
        cpu = cpu_baseline(mats)
        oracle_sc = oracle_single_component()
        cpu["single_component_n502_s"] = round(oracle_sc[1], 2)
        log("host library context (LAPACK)")
        hostlib = host_library(mats)
    latency = None
    if not args.no_latency:
        log("single-component latency (Table 1 sizes)")
        latency = single_component_latency(oracle_time=oracle_sc)

    out = {
        "metric": METRIC, "value": value, "unit": "components/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 2), "step_ms": spread64,
        "end_to_end_ms_incl_h2d_d2h": round(e2e64, 2), "higher_is_better": True, "scaling": "weak",
        "launch": "hipGraph replays (the eigenvalue launch and the identity launch, each recorded once)",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "n2048 pair: GOE (seed 4) + 16-cluster Q diag(lam) Q^T (seed 40); eigenvalues of "
                               "both matrices and all 2x2048 minors in one persistent launch, then all 2x2048^2 "
                               "|v_ij|^2", "n": N, "matrices": 2, "form": "fp64", "components_per_step": comps},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host_library": hostlib,
        "errors_vs_oracle": err64, "flags": flags64,
        "fp32_form": fp32,
        "identity_paired_form": paired,
        "single_component_latency": latency,
        "other_workloads": others,
        "kernel_sources_hash": kernel_sources_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
