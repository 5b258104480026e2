"""Per-phase time of the two-stage eigenvalue kernel on the n = 2048 pair.

Loads the library built with phase timers (libeeid_phase.so: build it with
``python -m paper_2002_04989_amd.build --phase-timers``), runs the eigenvalue
launch of the n = 2048 pair (GOE seed 4 + the 16-cluster matrix, seed 40)
once per form in a given kernel configuration, and prints each phase's share
of the workgroups' time and the corresponding part of the launch's wall time
(HIP events).  The timers cost a few percent themselves.

    python -m paper_2002_04989_amd.phase_report [--variant band32_nt256x2] [--forms fp64,fp32]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import sys

PHASES = ("gather", "panel QR", "symmetric product (Y = A V)", "W", "rank-2k update", "band to tridiagonal",
          "bisection", "queue and rest")


def main(argv=None) -> dict:
    ap = argparse.ArgumentParser()
    ap.add_argument("--variant", default="band32_nt256x2")
    ap.add_argument("--forms", default="fp64,fp32")
    args = ap.parse_args(argv)
    import torch
    from . import eeid, inputs
    lib = eeid.load_library(eeid.PHASE_LIB_PATH)
    mats = [torch.from_numpy(inputs.goe(2048, 4)).to("cuda:0"),
            torch.from_numpy(inputs.clustered(2048, 16, 1e-6, 40)[0]).to("cuda:0")]
    eeid.set_variant(args.variant)
    report = {"workload": "n2048 pair (GOE seed 4 + 16-cluster seed 40)", "variant": args.variant, "forms": {}}
    for form in args.forms.split(","):
        eeid.minor_eigvals(mats, form)              # warm-up (workspace, tables)
        torch.cuda.synchronize()
        if lib.eeid_phase_ticks(None, 1) != 0:
            raise RuntimeError("this library was built without phase timers")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        eeid.minor_eigvals(mats, form)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        ticks = (ctypes.c_ulonglong * 8)()
        if lib.eeid_phase_ticks(ticks, 0) != 0:
            raise RuntimeError("eeid_phase_ticks failed")
        total = sum(ticks)
        rows = {PHASES[q]: {"share": ticks[q] / total, "launch_ms": ms * ticks[q] / total,
                            "workgroup_seconds": ticks[q] / 1e8} for q in range(8)}
        report["forms"][form] = {"launch_ms": ms, "resident_workgroups": total / 1e8 / (ms * 1e-3), "phases": rows}
        print(f"{form}: launch {ms:.1f} ms, {total / 1e8 / (ms * 1e-3):.0f} workgroups busy on average")
        for name, r in rows.items():
            print(f"  {name:<30} {100 * r['share']:6.2f} %  {r['launch_ms']:8.1f} ms")
    print(json.dumps(report))
    return report


if __name__ == "__main__":
    main(sys.argv[1:])
