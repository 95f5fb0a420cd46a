"""Summaries of rocprofv3 output for the step kernel.

    python -m paper_2101_04847_amd.profiling trace <kernel_trace.csv> <kernel-regex> <n_last> [out.md]
    python -m paper_2101_04847_amd.profiling traffic <fetch.csv> <write.csv> <copy_fetch.csv> \
        <copy_write.csv> <kernel-regex> <copy-bytes> <storage> <nx> <ny> [out.json]
    python -m paper_2101_04847_amd.profiling sq <counter_collection.csv> <kernel-regex> <n_simd> <n_xcd>
    python -m paper_2101_04847_amd.profiling copy <bytes>

`copy` runs a plain device-to-device copy of the given size ten times (the
calibration kernel for the counters).

`trace` reports the duration statistics of the last n launches of the kernels
matching the regex (the timed steps of a bench run; earlier launches of the
same kernel belong to tile tuning and warm-up).

`traffic` turns FETCH_SIZE / WRITE_SIZE counter runs (KiB per dispatch) into
HBM bytes per launch, each counter scaled by the factor that makes it read
the known size of a plain copy kernel, and records the hash of the kernel
sources so that a stale record is ignored by bench.py.

`sq` turns one run of the shader-sequencer counters SQ_WAVE_CYCLES,
SQ_WAIT_INST_ANY, SQ_WAIT_ANY, SQ_ACTIVE_INST_ANY, SQ_ACTIVE_INST_VALU,
SQ_ACTIVE_INST_VMEM, SQ_INSTS_VALU and GRBM_GUI_ACTIVE (means per dispatch of
the matching kernel) into shares of the waves' lifetime (waiting on a memory
or other dependency, issuing any instruction, a VALU or a vector-memory
instruction) and the VALU busy fraction of the chip, SQ_ACTIVE_INST_VALU x 4
/ n_simd / (GRBM_GUI_ACTIVE / n_xcd): the usual rocprof definition, with
GRBM_GUI_ACTIVE summed over the n_xcd dies (n_simd = 4 per CU).  A second
estimate counts 4 cycles per wave-64 VALU instruction: SQ_INSTS_VALU x 4 /
n_simd / (GRBM_GUI_ACTIVE / n_xcd).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in ("paper_2101_04847_amd/csrc/lb_kernels.hpp", "paper_2101_04847_amd/csrc/lb.hip",
                "paper_2101_04847_amd/csrc/lb_internal.hpp", "paper_2101_04847_amd/csrc/lb_memory.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def trace_summary(path: str, regex: str, n_last: int) -> dict:
    rows = [r for r in _rows(path) if re.search(regex, r["Kernel_Name"])]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    rows = rows[-n_last:]
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in rows]
    return {"kernel": rows[-1]["Kernel_Name"], "launches": len(d), "mean_ms": statistics.fmean(d),
            "median_ms": statistics.median(d), "min_ms": min(d), "max_ms": max(d),
            "stdev_ms": statistics.pstdev(d), "grid": rows[-1]["Grid_Size_X"] if "Grid_Size_X" in rows[-1] else rows[-1].get("Grid_Size"),
            "workgroup": rows[-1].get("Workgroup_Size_X", rows[-1].get("Workgroup_Size")),
            "vgpr": rows[-1].get("VGPR_Count"), "lds": rows[-1].get("LDS_Block_Size")}


def _counter_mean(path, regex, counter):
    v = [float(r["Counter_Value"]) for r in _rows(path)
         if re.search(regex, r["Kernel_Name"]) and r["Counter_Name"] == counter]
    if not v:
        raise ValueError(f"no {counter} rows for {regex} in {path}")
    return statistics.fmean(v), len(v)


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, regex, copy_bytes, storage, nx, ny):
    f_kib, nf = _counter_mean(fetch_csv, regex, "FETCH_SIZE")
    w_kib, nw = _counter_mean(write_csv, regex, "WRITE_SIZE")
    cf_kib, _ = _counter_mean(copy_fetch_csv, "copy", "FETCH_SIZE")
    cw_kib, _ = _counter_mean(copy_write_csv, "copy", "WRITE_SIZE")
    kf = copy_bytes / (cf_kib * 1024.0)
    kw = copy_bytes / (cw_kib * 1024.0)
    read = f_kib * 1024.0 * kf
    write = w_kib * 1024.0 * kw
    bpl = {"f64": 288, "f32": 144, "f16s": 88, "bf16s": 88}[storage]
    alg = bpl * nx * ny
    return {"storage": storage, "nx": nx, "ny": ny, "source_hash": kernel_source_hash(),
            "bytes_per_launch": round(read + write), "read_bytes": round(read), "write_bytes": round(write),
            "algorithmic_bytes": alg, "read_over_algorithmic": read / (alg / 2), "write_over_algorithmic": write / (alg / 2),
            "fetch_factor": kf, "write_factor": kw, "dispatches": [nf, nw],
            "copy_bytes": copy_bytes}


SQ_COUNTERS = ("SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU",
               "SQ_ACTIVE_INST_VMEM", "SQ_INSTS_VALU", "GRBM_GUI_ACTIVE")


def sq_summary(path: str, regex: str, n_simd: int, n_xcd: int = 1) -> dict:
    m = {c: _counter_mean(path, regex, c)[0] for c in SQ_COUNTERS}
    w = m["SQ_WAVE_CYCLES"]
    cycles = m["GRBM_GUI_ACTIVE"] / n_xcd   # cycles of the kernel on one die
    return {"dispatches": _counter_mean(path, regex, "SQ_WAVE_CYCLES")[1],
            "wait_dependency": m["SQ_WAIT_INST_ANY"] / w, "wait_any": m["SQ_WAIT_ANY"] / w,
            "issue_any": m["SQ_ACTIVE_INST_ANY"] / w, "issue_valu": m["SQ_ACTIVE_INST_VALU"] / w,
            "issue_vmem": m["SQ_ACTIVE_INST_VMEM"] / w,
            "valu_busy": m["SQ_ACTIVE_INST_VALU"] * 4.0 / n_simd / cycles,
            "valu_busy_from_insts": m["SQ_INSTS_VALU"] * 4.0 / n_simd / cycles,
            "valu_insts": m["SQ_INSTS_VALU"], "cycles": cycles}


def copy_kernel(nbytes: float) -> None:
    import torch
    n = int(nbytes)
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n} bytes 10 times", flush=True)


def main(argv):
    if argv[0] == "copy":
        copy_kernel(float(argv[1]))
        return
    if argv[0] == "trace":
        s = trace_summary(argv[1], argv[2], int(argv[3]))
        text = json.dumps(s, indent=1)
    elif argv[0] == "sq":
        s = sq_summary(argv[1], argv[2], int(argv[3]), int(argv[4]))
        text = json.dumps(s, indent=1)
        argv = argv[:5]
    elif argv[0] == "traffic":
        s = traffic(argv[1], argv[2], argv[3], argv[4], argv[5], float(argv[6]), argv[7], int(argv[8]), int(argv[9]))
        text = json.dumps(s, indent=1)
        argv = argv[:10] + argv[10:]
    else:
        raise SystemExit(__doc__)
    out = argv[-1] if argv[-1].endswith((".md", ".json")) and len(argv) in (5, 11) else None
    if out:
        with open(out, "w") as fh:
            fh.write(text + "\n")
    print(text)


if __name__ == "__main__":
    main(sys.argv[1:])
