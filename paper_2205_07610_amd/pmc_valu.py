"""VALU issue and busy fractions per kernel from one rocprofv3 PMC run of bench.py.

Usage (from the repository root):

    rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_INSTS_LDS \
        SQ_INSTS_SALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE --output-format csv \
        -d <dir> -o run -- python3 bench.py --workload <w> --steps 1 --warmup 0 \
        --no-cpu-baseline > <bench_json>
    python -m paper_2205_07610_amd.pmc_valu <dir> <bench_json> <workload_name> [--write]

rocprofv3 reports every counter of a dispatch summed over its hardware
instances (shader engines, XCDs).  Per kernel group (the groups and the
launches that form one unit are those of pmc_traffic: all launches of the
timed learned step for the banded and feature kernels, the largest launch
for the full-DP kernels):

  gpu_cycles   = GRBM_GUI_ACTIVE / 8           (the 8 XCDs count the same cycles)
  issue_frac   = 4 * SQ_INSTS_VALU / (1024 * gpu_cycles)
                 a wave64 VALU instruction holds one of the 1024 SIMDs for 4
                 cycles, so this is the share of SIMD cycles that issued VALU
                 work: the measured counterpart of the algorithmic fraction
  busy_frac    = SQ_ACTIVE_INST_VALU / (256 * gpu_cycles)
                 (the VALUBusy expression; the counter is in quad-cycles
                 summed over a CU's 4 SIMDs)
  lane_util    = SQ_THREAD_CYCLES_VALU / (64 * SQ_ACTIVE_INST_VALU)  (the VALUUtilization expression)
  insts_per_cell = 64 * SQ_INSTS_VALU / cells  (lane-instructions per DP cell;
                 a packed 16-bit instruction covers two cells per lane)

`cells` comes from the bench JSON line of the same run (the cells the
kernel's unit computed).  With --write, one record per group goes to
profiles/<group>_valu_<workload_name>.json, keyed like the traffic records by the kernel
source, the routing sources and the workload, so bench.py reports it only
for the same build and workload.
"""
import csv
import json
import os
import sys

from paper_2205_07610_amd.pmc_traffic import GROUPS, ROOT, routing_sha, sha, short

COUNTERS = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_INSTS_LDS",
            "SQ_INSTS_SALU", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")
N_XCD = 8
N_SIMD = 1024
N_CU = 256


def load(d: str):
    """{dispatch id: (kernel short name, {counter: value})}."""
    out = {}
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            did = int(r["Dispatch_Id"])
            name, vals = out.setdefault(did, (short(r["Kernel_Name"]), {}))
            vals[r["Counter_Name"]] = vals.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def bench_cells(bench: dict):
    """Cells of each kernel group's unit, from the bench JSON line."""
    cells = {}
    for name, r in bench.get("roofline_band_kernels", {}).items():
        cells[name] = r.get("cells")
    for name, r in bench.get("full_dp", {}).get("roofline_per_kernel", {}).items():
        cells.setdefault(name, r.get("cells"))
    for name, r in bench.get("roofline_per_kernel", {}).items():
        cells.setdefault(name, r.get("cells"))
    return cells


def learned_step_window(D):
    """Dispatch ids of the timed learned step (as pmc_traffic selects them):
    from the first feature launch after the largest wavefront launch to the
    second band classification after it."""
    ids = sorted(D)
    longs = [i for i in ids if D[i][0].startswith(("long_dp_i32_kernel", "long_dp_i16_kernel"))]
    after = max(longs, key=lambda i: D[i][1].get("SQ_INSTS_VALU", 0)) if longs else -1
    feats = [i for i in ids if i > after and D[i][0].startswith("features_kernel")]
    start = feats[0] if feats else after + 1
    cls = [i for i in ids if i > start and D[i][0].startswith("band_classify_kernel")]
    end = cls[1] if len(cls) > 1 else float("inf")
    return start, end


def summarise(pmc_dir, bench_json, workload_name):
    D = load(pmc_dir)
    with open(bench_json) as f:
        lines = [ln for ln in f if ln.strip().startswith("{")]
    bench = json.loads(lines[-1])
    cells = bench_cells(bench)
    start, end = learned_step_window(D)
    out = {}
    for g, (pred, src, unit) in GROUPS.items():
        sel = [i for i in sorted(D) if pred(D[i][0])]
        if not sel:
            continue
        if unit == "largest":
            sel = [max(sel, key=lambda i: D[i][1].get("SQ_INSTS_VALU", 0))]
            note = "unit: the full-DP step's launch (largest of the run)"
        else:
            sel = [i for i in sel if start <= i < end]
            note = "unit: all launches of the one timed learned step (every class and round)"
        if not sel:
            continue
        tot = {c: sum(D[i][1].get(c, 0.0) for i in sel) for c in COUNTERS}
        cyc = tot["GRBM_GUI_ACTIVE"] / N_XCD
        rec = {"kernel": g, "source": src, "source_sha": sha(src), "routing_sha": routing_sha(),
               "workload_name": workload_name, "launches": len(sel), "note": note,
               "counters": {c: tot[c] for c in COUNTERS}, "gpu_cycles": cyc}
        if cyc > 0:
            rec["issue_frac"] = round(4 * tot["SQ_INSTS_VALU"] / (N_SIMD * cyc), 4)
            rec["busy_frac"] = round(tot["SQ_ACTIVE_INST_VALU"] / (N_CU * cyc), 4)
        if tot["SQ_ACTIVE_INST_VALU"] > 0:
            rec["lane_util"] = round(tot["SQ_THREAD_CYCLES_VALU"] / (64 * tot["SQ_ACTIVE_INST_VALU"]), 4)
        c = cells.get(g)
        if c:
            rec["cells"] = c
            rec["lane_insts_per_cell"] = round(64 * tot["SQ_INSTS_VALU"] / c, 4)
            rec["lds_insts_per_cell"] = round(64 * tot["SQ_INSTS_LDS"] / c, 4)
        out[g] = rec
    return out


def main(argv):
    if len(argv) < 3:
        raise SystemExit(__doc__)
    recs = summarise(argv[0], argv[1], argv[2])
    for g, rec in recs.items():
        print(g, json.dumps({k: v for k, v in rec.items() if k != "counters"}))
        if "--write" in argv:
            with open(os.path.join(ROOT, "profiles", f"{g}_valu_{argv[2]}.json"), "w") as f:
                json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
