"""HBM traffic per kernel from two rocprofv3 PMC runs of bench.py.

Usage (from the repository root, after the FETCH_SIZE and WRITE_SIZE runs of
`bench.py --copy-reference`, whose CSV output went to <fetch_dir> and
<write_dir>):

    python -m paper_2205_07610_amd.pmc_traffic <fetch_dir> <write_dir> <workload_name> \
        "<workload description>" [--write]

Both counters read in KiB per dispatch.  Each is scaled by what it reads for
the 1 GiB device copy that `--copy-reference` launches (rocclr's copyBuffer
with a grid of 131072 threads): the factor that makes the copy read, and
write, exactly 1 GiB.  With --write, one JSON record per kernel group goes to
profiles/<group>_traffic.json, keyed by the kernel source's SHA-1 and the
workload name (and the runtime's routing source) so that bench.py reports
it only for the same sources and workload.  The unit the bytes cover is the one bench.py's roofline uses for
that kernel: for the banded and feature kernels all launches of one step,
for the full-DP kernels the full-DP step's one launch.
"""
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_GRID = "131072"

# group -> (kernel-name predicate, source file, which launches form one unit)
GROUPS = {
    "band32": (lambda k: k.startswith("band_dp_i32_kernel") and ", false," in k,
               "paper_2205_07610_amd/csrc/band_dp_i32.hip", "all"),
    "band16": (lambda k: k.startswith("band_dp_i16_kernel"),
               "paper_2205_07610_amd/csrc/band_dp_i16x2.hip", "all"),
    "features": (lambda k: k.startswith("features_kernel"),
                 "paper_2205_07610_amd/csrc/features.hip", "all"),
    "long": (lambda k: k.startswith("long_dp_i32_kernel"),
             "paper_2205_07610_amd/csrc/long_dp_i32.hip", "largest"),
    "long16": (lambda k: k.startswith("long_dp_i16_kernel"),
               "paper_2205_07610_amd/csrc/long_dp_i16x2.hip", "largest"),
    "full32": (lambda k: k.startswith("full_dp_i32_kernel"),
               "paper_2205_07610_amd/csrc/full_dp_i32.hip", "largest"),
    # the packed kernel, or its all-against-all form (the same source and
    # timing phase; a workload runs one of them)
    "full16": (lambda k: k.startswith("full_dp_i16_kernel") or k.startswith("all_vs_all_i16_kernel"),
               "paper_2205_07610_amd/csrc/full_dp_i16x2.hip", "largest"),
}


def short(name: str) -> str:
    name = name.replace("void ", "").replace("asmi::(anonymous namespace)::", "")
    return re.sub(r"\(.*$", "", name)


def load(d: str):
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        return list(csv.DictReader(f))


def copy_scale(rows) -> float:
    copies = [float(r["Counter_Value"]) for r in rows
              if r["Kernel_Name"] == "__amd_rocclr_copyBuffer" and r["Grid_Size"] == COPY_GRID][:3]
    if not copies:
        raise SystemExit("no 1 GiB reference copy in the counter run (bench.py --copy-reference)")
    return (1 << 30) / (sum(copies) / len(copies) * 1024)


def sha(path: str) -> str:
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


# The runtime's routing decides which pairs each kernel gets, so a record also
# holds the hash of the runtime source and the shared header.
ROUTING_SOURCES = ("paper_2205_07610_amd/csrc/runtime.hip", "paper_2205_07610_amd/csrc/internal.h")


def routing_sha() -> str:
    h = hashlib.sha1()
    for path in ROUTING_SOURCES:
        with open(os.path.join(ROOT, path), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def summarise(fetch_dir, write_dir, workload_name, workload_desc):
    F, W = load(fetch_dir), load(write_dir)
    sf, sw = copy_scale(F), copy_scale(W)

    def rows_of(R, pred):
        return sorted(((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in R
                       if pred(short(r["Kernel_Name"]))), key=lambda x: x[0])

    # bench.py times the full DP, then the learned path, then the fixed-band
    # comparison.  The timed learned step starts with the first feature
    # launch after the full-DP step's wavefront launch (the largest
    # wavefront launch of the run, 32-bit or packed; earlier launches belong
    # to training and its diagnostics) and ends before the next call's band
    # classification (the step itself classifies once).
    def step_window(R):
        long_rows = rows_of(R, GROUPS["long"][0]) + rows_of(R, GROUPS["long16"][0])
        after = max(long_rows, key=lambda x: x[1])[0] if long_rows else -1
        feats = [d for d, _ in rows_of(R, GROUPS["features"][0]) if d > after]
        start = feats[0] if feats else after + 1
        classify = [d for d, _ in rows_of(R, lambda k: k.startswith("band_classify_kernel")) if d > start]
        return start, (classify[1] if len(classify) > 1 else float("inf"))

    # each pass's own window (launches after the learned step, such as the
    # fixed-band comparison chosen by timing, may differ between the passes)
    win_f, win_w = step_window(F), step_window(W)
    out = {}
    for g, (pred, src, unit) in GROUPS.items():
        fr, wr = rows_of(F, pred), rows_of(W, pred)
        if not fr or not wr:
            continue
        if unit == "largest":   # the full-DP step's launch is the largest of the run
            i = max(range(len(fr)), key=lambda k: fr[k][1])
            j = max(range(len(wr)), key=lambda k: wr[k][1])
            fr, wr = [fr[i]], [wr[j]]
            note = "unit: the full-DP step's launch (largest of the run)"
        else:
            fr = [x for x in fr if win_f[0] <= x[0] < win_f[1]]
            wr = [x for x in wr if win_w[0] <= x[0] < win_w[1]]
            note = "unit: all launches of the one timed learned step (every class and round)"
        if not fr or len(fr) != len(wr):
            continue
        n = len(fr)
        fb = sum(x[1] for x in fr) * 1024 * sf
        wb = sum(x[1] for x in wr) * 1024 * sw
        out[g] = {"kernel": g, "source": src, "source_sha": sha(src), "routing_sha": routing_sha(),
                  "launches": n, "note": note,
                  "fetch_bytes": fb, "write_bytes": wb, "bytes_per_unit": fb + wb,
                  "fetch_scale": round(sf, 4), "write_scale": round(sw, 4),
                  "workload": workload_desc, "workload_name": workload_name}
    return out


def main(argv):
    if len(argv) < 4:
        raise SystemExit(__doc__)
    recs = summarise(argv[0], argv[1], argv[2], argv[3])
    for g, rec in recs.items():
        print(g, json.dumps(rec))
        if "--write" in argv:
            with open(os.path.join(ROOT, "profiles", f"{g}_traffic.json"), "w") as f:
                json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
