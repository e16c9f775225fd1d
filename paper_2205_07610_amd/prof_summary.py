"""Kernel table of a rocprofv3 --kernel-trace run (its rocpd results database).

Usage (from the repository root):

    python -m paper_2205_07610_amd.prof_summary <run_results.db> [top]

Prints a markdown table of kernels by total time: calls, total, average and
largest duration (nanoseconds) and the share of the total, with kernel names
shortened to the function and template arguments.  Then, for each learned
call of the run (one feature launch, one band classification, the banded
rounds), the feature kernel's duration and the union of the packed banded
kernel's busy intervals: its classes run concurrently on several streams,
so their launch durations overlap.
"""
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = name.replace("void ", "").replace("asmi::(anonymous namespace)::", "")
    return re.sub(r"\(.*$", "", name)


def main(argv):
    if not argv:
        raise SystemExit(__doc__)
    top = int(argv[1]) if len(argv) > 1 else 30
    con = sqlite3.connect(argv[0])
    rows = {}
    for name, start, end in con.execute("select name, start, end from kernels"):
        k = short(name)
        d = int(end) - int(start)
        c, tot, mx = rows.get(k, (0, 0, 0))
        rows[k] = (c + 1, tot + d, max(mx, d))
    total = sum(v[1] for v in rows.values())
    print("| kernel | calls | total ns | average ns | max ns | % |")
    print("|---|---|---|---|---|---|")
    for k, (c, tot, mx) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:top]:
        print(f"| {k} | {c} | {tot:,} | {tot // c:,} | {mx:,} | {100.0 * tot / total:.2f} |")
    ks = sorted((int(s), int(e), short(n)) for n, s, e in con.execute("select name, start, end from kernels"))
    print()
    for i, (s0, e0, k) in enumerate(ks):
        if k != "features_kernel":
            continue
        # the call's launches: up to its second band classification (the
        # first is its own) or the next feature launch
        j, seen = i + 1, 0
        while j < len(ks) and ks[j][2] != "features_kernel":
            if ks[j][2].startswith("band_classify_kernel"):
                seen += 1
                if seen == 2:
                    break
            j += 1
        iv = sorted((s, e) for s, e, n in ks[i:j] if n.startswith("band_dp_i16_kernel"))
        busy, cur = 0, None
        for s, e in iv:
            if cur is None or s > cur[1]:
                busy += cur[1] - cur[0] if cur else 0
                cur = [s, e]
            else:
                cur[1] = max(cur[1], e)
        busy += cur[1] - cur[0] if cur else 0
        print(f"learned call at launch {i}: features {(e0 - s0) / 1e6:.2f} ms, packed banded kernel "
              f"{len(iv)} launches, busy {busy / 1e6:.2f} ms")


if __name__ == "__main__":
    main(sys.argv[1:])
