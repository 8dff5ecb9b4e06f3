"""Merge tuner record files into the shipped defaults (paper_1709_06350_amd/tuning_defaults.txt).

The record files come from separate processes that timed their candidates from scratch, e.g. on an
MI355X, three times:
    MR_TUNING_FILE=<out>/run<k>.txt MR_TUNING_DEFAULTS= python3 bench.py --no-cpu-baseline
For every key the choice made by most runs is kept (a tie goes to the earliest run), so one noisy
timing does not decide a shipped choice.

    python3 -m paper_1709_06350_amd.make_tuning_defaults out.txt run1.txt run2.txt run3.txt
"""
from __future__ import annotations

import collections
import sys


def read(path: str) -> dict[str, str]:
    out = {}
    for ln in open(path):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        key, _, vals = ln.rpartition("|")
        if key.count("|") == 4 and vals:
            out[key] = vals
    return out


def merge(paths: list[str]) -> dict[str, str]:
    runs = [read(p) for p in paths]
    keys = sorted(set().union(*runs))
    merged = {}
    for k in keys:
        votes = [r[k] for r in runs if k in r]
        counts = collections.Counter(votes)
        best = max(counts.values())
        merged[k] = next(v for v in votes if counts[v] == best)
    return merged


def main(argv: list[str]) -> None:
    out, paths = argv[0], argv[1:]
    merged = merge(paths)
    with open(out, "w") as f:
        f.write(f"# tuner choices shipped with libmr (majority of {len(paths)} runs that timed from scratch)\n")
        f.write("# kind|arch|device|compute units|n|values\n")
        for k, v in merged.items():
            f.write(f"{k}|{v}\n")


if __name__ == "__main__":
    main(sys.argv[1:])
