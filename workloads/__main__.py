"""Prints the run parameters of the named workloads as JSON, one object per
line: `python -m workloads C2`, `python -m workloads all` (C1, C2, C3, C4's 64
halos, C5, BLK)."""
import json
import sys

from . import batch_c4, config


def main(argv):
    names = argv or ["all"]
    if names == ["all"]:
        names = ["C1", "C2", "C3", "C4", "C5", "BLK"]
    for name in names:
        cfg = dict(name="C4", halos=batch_c4()) if name == "C4" else config(name)
        print(json.dumps(cfg))


if __name__ == "__main__":
    main(sys.argv[1:])
