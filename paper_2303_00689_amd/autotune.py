"""GEMM tile autotuner: times both kernel families of the Fermi and response
chains over a grid of orders, per arithmetic and output kind, and writes the
tile table the binding installs with the library (xlbomd_set_tile_table).

    python -m paper_2303_00689_amd.autotune [--out PATH] [--reps K]

For each (precision, output kind) and each order n of the grid, every family
that can run n is timed (FP64: small, large and compact tiles, large needing
n % 16 == 0; the splits: small, large and medium tiles, large needing
n % 32 == 0 and medium n % 4 == 0 (FP16x3 n % 32 == 0); large and medium
tiles n >= 128), and the
fastest is kept; runs of equal choices merge into one row covering (previous n, n].
Orders between grid points take the next grid point's row; orders a row's
family cannot run, and orders past the grid, take the library's built-in rule.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2303_00689_amd import binding  # noqa: E402

PRECS = {0: "fp64", 1: "bf16x3", 2: "bf16x6", 3: "fp16x3"}
# the ensemble's orbital counts (4 x 20..300 atoms) in steps of 32, then the
# larger single systems up to 4096
GRID = list(range(128, 1281, 32)) + [1536, 2048, 2560, 3072, 3360, 4096]


def tune(reps: int, grid=GRID, log=print):
    rows, timings = [], []
    for prec, pname in PRECS.items():
        for sym in (0, 1):
            choice = []
            fams = {"small": binding.GEMM_SMALL, "large": binding.GEMM_LARGE, "compact": binding.GEMM_COMPACT}
            if prec in (1, 2, 3):
                fams["medium"] = binding.GEMM_MEDIUM
            for n in grid:
                t = {name: binding.time_gemm(n, prec, sym, f, reps) for name, f in fams.items()}
                # the fastest family that can run n (small always can); ties keep the smaller tiles
                best = min((v, k) for k, v in t.items() if v is not None)[1]
                fam = fams[best]
                choice.append((n, fam))
                timings.append({"prec": pname, "sym": sym, "n": n, **{f"{k}_us": v for k, v in t.items()},
                                "family": fam})
            log(f"{pname} sym={sym}: " + " ".join(f"{n}:{'sLMC'[f - 1]}" for n, f in choice))
            # merge runs of one family into rows covering (previous n_max, n_max]
            for k, (n, fam) in enumerate(choice):
                if k + 1 < len(choice) and choice[k + 1][1] == fam:
                    continue
                rows.append([prec, sym, n, fam])
    return rows, timings


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=binding.TILE_TABLE_PATH)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    os.environ["XLBOMD_TILE_TABLE"] = "none"   # time the families, not an older table
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("autotune needs a GPU")
    t = time.perf_counter()
    rows, timings = tune(args.reps)
    if len(rows) > binding.TILE_TABLE_MAX:
        raise SystemExit(f"{len(rows)} rows exceed the table's {binding.TILE_TABLE_MAX}")
    out = {"device": torch.cuda.get_device_name(0), "reps": args.reps,
           "seconds": time.perf_counter() - t,
           "rows_format": "[prec (0 FP64, 1 BF16x3, 2 BF16x6, 3 FP16x3), sym, n_max, family (1 small, 2 large, "
                          "3 medium, 4 compact)]",
           "rows": rows, "timings": timings}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {len(rows)} rows to {args.out} ({out['seconds']:.1f} s)")


if __name__ == "__main__":
    main()
