"""GEMM autotuner: measures the tile, split-K and schedule choices of every distinct GEMM
launch of a division on this device and writes the fastest per launch key as a JSON
table, which ``load`` installs (the launcher then uses it for matching launches and its
built-in choices elsewhere).

    python -m paper_2203_08900_amd.autotune --m 2048 --precision mixed --basis core \\
        --out tuning.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys


def tune(m: int, precision: str = "mixed", basis: str = "core", seed: int = 1) -> dict:
    """Tune one division of the Casida-like workload (the benchmark's generator) at half
    size m; returns the table with its provenance."""
    import torch
    from . import api, inputs

    a, b = inputs.casida_like(m, seed)
    A = torch.tensor(a, dtype=torch.float64, device="cuda")
    B = torch.tensor(b, dtype=torch.float64, device="cuda")
    api.set_gemm_tuning([])                     # measure against the built-in choices
    entries = api.autotune_divide(A, B, precision=precision, basis=basis)
    gain = sum((e["ms_default"] - e["ms"]) * e["launches"] for e in entries)
    return {"device": torch.cuda.get_device_name(0), "m": m, "precision": precision,
            "basis": basis, "seed": seed,
            "predicted_saving_ms_per_divide": gain,
            "entries": [e for e in entries
                        if (e["tile"], e["ksplit"], e["streamk"]) != (0, 0, 0)]}


def load(path: str) -> int:
    """Install the table of a JSON file written by ``tune``; returns its entry count."""
    from . import api
    with open(path) as f:
        table = json.load(f)
    api.set_gemm_tuning(table["entries"])
    return len(table["entries"])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--m", type=int, default=2048)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--basis", default="core")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    table = tune(args.m, args.precision, args.basis)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"{len(table['entries'])} launch keys, predicted saving "
          f"{table['predicted_saving_ms_per_divide']:.3f} ms per divide -> {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
