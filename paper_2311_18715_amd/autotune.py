"""Table of tuned streaming-pass launch shapes, and the command that fills it.

The library's ``odmd_autotune`` times the candidate launch shapes of the
pass for one size; this module keeps the winners in a JSON table keyed by
(GPU architecture, basis type, snapshot type, rank-cap bucket, n bucket,
objective) and hands them to ``ODMD(shape=...)``:

- n bucket: the nearest power of two (tuned at that n; a shape is a rule,
  rows per workgroup and a workgroup cap, so it carries over to any n of
  the bucket);
- rank-cap bucket: r_max rounded up to a multiple of 16 (tuned at it);
- objective: 'latency' (one stream, time per update) or 'throughput'
  (``THROUGHPUT_STREAMS`` handles of the size advanced by batched steps,
  time per step).

The table shipped beside this module was written by this command on an
MI355X; ``ODMD_SHAPE_TABLE`` names another file to read.  A shape fixes the
order of the pass's sums, so handles built from different tables agree to
rounding, not bit for bit.

    python -m paper_2311_18715_amd.autotune --out table.json --basis f32 \\
        --objective throughput --nexp 13-20 --rmax 16,32,48,64
"""
from __future__ import annotations

import argparse
import json
import math
import os

from . import odmd

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pass_shapes.json")
THROUGHPUT_STREAMS = 16
OBJECTIVES = ("latency", "throughput")


def n_bucket(n: int) -> int:
    """Exponent of the power of two nearest to n (in log scale)."""
    if n < 1:
        raise ValueError("n must be positive")
    return int(round(math.log2(n)))


def r_bucket(r_max: int) -> int:
    if not 1 <= r_max <= odmd.RMAX:
        raise ValueError("r_max out of range")
    return min(odmd.RMAX, (r_max + 15) // 16 * 16)


def key(arch: str, basis: str, io: str, r_max: int, n: int, objective: str) -> str:
    if objective not in OBJECTIVES:
        raise ValueError(f"objective must be one of {OBJECTIVES}")
    return f"{arch}/{basis}/{io}/r{r_bucket(r_max)}/n2^{n_bucket(n)}/{objective}"


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def load_table(path: str | None = None) -> dict:
    path = path or os.environ.get("ODMD_SHAPE_TABLE") or TABLE_PATH
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data.get("shapes", {})


def save_table(shapes: dict, path: str, meta: dict | None = None) -> None:
    body = {"shapes": dict(sorted(shapes.items()))}
    if meta:
        body["meta"] = meta
    with open(path, "w") as f:
        json.dump(body, f, indent=1)
        f.write("\n")


def _valid(entry) -> bool:
    try:
        t, r, c = entry["shape"]
    except (KeyError, TypeError, ValueError):
        return False
    return t in (256, 512) and 16 <= r <= (1 << 24) and r % 16 == 0 and 1 <= c <= 65536


def lookup(n: int, r_max: int, basis: str = "f64", io: str | None = None,
           objective: str = "latency", table: dict | None = None, arch: str | None = None):
    """Tuned (threads, rows_per_block, max_blocks) for the stream, or None.

    None means no entry: the caller keeps the library's default rule.
    """
    io = io or ("f32" if basis == "bf16" else basis)
    table = load_table() if table is None else table
    arch = arch or device_arch()
    entry = table.get(key(arch, basis, io, r_max, n, objective))
    if entry is None or not _valid(entry):
        return None
    return tuple(int(v) for v in entry["shape"])


def tune_bucket(n_exp: int, r_max: int, basis: str, io: str | None, objective: str) -> dict:
    """Run odmd_autotune at the bucket's representative size."""
    streams = 1 if objective == "latency" else THROUGHPUT_STREAMS
    shape, us_best, us_default = odmd.autotune(1 << n_exp, r_bucket(r_max), basis, io, streams)
    return {"shape": list(shape), "us_best": round(us_best, 3), "us_default": round(us_default, 3),
            "streams": streams}


def _parse_range(text: str) -> list[int]:
    out: list[int] = []
    for part in text.split(","):
        if "-" in part:
            a, b = part.split("-")
            out.extend(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True, help="JSON table to write (entries are merged)")
    ap.add_argument("--basis", default="f32", choices=("f64", "f32", "bf16"))
    ap.add_argument("--io", default=None, choices=(None, "f64", "f32"))
    ap.add_argument("--objective", default="throughput", choices=OBJECTIVES)
    ap.add_argument("--nexp", default="13-20", help="n buckets as exponents of two, e.g. 13-20")
    ap.add_argument("--rmax", default="16,32,48,64", help="rank-cap buckets")
    a = ap.parse_args(argv)
    io = a.io or ("f32" if a.basis == "bf16" else a.basis)
    import torch
    shapes = load_table(a.out) if os.path.exists(a.out) else {}
    arch = device_arch()
    meta = {"device": torch.cuda.get_device_name(), "arch": arch,
            "written_by": "python -m paper_2311_18715_amd.autotune",
            "rule": "tuned shape kept only if more than 2 % faster than the default"}
    for r in _parse_range(a.rmax):
        for e in _parse_range(a.nexp):
            k = key(arch, a.basis, io, r, 1 << e, a.objective)
            shapes[k] = tune_bucket(e, r, a.basis, io, a.objective)
            s = shapes[k]
            print(f"{k}: {tuple(s['shape'])} {s['us_best']} us (default {s['us_default']} us)",
                  flush=True)
            save_table(shapes, a.out, meta)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
