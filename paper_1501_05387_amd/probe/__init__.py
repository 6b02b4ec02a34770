"""Memory-rate probe of one MI355X (``libgfrprobe.so``, built from ``probe.hip``).

Measures the rates that bound the engine's kernels: random 4- and 8-byte
gathers and 4-byte atomics over tables sized like the traversal state
(0.5 MB: an R-MAT s22 bitmap, L2-resident; 16.8 MB: a distance array, inside
the 256 MB MALL; 513 MB: a column array, HBM), random distance rows of 64, 128 and
256 bytes read one wave per row (with and without an atomicMin on every
word; 128-byte rows also as 64 lanes x 2 bytes and two rows per wave
instruction), and a stream copy.  ``python -m paper_1501_05387_amd.probe --out F``
writes the figures as JSON and prints a table.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfrprobe.so")

KINDS = {"gather4": 0, "gather8": 1, "atomic4": 2, "row256": 3, "row256_atomic": 4, "row128": 5,
         "row128_atomic": 6, "copy": 7, "row128_u16": 8, "row128_pair": 9, "row64": 10,
         "row64_u8": 11, "row64_quad": 12, "row64_quad_atomic1": 13, "row256_pair": 14}

MB = 1 << 20
# (name, kind, table bytes, operations)
CASES = [
    ("gather4 0.5MB", "gather4", MB // 2, 1 << 28),
    ("gather4 16.8MB", "gather4", 16 * MB + 800 * 1024, 1 << 28),
    ("gather4 513MB", "gather4", 513 * MB, 1 << 27),
    ("gather8 32MB", "gather8", 32 * MB, 1 << 27),
    ("gather8 1GB", "gather8", 1024 * MB, 1 << 27),
    ("atomic4 16.8MB", "atomic4", 16 * MB + 800 * 1024, 1 << 26),
    ("atomic4 513MB", "atomic4", 513 * MB, 1 << 26),
    ("row256 1GB", "row256", 1024 * MB, 1 << 25),
    ("row256_atomic 1GB", "row256_atomic", 1024 * MB, 1 << 25),
    ("row128 512MB", "row128", 512 * MB, 1 << 25),
    ("row128_atomic 512MB", "row128_atomic", 512 * MB, 1 << 25),
    ("row128_u16 512MB", "row128_u16", 512 * MB, 1 << 25),
    ("row128_pair 512MB", "row128_pair", 512 * MB, 1 << 25),
    ("row64 256MB", "row64", 256 * MB, 1 << 25),
    ("row64_u8 256MB", "row64_u8", 256 * MB, 1 << 25),
    ("row64_u8 1GB", "row64_u8", 1024 * MB, 1 << 25),
    ("row64_quad 256MB", "row64_quad", 256 * MB, 1 << 26),
    ("row64_quad 1GB", "row64_quad", 1024 * MB, 1 << 26),
    ("row64_quad_atomic1 256MB", "row64_quad_atomic1", 256 * MB, 1 << 26),
    ("row256_pair 1GB", "row256_pair", 1024 * MB, 1 << 25),
    ("copy 1GB", "copy", 1024 * MB, 0),
]


def lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgfrprobe.so is not built; run `python -m paper_1501_05387_amd.build`")
    import torch  # noqa: F401  (one HIP runtime for the process, as for libgfr.so)
    L = ctypes.CDLL(LIB_PATH)
    L.probe_run.restype = ctypes.c_float
    L.probe_run.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    return L


def run(cases=CASES):
    L = lib()
    out = []
    for name, kind, nbytes, count in cases:
        ms = float(L.probe_run(KINDS[kind], nbytes, count))
        if ms <= 0:
            raise RuntimeError("probe %s failed" % name)
        if kind == "copy":
            rate, unit, gbs = 2 * nbytes / (ms * 1e-3) / 1e9, "GB/s (read + write)", 2 * nbytes / (ms * 1e-3) / 1e9
        else:
            rate = count / (ms * 1e-3) / 1e9
            per = {"gather4": 4, "gather8": 8, "atomic4": 4, "row256": 256, "row256_atomic": 256,
                   "row128": 128, "row128_atomic": 128, "row128_u16": 128, "row128_pair": 128,
                   "row64": 64, "row64_u8": 64, "row64_quad": 64, "row64_quad_atomic1": 64,
                   "row256_pair": 256}[kind]
            unit = "G rows/s" if kind.startswith("row") else "G ops/s"
            gbs = rate * per
        rec = {"case": name, "kind": kind, "table_bytes": nbytes, "ops": count, "ms": round(ms, 4),
               "rate": round(rate, 2), "unit": unit, "useful_GBs": round(gbs, 1)}
        print("%-22s %9.3f ms  %8.2f %-20s %8.1f GB/s useful" % (name, ms, rate, unit, gbs), flush=True)
        out.append(rec)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=None, help="JSON file for the figures")
    args = ap.parse_args()
    res = run()
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
