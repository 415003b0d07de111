"""Write the FP64 oracle's fitted coefficients for the large seeded workloads.

The oracle fit costs P(P+1)/2 (4w+1)^2 n FP64 multiply-adds for its lag sums
(3e11 at 4096^2 with w = 7, DK = 2): minutes of host time, too long to repeat
inside every GPU test run. This script -- which calls only ``datagen`` (the
seeded inputs) and ``oracle`` -- stores the coefficients once as text, with
the sha256 of the generated input arrays. The GPU tests regenerate the same
inputs, check the hashes, and compare against these values; if an input hash
differs (a different numpy build), the tests fit the oracle live instead.

Run from the repository root:  python tests/golden/make_oracle_fits.py [name ...]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import datagen  # noqa: E402
import oracle  # noqa: E402


def _c3():
    return datagen.config3()


def _mix6144():
    return datagen.star_pair(1000 + 6144, 6144, 6144, w=7, dk=2, db=2)


def _c4(n0, n1):
    return lambda: datagen.star_pair(100 + n0 + n1, n0, n1, w=5, dk=1, db=1)


# name -> (generator, w0, w1, dk, db, description)
WORKLOADS = {
    "c3_4096": (_c3, 7, 7, 2, 2, "datagen.config3(): 4096x4096 FP32, 40000 Moffat stars, w=7, DK=DB=2"),
    "mix_6144": (_mix6144, 7, 7, 2, 2,
                 "datagen.star_pair(1000 + 6144, 6144, 6144, w=7, dk=2, db=2): FP32, w=7, DK=DB=2"),
    "c4_2048x2048": (_c4(2048, 2048), 5, 5, 1, 1,
                     "datagen.star_pair(100 + 4096, 2048, 2048, w=5, dk=1, db=1): FP32, w=5, DK=DB=1"),
    "c4_2048x4096": (_c4(2048, 4096), 5, 5, 1, 1,
                     "datagen.star_pair(100 + 6144, 2048, 4096, w=5, dk=1, db=1): FP32, w=5, DK=DB=1"),
}


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def path_of(name: str) -> str:
    return os.path.join(HERE, f"oracle_fit_{name}.txt")


def read(name: str):
    """(r_sha256, s_sha256, coefficients) of a stored fit, or None."""
    try:
        lines = open(path_of(name)).read().splitlines()
    except OSError:
        return None
    meta = {}
    vals = []
    for ln in lines:
        if ln.startswith("#"):
            if ":" in ln:
                k, v = ln[1:].split(":", 1)
                meta[k.strip()] = v.strip()
        elif ln.strip():
            vals.append(float(ln))
    return meta.get("r_sha256"), meta.get("s_sha256"), np.array(vals)


def write(name: str) -> None:
    make, w0, w1, dk, db, desc = WORKLOADS[name]
    t = time.time()
    pair = make()
    r = pair.r.astype(np.float64)
    s = pair.s.astype(np.float64)
    t_gen = time.time() - t
    t = time.time()
    coef = oracle.fit(r, s, w0, w1, dk, db)
    t_fit = time.time() - t
    with open(path_of(name), "w") as f:
        f.write("# oracle.fit coefficients (FP64, pixel units, library unknown order)\n")
        f.write("# written by tests/golden/make_oracle_fits.py: calls datagen and oracle only\n")
        f.write(f"# workload: {desc}\n")
        f.write(f"# params: w0={w0} w1={w1} dk={dk} db={db} const_phot=0\n")
        f.write(f"# r_sha256: {sha256(pair.r)}\n")
        f.write(f"# s_sha256: {sha256(pair.s)}\n")
        f.write(f"# n_unknowns: {len(coef)}\n")
        for v in coef:
            f.write(f"{v:.17e}\n")
    print(f"{name}: generated in {t_gen:.1f}s, oracle fit in {t_fit:.1f}s "
          f"({oracle.num_threads()} threads)", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    for nm in names:
        write(nm)
