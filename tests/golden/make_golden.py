"""Write the oracle's expected values for the long GPU parity runs.

    python tests/golden/make_golden.py [case ...]

The cases run the FP64 oracle (``oracle/``) on seeded synthetic inputs from
``paper_2302_05804_amd.synth`` and store its iterates and log-likelihood trace
as ``tests/golden/<case>.npz``.  Nothing here comes from the GPU path.  Every
file also stores a SHA-256 of the inputs it was computed from, so that a test
can tell when the generator no longer reproduces them.

Cases (Sec. 2, Eq. (2); Eq. (3) for sr = 2):
  c3crop  the HSC-shaped recipe (33 frames, 43 x 43 Moffat PSFs, 1% masked as
          cosmic-ray streaks and bad columns) on a 272 x 200 crop: three tiles of
          128 rows (the last one ragged) by two of 128 columns (ragged), 100
          iterations from the flat start; x after 10, 50 and 100 iterations
          (binary32 for 10 and 50, binary64 for 100) and l(x^(k-1)), k = 1..100.
  sr2job  a super-resolution x2 job of the serving stream's kind: 4 frames of
          72 x 152 on a 144 x 304 latent grid (wider than two 128-column tiles,
          not a multiple of 128), 60 iterations from the flat start.
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

import oracle  # noqa: E402
from paper_2302_05804_amd import synth  # noqa: E402

CASES = {
    "c3crop": dict(recipe="c3", H=272, W=200, seed=3272, n_iter=100, snaps=(10, 50)),
    "sr2job": dict(recipe="c4", H=144, W=304, n=4, seed=4144, n_iter=60, snaps=(20,)),
}


def inputs(case: str):
    """The seeded problem of a case and its flat starting image (binary32)."""
    c = CASES[case]
    over = {k: c[k] for k in ("H", "W", "n") if k in c}
    p = synth.make_problem(c["recipe"], seed=c["seed"], **over)
    x0 = np.full(p.latent_shape, np.float32(oracle.flat_x0(p.y, p.v, p.sr)), np.float32)
    return p, x0


def input_digest(p) -> str:
    h = hashlib.sha256()
    for a in (p.y, p.v, p.psf):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def make(case: str) -> str:
    c = CASES[case]
    p, x0 = inputs(case)
    t0 = time.time()
    x = x0.astype(np.float64)
    done = 0
    snaps = {}
    trace = []
    for stop in list(c["snaps"]) + [c["n_iter"]]:
        x, tr, _ = oracle.run(p.y, p.v, p.psf, x, stop - done, sr=p.sr, trace=True)
        trace.append(tr)
        done = stop
        snaps[stop] = x.copy()
        print(f"{case}: {done} iterations, {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, f"{case}.npz")
    arrays = {f"x{k}": (v if k == c["n_iter"] else v.astype(np.float32)) for k, v in snaps.items()}
    np.savez_compressed(out, trace=np.concatenate(trace), x0=x0, digest=np.array(input_digest(p)),
                        **arrays)
    return out


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        print("wrote", make(name), flush=True)
