"""Write the FP64 oracle's heights of the 4-layer 512^2 crop (the [0:512,
0:512] window of the 4-layer workload's seeded 4096^2 fields, run as its
own periodic domain) at t = 10^4, 2 10^4 and 5 10^4 steps to
``film4_512_long.npz`` (test fixture for the long-horizon accuracy of the
storage formats; calls only ``oracle/`` and the seeded input generator).

Stored (FP64 unless noted):
  rows     row indices kept (every 8th row)
  t        checkpoint steps, int64 [3]
  h        h_i on the kept rows at each checkpoint, [3][N][len(rows)][nx]
  mass0    per-layer mass of the initial state
  mass     per-layer mass at each checkpoint, [3][N]

Run from the repository root: ``python tests/golden/make_film4_512_long.py``
(about 45 minutes on 8 host cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2409_16659_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "film4_512_long.npz")
CHECKPOINTS = (10_000, 20_000, 50_000)
CHUNK = 1000


def main():
    film, h0, _ = inputs.workload("film4_2d_512")
    o = oracle.Oracle(film)
    o.init(h0)
    mass0 = o.mass()
    rows = np.arange(0, film["ny"], 8)
    hs, masses = [], []
    t0 = time.perf_counter()
    for tc in CHECKPOINTS:
        while o.steps_done < tc:
            o.step(min(CHUNK, tc - o.steps_done))
            print(f"{o.steps_done} steps, {time.perf_counter() - t0:.0f} s", flush=True)
        h, _, _ = o.read()
        hs.append(np.ascontiguousarray(h[:, rows]))
        masses.append(o.mass())
    np.savez(OUT, rows=rows, t=np.array(CHECKPOINTS, dtype=np.int64), h=np.stack(hs), mass0=mass0,
             mass=np.stack(masses))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
