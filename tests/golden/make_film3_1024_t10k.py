"""Write the FP64 oracle's state of the 3-layer 1024^2 workload after 10^4
steps to ``film3_1024_t10k.npz`` (test fixture; calls only ``oracle/`` and
the seeded input generator).

Stored (all FP64):
  rows_h   row indices of the height rows kept (every 16th row)
  h        h_i on those rows, [N][len(rows_h)][nx]
  rows_u   row indices of the velocity rows kept (every 64th row)
  ux, uy   U_i on those rows, [N][len(rows_u)][nx]
  mass0    per-layer mass of the initial state
  mass     per-layer mass after the run
  steps    number of steps

Run from the repository root: ``python tests/golden/make_film3_1024_t10k.py``
(about 25 minutes on 8 host cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2409_16659_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "film3_1024_t10k.npz")
STEPS = 10_000
CHUNK = 500


def main():
    film, h0, _ = inputs.workload("film3_2d_1024")
    o = oracle.Oracle(film)
    o.init(h0)
    mass0 = o.mass()
    t0 = time.perf_counter()
    while o.steps_done < STEPS:
        o.step(min(CHUNK, STEPS - o.steps_done))
        print(f"{o.steps_done} steps, {time.perf_counter() - t0:.0f} s", flush=True)
    h, ux, uy = o.read()
    rows_h = np.arange(0, film["ny"], 16)
    rows_u = np.arange(0, film["ny"], 64)
    np.savez(OUT, rows_h=rows_h, h=np.ascontiguousarray(h[:, rows_h]), rows_u=rows_u,
             ux=np.ascontiguousarray(ux[:, rows_u]), uy=np.ascontiguousarray(uy[:, rows_u]),
             mass0=mass0, mass=o.mass(), steps=np.int64(STEPS))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
