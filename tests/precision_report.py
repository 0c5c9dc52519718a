"""Accuracy of the reduced-precision storage formats against the FP64 oracle
over time, on the 512 x 512 crop of the 4-layer workload (the [0:512, 0:512]
window of its seeded 4096^2 fields, run as its own periodic domain).

For each format (FP64 and FP32; FP32 rest with IEEE-half or bfloat16 moving
populations; all-IEEE-half or all-bfloat16 deviations) and each time t it
prints, per layer, the relative L2 error of the heights
||h - h_ref|| / ||h_ref||, the same error relative to the perturbation
||h - h_ref|| / ||h_ref - mean(h_ref)||, and the relative mass change since
t = 0.  Up to --oracle-steps the oracle runs alongside; at 10^4, 2 10^4
and 5 10^4 steps the reference is the oracle's stored state
(tests/golden/film4_512_long.npz, every 8th row, written by
tests/golden/make_film4_512_long.py).

    python tests/precision_report.py [--oracle-steps 3000] [--long-steps 50000]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2409_16659_amd import inputs  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden", "film4_512_long.npz")


def errors(h, ref):
    out = []
    for i in range(h.shape[0]):
        d = np.linalg.norm(h[i] - ref[i])
        out.append((float(d / np.linalg.norm(ref[i])),
                    float(d / max(np.linalg.norm(ref[i] - ref[i].mean()), 1e-300))))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--oracle-steps", type=int, default=3000)
    ap.add_argument("--long-steps", type=int, default=50_000)
    args = ap.parse_args()

    import oracle
    from paper_2409_16659_amd import mlfilm

    mlfilm.load_library()
    film, h0, _ = inputs.workload("film4_2d_512")
    gold = np.load(GOLDEN)
    stored = {int(t): k for k, t in enumerate(gold["t"])}
    checkpoints = [t for t in (100, 300, 1000, 3000) if t <= args.oracle_steps]
    checkpoints += [t for t in sorted(stored) if t <= args.long_steps]
    precs = ["f64", "f32", "f16mix", "bf16mix", "f16", "bf16"]
    films = {p: mlfilm.Film(film, p, check_every=-1) for p in precs}
    for f in films.values():
        f.init(h0)
    m0 = {p: films[p].mass() for p in precs}
    o = oracle.Oracle(film)
    o.init(h0)
    mo0 = o.mass()
    rows_kept = gold["rows"]
    t = 0
    rows = []
    for tc in checkpoints:
        for f in films.values():
            f.step(tc - t)
        if tc in stored:
            ref_name, sel = "oracle (stored)", rows_kept
            ref = gold["h"][stored[tc]]
            mo = gold["mass"][stored[tc]]
        else:
            t0 = time.perf_counter()
            o.step(tc - o.steps_done)
            print(f"[report] oracle reached t={tc} ({time.perf_counter() - t0:.1f} s)", flush=True)
            ref_name, sel = "oracle", slice(None)
            ref, _, _ = o.read()
            mo = o.mass()
        t = tc
        for p in precs:
            h, _, _ = films[p].read()
            m = films[p].mass()
            e = errors(h[:, sel], ref)
            row = {"t": tc, "storage": p, "against": ref_name,
                   "l2": [a for a, _ in e], "l2_pert": [b for _, b in e],
                   "mass_drift": [float(abs(m[i] - m0[p][i]) / m0[p][i]) for i in range(len(m))],
                   "oracle_mass_drift": [float(abs(mo[i] - mo0[i]) / mo0[i]) for i in range(len(mo))]}
            rows.append(row)
            print(json.dumps(row), flush=True)
    print()
    print("| t | storage | vs | max rel L2 (h) | max L2 / perturbation | max mass drift |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['t']} | {r['storage']} | {r['against']} | {max(r['l2']):.2e} | "
              f"{max(r['l2_pert']):.2e} | {max(r['mass_drift']):.2e} |")


if __name__ == "__main__":
    main()
