"""Write tests/golden/long_runs.json: oracle summaries of full-length runs.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``paper_1603_09577_amd.workloads``, which hold none of the method's
arithmetic).  For each case the oracle runs the whole step count in FP64 and
stores, at every snapshot:

* ``sum``, ``sumsq`` -- sum over all nodes of phi and phi^2,
* ``blocks``        -- means of phi over a coarse grid of equal blocks,
* ``vals``          -- phi at seeded sample nodes (flat C-order indices ``idx``).

The GPU tests compute the same summaries from their own runs and compare.

    python tests/golden/make_long_runs.py [--threads N] [--cases a,b]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
from paper_1603_09577_amd import workloads as W  # noqa: E402

NSAMPLES = 512


def cases():
    """name -> (spec, phi0, snapshots, block edge)"""
    spec2, phi2, T2 = W.nonlinear_2d(1024)
    spec3, phi3, T3 = W.d3q19_walls((64, 64, 64))
    spec4, phi4, T4 = W.d3q19_walls((128, 128, 128))
    spec5, phi5, T5 = W.nonlinear_2d_walls_rates(1024)
    spec6, phi6, T6 = W.d3q19_walls_source((128, 128, 128))
    spec7, phi7, _ = W.d3q19_walls((256, 256, 256))
    return {
        "nonlinear2d-1024": (spec2, phi2, (1, 10, 100, 1000, T2), 64),
        "d3q19-walls-64": (spec3, phi3, (1, 10, 100, 1000, T3), 16),
        "d3q19-walls-128": (spec4, phi4, (1, 10, 100, 1000, T4), 16),
        "nonlinear2d-1024-scheme-b": (dict(spec2, scheme="B"), phi2, (1, 10, 100, 1000, T2), 64),
        "nonlinear2d-1024-walls-rates": (spec5, phi5, (1, 10, 100, 1000, T5), 64),
        "d3q19-128-source": (spec6, phi6, (1, 10, 100, T6), 16),
        # the full 256^3 grid for the first 200 of its 2000 steps (the whole
        # run would take the host oracle hours; 128^3 covers the full length)
        "d3q19-walls-256": (spec7, phi7, (1, 10, 100, 200), 32),
    }


def block_means(field, edge):
    """Means over blocks of edge^d nodes (field axes divisible by edge)."""
    shp = []
    for n in field.shape:
        assert n % edge == 0
        shp += [n // edge, edge]
    return field.reshape(shp).mean(axis=tuple(range(1, 2 * field.ndim, 2)))


def summarize(field, edge, idx):
    f = np.asarray(field, dtype=np.float64)
    return {
        "sum": float(f.sum()),
        "sumsq": float((f * f).sum()),
        "blocks": block_means(f, edge).ravel().tolist(),
        "vals": f.ravel()[idx].tolist(),
    }


def sample_indices(nodes, seed=99):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(nodes, size=NSAMPLES, replace=False))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--cases", default="")
    args = ap.parse_args()
    out_path = os.path.join(HERE, "long_runs.json")
    data = json.load(open(out_path)) if os.path.exists(out_path) else {}
    want = set(c for c in args.cases.split(",") if c)
    for name, (spec, phi0, snaps, edge) in cases().items():
        if want and name not in want:
            continue
        p = orc.params_from_spec(spec)
        idx = sample_indices(phi0.size)
        t0 = time.time()
        _, got = orc.run(p, phi0, max(snaps), snapshots=snaps, nthreads=args.threads)
        print(f"{name}: {max(snaps)} steps in {time.time() - t0:.0f} s", flush=True)
        data[name] = {
            "shape": list(phi0.shape), "block_edge": edge, "idx": idx.tolist(),
            "snapshots": {str(s): summarize(got[s], edge, idx) for s in snaps},
        }
        with open(out_path, "w") as fh:
            json.dump(data, fh, separators=(",", ":"))


if __name__ == "__main__":
    main()
