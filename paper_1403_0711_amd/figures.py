"""The charge configurations of the paper's two accuracy figures, sampled on
one field chain with the library (several charge sets per chain).

Fig. 1 (two-body energy on an L = 128 box): unit charges at the centre and at
(nx, L/2, L/2) for every nx on the line.  Fig. 2 (error against the number of
samples M): solid cubes of N = 8 .. 32768 unit charges about the centre.  The
paper samples one configuration every 1000 sweeps; here every set is sampled
after every sweep of one chain, and the statistical error of each running
estimate comes from bins long against the chain's correlation time.

Usage: ``python -m paper_1403_0711_amd.figures --therm 5000 --sweeps 200000``
prints one JSON object: for every set and every checkpoint M, the running
mean of the samples and its binned error.
"""

from __future__ import annotations

import argparse
import json
import time

from . import workloads


def figure_sets(L: int = 128, cube_sides=(2, 4, 8, 16, 32)):
    """Charge sets of Figs. 1 and 2 on an L^3 box: (name, ChargeSet) pairs,
    the pair scan first (nx = 0 .. L-1 except the centre), then the cubes."""
    c = L // 2
    sets = [(f"pair_nx{x}", workloads.pair_scan(L=L, nx=x)) for x in range(L) if x != c]
    sets += [(f"cube_N{s ** 3}", workloads.solid_cube(L=L, side=s)) for s in cube_sides]
    return sets


def run(L: int = 128, therm: int = 5000, sweeps: int = 200000, bin_size: int = 2000, checkpoints=None,
        storage: str = "fp32", seed: int = 0, cube_sides=(2, 4, 8, 16, 32), progress=None):
    """Thermalise, then sample every set after every sweep; at each checkpoint
    (a number of samples, a multiple of bin_size) record every set's running
    mean, binned error and number of full bins; ``progress(row)`` is called
    with each checkpoint's record as it completes.  Returns a dict."""
    import torch

    from . import lattice

    sets = figure_sets(L, cube_sides)
    if checkpoints is None:
        checkpoints = [m for m in (10 * bin_size, 20 * bin_size, 50 * bin_size, 100 * bin_size) if m <= sweeps]
        if not checkpoints or checkpoints[-1] != sweeps:
            checkpoints.append(sweeps)
    checkpoints = sorted(int(m) for m in checkpoints)
    lat = lattice.Lattice((L, L, L), storage, seed=seed)
    lat.set_charge_sets([(cs.xyz, cs.q) for _, cs in sets])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.thermalise(therm)
    done = 0
    rows = []
    for m in checkpoints:
        lat.sweep_and_measure(m - done, 1, bin_size)
        done = m
        est = [lat.energy_estimate(allow_few_bins=True, charge_set=k) for k in range(len(sets))]
        rows.append({"M": m, "mean": [e[0] for e in est], "stderr": [e[1] for e in est],
                     "bins": est[0][3], "seconds": time.perf_counter() - t0})
        if progress:
            progress(rows[-1])
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    lat.close()
    return {"L": L, "storage": storage, "therm": therm, "sweeps": sweeps, "bin_size": bin_size,
            "sets": [name for name, _ in sets], "checkpoints": rows, "seconds": seconds,
            "ms_per_sweep": 1e3 * seconds / (therm + sweeps)}


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--L", type=int, default=128)
    p.add_argument("--therm", type=int, default=5000)
    p.add_argument("--sweeps", type=int, default=200000)
    p.add_argument("--bin-size", type=int, default=2000)
    p.add_argument("--storage", default="fp32", choices=["fp32", "bf16", "fp16"])
    p.add_argument("--checkpoints", type=str, default=None,
                   help="comma-separated sample counts (multiples of --bin-size); default: 10, 20, 50, 100 bins and the end")
    a = p.parse_args()
    cps = [int(float(v)) for v in a.checkpoints.split(",")] if a.checkpoints else None
    res = run(a.L, a.therm, a.sweeps, a.bin_size, checkpoints=cps, storage=a.storage,
              progress=lambda row: print(json.dumps({"checkpoint": row["M"], "seconds": row["seconds"]}), flush=True))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
