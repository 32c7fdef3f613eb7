"""Write exact_energies.json: the exact lattice energy E_lat of each named
synthetic workload, from the oracle's exact Green's-function routes only
(DST-I solve of q^T G q plus the heat-kernel diagonal; dense Cholesky for the
16^3 box), and of the charge sets of the paper's two accuracy figures on the
128^3 box (the two-body scan of Fig. 1, the solid cubes of Fig. 2), with the
continuum energy of Eq. (s1) beside them.
Run: python tests/golden/make_exact_energies.py [--skip-768] [--figures-only]
[--batched-only] (--figures-only and --batched-only keep the other entries of
an existing file)."""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402
from paper_1403_0711_amd import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_energies.json")


def figures(res):
    """Fig. 1: unit charges at the centre c = L/2 and at (nx, c, c), every nx
    != c; Fig. 2: solid cubes of side 2 .. 32 (N = 8 .. 32768) about the
    centre.  L = 128, Dirichlet box."""
    L = 128
    c = L // 2
    xs = [x for x in range(L) if x != c]
    e_lat, e_cont = [], []
    t = time.time()
    for x in xs:
        p = workloads.pair_scan(L=L, nx=x)
        e_lat.append(exact.energy_dst(p.shape, p.xyz, p.q))
        e_cont.append(exact.energy_continuum(p.xyz, p.q))
    res["fig1_pair_scan_128"] = {"route": "DST-I + heat-kernel diagonal", "nx": xs, "E_lat": e_lat,
                                 "E_continuum": e_cont, "seconds": round(time.time() - t, 1)}
    print("fig1", round(time.time() - t, 1), "s", flush=True)
    sides = [2, 4, 8, 16, 32]
    e_lat, e_cont = [], []
    for side in sides:
        t = time.time()
        cube = workloads.solid_cube(L=L, side=side)
        e_lat.append(exact.energy_dst(cube.shape, cube.xyz, cube.q))
        e_cont.append(exact.energy_continuum(cube.xyz, cube.q))
        print("fig2 side", side, e_lat[-1], e_cont[-1], round(time.time() - t, 1), "s", flush=True)
    res["fig2_cubes_128"] = {"route": "DST-I + heat-kernel diagonal", "side": sides,
                             "N": [s ** 3 for s in sides], "E_lat": e_lat, "E_continuum": e_cont}


def batched(res):
    """The 512 chains of the batched workload (edges 24 .. 64, 16 .. 512
    charges each), every chain."""
    t = time.time()
    chains = workloads.batched_chains(seed=0)
    res["batched_512"] = {"route": "DST-I + heat-kernel diagonal per chain",
                          "E_lat": [exact.energy_dst(ch.shape, ch.xyz, ch.q) for ch in chains],
                          "chains": "all 512, in order", "seconds": round(time.time() - t, 1)}
    print("batched_512", round(time.time() - t, 1), "s", flush=True)


def main():
    if "--batched-only" in sys.argv:
        with open(OUT) as f:
            res = json.load(f)
        batched(res)
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1)
        print("wrote", OUT)
        return
    if "--figures-only" in sys.argv:
        with open(OUT) as f:
            res = json.load(f)
        figures(res)
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1)
        print("wrote", OUT)
        return
    res = {"note": "E_lat = sum_{i != j} q_i q_j G(n_i, n_j), G = (-Delta_L)^{-1} on the Dirichlet box, "
                   "for the seed-0 charge sets of paper_1403_0711_amd.workloads; written by "
                   "tests/golden/make_exact_energies.py from oracle.exact only."}
    c = workloads.small_neutral(seed=0)
    res["small_neutral_16"] = {"route": "dense Cholesky", "E_lat": exact.energy_dense(c.shape, c.xyz, c.q),
                               "E_continuum": exact.energy_continuum(c.xyz, c.q)}
    for name, make in (("large_neutral_256", workloads.large_neutral),
                       ("gaussian_blob_384", workloads.gaussian_blob),
                       ("largest_subdomain_768", workloads.largest_subdomain)):
        if name.endswith("768") and "--skip-768" in sys.argv:
            continue
        t = time.time()
        c = make()
        e = exact.energy_dst(c.shape, c.xyz, c.q)
        res[name] = {"route": "DST-I + heat-kernel diagonal", "E_lat": e, "seconds": round(time.time() - t, 1)}
        print(name, e, round(time.time() - t, 1), "s", flush=True)
    batched(res)
    figures(res)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
