"""Write exact_energies.json: the exact lattice energy E_lat of each named
synthetic workload, from the oracle's exact Green's-function routes only
(DST-I solve of q^T G q plus the heat-kernel diagonal; dense Cholesky for the
16^3 box).  Run: python tests/golden/make_exact_energies.py [--skip-768]."""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402
from paper_1403_0711_amd import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_energies.json")


def main():
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
    chains = workloads.batched_chains(seed=0)
    res["batched_512"] = {"route": "DST-I + heat-kernel diagonal per chain",
                          "E_lat": [exact.energy_dst(ch.shape, ch.xyz, ch.q) for ch in chains[:16]],
                          "chains": "first 16 of 512"}
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
