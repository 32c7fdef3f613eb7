"""Throughput of the heat-bath lattice Coulomb-energy estimator on one MI355X.

One step = one measured sweep of the whole path: both red-black half-sweeps
(Philox4x32-10 in registers, inverse-CDF Gaussian, 7-point update) over the
lattice, then the gather of X = sum q phi and Y = sum q^2 phi^2 over the
charges, O = X^2 - Y and its compensated accumulation into a bin.

Default workload: the largest lattice one GPU holds here, 768^3 sites (FP32 field 1.69 GiB),
1.1e6 charges (1e6 of +-1, 1e5 drawn from N(0, 0.5^2)), seeded synthetic
input (the paper's tests use synthetic charge placements only).

Prints one JSON line: whole-job site updates/s, the roofline of the dominant
kernel (the library's default sweep kernel for the box, or the autotuner's
pick with --variant tuned) from HIP events around its own launches on the
library's stream, the time to a 1% statistical error on E_N
(extrapolated from the measured binned error and the exact lattice energy
stored in tests/golden/exact_energies.json), the same sweep with FP16 field
storage, the 512-chain batched workload, a dense batch (256 chains of 64^3), the time to a 1% error on the 16^3
workload (256 batched chains against one chain) for comparison, and the CPU oracle
timed on a bounded sample of the same workload; with extras, also a coupled
FP32 / BF16 / FP16 comparison on the 384^3 Gaussian blob (bias of the 16-bit
chains and their cost per sweep), four charge sets sampled on one chain, the
paper's two accuracy figures (132 charge sets on one 128^3 chain), and the
charges moved off the lattice with force estimates.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "site updates/s + HBM GB/s; time to E_N at 1% stat error vs plain FP32 sweep"
HBM_PEAK_GBPS = 8000.0
# Vector ALU peak: 256 CUs x 128 lanes per clock x 2.4 GHz = 78.6e12 lane
# slots/s at the FP32 FMA rate (157.3 TFLOP/s at 2 flops per FMA).  Measured
# on gfx950, 32-bit integer ops (multiply, three-input xor, convert) issue at
# half that rate and v_log_f32 at a quarter, so they count 2 and 4 slots.
ALU_PEAK_TSLOTS = 256 * 128 * 2.4e9 / 1e12
# Algorithmic slots per site update: the stencil sum and update (5 adds + 1
# FMA = 6), the inverse-CDF noise (grid value: 2 integer ops = 4, scale and
# 1 - s^2: 2, log: 4, w and the degree-8 polynomial: 9, times s: 1 = 20)
# and a quarter of a Philox4x32-10 call (10 rounds x (2 multiplies + 2
# three-input xors) / 4 = 10 integer ops = 20).
ALU_SLOTS_PER_SITE = 6 + 20 + 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
EXACT_FILE = os.path.join(ROOT, "tests", "golden", "exact_energies.json")


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=500)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="largest_subdomain_768",
                   choices=["largest_subdomain_768", "large_neutral_256", "gaussian_blob_384",
                            "small_neutral_16"])
    p.add_argument("--storage", default="fp32", choices=["fp32", "bf16", "fp16", "bf16sr", "fp16sr"])
    p.add_argument("--variant", default="auto",
                   choices=["auto", "tuned", "quad", "generic", "zslab", "stream", "fused", "resident", "blocked"],
                   help="auto: the library's default kernel and tuning for the box; "
                        "tuned: the library's autotuner picks kernel, slab depth and tile")
    p.add_argument("--bin-size", type=int, default=None,
                   help="samples per bin of the headline estimate (default: a tenth of the samples, so that "
                        "the binned error exists)")
    p.add_argument("--therm", type=int, default=None,
                   help="thermalisation sweeps before the warmup (default: the workload recipe's)")
    p.add_argument("--no-extras", action="store_true", help="skip the FP16 and batched comparisons")
    p.add_argument("--planes", type=int, default=None, help="slab kernels: planes per workgroup")
    p.add_argument("--tile", type=int, default=-1, help="slab kernels: tile configuration (-1: library default)")
    p.add_argument("--xcd-order", type=int, default=None, choices=[0, 1, 2],
                   help="slab kernels' workgroup order over the XCDs: 0 as dealt, 1 a run of tiles per XCD, "
                        "2 a band of each slab's tiles per XCD (default: the library's)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a plain device copy of the workload's colour-array size (counter calibration)")
    p.add_argument("--kernel-reps", type=int, default=50,
                   help="sweeps timed for the per-kernel (half-sweep) duration")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--figures-sweeps", type=int, default=200000,
                   help="measured sweeps of the figures comparison (128^3, 132 charge sets)")
    p.add_argument("--precision-128", type=int, default=0, metavar="SWEEPS",
                   help="only the coupled precision comparison on a 128^3 Gaussian blob (7400 charges of +1, "
                        "sigma 16; 1e5 FP32 thermalisation sweeps) with SWEEPS sweeps per format")
    p.add_argument("--coupled-sweeps", type=int, default=100000,
                   help="sweeps per storage format of the coupled precision comparison")
    return p.parse_args()


# Device sources of each timed kernel: stored counters are valid while these
# are unchanged (host-side launch structs are not part of a kernel's code).
_COMMON_SOURCES = ["device_common.hpp", "erfinv_coeffs.h"]
KERNEL_SOURCES = {
    "sweep_blocked": ["blocked_sweep.hip", "lds_pipe.hpp"],
    "halfsweep_stream": ["stream_sweep.hip", "lds_pipe.hpp"],
    "halfsweep_zslab": ["sweep_kernels.hip"],
    "halfsweep_quad": ["sweep_kernels.hip"],
    "halfsweep_generic": ["sweep_kernels.hip"],
    "fused_sweep": ["fused_sweep.hip"],
    "resident_chain": ["batch_kernels.hip"],
}


def _code_only(text: str) -> str:
    """C++ source without comments and whitespace (the sources contain no
    string literal with a comment marker)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return "".join(text.split())


def sources_hash(kname: str) -> str:
    """Hash of the code (comments and whitespace removed) of the HIP sources a
    kernel is built from, to tell whether stored counters are stale."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1403_0711_amd", "csrc")
    for n in KERNEL_SOURCES.get(kname, []) + _COMMON_SOURCES:
        with open(os.path.join(csrc, n), encoding="utf-8") as f:
            h.update(n.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def stored_entry(kname: str, key: str):
    """The stored rocprofv3 --pmc record of a kernel configuration, if taken
    on the kernel's current sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(key)
    if not e or e.get("sources_hash") != sources_hash(kname):
        return None
    return e


def stored_traffic(kname: str, key: str):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE and
    WRITE_SIZE, scaled by a copy kernel of known size), if taken on the
    kernel's current sources."""
    e = stored_entry(kname, key)
    return e.get("bytes_per_launch") if e else None


def roofline(kname: str, V: int, launch_ms: float, gbps: float, bytes_per_launch: int, traffic, stored):
    """The dominant kernel against its ceiling.  The blocked sweep moves 4 B
    per FP32 site update (half the plain sweep's): it is bound by the vector
    ALU, reported in algorithmic slots per second with its HBM rate beside
    it; the other kernels are bound by HBM."""
    hbm = {"achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
           "bytes_per_launch": bytes_per_launch, "launch_ms": launch_ms, "traffic": traffic}
    if kname != "sweep_blocked":
        return {"bound": "hbm", "kernel": kname, **hbm}
    slots = ALU_SLOTS_PER_SITE * V / (launch_ms * 1e-3) / 1e12
    out = {"bound": "alu", "kernel": kname, "achieved": slots, "peak": ALU_PEAK_TSLOTS, "unit": "Tslot/s",
           "frac": slots / ALU_PEAK_TSLOTS, "slots_per_site_update": ALU_SLOTS_PER_SITE,
           "site_updates_per_launch": V, "launch_ms": launch_ms, "traffic": traffic, "hbm": hbm}
    if stored and "valu" in stored:
        out["valu_counters"] = stored["valu"]
    return out


def exact_energy(workload: str):
    try:
        with open(EXACT_FILE) as f:
            return json.load(f)[workload]["E_lat"]
    except (OSError, ValueError, KeyError):
        return None


def time_to_1pct(t_run_s: float, stderr: float, e_exact):
    """t_run (eps_run / 0.01)^2 with eps_run = binned stderr / |E_exact|:
    samples needed for a 1% relative error, at the measured cost per sample
    (the binned error already carries the autocorrelation)."""
    if e_exact is None or not math.isfinite(stderr) or e_exact == 0:
        return None
    eps = stderr / abs(e_exact)
    return {"seconds": t_run_s * (eps / 0.01) ** 2, "eps_run": eps, "E_exact": e_exact,
            "kind": "extrapolated"}


def kernel_roofline(lat, stream, V: int, esz: int, variant: str, reps: int, torch):
    """Average duration of the dominant sweep kernel, from HIP events around
    `reps` unmeasured sweeps on the library's stream, and its algorithmic
    bytes per launch."""
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if V <= (1 << 24):  # sweeps replayed from a captured graph: capture it before timing
        lat.thermalise(reps)
    ev0.record(stream)
    lat.thermalise(reps)
    ev1.record(stream)
    ev1.synchronize()
    sweep_ms = ev0.elapsed_time(ev1) / reps
    if variant == "fused":
        return sweep_ms, sweep_ms, 3 * (V // 2) * esz, "fused_sweep"  # read colour 1, write both colours
    if variant == "blocked":  # read colour 1, write colour 1 (colour 0 stays on chip)
        return sweep_ms, sweep_ms, 2 * (V // 2) * esz, "sweep_blocked"
    if variant == "resident":
        return sweep_ms, sweep_ms, 2 * (V // 2) * 2 * esz, "resident_chain"
    return sweep_ms, sweep_ms / 2.0, (V // 2) * 2 * esz, f"halfsweep_{variant}"  # read other colour, write own


def kernel_key(kname: str, lat_tuning: dict, workload: str, storage: str) -> str:
    """Key of the stored counters: kernel, slab planes and tile, workload, storage."""
    t = lat_tuning or {}
    return f"{kname}_p{t.get('planes', 0)}_t{t.get('tile', 0)}_{workload}_{storage}"


def fp16_comparison(cs, seed, steps, bin_size, torch, lattice, tuned: bool, storage: str = "fp16"):
    """The same workload with 16-bit field storage (FP16 or BF16; FP32
    arithmetic): per-step time after the workload's thermalisation-free
    warm-up, the library's default kernel for that storage."""
    lat = lattice.Lattice(cs.shape, storage, seed=seed)
    if tuned:
        lat.autotune(5)
    tune = lat.tuning()
    lat.set_charges(cs.xyz, cs.q)
    lat.sweep_and_measure(5, 1, bin_size)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep_and_measure(steps, 1, bin_size)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat.close()
    return {"ms_per_step": 1e3 * dt / steps, "site_updates_per_s": int(np.prod(cs.shape)) * steps / dt,
            "tuning": tune}


def batched_comparison(sweeps, torch, lattice, workloads):
    """512 chains (edges 24..64, 16..512 charges) in one persistent launch,
    the half-sweep form chosen per box by the batch autotuner.  Against the
    vector-ALU ceiling (the same algorithmic slots per site update as the
    single lattice), and against the bound of its largest chains: one
    workgroup sweeps a chain, so the launch lasts at least as long as a 64^3
    chain takes on one CU (reported as the workgroup's rate)."""
    chains = workloads.batched_chains(seed=0)
    b = lattice.Batch([c.shape for c in chains], "fp32", seed=0)
    for k, c in enumerate(chains):
        b.set_charges(k, c.xyz, c.q)
    n_ring = b.autotune(3)
    b.run(5, 10, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(0, sweeps, 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sites = sum(int(np.prod(c.shape)) for c in chains)
    b.close()
    rate = sites * sweeps / dt
    slots = ALU_SLOTS_PER_SITE * rate / 1e12
    return {"chains": len(chains), "sites": sites, "sweeps": sweeps, "seconds": dt, "site_updates_per_s": rate,
            "chains_on_the_lds_ring": n_ring,
            "roofline": {"bound": "alu", "achieved": slots, "peak": ALU_PEAK_TSLOTS, "unit": "Tslot/s",
                         "frac": slots / ALU_PEAK_TSLOTS},
            "largest_chain": {"edge": 64, "sites": 64 ** 3,
                              "sweep_time_bound_ms": 1e3 * dt / sweeps,
                              "one_workgroup_site_updates_per_s": 64 ** 3 * sweeps / dt}}


def dense_batch(sweeps, torch, lattice):
    """256 chains of 64^3 with no charges (1 MiB of FP32 field each, 256 MiB
    in all: the size from which a batch sweeps through the LDS ring)."""
    shapes = [(64, 64, 64)] * 256
    b = lattice.Batch(shapes, "fp32", seed=0)
    b.run(2, 10, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(0, sweeps, 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    sites = 256 * 64 ** 3
    return {"chains": 256, "edge": 64, "sweeps": sweeps, "ms_per_sweep": 1e3 * dt / sweeps,
            "site_updates_per_s": sites * sweeps / dt}


def calibrate_copy(spec, torch):
    """A plain copy of one colour array of the workload (read n*4 B, write
    n*4 B, n = V/2 FP32 values), three times: run under rocprofv3 --pmc, its
    FETCH_SIZE / WRITE_SIZE per dispatch against the known bytes give the
    counters' scale factors."""
    cs = spec["make"]()
    n = int(np.prod(cs.shape)) // 2
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": n * 4, "calibrate_copy_bytes_written": n * 4}), flush=True)


def binning_curve(series: np.ndarray):
    """Standard error of the mean of a correlated series from blocks of
    1, 2, 4, ... samples (at least 16 blocks): the plateau is the error with
    the autocorrelation included; tau_int = (plateau / naive)^2 / 2."""
    out = []
    b = 1
    while len(series) // b >= 16:
        n = len(series) // b
        m = series[: n * b].reshape(n, b).mean(axis=1)
        out.append((b, float(m.std(ddof=1) / math.sqrt(n))))
        b *= 2
    return out


def tau_and_error(series: np.ndarray):
    """The binning curve's largest error (its plateau, or a lower bound when
    the series is shorter than a few autocorrelation times) and tau_int."""
    curve = binning_curve(series)
    if not curve:
        return None, None, curve
    err = max(e for _, e in curve)
    return err, 0.5 * (err / curve[0][1]) ** 2, curve


def precision_coupled(sweeps, torch, lattice, workloads, therm=40000, small=None):
    """Reduced-precision storage at equal accuracy, on the 384^3 Gaussian blob
    (2e5 charges of +1).  One FP32 chain is thermalised (`therm` sweeps from
    phi = 0, about 5 e-folds of the slowest mode's variance); its field is the
    common start of an FP32 chain and of BF16 and FP16 chains, each rounded
    to nearest even and stochastically, on one Philox stream (same seed and
    chain id; the 16-bit copies round it), one sample per sweep.  The chains move together, so the per-sweep difference of a 16-bit
    chain's sample from the FP32 chain's measures its bias with an error far
    below the chains' own statistical error; each format also reports its
    mean against the exact E_lat with the binning curve's error (a lower
    bound when `sweeps` is only a few autocorrelation times, about 1300
    sweeps here).  Storage rounding shrinks stored values slightly toward
    zero (round-to-nearest-even cells are asymmetric at each power of two),
    a weak mass term whose effect on E_N grows as u^2 L^2: the BF16 chain's
    difference is several percent at 384^3, FP16's 64 times smaller.
    Stochastic rounding (the low byte of each site's Philox word) has no
    such shrinkage, so its chains' differences are zero within error.  With
    equal statistics, time to a given error scales as the cost per sweep.  Each
    format runs the sweep configuration the library's autotuner picks for it
    on this machine (kernel choice does not change the chain: every kernel
    computes the same update).  With `small` (a charge set), the same on
    that set instead (the 128^3 blob of --precision-128: long runs resolve
    biases of 1e-4 of E_N)."""
    name = "gaussian_blob_384" if small is None else "gaussian_blob_128"
    if small is None:
        spec = workloads.WORKLOADS[name]
        cs, seed, E = spec["make"](), spec["philox_seed"], exact_energy(name)
    else:
        cs, seed, E = small, 0, None
    out, series = {"workload": name, "sweeps": sweeps, "thermalisation_fp32": therm, "E_exact": E}, {}
    lat = lattice.Lattice(cs.shape, "fp32", seed=seed, chain_id=7)
    lat.thermalise(therm)
    phi0 = lat.get_field()
    lat.close()
    formats = ("fp32", "bf16", "fp16", "bf16sr", "fp16sr")
    for st in formats:
        lat = lattice.Lattice(cs.shape, st, seed=seed)
        lat.set_field(phi0)
        lat.set_charges(cs.xyz, cs.q)
        lat.autotune(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for done in range(0, sweeps, 200000):  # calls of at most 2e5 sweeps (progress lines)
            lat.sweep_and_measure(min(200000, sweeps - done), 1, 1)
            if sweeps > 200000:
                print(f"precision {name} {st}: {min(done + 200000, sweeps)} sweeps", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _, n, bins = lat.get_state()
        series[st] = bins[:, 0] - bins[:, 1]  # one sample per bin
        err, tau, _ = tau_and_error(series[st])
        mean = float(series[st].mean())
        out[st] = {"ms_per_sweep": 1e3 * dt / sweeps, "mean_O": mean, "stderr_binned": err, "tau_int": tau,
                   "tuning": lat.tuning()}
        if E:
            out[st]["rel_error_vs_exact"] = (mean - E) / E
            out[st]["rel_stderr"] = err / abs(E) if err is not None else None
        lat.close()
    del phi0
    out["sd_O"] = float(series["fp32"].std())
    for st in formats[1:]:
        # the difference of two coupled chains drifts in the slowest modes
        # (rounding errors accumulate there over their relaxation time, about
        # 1e4 sweeps on this machine): its error is the binning curve's largest,
        # a lower bound when the run is not much longer than that time
        d = series[st] - series["fp32"]
        err, tau, _ = tau_and_error(d)
        out[st].update({"bias_vs_fp32": float(d.mean()), "bias_stderr": err, "bias_tau_int": tau,
                        "bias_rel_to_exact": float(d.mean()) / E if E else None,
                        "bias_rel_to_fp32_mean": float(d.mean()) / out["fp32"]["mean_O"],
                        "sd_of_difference": float(d.std()),
                        "cost_vs_fp32": out[st]["ms_per_sweep"] / out["fp32"]["ms_per_sweep"]})
    return out


def time_to_1pct_256(torch, lattice, workloads, therm=2000, sweeps=4000):
    """Time to a 1% statistical error on E_N for the 256^3 chain with 65,536
    charges of +-1 (E_lat = 12.0, sd(O) about 2e4: billions of samples, so
    extrapolated): the library's default sweep, one sample per sweep after
    `therm` sweeps; the error of the mean from the binning curve (tau_int
    from its plateau), time = t_run (error / 1%)^2."""
    name = "large_neutral_256"
    spec = workloads.WORKLOADS[name]
    cs = spec["make"]()
    E = exact_energy(name)
    lat = lattice.Lattice(cs.shape, "fp32", seed=spec["philox_seed"])
    lat.set_charges(cs.xyz, cs.q)
    lat.thermalise(therm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep_and_measure(sweeps, 1, 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, _, bins = lat.get_state()
    tuning = lat.tuning()
    lat.close()
    O = bins[:, 0] - bins[:, 1]
    err, tau, curve = tau_and_error(O)
    out = {"workload": name, "thermalisation": therm, "sweeps": sweeps, "seconds_run": dt,
           "ms_per_sweep": 1e3 * dt / sweeps, "mean": float(O.mean()), "stderr": err, "tau_int": tau,
           "binning_curve": curve, "E_exact": E, "tuning": tuning}
    if E and err:
        out["time_to_1pct_s"] = dt * (err / (0.01 * abs(E))) ** 2
        out["kind"] = "extrapolated"
    return out


def batched_time_to_1pct(torch, lattice, workloads, therm=1000, sweeps=2000, bin_size=100, sample=32):
    """Time to 1% on the 512-chain batch (edges 24..64, 16..512 charges):
    all chains in one persistent launch against the same chains run one by
    one with the single-lattice library (the library's default sweep per
    box).  Both give each chain the same field and samples (same kernel
    arithmetic, same Philox streams), so their errors are equal and time to
    1% scales as wall time: t_run (error / 1%)^2 per chain, its median over
    the chains with an exact energy reported.  One by one is timed on every
    (512 / sample)-th chain and scaled to the 512."""
    chains = workloads.batched_chains(seed=0)
    with open(EXACT_FILE) as f:
        E = json.load(f).get("batched_512", {}).get("E_lat", [])
    b = lattice.Batch([c.shape for c in chains], "fp32", seed=0)
    for k, c in enumerate(chains):
        b.set_charges(k, c.xyz, c.q)
    b.run(therm, 0, bin_size)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(0, sweeps, bin_size)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ratios = []
    for k in range(min(len(E), len(chains))):
        m, se = b.energy_estimate(k)[:2]
        if E[k] and math.isfinite(se):
            ratios.append((se / (0.01 * abs(E[k]))) ** 2)
    b.close()
    step = max(1, len(chains) // sample)
    picked = list(range(0, len(chains), step))
    t0 = time.perf_counter()
    for k in picked:
        c = chains[k]
        lat = lattice.Lattice(c.shape, "fp32", seed=0, chain_id=k)
        lat.set_charges(c.xyz, c.q)
        lat.thermalise(therm)
        lat.sweep_and_measure(sweeps, 1, bin_size)
        lat.energy_estimate(allow_few_bins=True)
        lat.close()
    torch.cuda.synchronize()
    t_one = (time.perf_counter() - t0) * len(chains) / len(picked)
    t_batch_all = t_batch * (therm + sweeps) / sweeps  # the batch's thermalisation too, as one by one
    med = float(np.median(ratios)) if ratios else None
    out = {"chains": len(chains), "thermalisation": therm, "sweeps": sweeps, "bin_size": bin_size,
           "batched_seconds": t_batch_all, "one_by_one_seconds": t_one,
           "one_by_one_timed_chains": len(picked), "speedup": t_one / t_batch_all,
           "chains_with_exact_energy": len(ratios), "median_error_over_1pct_squared": med}
    if med:
        out["time_to_1pct_batched_s"] = t_batch_all * med
        out["time_to_1pct_one_by_one_s"] = t_one * med
        out["kind"] = "extrapolated"
    return out


def time_to_1pct_measured(torch, lattice, workloads, chains=256, call_s=5.0, cap_s=60.0):
    """Time to a 1% statistical error on E_N on the 16^3 neutral workload (8
    charges of +-1, E_lat = 0.029, so about 1e8 samples): `chains`
    independent chains of the same system in one batched launch, run until
    the error of their pooled mean (spread of the chains' means over
    sqrt(chains)) is below 1% of |E_exact|, timed by wall clock; against one
    chain (the plain sweep) timed over a bounded run and extrapolated as
    t_run (error / 1%)^2 from its binned error.  Both after 1e3
    thermalisation sweeps.  Sweeps go in calls of at most `call_s` seconds,
    sized from the rate measured so far, each reported on stderr."""
    name = "small_neutral_16"
    cs = workloads.WORKLOADS[name]["make"]()
    E = exact_energy(name)
    if not E:
        return None
    target, bin_size = 0.01 * abs(E), 1000

    lat = lattice.Lattice(cs.shape, "fp32", seed=0)
    lat.set_charges(cs.xyz, cs.q)
    lat.thermalise(1000)
    torch.cuda.synchronize()
    n_plain = 200 * bin_size
    t0 = time.perf_counter()
    lat.sweep_and_measure(n_plain, 1, bin_size)
    mean, se, _, _ = lat.energy_estimate()
    dt = time.perf_counter() - t0
    lat.close()
    plain = {"seconds_run": dt, "sweeps": n_plain, "mean": mean, "stderr": se,
             "time_to_1pct_s": dt * (se / target) ** 2, "kind": "extrapolated"}
    print(f"time to 1% (16^3): one chain, {n_plain} sweeps in {dt:.2f} s, stderr {se:.3g}",
          file=sys.stderr, flush=True)

    b = lattice.Batch([cs.shape] * chains, "fp32", seed=0, chain_ids=list(range(1, chains + 1)))
    for k in range(chains):
        b.set_charges(k, cs.xyz, cs.q)
    b.run(1000, 0, bin_size)
    torch.cuda.synchronize()

    def pooled():
        means = np.array([b.energy_estimate(k)[0] for k in range(chains)])
        return float(means.mean()), float(means.std(ddof=1) / math.sqrt(chains))

    t0 = time.perf_counter()
    done, step = 0, 2 * bin_size
    while True:
        t1 = time.perf_counter()
        b.run(0, step, bin_size)
        torch.cuda.synchronize()
        rate = step / (time.perf_counter() - t1)  # sweeps per chain and second
        done += step
        mean_b, se_b = pooled()
        print(f"time to 1% (16^3): {chains} chains, {done} sweeps each, stderr {se_b:.3g}",
              file=sys.stderr, flush=True)
        if se_b <= target or time.perf_counter() - t0 > cap_s:
            break
        need = int(done * (se_b / target) ** 2 * 1.1) - done
        step = max(bin_size, min(need, int(rate * call_s)) // bin_size * bin_size)
    batched = {"seconds": time.perf_counter() - t0, "sweeps_per_chain": done, "chains": chains, "mean": mean_b,
               "stderr": se_b, "reached": se_b <= target, "kind": "measured"}
    b.close()
    out = {"workload": name, "E_exact": E, "target_stderr": target, "plain": plain, "batched": batched}
    if batched["reached"]:
        out["batched_speedup"] = plain["time_to_1pct_s"] / batched["seconds"]
    return out


def charge_sets_comparison(cs, spec, workloads, steps, bin_size, torch, lattice, n_sets=4):
    """Several charge sets on one field chain: the workload's set plus
    n_sets - 1 more drawn with other seeds, every set sampled every sweep.
    Sample rate per set against the one-set run: the sweeps are shared."""
    sets = [cs] + [spec["make"](seed=s) for s in range(1, n_sets)]
    lat = lattice.Lattice(cs.shape, "fp32", seed=spec["philox_seed"])
    lat.set_charge_sets([(c.xyz, c.q) for c in sets])
    lat.sweep_and_measure(5, 1, bin_size)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep_and_measure(steps, 1, bin_size)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat.close()
    return {"sets": n_sets, "charges_per_set": [int(c.n) for c in sets], "ms_per_step": 1e3 * dt / steps,
            "set_samples_per_s": n_sets * steps / dt}


def figures_comparison(sweeps: int = 200000):
    """The paper's accuracy figures on the 128^3 box, all 132 charge sets
    (two-body scan, solid cubes N = 8 .. 32768) sampled on one chain: for the
    cubes, delta = |estimate - E| / |E| against the exact lattice energy and
    against the continuum energy of Eq. (s1) (the paper's reference, which
    the open box misses for large cubes) at each checkpoint M; for the pairs,
    the largest |estimate - E_lat| / stderr."""
    from paper_1403_0711_amd import figures

    with open(EXACT_FILE) as f:
        ex = json.load(f)
    res = figures.run(L=128, therm=min(5000, sweeps), sweeps=sweeps, bin_size=min(2000, max(sweeps // 10, 1)))
    n_pair = len(ex["fig1_pair_scan_128"]["E_lat"])
    e_lat = np.array(ex["fig1_pair_scan_128"]["E_lat"] + ex["fig2_cubes_128"]["E_lat"])
    e_s1 = np.array(ex["fig1_pair_scan_128"]["E_continuum"] + ex["fig2_cubes_128"]["E_continuum"])
    out = {"sweeps": sweeps, "sets": len(res["sets"]), "ms_per_sweep": res["ms_per_sweep"],
           "cube_N": ex["fig2_cubes_128"]["N"], "checkpoints": []}
    for row in res["checkpoints"]:
        mean, se = np.array(row["mean"]), np.array(row["stderr"])
        out["checkpoints"].append({
            "M": row["M"],
            "cube_delta_lattice": [float(v) for v in np.abs(mean[n_pair:] - e_lat[n_pair:]) / np.abs(e_lat[n_pair:])],
            "cube_delta_eq_s1": [float(v) for v in np.abs(mean[n_pair:] - e_s1[n_pair:]) / np.abs(e_s1[n_pair:])],
            "pair_max_abs_z": float(np.max(np.abs(mean[:n_pair] - e_lat[:n_pair]) / se[:n_pair]))})
    return out


def offlattice_comparison(cs, spec, steps, bin_size, torch, lattice):
    """The workload's charges moved off the lattice (each by a seeded uniform
    offset in [0, 1) per axis, kept in the box) with force estimates on:
    cost per step against the on-lattice step."""
    rng = np.random.default_rng(1)
    hi = np.array(cs.shape, dtype=np.float64) - 1.0
    r = np.minimum(cs.xyz + rng.uniform(size=cs.xyz.shape), hi)
    lat = lattice.Lattice(cs.shape, "fp32", seed=spec["philox_seed"])
    lat.set_offlattice_charges(r, cs.q, forces=True)
    lat.sweep_and_measure(5, 1, bin_size)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep_and_measure(steps, 1, bin_size)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g, se, n = lat.force_estimate()
    lat.close()
    return {"charges": int(cs.n), "forces": True, "ms_per_step": 1e3 * dt / steps,
            "force_samples": int(n), "median_force_stderr_rel": float(np.median(se / np.maximum(np.abs(g), 1e-30)))}


def copy_reference(n_bytes: int, torch, reps: int = 10):
    """A device-to-device copy of n_bytes (read n_bytes, write n_bytes), timed
    with HIP events: the practical ceiling for a kernel that streams one array
    into another."""
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    return {"bytes_read": n_bytes, "bytes_written": n_bytes, "ms": ms, "GBps": 2 * n_bytes / (ms * 1e-3) / 1e9}


def cpu_baseline(cs, storage: str, seed: int):
    """The CPU oracle on a bounded sample of the workload: one full sweep of
    the whole lattice plus one gather of all charges."""
    import oracle

    lib = oracle.load()
    ch = oracle.OracleChain(cs.shape, storage=storage, seed=seed)
    ch.set_charges(cs.xyz, cs.q)
    V = int(np.prod(cs.shape))
    cores = int(lib.orc_max_threads())
    t0 = time.perf_counter()
    ch.sweeps(1, 1)
    dt = time.perf_counter() - t0
    del ch
    # the same oracle on one thread, on a smaller box of the same kind (one
    # unmeasured sweep of 192^3, a few seconds)
    small = (192, 192, 192)
    lib.orc_set_threads(1)
    try:
        one = oracle.OracleChain(small, storage=storage, seed=seed)
        t1 = time.perf_counter()
        one.sweeps(1, 0)
        dt1 = time.perf_counter() - t1
    finally:
        lib.orc_set_threads(cores)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": V / dt, "unit": "site updates/s", "cores": cores, "host_cpu": model,
            "host_cpus_online": os.cpu_count(),
            "kind": "oracle",
            "sample": f"1 measured sweep of the full {cs.shape[0]}x{cs.shape[1]}x{cs.shape[2]} "
                      f"box with all {cs.n} charges ({dt:.1f} s)",
            "single_thread": {"value": int(np.prod(small)) / dt1, "unit": "site updates/s",
                              "sample": f"1 sweep of a {small[0]}^3 box on 1 thread ({dt1:.1f} s)"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only: the lattice is one GPU's "
                          "subdomain; multi-GPU sharding is not implemented"}))
        sys.exit(2)
    import torch

    from paper_1403_0711_amd import lattice, workloads

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    lattice.load_library()
    spec = workloads.WORKLOADS[args.workload]
    if args.calibrate_copy:
        calibrate_copy(spec, torch)
        return
    if args.precision_128:
        blob = workloads.gaussian_blob(seed=0, L=128, n=7400, sigma=16.0)
        print(json.dumps({"precision_coupled_128": precision_coupled(args.precision_128, torch, lattice, workloads,
                                                                     therm=100000, small=blob)}), flush=True)
        return
    cs = spec["make"]()
    seed = spec["philox_seed"]
    V = int(np.prod(cs.shape))
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    lat = lattice.Lattice(cs.shape, args.storage, seed=seed, chain_id=0, device=0, stream=stream)
    if args.variant == "tuned":
        lat.autotune(5)
    else:
        lat.set_variant(args.variant)
        if args.planes is not None or args.tile != -1 or args.xcd_order is not None:
            lat.set_tuning(args.planes or 0, args.tile, args.xcd_order)
    tuning = lat.tuning()  # what runs: library defaults or the autotuner's choice, resolved
    variant = tuning["variant"]
    lat.set_charges(cs.xyz, cs.q)
    # the workload's thermalisation (untimed; the chain starts from phi = 0),
    # enqueued right before the warmup: the GPU runs from the thermalisation
    # into the timed steps without an idle gap (after one, its clocks take
    # ~25 ms to settle and a short timed region would measure that)
    therm = spec["therm"] if args.therm is None else args.therm
    lat.thermalise(therm)

    # warmup: W measured sweeps (untimed).  Boxes of at most 2^24 sites run
    # their sweeps as replays of a captured hipGraph chunk (32 sweeps): the
    # warmup then covers two chunks, so that the one-off capture is not timed
    warmup = args.warmup if V > (1 << 24) else max(args.warmup, 64)
    bin_size = args.bin_size or max(1, (warmup + args.steps) // 10)
    lat.sweep_and_measure(warmup, 1, bin_size)
    torch.cuda.synchronize()

    # timed: exactly K steps
    t0 = time.perf_counter()
    lat.sweep_and_measure(args.steps, 1, bin_size)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = V * args.steps / elapsed

    esz = 4 if args.storage == "fp32" else 2
    sweep_ms, launch_ms, bytes_per_launch, kname = kernel_roofline(
        lat, stream, V, esz, variant, args.kernel_reps, torch)
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    measure_ms = max(ms_per_step - sweep_ms, 0.0)
    traffic = stored_traffic(kname, kernel_key(kname, tuning, args.workload, args.storage))

    m, se, M, nb = lat.energy_estimate(allow_few_bins=True)
    e_exact = exact_energy(args.workload)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else f"f32 arithmetic, {args.storage} storage",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": list(cs.shape), "charges": cs.n,
                   "storage": args.storage, "variant": variant, "tuning": tuning,
                   "measure_every": 1, "bin_size": bin_size, "thermalisation": therm,
                   "philox_seed": seed},
        "hbm_gbps": achieved,
        "sweep_ms": sweep_ms,
        "measure_ms": measure_ms,
        "samples": M,
        "estimate": {"mean": m, "stderr": se if math.isfinite(se) else None, "bins": nb,
                     "E_exact": e_exact},
        "time_to_1pct": time_to_1pct(ms_per_step * 1e-3 * M, se, e_exact),
        "roofline": roofline(kname, V, launch_ms, achieved, bytes_per_launch, traffic,
                             stored_entry(kname, kernel_key(kname, tuning, args.workload, args.storage))),
    }
    lat.close()
    del lat
    torch.cuda.synchronize()
    if not args.no_extras:
        try:
            out["copy_same_bytes"] = copy_reference(bytes_per_launch // 2, torch)
            out["copy_same_bytes"]["kernel_vs_copy"] = out["copy_same_bytes"]["ms"] / launch_ms
            if args.storage == "fp32":
                for st in ("fp16", "bf16", "fp16sr", "bf16sr"):
                    r = fp16_comparison(cs, seed, min(args.steps, 200), bin_size, torch, lattice,
                                        args.variant == "tuned", storage=st)
                    r["speedup_vs_fp32"] = ms_per_step / r["ms_per_step"]
                    out[f"{st}_storage"] = r
            out["batched_512"] = batched_comparison(200, torch, lattice, workloads)
            out["batched_256x64"] = dense_batch(100, torch, lattice)
            out["time_to_1pct_16"] = time_to_1pct_measured(torch, lattice, workloads)
            out["time_to_1pct_256"] = time_to_1pct_256(torch, lattice, workloads)
            out["time_to_1pct_batched_512"] = batched_time_to_1pct(torch, lattice, workloads)
            out["precision_coupled"] = precision_coupled(args.coupled_sweeps, torch, lattice, workloads)
            out["figures_128"] = figures_comparison(args.figures_sweeps)
            if args.storage == "fp32":
                sets = charge_sets_comparison(cs, spec, workloads, min(args.steps, 200), bin_size, torch,
                                              lattice)
                sets["set_samples_vs_one_set"] = sets["set_samples_per_s"] / (1e3 / ms_per_step)
                out["charge_sets"] = sets
                off = offlattice_comparison(cs, spec, min(args.steps, 200), bin_size, torch, lattice)
                off["cost_vs_on_lattice"] = off["ms_per_step"] / ms_per_step
                out["offlattice_forces"] = off
        except Exception as exc:  # comparisons must not hide the headline line
            out["extras_error"] = repr(exc)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cs, args.storage, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
