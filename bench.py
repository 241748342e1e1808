"""Throughput of the CCD sweep on one MI355X.

Workload: pure neutron matter, N = 66, plane waves with n^2 <= 20 (778 states),
Minnesota interaction, the ten densities 0.02, 0.04, ..., 0.20 fm^-3 as one
batch, FP64 contractions, linear mixing 0.5, started from the MBPT2 amplitudes.
One step = one Jacobi sweep of all ten solves (every term of eq. ccd3).

value = CCD iterations per second, counting one iteration per solve per sweep
(10 per step).  Inputs are resident in HBM before the timed region.  Per-kernel
durations come from HIP events recorded by the library on its own stream during
a second, identical region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DENSITIES = [round(0.02 * (k + 1), 2) for k in range(10)]
N, NMAX2, MIXING = 66, 20, 0.5

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1611_06765_amd", "csrc", "ccd_device.hip")


def measured_traffic(family):
    """HBM bytes per launch of a kernel family from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (scaled by a plain copy of known size), or
    None if the kernel source changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha or rec.get("kernel_family") != family:
        return None
    return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0


def cpu_baseline(budget_s=20.0):
    """The oracle (intermediates form, fourth index deduced) timed on the host
    cores: one density of the same workload, sweeps until the budget is spent."""
    from oracle import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    p = oracle.PNM(N, NMAX2, 0.16)
    o3 = oracle.O3(p)
    t0 = time.perf_counter()
    sweeps = 0
    while True:
        o3.sweep(MIXING)
        sweeps += 1
        el = time.perf_counter() - t0
        if el > budget_s or sweeps >= 50:
            break
    return {"value": sweeps / el, "unit": "CCD iterations/s", "cores": threads, "kind": "oracle",
            "sample": f"{sweeps} sweeps of one solve (N=66, n^2<=20, rho=0.16, mixing 0.5) "
                      f"in {el:.1f} s, OpenMP threads={threads}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "see DESIGN.md for how the sweep would shard", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1611_06765_amd import ccd

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    ctx = ccd.Context([ccd.problem(N, NMAX2, r) for r in DENSITIES], stream=stream.cuda_stream)
    ctx.bind(dev)
    info = ctx.info(0)
    nsolve = len(DENSITIES)

    if args.copy_probe:
        x = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    ctx.iterate(mixing=MIXING, tol=0.0, max_iter=max(1, args.warmup))
    torch.cuda.synchronize()

    # timed region
    t0 = time.perf_counter()
    ctx.iterate(mixing=MIXING, tol=0.0, max_iter=args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el * 1e3 / args.steps

    # identical region with per-kernel HIP events on the library's stream
    ctx.set_timing(True)
    ctx.kernel_times(reset=True)
    t1 = time.perf_counter()
    ctx.iterate(mixing=MIXING, tol=0.0, max_iter=args.steps)
    torch.cuda.synchronize()
    el_ev = time.perf_counter() - t1
    kt = ctx.kernel_times(reset=True)
    ctx.set_timing(False)

    flops_exec = nsolve * (info["flops_pp"] + info["flops_hh"] + info["flops_ring"])
    flops_ord = nsolve * info["flops_ordered"]
    # per-step time of each kernel family (a family may launch several times a step)
    kernels = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
               for k, v in kt.items() if v[1]}
    total_ms = sum(v["ms_per_step"] for v in kernels.values())
    for v in kernels.values():
        v["share"] = v["ms_per_step"] / total_ms
    # useful FP64 flops of one step, per family (unordered pairs, as executed)
    fam_flops = {"ladder_update": nsolve * (info["flops_pp"] + info["flops_hh"] / 2),
                 "direct": nsolve * info["flops_hh"] / 2,
                 "ring": nsolve * info["flops_ring"]}
    ring_ms = sum(kernels.get(k, {}).get("ms_per_step", 0.0) for k in ("ring", "ring_small"))
    fam_ms = {"ladder_update": kernels.get("ladder_update", {}).get("ms_per_step", 0.0),
              "direct": kernels.get("direct", {}).get("ms_per_step", 0.0), "ring": ring_ms}
    for k in fam_ms:
        if fam_ms[k] > 0:
            kernels.setdefault(k, {})["tflops"] = fam_flops[k] / (fam_ms[k] * 1e-3) / 1e12
    dom = max(fam_ms, key=lambda k: fam_ms[k])
    achieved = fam_flops[dom] / (fam_ms[dom] * 1e-3) / 1e12
    roof = {"kernel": dom if dom != "ring" else "ring (ring_small + ring)", "bound": "mfma",
            "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(dom),
            "ms_per_step": fam_ms[dom], "flops_per_step": fam_flops[dom]}

    energies = [ctx.energy(p)[2] for p in range(nsolve)]
    out = {
        "metric": "CCD iterations/s + TFLOP/s, N=66 PNM; mixed/learned vs FP64 at 1e-6 rel E",
        "value": nsolve * args.steps / el,
        "unit": "CCD iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "PNM CCD sweep, N=66, n^2<=20 (778 states), Minnesota, "
                               "10 densities 0.02-0.20 fm^-3 batched, FP64, mixing 0.5",
                   "solves_per_step": nsolve, "states": info["n_states"],
                   "amplitudes_per_solve": info["n_amplitudes"]},
        "tflops_effective_ordered": flops_ord / (ms_step * 1e-3) / 1e12,
        "tflops_executed": flops_exec / (ms_step * 1e-3) / 1e12,
        "ms_per_step_with_events": el_ev * 1e3 / args.steps,
        "kernels": kernels,
        "roofline": roof,
        "e_corr_last": energies,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
