"""Throughput of the CCD sweep on one MI355X.

Workload: pure neutron matter, N = 66, plane waves with n^2 <= 20 (778 states),
Minnesota interaction, the ten densities 0.02, 0.04, ..., 0.20 fm^-3 as one
batch, FP64 contractions, linear mixing 0.5, started from the MBPT2 amplitudes.
One step = one Jacobi sweep of all ten solves (every term of eq. ccd3).

value = CCD iterations per second, counting one iteration per solve per sweep
(10 per step).  Inputs are resident in HBM before the timed region.  Per-kernel
durations come from HIP events recorded by the library on its own stream during
a second, identical region.  The same measurement at N=66, n^2<=36, rho=0.16
(one solve) is reported as c3_fp64.

Beside the throughput line, wall time to convergence of the three other forms
against the plain FP64 GPU path on the same GPU.  Every timed solve stops when
both |dE_n - dE_(n-1)| and the estimate |dE_n| r / (1 - r) of the remaining
change (r = |dE_n / dE_(n-1)|) are below CONV_REL |dE_n|, which leaves the
energy within 1e-6 of its limit.  Errors are reported against the CPU oracle's
converged energies committed under tests/golden/ (the twist form, which has no
oracle energies, against a GPU FP64 solve converged to 1e-10 MeV).  Both
sides of every comparison use the same flag-read interval and tuning policy:
  mixed_c3    N=66, n^2<=36, rho=0.16: FP32 or BF16 contractions, then FP64
              refinement;
  batched_c4  40 solves (N in {14,38,54,66} x 10 densities, seeded cutoffs
              12..36) in one context with tuned launch shapes,
              against the same 40 solved one after another in plain FP64;
  learned_c5  a network trained on converged N=66, n^2<=20 amplitudes at 24
              seeded densities warm-starts 16 held-out densities at n^2<=36,
              against the MBPT2 start;
  twist_averaged  N=66, n^2<=20, rho=0.16 under twisted boundary conditions on
              a 5-point Gauss-Legendre mesh per direction (125 solves) in one
              context, against the 125 solved one after another; twist-averaged
              T/N, HF/N and E/N beside the periodic box and infinite matter.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-forms]
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
CONV_REL = 1e-7          # relative stop threshold of every timed solve
STOP_RULE = 1            # with the geometric-tail estimate of the remaining change
REF_TOL = 1e-10          # MeV: the FP64 reference the errors are taken against
# Chunks of sweeps are issued eagerly with one flag read per chunk: on this
# ROCm, replaying a chunk as a HIP graph loses the concurrency of the sweep's
# forked streams (about 10% slower per sweep); graphs stay available.
GRAPH = False
C4_SEED = 20161121

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
TRAFFIC_C2 = "N=66, n^2<=20, 10 densities, FP64"
TRAFFIC_C3 = "N=66, n^2<=36, rho=0.16, FP64"
KERNEL_SRC = os.path.join(ROOT, "paper_1611_06765_amd", "csrc", "ccd_device.hip")


def source_digest(path=KERNEL_SRC):
    """sha256 of the sweep's device code with its comments and blank space
    removed, so that a comment-only edit keeps the counters valid and any code
    edit does not.  The set-up kernels (MBPT2 start, network warm start,
    features), which do not run in a sweep, and the host code after the device
    code are left out."""
    import hashlib
    import re
    src = open(path).read()
    a, b = src.find("\n// set-up kernels\n"), src.find("\n// sweep kernels\n")
    if 0 <= a < b:
        src = src[:a] + src[b:]
    h = src.find("\n// context\n")
    if h >= 0:
        src = src[:h]
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    src = re.sub(r"\s+", " ", src).strip()
    return hashlib.sha256(src.encode()).hexdigest()


def measured_traffic(family, workload):
    """HBM bytes per launch of a kernel family at a workload, from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by a plain copy of known
    size), or None if no record matches or the kernel code changed since the
    counters were taken."""
    try:
        recs = json.load(open(TRAFFIC_FILE))
        sha = source_digest()
    except (OSError, ValueError):
        return None
    for rec in recs if isinstance(recs, list) else [recs]:
        if (rec.get("source_sha256") == sha and rec.get("kernel_family") == family
                and rec.get("workload") == workload):
            return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0
    return None


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def oracle_energies(name):
    """Converged correlation energies {(N, nmax2, rho): E} that the CPU oracle
    wrote under tests/golden/ (the last sweep of a history file, or the E_CCD
    column of a converged-energy file); empty if the file is absent."""
    out = {}
    try:
        lines = open(os.path.join(GOLDEN_DIR, name)).read().splitlines()
    except OSError:
        return out
    for line in lines:
        f = line.split("#", 1)[0].split()
        if not f:
            continue
        key = (int(f[0]), int(f[1]), float(f[2]))
        out[key] = float(f[-1]) if "history" in name else float(f[6])
    return out


def _err_vs_oracle(energies, keys, ref):
    """Largest relative error of the energies against the oracle's, or None."""
    if not ref or any(k not in ref for k in keys):
        return None
    return max(_rel(e, ref[k]) for e, k in zip(energies, keys))


def ring_class_flops(ccd, ctx, p=0):
    """FP64 flops of one sweep's ring per kernel (ring_small and the pair
    blocks of padded order 32 .. 80), from problem p's cross channels."""
    ph = ctx.export_map(ccd.CCD_MAP_PH_CHANNELS, p).reshape(-1, 6)
    out = {}
    for x in range(len(ph)):
        y = int(ph[x, 5])
        if y < x:
            continue
        n, m = float(ph[x, 4]), float(ph[y, 4])
        nb = int(max(n, m))
        k = "ring_small" if nb <= 16 else "ring%d" % (16 * ((nb + 15) // 16))
        out[k] = out.get(k, 0.0) + (4 * n * m * m + (4 * m * n * n if y != x else 0.0))
    return out


def kernel_symbol(family, tuning, precision=0):
    """The kernel a family's single launch runs in the sweep, as rocprofv3
    names it (the ring variant follows the tuned waves per block)."""
    if family == "ladder":
        return "k_ladder64" if precision == 0 else "void k_ladder<%d>" % precision
    if family == "direct":
        return "void k_direct<%d>" % precision
    n16 = int(family[4:])
    k = (n16 - 32) // 16
    nwa, nwb = {32: (4, 2), 48: (9, 3), 64: (16, 8), 80: (16, 9)}[n16]
    return "void k_ringp<%d, %d, %d>" % (precision, n16, nwb if tuning[6 + k] else nwa)


def measure_sweeps(ccd, ctx, steps, warmup, tuning, ceilings, workload, precision=0):
    """Time `steps` FP64 sweeps of every problem of ctx (inputs resident), then
    the same sweeps again with the library's per-kernel HIP events on its own
    stream; per-family times, the useful FP64 flops of each contraction family
    and the roofline of the longest single launch."""
    import torch
    info = ctx.info(0)
    nsolve = ctx.n
    ctx.iterate(mixing=MIXING, tol=0.0, max_iter=max(1, warmup), precision=precision)
    ctx.set_tuning(tuning)
    ctx.iterate(mixing=MIXING, tol=0.0, max_iter=2, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.iterate(mixing=MIXING, tol=0.0, max_iter=steps, precision=precision)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.set_timing(True)
    ctx.kernel_times(reset=True)
    t1 = time.perf_counter()
    ctx.iterate(mixing=MIXING, tol=0.0, max_iter=steps, precision=precision)
    torch.cuda.synchronize()
    el_ev = time.perf_counter() - t1
    kt = ctx.kernel_times(reset=True)
    ctx.set_timing(False)
    # per-step time of each kernel family (a family may launch several times a step)
    kernels = {k: {"ms_per_step": v[0] / steps, "launches_per_step": v[1] / steps}
               for k, v in kt.items() if v[1]}
    total_ms = sum(v["ms_per_step"] for v in kernels.values())
    for v in kernels.values():
        v["share"] = v["ms_per_step"] / total_ms
    # useful FP64 flops of one step, per family (unordered pairs, as executed;
    # the pp ladder over momentum pairs); the ring per size class of its pair
    # blocks {Q, -Q}: 4 n m (n + m) for cross channels of n and m pairs
    ring_cls = ring_class_flops(ccd, ctx)
    fam_flops = {"ladder": nsolve * (info["flops_pp"] + info["flops_hh"] / 2),
                 "direct": nsolve * info["flops_hh"] / 2}
    for k, f in ring_cls.items():
        fam_flops[k] = nsolve * f
    fam_ms = {k: kernels.get(k, {}).get("ms_per_step", 0.0) for k in fam_flops}
    for k in fam_ms:
        if fam_ms[k] > 0:
            kernels[k]["tflops"] = fam_flops[k] / (fam_ms[k] * 1e-3) / 1e12
    # dominant kernel: the longest single launch among the contraction kernels
    per_launch = {k: fam_ms[k] / max(1.0, kernels[k]["launches_per_step"])
                  for k in fam_ms if fam_ms[k] > 0 and k != "ring_small"}
    dom = max(per_launch, key=lambda k: per_launch[k])
    achieved = fam_flops[dom] / (per_launch[dom] * 1e-3) / 1e12
    # the contraction precision's published dense peak: FP64 (the direct
    # product and the one-body terms stay FP64 in every mode), FP32 or BF16
    peak = PEAK_FP64_TFLOPS if precision == 0 or dom == "direct" else {1: 157.3, 2: 2500.0}[precision]
    roof = {"kernel": kernel_symbol(dom, tuning, precision), "bound": "mfma",
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": measured_traffic(dom, workload) if workload else None,
            "family": dom, "ms_per_launch": per_launch[dom], "flops_per_launch": fam_flops[dom]}
    # the same rate against what this part's matrix cores reach in a resident
    # loop of the instruction the kernel uses (context, not the peak)
    if precision == 0 or dom == "direct":
        meas = ceilings["fp64_mfma_4x4x4_tflops"] if dom == "ladder" else ceilings["fp64_mfma_16x16x4_tflops"]
    else:
        meas = ceilings.get("fp32_mfma_16x16x4_tflops" if precision == 1 else "bf16_mfma_16x16x32_tflops", 1.0)
    roof["measured_ceiling"] = meas
    roof["frac_of_measured_ceiling"] = achieved / meas
    return {"elapsed_s": el, "ms_per_step": el * 1e3 / steps, "ms_per_step_with_events": el_ev * 1e3 / steps,
            "kernels": kernels, "roofline": roof}


def sweep_rate_c3(ccd, stream, steps, warmup, ceilings, precision=0):
    """Sweeps of one solve at N=66, n^2<=36 (1850 states), rho=0.16 (FP64, or
    the given contraction precision), with its per-kernel times and the
    roofline of its longest launch (against the FP64 peak)."""
    c = ccd.Context([ccd.problem(66, 36, 0.16)], stream=stream).bind()
    info = c.info(0)
    m = measure_sweeps(ccd, c, steps, warmup, [0] * 10, ceilings, TRAFFIC_C3 if precision == 0 else None,
                       precision)
    c.close()
    fl = info["flops_pp"] + info["flops_hh"] + info["flops_ring"]
    return {"workload": "PNM N=66, n^2<=36 (1850 states), rho=0.16, %s, mixing 0.5, one solve"
                        % {0: "FP64", 1: "FP32 contractions", 2: "BF16 contractions"}[precision],
            "ccd_iterations_per_s": 1e3 / m["ms_per_step"], "ms_per_sweep": m["ms_per_step"],
            "tflops": fl / (m["ms_per_step"] * 1e-3) / 1e12,
            "context_tflops_ordered_pair_form": info["flops_ordered"] / (m["ms_per_step"] * 1e-3) / 1e12,
            "amplitudes": info["n_amplitudes"], "kernels": m["kernels"], "roofline": m["roofline"]}


def snm_rate(ccd, stream, steps, warmup):
    """Symmetric nuclear matter through the isospin path: A = 108 (54 protons,
    54 neutrons), n^2 <= 20 (1556 states), rho = 0.16, FP64, mixing 0.5: sweeps
    per second, the executed FP64 rate and the roofline of its longest launch
    (per-launch HIP events on the library's stream).  (At A = 76 and 132 the
    iteration diverges in this basis through the V_T channel.)"""
    import torch
    c = ccd.NMContext(ccd.nm_problem(108, 20, 0.16), stream=stream).bind()
    info = c.info()
    c.iterate(mixing=MIXING, max_iter=max(1, warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = c.iterate(mixing=MIXING, max_iter=steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    c.set_timing(True)
    c.kernel_times(reset=True)
    c.iterate(mixing=MIXING, max_iter=steps)
    kt = c.kernel_times(reset=True)
    c.set_timing(False)
    er, e2, ec = c.energy()
    c.close()
    kernels = {k: {"ms_per_sweep": v[0] / steps, "launches_per_sweep": v[1] / steps} for k, v in kt.items() if v[1]}
    per_launch = {k: kt[k][0] / kt[k][1] for k in kt if kt[k][1] and kt[k][2] > 0}
    dom = max(per_launch, key=lambda k: per_launch[k])
    achieved = kt[dom][2] / (per_launch[dom] * 1e-3) / 1e12
    return {"workload": "SNM A=108 (54 p + 54 n), n^2<=20 (1556 states), rho=0.16, Minnesota with V_T, FP64, "
                        "mixing 0.5, one solve",
            "ccd_iterations_per_s": steps / el, "ms_per_sweep": el * 1e3 / steps,
            "gpu_ms_per_sweep": r["gpu_ms"] / steps,
            "tflops": info["flops_per_sweep"] / (el / steps) / 1e12, "amplitudes": info["n_amplitudes"],
            "e_per_nucleon_after_mev": (er + ec) / 108, "sweeps_run": steps + warmup,
            "kernels": kernels,
            "roofline": {"kernel": "k_nm_gemm (" + dom + ")", "bound": "mfma", "achieved": achieved,
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                         "ms_per_launch": per_launch[dom], "flops_per_launch": kt[dom][2]}}


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


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def _rel(a, b):
    return abs(a - b) / abs(b)


def convergence_c2(ccd, stream):
    """The throughput workload solved to the paper's test |dE_n - dE_(n-1)| <
    1e-8 MeV: the ten densities batched and one after another, both with
    default launch shapes and flags read every 8 sweeps."""
    probs = [ccd.problem(N, NMAX2, r) for r in DENSITIES]
    c = ccd.Context(probs, stream=stream).bind()
    r, el = _timed(lambda: c.iterate(mixing=MIXING, tol=1e-8, max_iter=2000, check_every=8, graph=GRAPH))
    e = [c.energy(p)[2] for p in range(len(probs))]
    c.close()
    singles = [ccd.Context([p], stream=stream).bind() for p in probs]
    sw, el1 = _timed(lambda: [int(s.iterate(mixing=MIXING, tol=1e-8, max_iter=2000, check_every=8,
                                            graph=GRAPH)["sweeps"][0]) for s in singles])
    for s in singles:
        s.close()
    keys = [(N, NMAX2, r) for r in DENSITIES]
    return {"workload": "N=66, n^2<=20, 10 densities, FP64, mixing 0.5, MBPT2 start, |dE| < 1e-8 MeV",
            "batched_wall_s": el, "batched_sweeps": [int(x) for x in r["sweeps"]], "status": int(r["status"]),
            "one_at_a_time_wall_s": el1, "one_at_a_time_sweeps": sw,
            "e_corr_per_particle_mev": [x / N for x in e],
            "max_rel_err_vs_oracle": _err_vs_oracle(e, keys, oracle_energies("oracle_c2_history.txt"))}


def form_mixed_c3(ccd, stream):
    """N=66, n^2<=36, rho=0.16: plain FP64 vs FP32 / BF16 contractions + FP64
    refinement, every context autotuned for its precision; wall time to the
    CONV_REL stop and error against the oracle's converged energy."""
    key = (66, 36, 0.16)
    prob = [ccd.problem(*key)]
    e_orc = oracle_energies("oracle_c3_history.txt").get(key)
    out = {"workload": "PNM N=66, n^2<=36 (1850 states), rho=0.16, mixing 0.5, MBPT2 start",
           "conv_rel": CONV_REL, "e_corr_oracle": e_orc}
    runs = [("fp64", ccd.CCD_PREC_FP64, 0.0), ("fp32_refined", ccd.CCD_PREC_FP32, 1e-4),
            ("bf16_refined", ccd.CCD_PREC_BF16, 1e-2)]
    for name, prec, mtol in runs:
        c = ccd.Context(prob, stream=stream).bind()
        tab, _ = c.autotune(prec, reps=3)
        r, el = _timed(lambda: c.iterate(mixing=MIXING, tol=0.0, tol_rel=CONV_REL, stop_rule=STOP_RULE,
                                         max_iter=2000, precision=prec, mixed_tol=mtol, refine_sweeps=2,
                                         check_every=8, graph=GRAPH))
        n = int(r["sweeps"][0])
        e = c.energy()[2]
        out[name] = {"wall_s": el, "sweeps": n, "e_corr": e,
                     "rel_err_vs_oracle": _rel(e, e_orc) if e_orc is not None else None,
                     "status": int(r["status"]), "mixed_tol_mev": mtol or None, "tuning": [int(x) for x in tab]}
        c.close()
    f = out["fp64"]["wall_s"]
    for name in ("fp32_refined", "bf16_refined"):
        out[name]["speedup_vs_fp64"] = f / out[name]["wall_s"]
    return out


def c4_problems(ccd, seed=C4_SEED):
    import numpy as np
    cut = np.random.default_rng(seed).integers(12, 37, size=40)
    probs = []
    for a, n in enumerate([14, 38, 54, 66]):
        for b, r in enumerate(DENSITIES):
            probs.append(ccd.problem(n, int(cut[10 * a + b]), r))
    return probs, [int(x) for x in cut]


def form_batched_c4(ccd, stream):
    """40 solves: one context each, solved one after another in plain FP64, vs
    one batched context (FP64, and BF16 + FP64 refinement); every context
    autotuned, flags read every 8 sweeps on both sides."""
    probs, cut = c4_problems(ccd)
    keys = [(p.n_particles, p.nmax2, round(p.density, 2)) for p in probs]
    e_orc = oracle_energies("oracle_c4_converged.txt")
    singles = [ccd.Context([p], stream=stream).bind() for p in probs]
    for s in singles:
        s.autotune(ccd.CCD_PREC_FP64, reps=3)

    def seq():
        return [s.iterate(mixing=MIXING, tol=0.0, tol_rel=CONV_REL, stop_rule=STOP_RULE, max_iter=4000,
                          check_every=8, graph=GRAPH)["sweeps"][0] for s in singles]
    sw, t_seq = _timed(seq)
    e_seq = [s.energy()[2] for s in singles]
    for s in singles:
        s.close()
    out = {"workload": "40 PNM solves, N in {14,38,54,66} x rho 0.02..0.20, n^2 cutoffs drawn from "
                       f"numpy default_rng({C4_SEED}).integers(12, 37)", "seed": C4_SEED, "cutoffs": cut,
           "conv_rel": CONV_REL,
           "sequential_fp64": {"wall_s": t_seq, "sweeps_total": int(sum(sw)),
                               "max_rel_err_vs_oracle": _err_vs_oracle(e_seq, keys, e_orc)}}
    for name, prec, mtol in [("batched_fp64", ccd.CCD_PREC_FP64, 0.0),
                             ("batched_bf16_refined", ccd.CCD_PREC_BF16, 1e-2)]:
        c = ccd.Context(probs, stream=stream).bind()
        tab, _ = c.autotune(prec, reps=3)
        r, el = _timed(lambda: c.iterate(mixing=MIXING, tol=0.0, tol_rel=CONV_REL, stop_rule=STOP_RULE, max_iter=4000, precision=prec,
                                         mixed_tol=mtol, refine_sweeps=2, check_every=8, graph=GRAPH))
        e = [c.energy(p)[2] for p in range(len(probs))]
        out[name] = {"wall_s": el, "speedup_vs_sequential_fp64": t_seq / el,
                     "sweeps_max": int(max(r["sweeps"])), "status": int(r["status"]),
                     "max_rel_err_vs_oracle": _err_vs_oracle(e, keys, e_orc),
                     "tuning": [int(x) for x in tab]}
        c.close()
    return out


def infinite_matter(ccd, rho):
    """Kinetic and first-order (Hartree-Fock) energy per particle of infinite
    neutron matter with the Minnesota force: 3 hbar^2 k_F^2 / 10m, and the
    spin-summed direct + exchange integral over two Fermi spheres,
    rho W0 / 8 + (1 / 2 rho (2pi)^6) sum_a V_a (pi/kappa_a)^{3/2}
    int_0^{2k_F} 4 pi q^2 V_ov(q) exp(-q^2 / 4 kappa_a) dq, with V_ov the
    overlap volume of two Fermi spheres a distance q apart."""
    import numpy as np
    kf = (3.0 * np.pi ** 2 * rho) ** (1.0 / 3.0)
    t_inf = 3.0 * ccd.HBAR2_OVER_M * kf ** 2 / 10.0
    x, w = np.polynomial.legendre.leggauss(96)
    q = kf * (x + 1.0)
    wq = kf * w
    vov = np.pi / 12.0 * (4 * kf + q) * (2 * kf - q) ** 2
    m = ccd.MINNESOTA
    hf = 0.0
    for V, k in ((m["V_R"], m["kappa_R"]), (m["V_S"], m["kappa_S"])):
        amp = V * (np.pi / k) ** 1.5
        hf += rho * amp / 8.0
        hf += amp * np.sum(wq * 4 * np.pi * q * q * vov * np.exp(-q * q / (4 * k))) / (2 * rho * (2 * np.pi) ** 6)
    return t_inf, hf


def form_twist_averaged(ccd, stream, n_mesh=5, rho=0.16):
    """Twist-averaged boundary conditions (the paper's TABC5): one solve per
    twist of a Gauss-Legendre mesh, holes filled by energy per twist, batched in
    one context; FP64 to the CONV_REL stop."""
    import numpy as np
    th, w = ccd.twist_mesh(n_mesh)
    probs = [ccd.problem(N, NMAX2, rho, twist=t) for t in th]
    t0 = time.perf_counter()
    ref = ccd.Context(probs, stream=stream)
    plan_s = time.perf_counter() - t0
    ref.bind()
    ref.iterate(mixing=MIXING, tol=REF_TOL, max_iter=4000, check_every=16, graph=GRAPH)
    e_ref = [ref.energy(p)[2] for p in range(len(probs))]
    ref.close()
    singles = [ccd.Context([p], stream=stream).bind() for p in probs]
    sw, t_seq = _timed(lambda: [int(s.iterate(mixing=MIXING, tol=0.0, tol_rel=CONV_REL, stop_rule=STOP_RULE,
                                               max_iter=4000, check_every=8, graph=GRAPH)["sweeps"][0])
                                for s in singles])
    for s in singles:
        s.close()
    c = ccd.Context(probs, stream=stream).bind()
    tab = c.get_tuning()
    r, el = _timed(lambda: c.iterate(mixing=MIXING, tol=0.0, tol_rel=CONV_REL, stop_rule=STOP_RULE, max_iter=4000,
                                     check_every=8, graph=GRAPH))
    e = [c.energy(p)[2] for p in range(len(probs))]
    T, V, Eref, Emp2, Ecc = (x / N for x in c.twist_average(w))
    c.close()
    pbc = ccd.Context([ccd.problem(N, NMAX2, rho)], stream=stream).bind()
    pbc.iterate(mixing=MIXING, tol=REF_TOL, max_iter=4000, check_every=16)
    pt, pv = pbc.reference_parts()
    per, pmp2, pcc = pbc.energy()
    pbc.close()
    t_inf, hf_inf = infinite_matter(ccd, rho)
    return {"workload": f"PNM N=66, n^2<=20, rho={rho}, twists on a {n_mesh}-point Gauss-Legendre mesh per "
                        f"direction over [0, pi] ({len(probs)} solves), FP64, mixing 0.5, MBPT2 start",
            "conv_rel": CONV_REL, "plan_s": plan_s,
            "batched_fp64": {"wall_s": el, "speedup_vs_one_at_a_time": t_seq / el, "status": int(r["status"]),
                             "sweeps_max": int(max(r["sweeps"])), "sweeps_mean": float(np.mean(r["sweeps"])),
                             "max_rel_err_vs_gpu_fp64_ref": max(_rel(a, b) for a, b in zip(e, e_ref)),
                             "tuning": [int(x) for x in tab]},
            "one_at_a_time_fp64": {"wall_s": t_seq, "sweeps_total": int(sum(sw))},
            "per_particle_mev": {
                "twist_averaged": {"T": T, "HF_potential": V, "E_ref": Eref, "dE_mbpt2": Emp2, "dE_ccd": Ecc,
                                   "E_ccd": Eref + Ecc},
                "periodic": {"T": pt / N, "HF_potential": pv / N, "E_ref": per / N, "dE_mbpt2": pmp2 / N,
                             "dE_ccd": pcc / N, "E_ccd": (per + pcc) / N},
                "infinite_matter": {"T": t_inf, "HF_potential": hf_inf}}}


def form_learned_c5(ccd, stream, epochs=72, batch=16384, lr=2e-3):
    """Train the warm-start network on the method's converged amplitudes
    (N=66, n^2<=20, 24 seeded densities), then solve 16 held-out densities at
    n^2<=36 from the MBPT2 start and from the network (BF16 inference)."""
    import torch
    from paper_1611_06765_amd import inputs, warmstart
    train_d, held = inputs.c5_densities()
    (ctx, r), t_conv = _timed(lambda: warmstart.converged_context([(66, 20, d) for d in train_d], stream))
    (feat, tgt), t_feat = _timed(lambda: warmstart.training_set(ctx))
    ctx.close()
    (params, losses), t_train = _timed(lambda: warmstart.train(feat, tgt, epochs=epochs, batch=batch, lr=lr))
    n_train = int(feat.shape[0])
    del feat, tgt
    specs = [(66, 36, d) for d in held]
    e_orc = oracle_energies("oracle_c5_converged.txt")
    out = {"workload": "train: N=66, n^2<=20, 24 densities U[0.02,0.20] (seed %d); evaluate: 16 held-out "
                       "densities, N=66, n^2<=36 (1850 states), mixing 0.5" % inputs.C5_SEED,
           "train_densities": train_d, "heldout_densities": held, "conv_rel": CONV_REL,
           "training": {"amplitudes": n_train, "epochs": epochs, "batch": batch, "lr": lr,
                        "converge_s": t_conv, "features_s": t_feat, "train_s": t_train,
                        "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1]}}
    for name in ("mbpt2_start", "learned_start"):
        c = ccd.Context([ccd.problem(*s) for s in specs], stream=stream).bind()

        t_ws = [0.0]

        e_start = []

        def run():
            used = None
            if name == "learned_start":
                used, t_ws[0] = _timed(lambda: c.warm_start(params, ccd.CCD_PREC_BF16))
            e_start.extend(c.energy(p)[2] for p in range(len(specs)))
            return used, c.iterate(mixing=MIXING, tol=0.0, tol_rel=CONV_REL, stop_rule=STOP_RULE, max_iter=3000,
                                   check_every=8, graph=GRAPH)
        (used, r), el = _timed(run)
        e = [c.energy(p)[2] for p in range(len(specs))]
        out[name] = {"wall_s": el, "sweeps": [int(x) for x in r["sweeps"]], "sweeps_total": int(r["sweeps"].sum()),
                     "status": int(r["status"]), "max_rel_err_vs_oracle": _err_vs_oracle(e, specs, e_orc),
                     # the starting correlation energy's relative error against the oracle's converged one
                     "start_rel_err_vs_oracle": ([_rel(a, e_orc[k]) for a, k in zip(e_start, specs)]
                                                 if all(k in e_orc for k in specs) else None)}
        if used is not None:
            out[name]["network_kept"] = int(used.sum())
            out[name]["warm_start_s"] = t_ws[0]
        c.close()
    out["speedup_vs_mbpt2_start"] = out["mbpt2_start"]["wall_s"] / out["learned_start"]["wall_s"]
    out["sweep_ratio"] = out["learned_start"]["sweeps_total"] / out["mbpt2_start"]["sweeps_total"]
    # the same 16 solves one at a time (the batch above waits for its slowest member)
    seq = {}
    for name in ("mbpt2_start", "learned_start"):
        ctxs = [ccd.Context([ccd.problem(*s)], stream=stream).bind() for s in specs]

        def run():
            sw = 0
            for c in ctxs:
                if name == "learned_start":
                    c.warm_start(params, ccd.CCD_PREC_BF16)
                sw += int(c.iterate(mixing=MIXING, tol=0.0, tol_rel=CONV_REL, stop_rule=STOP_RULE, max_iter=3000,
                                    check_every=8, graph=GRAPH)["sweeps"][0])
            return sw
        sw, el = _timed(run)
        e = [c.energy()[2] for c in ctxs]
        seq[name] = {"wall_s": el, "sweeps_total": sw, "max_rel_err_vs_oracle": _err_vs_oracle(e, specs, e_orc)}
        for c in ctxs:
            c.close()
    seq["speedup"] = seq["mbpt2_start"]["wall_s"] / seq["learned_start"]["wall_s"]
    out["one_at_a_time"] = seq
    del params
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed / batched / learned wall-time comparisons")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--only", choices=["c2", "c3", "c3bf16", "snm", "warm"], default=None,
                    help="profiling runs: only this sweep measurement (no JSON line)")
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
    if args.only:
        # one workload's sweeps alone, for counter and trace runs of the profiler
        if args.copy_probe:
            x = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
            y = torch.empty_like(x)
            y.copy_(x)
            torch.cuda.synchronize()
            del x, y
        fake = {"fp64_mfma_4x4x4_tflops": 1.0, "fp64_mfma_16x16x4_tflops": 1.0}
        if args.only == "c2":
            c = ccd.Context([ccd.problem(N, NMAX2, r) for r in DENSITIES], stream=stream.cuda_stream).bind(dev)
            measure_sweeps(ccd, c, args.steps, args.warmup, [0] * 10, fake, TRAFFIC_C2)
            c.close()
        elif args.only == "c3":
            sweep_rate_c3(ccd, stream.cuda_stream, args.steps, args.warmup, fake)
        elif args.only == "c3bf16":
            sweep_rate_c3(ccd, stream.cuda_stream, args.steps, args.warmup, fake, ccd.CCD_PREC_BF16)
        elif args.only == "warm":
            # the network warm start of the 16 held-out densities (seeded
            # initial parameters: the inference cost does not depend on them)
            from paper_1611_06765_amd import inputs
            c = ccd.Context([ccd.problem(66, 36, r) for r in inputs.c5_densities()[1]], stream=stream.cuda_stream).bind(dev)
            params = torch.tensor(inputs.mlp_init(inputs.MLP_SEED), device=dev)
            for _ in range(args.steps):
                c.warm_start(params, ccd.CCD_PREC_BF16)
            c.close()
        else:
            snm_rate(ccd, stream.cuda_stream, args.steps, args.warmup)
        torch.cuda.synchronize()
        print(f"bench.py --only {args.only}: done", flush=True)
        return
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

    # measured ceilings of this GPU (HBM copy, resident MFMA loops), outside the timed region
    ceilings = ccd.measure_ceilings(1 << 30, stream=stream.cuda_stream, device=dev)
    # the default launch shapes: the autotuner's choices on this workload vary
    # from run to run within the noise (~2%), and a fixed shape keeps the
    # profiled kernels the ones reported here
    tuning = [0] * 10
    m = measure_sweeps(ccd, ctx, args.steps, args.warmup, tuning, ceilings, TRAFFIC_C2)
    el, ms_step, kernels, roof = m["elapsed_s"], m["ms_per_step"], m["kernels"], m["roofline"]
    flops_exec = nsolve * (info["flops_pp"] + info["flops_hh"] + info["flops_ring"])
    flops_ord = nsolve * info["flops_ordered"]

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
                   "amplitudes_per_solve": info["n_amplitudes"], "tuning": [int(x) for x in tuning]},
        # the metric's TFLOP/s: FP64 flops the kernels execute (unordered pairs,
        # the pp ladder over momentum pairs) per second of the timed region
        "tflops": flops_exec / (ms_step * 1e-3) / 1e12,
        "tflops_unit_note": "executed FP64 flops of the sweep / timed-region wall time",
        # context only: the same sweep counted in the paper's unrestricted
        # ordered-pair GEMM form (4.5x the executed flops at this workload)
        "context_tflops_ordered_pair_form": flops_ord / (ms_step * 1e-3) / 1e12,
        "ms_per_step_with_events": m["ms_per_step_with_events"],
        "kernels": kernels,
        "roofline": roof,
        "ceilings": ceilings,
        "e_corr_last": energies,
    }
    ctx.close()
    out["c3_fp64"] = sweep_rate_c3(ccd, stream.cuda_stream, args.steps, args.warmup, ceilings)
    out["c3_bf16"] = sweep_rate_c3(ccd, stream.cuda_stream, args.steps, args.warmup, ceilings, ccd.CCD_PREC_BF16)
    out["snm"] = snm_rate(ccd, stream.cuda_stream, min(args.steps, 40), min(args.warmup, 5))
    if not args.no_forms:
        out["convergence_c2"] = convergence_c2(ccd, stream.cuda_stream)
        out["mixed_c3"] = form_mixed_c3(ccd, stream.cuda_stream)
        out["batched_c4"] = form_batched_c4(ccd, stream.cuda_stream)
        out["learned_c5"] = form_learned_c5(ccd, stream.cuda_stream)
        out["twist_averaged"] = form_twist_averaged(ccd, stream.cuda_stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
