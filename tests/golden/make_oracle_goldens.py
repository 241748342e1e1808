"""Write the oracle's reference energies under tests/golden/.

    python tests/golden/make_oracle_goldens.py [c3] [c2] [c4] [c5]

Calls only the CPU oracle (oracle/, the intermediates form of the CCD
equations with the fourth index deduced) and the seeded workload parameters
of paper_1611_06765_amd/inputs.py, which compute nothing of the method.  Every
solve starts from the MBPT2 amplitudes (eq. ccdGuess), runs Jacobi sweeps of
eq. ccd3 with linear mixing and stops when the correlation energy of eq.
ccdcorr changes by less than the tolerance, the paper's test (sec.
"Approximations to the full CCD equations", the iteration algorithm).

Files (energies are box totals in MeV, repr of the FP64 value):
  oracle_c3_history.txt     N=66, n^2<=36, rho=0.16, mixing 0.5, |dE| < 1e-10:
                            every sweep's energy
  oracle_c2_history.txt     N=66, n^2<=20, rho=0.02..0.20, mixing 0.5,
                            |dE| < 1e-8: every sweep's energy
  oracle_c4_converged.txt   the 40 seeded solves (N in {14,38,54,66} x 10
                            densities, cutoffs 12..36), mixing 0.5, |dE| < 1e-9
  oracle_c5_converged.txt   the 16 held-out densities at N=66, n^2<=36,
                            mixing 0.5, |dE| < 1e-9
A solve already present in a file is kept, so an interrupted run resumes.
Takes hours on eight cores (C5 dominates); OMP_NUM_THREADS sets the threads.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_1611_06765_amd import inputs  # noqa: E402

MIXING = 0.5


def _done(path):
    keys = set()
    if os.path.exists(path):
        for line in open(path):
            line = line.split("#", 1)[0].split()
            if line:
                keys.add((int(line[0]), int(line[1]), float(line[2])))
    return keys


def _header(path, lines):
    if not os.path.exists(path):
        with open(path, "w") as f:
            for x in lines:
                f.write("# " + x + "\n")


def _solve(N, n2, rho, tol):
    t0 = time.time()
    o3 = oracle.O3(oracle.PNM(N, n2, rho))
    hist = o3.solve(MIXING, tol, max_iter=2000)
    print(f"  N={N} n2<={n2} rho={rho}: {len(hist) - 1} sweeps, E_corr {hist[-1]!r} "
          f"({time.time() - t0:.0f} s)", flush=True)
    return o3, hist


def histories(name, specs, tol):
    path = os.path.join(HERE, name)
    _header(path, [
        "Oracle energy histories (tests/golden/make_oracle_goldens.py, oracle O3 only).",
        f"MBPT2 start (eq. ccdGuess), Jacobi sweeps of eq. ccd3, mixing {MIXING}, stop when",
        f"|dE_n - dE_(n-1)| < {tol} MeV (the iteration algorithm); energies are box totals in MeV.",
        "columns: N  nmax2  rho  sweeps  E_ref  E_MBPT2  E_1 ... E_sweeps"])
    have = _done(path)
    for N, n2, rho in specs:
        if (N, n2, rho) in have:
            continue
        o3, hist = _solve(N, n2, rho, tol)
        with open(path, "a") as f:
            f.write(" ".join([str(N), str(n2), repr(rho), str(len(hist) - 1), repr(o3.eref)]
                             + [repr(x) for x in hist]) + "\n")


def converged(name, specs, tol, what):
    path = os.path.join(HERE, name)
    _header(path, [
        f"Oracle converged energies of {what} (tests/golden/make_oracle_goldens.py, oracle O3 only).",
        f"MBPT2 start (eq. ccdGuess), Jacobi sweeps of eq. ccd3, mixing {MIXING}, stop when",
        f"|dE_n - dE_(n-1)| < {tol} MeV; energies are box totals in MeV.",
        "columns: N  nmax2  rho  sweeps  E_ref  E_MBPT2  E_CCD  last |dE|"])
    have = _done(path)
    for N, n2, rho in specs:
        if (N, n2, rho) in have:
            continue
        o3, hist = _solve(N, n2, rho, tol)
        with open(path, "a") as f:
            f.write(" ".join([str(N), str(n2), repr(rho), str(len(hist) - 1), repr(o3.eref),
                              repr(hist[0]), repr(hist[-1]), repr(abs(hist[-1] - hist[-2]))]) + "\n")


def main(which):
    oracle.lib()
    if "c3" in which:
        histories("oracle_c3_history.txt", [(66, 36, 0.16)], 1e-10)
    if "c2" in which:
        histories("oracle_c2_history.txt", [(66, 20, r) for r in inputs.DENSITIES_10], 1e-8)
    if "c4" in which:
        converged("oracle_c4_converged.txt", inputs.c4_specs(), 1e-9,
                  f"the 40 batched solves (cutoffs from seed {inputs.C4_SEED})")
    if "c5" in which:
        _, held = inputs.c5_densities()
        converged("oracle_c5_converged.txt", [(66, 36, d) for d in held], 1e-9,
                  f"the 16 held-out densities (seed {inputs.C5_SEED})")


if __name__ == "__main__":
    main(sys.argv[1:] or ["c3", "c2", "c4", "c5"])
