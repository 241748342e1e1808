"""Python access to the CPU oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It wraps ``ccd_oracle.c`` through ctypes
and adds the pairing-model Hamiltonian (sec. "Developing a CCD code for infinite
matter", eqs. sppairing / intpairing) as dense numpy arrays.  Nothing here is
shared with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccd_oracle.c")
_LIB = os.path.join(_HERE, "libccd_oracle.so")

# Term bits of eq. ccd3 (same meaning in both oracle forms and on the GPU path).
T_PP, T_HH, T_RING, T_QHH, T_QRING, T_QHOLE, T_QPART = 1, 2, 4, 8, 16, 32, 64
T_LINEAR = T_PP | T_HH | T_RING
T_ALL = 127

# Minnesota parameters (Table "Parameters used to define the Minnesota
# interaction model"; V_T and V_S are attractive, hbar^2/m = 41.47 MeV fm^2).
# The table prints both without a sign.  Between two neutrons the V_T channel
# vanishes, so its sign matters only with protons and neutrons.
MINNESOTA = dict(VR=200.0, kR=1.487, VT=-178.0, kT=0.639, VS=-91.85, kS=0.465)
HBAR2_OVER_M = 41.47


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        sig = {
            "orc_pnm_new": (vp, [i, i, d, d, d, d, d, d, d, d]),
            "orc_pnm_new_twist": (vp, [i, i, d, d, d, d, d, d, d, d, d, d, d]),
            "orc_nm_new": (vp, [i, i, i, d, d, d, d, d, d, d, d, i]),
            "orc_pnm_isospins": (None, [vp, ip]),
            "orc_pnm_species": (i, [vp]),
            "orc_pnm_free": (None, [vp]),
            "orc_pnm_vas_direct": (d, [vp, i, i, i, i]),
            "orc_pnm_vas_fast": (d, [vp, i, i, i, i]),
            "orc_pnm_nstates": (i, [vp]),
            "orc_pnm_L": (d, [vp]),
            "orc_pnm_states": (None, [vp, ip, ip, ip, ip]),
            "orc_pnm_kinetic": (None, [vp, dp]),
            "orc_pnm_fock": (None, [vp, dp]),
            "orc_pnm_eref": (d, [vp]),
            "orc_pnm_dense_v": (None, [vp, dp]),
            "orc_o1_new": (vp, [i, i, dp, dp]),
            "orc_o1_free": (None, [vp]),
            "orc_o1_eref": (d, [vp]),
            "orc_o1_emp2": (d, [vp]),
            "orc_o1_ecorr": (d, [vp]),
            "orc_o1_eps": (None, [vp, dp]),
            "orc_o1_t": (d, [vp, i, i, i, i]),
            "orc_o1_sweep": (d, [vp, d, C.c_uint]),
            "orc_o3_new": (vp, [vp]),
            "orc_o3_free": (None, [vp]),
            "orc_o3_eref": (d, [vp]),
            "orc_o3_emp2": (d, [vp]),
            "orc_o3_ecorr": (d, [vp]),
            "orc_o3_t": (d, [vp, i, i, i, i]),
            "orc_o3_count": (C.c_long, [vp]),
            "orc_o3_export": (None, [vp, ip, dp]),
            "orc_o3_set_t": (None, [vp, dp]),
            "orc_o3_sweep": (d, [vp, d, C.c_uint]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


class PNM:
    """Pure neutron matter model space and Minnesota interaction; `twist` =
    (theta_x, theta_y, theta_z) in radians gives momenta (2 pi n + theta) / L
    and the holes filled by energy for that twist."""

    def __init__(self, n_particles: int, nmax2: int, rho: float,
                 hbar2_over_m: float = HBAR2_OVER_M, twist=(0.0, 0.0, 0.0), **pot):
        p = dict(MINNESOTA)
        p.update(pot)
        self.N, self.nmax2, self.rho = n_particles, nmax2, rho
        self.twist = tuple(float(x) for x in twist)
        self.h = lib().orc_pnm_new_twist(nmax2, n_particles, rho, hbar2_over_m,
                                         p["VR"], p["kR"], p["VT"], p["kT"], p["VS"], p["kS"],
                                         *self.twist)
        if not self.h:
            raise ValueError("N is odd, leaves no particle states, or (untwisted) does not close a shell")
        self.ns = lib().orc_pnm_nstates(self.h)
        self.L = lib().orc_pnm_L(self.h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_pnm_free(self.h)
            self.h = None

    def states(self):
        a = [np.zeros(self.ns, dtype=np.int32) for _ in range(4)]
        lib().orc_pnm_states(self.h, *[_ip(x) for x in a])
        return np.stack(a, axis=1)  # columns nx, ny, nz, 2*s_z

    def kinetic(self):
        out = np.zeros(self.ns)
        lib().orc_pnm_kinetic(self.h, _dp(out))
        return out

    def fock(self):
        out = np.zeros(self.ns)
        lib().orc_pnm_fock(self.h, _dp(out))
        return out

    def eref(self) -> float:
        return lib().orc_pnm_eref(self.h)

    def v(self, p, q, r, s) -> float:
        return lib().orc_pnm_vas_direct(self.h, p, q, r, s)

    def v_fast(self, p, q, r, s) -> float:
        return lib().orc_pnm_vas_fast(self.h, p, q, r, s)

    def dense_v(self):
        n = self.ns
        out = np.zeros(n ** 4)
        lib().orc_pnm_dense_v(self.h, _dp(out))
        return out.reshape(n, n, n, n)


class NM(PNM):
    """Nuclear matter: species = 2 gives symmetric nuclear matter (A/2
    protons and A/2 neutrons when A fills whole momenta; Table 1's magic
    numbers doubled), species = 1 pure neutron matter.  open_ok accepts a
    nucleon number that does not close a shell (small exact test systems).
    Periodic box."""

    def __init__(self, n_particles: int, nmax2: int, rho: float, species: int = 2, open_ok: bool = False,
                 hbar2_over_m: float = HBAR2_OVER_M, **pot):
        p = dict(MINNESOTA)
        p.update(pot)
        self.N, self.nmax2, self.rho = n_particles, nmax2, rho
        self.twist = (0.0, 0.0, 0.0)
        self.h = lib().orc_nm_new(nmax2, n_particles, species, rho, hbar2_over_m,
                                  p["VR"], p["kR"], p["VT"], p["kT"], p["VS"], p["kS"], int(bool(open_ok)))
        if not self.h:
            raise ValueError("A leaves no particle states or does not close a shell")
        self.ns = lib().orc_pnm_nstates(self.h)
        self.L = lib().orc_pnm_L(self.h)

    def isospins(self):
        """twice t_z per state: -1 proton, +1 neutron"""
        a = np.zeros(self.ns, dtype=np.int32)
        lib().orc_pnm_isospins(self.h, _ip(a))
        return a


class O1:
    """Dense eq. ccd3 iteration for any Hamiltonian given as dense arrays."""

    def __init__(self, hdiag, v, nh: int):
        self.n = len(hdiag)
        self._h = np.ascontiguousarray(hdiag, dtype=np.float64)
        self._v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        self.nh = nh
        self.o = lib().orc_o1_new(self.n, nh, _dp(self._h), _dp(self._v))

    def __del__(self):
        if getattr(self, "o", None) and _lib is not None:
            _lib.orc_o1_free(self.o)
            self.o = None

    eref = property(lambda s: lib().orc_o1_eref(s.o))
    emp2 = property(lambda s: lib().orc_o1_emp2(s.o))
    ecorr = property(lambda s: lib().orc_o1_ecorr(s.o))

    def eps(self):
        out = np.zeros(self.n)
        lib().orc_o1_eps(self.o, _dp(out))
        return out

    def t(self, a, b, i, j) -> float:
        return lib().orc_o1_t(self.o, a, b, i, j)

    def sweep(self, alpha: float = 1.0, mask: int = T_ALL) -> float:
        return lib().orc_o1_sweep(self.o, alpha, mask)


class O3:
    """PNM CCD in the intermediates form with the fourth index deduced."""

    def __init__(self, pnm: PNM):
        self.pnm = pnm
        self.o = lib().orc_o3_new(pnm.h)

    def __del__(self):
        if getattr(self, "o", None) and _lib is not None:
            _lib.orc_o3_free(self.o)
            self.o = None

    eref = property(lambda s: lib().orc_o3_eref(s.o))
    emp2 = property(lambda s: lib().orc_o3_emp2(s.o))
    ecorr = property(lambda s: lib().orc_o3_ecorr(s.o))

    def t(self, a, b, i, j) -> float:
        return lib().orc_o3_t(self.o, a, b, i, j)

    def export(self):
        n = lib().orc_o3_count(self.o)
        ijab = np.zeros((n, 4), dtype=np.int32)
        tv = np.zeros(n)
        lib().orc_o3_export(self.o, _ip(ijab), _dp(tv))
        return ijab, tv

    def set_t(self, tv):
        tv = np.ascontiguousarray(tv, dtype=np.float64)
        lib().orc_o3_set_t(self.o, _dp(tv))

    def sweep(self, alpha: float = 1.0, mask: int = T_ALL) -> float:
        return lib().orc_o3_sweep(self.o, alpha, mask)

    def solve(self, alpha: float, tol: float, max_iter: int = 500, mask: int = T_ALL):
        """Iterate until |dE_n - dE_(n-1)| < tol; returns the energy history
        [E_MBPT2, E_1, E_2, ...] (sec. "Developing a CCD code ...")."""
        hist = [self.ecorr]
        for _ in range(max_iter):
            hist.append(self.sweep(alpha, mask))
            if abs(hist[-1] - hist[-2]) < tol:
                break
        return hist


def pairing_model(g: float, delta: float = 1.0, nlevels: int = 4):
    """Pairing Hamiltonian as dense arrays: h_pp = delta (p-1) per level p, and
    <p+ p-||q+ q-> = -g/2 with the antisymmetry signs (eqs. sppairing and
    intpairing).  States: 2*(p-1) is spin up, 2*(p-1)+1 spin down."""
    n = 2 * nlevels
    h = np.array([delta * (s // 2) for s in range(n)], dtype=np.float64)
    v = np.zeros((n, n, n, n))

    def sig(p, q):
        if p // 2 != q // 2 or p == q:
            return 0.0
        return 1.0 if p % 2 == 0 else -1.0

    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s in range(n):
                    v[p, q, r, s] = -0.5 * g * sig(p, q) * sig(r, s)
    return h, v


def twist_grid(n_per_dir: int):
    """Gauss-Legendre twist angles on [0, pi] in each direction and the weights
    w_x w_y w_z / pi^3 of the twist average (they sum to 1), from numpy's
    Gauss-Legendre rule (the twist-averaging algorithm)."""
    x, w = np.polynomial.legendre.leggauss(n_per_dir)
    th = 0.5 * np.pi * (x + 1.0)
    wt = 0.5 * np.pi * w
    thetas, weights = [], []
    for a in range(n_per_dir):
        for b in range(n_per_dir):
            for c in range(n_per_dir):
                thetas.append((th[a], th[b], th[c]))
                weights.append(wt[a] * wt[b] * wt[c] / np.pi ** 3)
    return np.array(thetas), np.array(weights)

