"""ctypes binding of libccd.so (include/ccd.h): argument marshalling only.

Every step of the CCD sweep runs in the library's HIP kernels.  PyTorch is used
for device memory (the workspace tensor) and for the stream the library works
on.  If the shared library is missing this module raises at import time: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1611_06765_amd.build_lib`")

# torch brings its own HIP runtime (same soname, libamdhip64.so.7).  Loading it
# first makes the library bind to that runtime instead of a second copy from
# /opt/rocm: two HIP runtimes in one process do not share the device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

CCD_OK, CCD_NOT_CONVERGED, CCD_DIVERGED = 0, 1, 2
CCD_EINVAL, CCD_ENOTMAGIC, CCD_ENOMEM, CCD_EHIP, CCD_ESTATE = -1, -2, -3, -4, -5
STATUS_NAMES = {0: "CCD_OK", 1: "CCD_NOT_CONVERGED", 2: "CCD_DIVERGED", -1: "CCD_EINVAL",
                -2: "CCD_ENOTMAGIC", -3: "CCD_ENOMEM", -4: "CCD_EHIP", -5: "CCD_ESTATE"}

CCD_T_PP, CCD_T_HH, CCD_T_RING, CCD_T_QHH = 1, 2, 4, 8
CCD_T_QRING, CCD_T_QHOLE, CCD_T_QPART, CCD_T_ALL = 16, 32, 64, 127
CCD_PREC_FP64, CCD_PREC_FP32, CCD_PREC_BF16 = 0, 1, 2
CCD_MAP_STATES, CCD_MAP_CHANNELS, CCD_MAP_HH, CCD_MAP_PP, CCD_MAP_PH_CHANNELS, CCD_MAP_PH = range(6)
(CCD_TUNE_DIRECT, CCD_TUNE_DCHI, CCD_TUNE_RING_SMALL, CCD_TUNE_RING, CCD_TUNE_LADDER, CCD_TUNE_UPDATE,
 CCD_TUNE_RING_NW32, CCD_TUNE_RING_NW48, CCD_TUNE_RING_NW64, CCD_TUNE_RING_NW80) = range(10)
CCD_TUNE_LEN = 10


class ccd_problem(C.Structure):
    _fields_ = [("n_particles", C.c_int32), ("nmax2", C.c_int32), ("density", C.c_double),
                ("hbar2_over_m", C.c_double), ("V_R", C.c_double), ("kappa_R", C.c_double),
                ("V_S", C.c_double), ("kappa_S", C.c_double), ("twist", C.c_double * 3)]


class ccd_solver_opts(C.Structure):
    _fields_ = [("mixing", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("refine_sweeps", C.c_int32), ("terms", C.c_uint32),
                ("mixed_tol", C.c_double), ("check_every", C.c_int32), ("use_graph", C.c_int32),
                ("tol_rel", C.c_double), ("stop_rule", C.c_int32)]


class ccd_info(C.Structure):
    _fields_ = [("n_states", C.c_int32), ("n_holes", C.c_int32), ("n_particles_states", C.c_int32),
                ("n_channels", C.c_int32), ("n_channels_sz0", C.c_int32), ("n_ph_channels", C.c_int32),
                ("max_hh", C.c_int32), ("max_pp", C.c_int32), ("max_ph", C.c_int32),
                ("n_amplitudes", C.c_int64), ("lut_size", C.c_int32), ("box_L", C.c_double),
                ("flops_pp", C.c_double), ("flops_hh", C.c_double), ("flops_ring", C.c_double),
                ("flops_ordered", C.c_double)]


class ccd_adam_opts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("batch", C.c_int32)]


class ccd_nm_problem(C.Structure):
    _fields_ = [("n_nucleons", C.c_int32), ("species", C.c_int32), ("nmax2", C.c_int32),
                ("density", C.c_double), ("hbar2_over_m", C.c_double), ("V_R", C.c_double),
                ("kappa_R", C.c_double), ("V_T", C.c_double), ("kappa_T", C.c_double),
                ("V_S", C.c_double), ("kappa_S", C.c_double)]


class ccd_nm_info(C.Structure):
    _fields_ = [("n_states", C.c_int32), ("n_holes", C.c_int32), ("n_channels", C.c_int32),
                ("n_ph_channels", C.c_int32), ("max_hh", C.c_int32), ("max_pp", C.c_int32),
                ("max_ph", C.c_int32), ("n_amplitudes", C.c_int64), ("box_L", C.c_double),
                ("flops_per_sweep", C.c_double)]


CCD_NM_MAP_STATES, CCD_NM_MAP_CHANNELS, CCD_NM_MAP_HH, CCD_NM_MAP_PP = range(4)
CCD_MLP_NPACK, CCD_MLP_NPARAM = 8, 17800

_vp, _i32, _sz = C.c_void_p, C.c_int32, C.c_size_t
_dp, _ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
_SIGS = {
    "ccd_build_channels": (_i32, [C.POINTER(ccd_problem), _i32, _vp, C.POINTER(_vp)]),
    "ccd_workspace_size": (_i32, [_vp, C.POINTER(_sz)]),
    "ccd_bind_workspace": (_i32, [_vp, _vp, _sz]),
    "ccd_iterate": (_i32, [_vp, C.POINTER(ccd_solver_opts), _ip, _dp]),
    "ccd_energy": (_i32, [_vp, _i32, _dp, _dp, _dp]),
    "ccd_problem_info": (_i32, [_vp, _i32, C.POINTER(ccd_info)]),
    "ccd_mbpt3": (_i32, [_vp, _dp]),
    "ccd_measure_ceilings": (_i32, [_vp, _sz, _vp, _dp]),
    "ccd_dense_workspace_size": (_i32, [_i32, _i32, C.POINTER(_sz)]),
    "ccd_dense_solve": (_i32, [_dp, _dp, _i32, _i32, C.POINTER(ccd_solver_opts), _vp, _sz, _vp, _dp, _dp, _dp,
                               _ip, _dp]),
    "ccd_dense_solve_static": (_i32, [_dp, _dp, _i32, _i32, C.POINTER(ccd_solver_opts), _vp, _dp, _dp, _dp,
                                      _ip, _dp]),
    "ccd_reference_parts": (_i32, [_vp, _i32, _dp, _dp]),
    "ccd_twist_mesh": (_i32, [_i32, _dp, _dp]),
    "ccd_twist_average": (_i32, [_vp, _dp, _dp]),
    "ccd_get_amplitudes": (_i32, [_vp, _i32, _dp, _sz]),
    "ccd_set_amplitudes": (_i32, [_vp, _i32, _dp, _sz]),
    "ccd_reset_amplitudes": (_i32, [_vp]),
    "ccd_export_maps": (_i32, [_vp, _i32, _i32, _ip, _sz, C.POINTER(_sz)]),
    "ccd_export_tables": (_i32, [_vp, _i32, _dp, _dp, _dp]),
    "ccd_mlp_features": (_i32, [_vp, _i32, _vp, _vp]),
    "ccd_mlp_forward": (_i32, [_vp, _vp, C.c_int64, _i32, _vp, _vp]),
    "ccd_mlp_work_size": (_i32, [C.c_int64, C.POINTER(_sz)]),
    "ccd_mlp_loss_grad": (_i32, [_vp, _vp, _vp, C.c_int64, _vp, _dp, _vp, _sz, _vp]),
    "ccd_mlp_train": (_i32, [_vp, _vp, _vp, C.POINTER(C.c_int64), _vp, _vp, C.c_int64, _vp, C.c_int64,
                             C.POINTER(ccd_adam_opts), _vp, _sz, _dp, _vp]),
    "ccd_warm_start": (_i32, [_vp, _vp, _i32, _ip]),
    "ccd_autotune": (_i32, [_vp, _i32, _i32, _dp]),
    "ccd_get_tuning": (_i32, [_vp, _ip, _i32]),
    "ccd_set_tuning": (_i32, [_vp, _ip, _i32]),
    "ccd_set_timing": (_i32, [_vp, _i32]),
    "ccd_kernel_families": (_i32, []),
    "ccd_kernel_name": (C.c_char_p, [_i32]),
    "ccd_kernel_times": (_i32, [_vp, _dp, C.POINTER(C.c_int64), _i32]),
    "ccd_nm_build": (_i32, [C.POINTER(ccd_nm_problem), _vp, C.POINTER(_vp)]),
    "ccd_nm_info_get": (_i32, [_vp, C.POINTER(ccd_nm_info)]),
    "ccd_nm_workspace_size": (_i32, [_vp, C.POINTER(_sz)]),
    "ccd_nm_bind_workspace": (_i32, [_vp, _vp, _sz]),
    "ccd_nm_iterate": (_i32, [_vp, C.POINTER(ccd_solver_opts), _ip, _dp]),
    "ccd_nm_energy": (_i32, [_vp, _dp, _dp, _dp]),
    "ccd_nm_get_amplitudes": (_i32, [_vp, _dp, _sz]),
    "ccd_nm_set_amplitudes": (_i32, [_vp, _dp, _sz]),
    "ccd_nm_export_maps": (_i32, [_vp, _i32, _ip, _sz, C.POINTER(_sz)]),
    "ccd_nm_export_tables": (_i32, [_vp, _dp, _dp, _dp]),
    "ccd_nm_element": (_i32, [_vp, _i32, _i32, _i32, _i32, _dp]),
    "ccd_nm_last_ms": (_i32, [_vp, _dp]),
    "ccd_nm_set_timing": (_i32, [_vp, _i32]),
    "ccd_nm_kernel_times": (_i32, [_vp, _dp, C.POINTER(C.c_int64), _dp, _i32]),
    "ccd_nm_kernel_name": (C.c_char_p, [_i32]),
    "ccd_nm_destroy": (None, [_vp]),
    "ccd_last_error": (C.c_char_p, []),
    "ccd_version": (C.c_char_p, []),
    "ccd_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class CCDError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.ccd_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _check(status, where, ok=(CCD_OK,)):
    if status not in ok:
        raise CCDError(status, where)
    return status


MINNESOTA = dict(V_R=200.0, kappa_R=1.487, V_S=-91.85, kappa_S=0.465)
HBAR2_OVER_M = 41.47


def problem(n_particles, nmax2, density, hbar2_over_m=HBAR2_OVER_M, twist=(0.0, 0.0, 0.0), **pot):
    """ccd_problem; twist = (theta_x, theta_y, theta_z) in radians (0 = periodic)."""
    p = dict(MINNESOTA)
    p.update(pot)
    return ccd_problem(n_particles, nmax2, density, hbar2_over_m,
                       p["V_R"], p["kappa_R"], p["V_S"], p["kappa_S"],
                       (C.c_double * 3)(*(float(x) for x in twist)))


def measure_ceilings(nbytes=1 << 30, stream=None, device="cuda"):
    """Measured ceilings of the GPU: dict of HBM copy GB/s and the FP64 / FP32 /
    BF16 MFMA TFLOP/s of resident loops (ccd_measure_ceilings)."""
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = (buf.data_ptr() + 255) & ~255
    out = np.zeros(5)
    sp = None if stream is None else _vp(stream)
    _check(_lib.ccd_measure_ceilings(_vp(ptr), nbytes, sp, _dptr(out)), "ccd_measure_ceilings")
    del buf
    return {"hbm_copy_gbs": out[0], "fp64_mfma_16x16x4_tflops": out[1], "fp64_mfma_4x4x4_tflops": out[2],
            "fp32_mfma_16x16x4_tflops": out[3], "bf16_mfma_16x16x32_tflops": out[4]}


def dense_solve(h, v, n_holes, mixing=1.0, tol=1e-10, max_iter=500, terms=CCD_T_ALL, tol_rel=0.0,
                stream=None, device="cuda"):
    """CCD of a small dense Hamiltonian (ccd_dense_solve): h[n] one-body
    diagonal, v[n,n,n,n] antisymmetrised elements, the lowest n_holes states
    holes.  Returns dict(status, e_ref, e_mbpt2, e_ccd, sweeps, history)."""
    import torch
    h = np.ascontiguousarray(h, dtype=np.float64)
    n = h.size
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
    if v.size != n ** 4:
        raise ValueError("v must hold n^4 elements")
    need = _sz()
    _check(_lib.ccd_dense_workspace_size(n, n_holes, C.byref(need)), "ccd_dense_workspace_size")
    buf = torch.empty(need.value + 256, dtype=torch.uint8, device=device)
    ptr = (buf.data_ptr() + 255) & ~255
    o = ccd_solver_opts(mixing, tol, max_iter, CCD_PREC_FP64, 0, terms, 0.0, 1, 0, tol_rel, 0)
    er, e2, ec = C.c_double(), C.c_double(), C.c_double()
    sw = C.c_int32()
    hist = np.zeros(max_iter)
    sp = None if stream is None else _vp(stream)
    st = _lib.ccd_dense_solve(_dptr(h), _dptr(v), n, n_holes, C.byref(o), _vp(ptr), need.value, sp,
                              C.byref(er), C.byref(e2), C.byref(ec), C.byref(sw), _dptr(hist))
    _check(st, "ccd_dense_solve", ok=(CCD_OK, CCD_NOT_CONVERGED, CCD_DIVERGED))
    del buf
    return {"status": st, "e_ref": er.value, "e_mbpt2": e2.value, "e_ccd": ec.value, "sweeps": sw.value,
            "history": hist[:sw.value]}


def dense_solve_static(h, v, n_holes, mixing=1.0, tol=1e-10, max_iter=500, terms=CCD_T_ALL, tol_rel=0.0,
                       stream=None):
    """dense_solve through ccd_dense_solve_static: no device memory is
    allocated, the library's static work area of the current device is used."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    n = h.size
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
    if v.size != n ** 4:
        raise ValueError("v must hold n^4 elements")
    o = ccd_solver_opts(mixing, tol, max_iter, CCD_PREC_FP64, 0, terms, 0.0, 1, 0, tol_rel, 0)
    er, e2, ec = C.c_double(), C.c_double(), C.c_double()
    sw = C.c_int32()
    hist = np.zeros(max_iter)
    sp = None if stream is None else _vp(stream)
    st = _lib.ccd_dense_solve_static(_dptr(h), _dptr(v), n, n_holes, C.byref(o), sp,
                                     C.byref(er), C.byref(e2), C.byref(ec), C.byref(sw), _dptr(hist))
    _check(st, "ccd_dense_solve_static", ok=(CCD_OK, CCD_NOT_CONVERGED, CCD_DIVERGED))
    return {"status": st, "e_ref": er.value, "e_mbpt2": e2.value, "e_ccd": ec.value, "sweeps": sw.value,
            "history": hist[:sw.value]}


def twist_mesh(n):
    """Gauss-Legendre twist mesh: (n^3 x 3 angles on [0, pi], n^3 weights summing to 1)."""
    th = np.zeros(3 * n ** 3)
    w = np.zeros(n ** 3)
    _check(_lib.ccd_twist_mesh(n, _dptr(th), _dptr(w)), "ccd_twist_mesh")
    return th.reshape(-1, 3), w


def _dptr(a):
    return a.ctypes.data_as(_dp)


class Context:
    """One ccd_ctx: a batch of independent problems sharing one stream."""

    def __init__(self, problems, stream=None):
        probs = (ccd_problem * len(problems))(*problems)
        self._h = _vp()
        sp = None if stream is None else _vp(stream)
        _check(_lib.ccd_build_channels(probs, len(problems), sp, C.byref(self._h)), "ccd_build_channels")
        self.n = len(problems)
        self.workspace = None

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.ccd_destroy(self._h)
            self._h = _vp()

    # ---- host-side plan (no GPU) ------------------------------------------
    def workspace_size(self):
        n = _sz()
        _check(_lib.ccd_workspace_size(self._h, C.byref(n)), "ccd_workspace_size")
        return n.value

    def info(self, p=0):
        i = ccd_info()
        _check(_lib.ccd_problem_info(self._h, p, C.byref(i)), "ccd_problem_info")
        return {k: getattr(i, k) for k, _ in ccd_info._fields_}

    def export_map(self, which, p=0):
        need = _sz()
        _check(_lib.ccd_export_maps(self._h, p, which, None, 0, C.byref(need)), "ccd_export_maps")
        out = np.zeros(need.value, dtype=np.int32)
        _check(_lib.ccd_export_maps(self._h, p, which, out.ctypes.data_as(_ip), out.size, None),
               "ccd_export_maps")
        return out

    def export_tables(self, p=0):
        inf = self.info(p)
        tk = np.zeros(inf["n_states"])
        eps = np.zeros(inf["n_states"])
        w = np.zeros(inf["lut_size"])
        _check(_lib.ccd_export_tables(self._h, p, _dptr(tk), _dptr(eps), _dptr(w)), "ccd_export_tables")
        return tk, eps, w

    # ---- device -------------------------------------------------------------
    def bind(self, device="cuda"):
        """Allocate the workspace as a torch uint8 tensor and bind it."""
        import torch
        nbytes = self.workspace_size()
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = self.workspace.data_ptr()
        ptr = (ptr + 255) & ~255
        _check(_lib.ccd_bind_workspace(self._h, _vp(ptr), nbytes), "ccd_bind_workspace")
        return self

    def iterate(self, mixing=1.0, tol=0.0, max_iter=1, precision=CCD_PREC_FP64, refine_sweeps=0,
                terms=CCD_T_ALL, history=False, mixed_tol=0.0, check_every=1, graph=False, tol_rel=0.0,
                stop_rule=0):
        o = ccd_solver_opts(mixing, tol, max_iter, precision, refine_sweeps, terms, mixed_tol,
                            check_every, int(bool(graph)), tol_rel, stop_rule)
        sweeps = np.zeros(self.n, dtype=np.int32)
        hist = np.zeros(self.n * max_iter) if history else None
        st = _lib.ccd_iterate(self._h, C.byref(o), sweeps.ctypes.data_as(_ip),
                              _dptr(hist) if history else None)
        _check(st, "ccd_iterate", ok=(CCD_OK, CCD_NOT_CONVERGED))
        res = {"status": st, "sweeps": sweeps}
        if history:
            res["history"] = hist.reshape(self.n, max_iter)
        return res

    def energy(self, p=0):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(_lib.ccd_energy(self._h, p, C.byref(a), C.byref(b), C.byref(c)), "ccd_energy")
        return a.value, b.value, c.value

    def mbpt3(self):
        """Third-order energies [n_problems][4] = (pp, hh, ring, total) in MeV;
        leaves the context at its MBPT2 amplitudes."""
        out = np.zeros((self.n, 4))
        _check(_lib.ccd_mbpt3(self._h, _dptr(out)), "ccd_mbpt3")
        return out

    def reference_parts(self, p=0):
        """(kinetic energy, Hartree-Fock potential energy) of the Fermi sea (host plan)."""
        a, b = C.c_double(), C.c_double()
        _check(_lib.ccd_reference_parts(self._h, p, C.byref(a), C.byref(b)), "ccd_reference_parts")
        return a.value, b.value

    def twist_average(self, weights):
        """Weighted sums of (T, E_ref - T, E_ref, MBPT2, correlation energy) over the problems."""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        if w.shape != (self.n,):
            raise ValueError("one weight per problem")
        out = np.zeros(5)
        _check(_lib.ccd_twist_average(self._h, _dptr(w), _dptr(out)), "ccd_twist_average")
        return out

    def eref(self, p=0):
        """Reference energy (host plan; no GPU needed)."""
        a = C.c_double()
        _check(_lib.ccd_energy(self._h, p, C.byref(a), None, None), "ccd_energy")
        return a.value

    def get_amplitudes(self, p=0):
        n = self.info(p)["n_amplitudes"]
        out = np.zeros(n)
        _check(_lib.ccd_get_amplitudes(self._h, p, _dptr(out), n), "ccd_get_amplitudes")
        return out

    def set_amplitudes(self, t, p=0):
        t = np.ascontiguousarray(t, dtype=np.float64)
        _check(_lib.ccd_set_amplitudes(self._h, p, _dptr(t), t.size), "ccd_set_amplitudes")

    def reset_amplitudes(self):
        _check(_lib.ccd_reset_amplitudes(self._h), "ccd_reset_amplitudes")

    def autotune(self, precision=CCD_PREC_FP64, reps=10):
        """Time the launch shapes of every tuning slot and keep the fastest;
        returns (table, best ms per launch of each slot)."""
        best = np.zeros(CCD_TUNE_LEN)
        _check(_lib.ccd_autotune(self._h, precision, reps, _dptr(best)), "ccd_autotune")
        return self.get_tuning(), best

    def get_tuning(self):
        t = np.zeros(CCD_TUNE_LEN, dtype=np.int32)
        _check(_lib.ccd_get_tuning(self._h, t.ctypes.data_as(_ip), CCD_TUNE_LEN), "ccd_get_tuning")
        return t

    def set_tuning(self, table):
        t = np.ascontiguousarray(table, dtype=np.int32)
        _check(_lib.ccd_set_tuning(self._h, t.ctypes.data_as(_ip), t.size), "ccd_set_tuning")

    # ---- learned warm start ---------------------------------------------------
    def mlp_features(self, p=0, targets=False):
        """Packed features [n_amp, 8] (and targets y*) of problem p as float32
        device tensors."""
        import torch
        n = self.info(p)["n_amplitudes"]
        dev = self.workspace.device
        feat = torch.empty((n, CCD_MLP_NPACK), dtype=torch.float32, device=dev)
        tgt = torch.empty(n, dtype=torch.float32, device=dev) if targets else None
        _check(_lib.ccd_mlp_features(self._h, p, _vp(feat.data_ptr()),
                                     _vp(tgt.data_ptr()) if targets else None), "ccd_mlp_features")
        return (feat, tgt) if targets else feat

    def warm_start(self, params=None, precision=CCD_PREC_BF16):
        """Network warm start of every problem (params: float32 device tensor of
        CCD_MLP_NPARAM entries; None restores the MBPT2 start); returns per
        problem whether the network's amplitudes were kept."""
        used = np.zeros(self.n, dtype=np.int32)
        ptr = None if params is None else _vp(params.data_ptr())
        _check(_lib.ccd_warm_start(self._h, ptr, precision, used.ctypes.data_as(_ip)), "ccd_warm_start")
        return used.astype(bool)

    def set_timing(self, on=True):
        _check(_lib.ccd_set_timing(self._h, int(on)), "ccd_set_timing")

    def kernel_times(self, reset=False):
        nf = _lib.ccd_kernel_families()
        ms = np.zeros(nf)
        cnt = np.zeros(nf, dtype=np.int64)
        _check(_lib.ccd_kernel_times(self._h, _dptr(ms), cnt.ctypes.data_as(C.POINTER(C.c_int64)),
                                     int(reset)), "ccd_kernel_times")
        return {_lib.ccd_kernel_name(f).decode(): (float(ms[f]), int(cnt[f])) for f in range(nf)}


def _stream_of(t):
    import torch
    return _vp(torch.cuda.current_stream(t.device).cuda_stream)


def mlp_forward(params, feat, precision=CCD_PREC_BF16):
    """Network prediction y for packed features feat [n, 8] (device tensors)."""
    import torch
    n = feat.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=feat.device)
    _check(_lib.ccd_mlp_forward(_vp(params.data_ptr()), _vp(feat.data_ptr()), n, precision,
                                _vp(y.data_ptr()), _stream_of(feat)), "ccd_mlp_forward")
    return y


def mlp_work_buffer(n, device):
    import torch
    nb = _sz()
    _check(_lib.ccd_mlp_work_size(n, C.byref(nb)), "ccd_mlp_work_size")
    w = torch.empty(nb.value + 256, dtype=torch.uint8, device=device)
    ptr = (w.data_ptr() + 255) & ~255
    return w, ptr, nb.value


def mlp_loss_grad(params, feat, target):
    """(loss, gradient tensor) of the mean squared error over all rows."""
    import torch
    n = feat.shape[0]
    g = torch.empty(CCD_MLP_NPARAM, dtype=torch.float32, device=feat.device)
    w, ptr, nb = mlp_work_buffer(n, feat.device)
    loss = C.c_double()
    _check(_lib.ccd_mlp_loss_grad(_vp(params.data_ptr()), _vp(feat.data_ptr()), _vp(target.data_ptr()), n,
                                  _vp(g.data_ptr()), C.byref(loss), _vp(ptr), nb, _stream_of(feat)),
           "ccd_mlp_loss_grad")
    del w
    return loss.value, g


class AdamState:
    """Adam moments and step counter of one parameter tensor."""

    def __init__(self, params):
        import torch
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = C.c_int64(0)


def mlp_train(params, state, feat, target, order, batch, lr, beta1=0.9, beta2=0.999, eps=1e-8, work=None):
    """len(order) // batch Adam steps over minibatches order[s*batch:(s+1)*batch]
    (int32 device tensor of row indices); returns the mean minibatch loss."""
    o = ccd_adam_opts(lr, beta1, beta2, eps, batch)
    if work is None:
        work = mlp_work_buffer(batch, feat.device)
    _, ptr, nb = work
    loss = C.c_double()
    _check(_lib.ccd_mlp_train(_vp(params.data_ptr()), _vp(state.m.data_ptr()), _vp(state.v.data_ptr()),
                              C.byref(state.step), _vp(feat.data_ptr()), _vp(target.data_ptr()), feat.shape[0],
                              _vp(order.data_ptr()), order.shape[0], C.byref(o), _vp(ptr), nb, C.byref(loss),
                              _stream_of(feat)), "ccd_mlp_train")
    return loss.value


MINNESOTA_NM = dict(V_R=200.0, kappa_R=1.487, V_T=-178.0, kappa_T=0.639, V_S=-91.85, kappa_S=0.465)


def nm_problem(n_nucleons, nmax2, density, species=2, hbar2_over_m=HBAR2_OVER_M, **pot):
    """ccd_nm_problem: species 2 = A/2 protons and A/2 neutrons, 1 = neutrons."""
    p = dict(MINNESOTA_NM)
    p.update(pot)
    return ccd_nm_problem(n_nucleons, species, nmax2, density, hbar2_over_m, p["V_R"], p["kappa_R"],
                          p["V_T"], p["kappa_T"], p["V_S"], p["kappa_S"])


class NMContext:
    """One ccd_nm_ctx: a nuclear-matter problem with isospin (include/ccd_nm.h)."""

    def __init__(self, problem, stream=None):
        self._h = _vp()
        sp = None if stream is None else _vp(stream)
        _check(_lib.ccd_nm_build(C.byref(problem), sp, C.byref(self._h)), "ccd_nm_build")
        self.workspace = None

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.ccd_nm_destroy(self._h)
            self._h = _vp()

    def info(self):
        i = ccd_nm_info()
        _check(_lib.ccd_nm_info_get(self._h, C.byref(i)), "ccd_nm_info_get")
        return {k: getattr(i, k) for k, _ in ccd_nm_info._fields_}

    def export_map(self, which):
        need = _sz()
        _check(_lib.ccd_nm_export_maps(self._h, which, None, 0, C.byref(need)), "ccd_nm_export_maps")
        out = np.zeros(need.value, dtype=np.int32)
        _check(_lib.ccd_nm_export_maps(self._h, which, out.ctypes.data_as(_ip), out.size, None),
               "ccd_nm_export_maps")
        return out

    def export_tables(self):
        n = self.info()["n_states"]
        tk, eps, er = np.zeros(n), np.zeros(n), C.c_double()
        _check(_lib.ccd_nm_export_tables(self._h, _dptr(tk), _dptr(eps), C.byref(er)), "ccd_nm_export_tables")
        return tk, eps, er.value

    def element(self, p, q, r, s):
        v = C.c_double()
        _check(_lib.ccd_nm_element(self._h, p, q, r, s, C.byref(v)), "ccd_nm_element")
        return v.value

    def canonical_index(self):
        """(i, j, a, b) of every canonical amplitude."""
        ch = self.export_map(CCD_NM_MAP_CHANNELS).reshape(-1, 7)
        hh = self.export_map(CCD_NM_MAP_HH).reshape(-1, 2)
        pp = self.export_map(CCD_NM_MAP_PP).reshape(-1, 2)
        out, ho, po = [], 0, 0
        for *_, nhh, npp in ch:
            out.append(np.concatenate([np.tile(hh[ho:ho + nhh], (npp, 1)), np.repeat(pp[po:po + npp], nhh, axis=0)],
                                      axis=1))
            ho += nhh
            po += npp
        return np.concatenate(out, axis=0)

    def bind(self, device="cuda"):
        import torch
        n = _sz()
        _check(_lib.ccd_nm_workspace_size(self._h, C.byref(n)), "ccd_nm_workspace_size")
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) & ~255
        _check(_lib.ccd_nm_bind_workspace(self._h, _vp(ptr), n.value), "ccd_nm_bind_workspace")
        return self

    def iterate(self, mixing=1.0, tol=0.0, max_iter=1, terms=CCD_T_ALL, tol_rel=0.0):
        o = ccd_solver_opts(mixing, tol, max_iter, CCD_PREC_FP64, 0, terms, 0.0, 1, 0, tol_rel, 0)
        sw = C.c_int32()
        hist = np.zeros(max_iter)
        st = _lib.ccd_nm_iterate(self._h, C.byref(o), C.byref(sw), _dptr(hist))
        _check(st, "ccd_nm_iterate", ok=(CCD_OK, CCD_NOT_CONVERGED))
        ms = C.c_double()
        _check(_lib.ccd_nm_last_ms(self._h, C.byref(ms)), "ccd_nm_last_ms")
        return {"status": st, "sweeps": sw.value, "history": hist, "gpu_ms": ms.value}

    def set_timing(self, on):
        _check(_lib.ccd_nm_set_timing(self._h, int(bool(on))), "ccd_nm_set_timing")

    def kernel_times(self, reset=False):
        """{family: (ms summed, launches, FP64 flops per launch)}"""
        n = 8
        ms, ln, fl = np.zeros(n), np.zeros(n, dtype=np.int64), np.zeros(n)
        _check(_lib.ccd_nm_kernel_times(self._h, _dptr(ms), ln.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(fl),
                                        int(bool(reset))), "ccd_nm_kernel_times")
        return {_lib.ccd_nm_kernel_name(f).decode(): (ms[f], int(ln[f]), fl[f]) for f in range(n)}

    def energy(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(_lib.ccd_nm_energy(self._h, C.byref(a), C.byref(b), C.byref(c)), "ccd_nm_energy")
        return a.value, b.value, c.value

    def get_amplitudes(self):
        out = np.zeros(self.info()["n_amplitudes"])
        _check(_lib.ccd_nm_get_amplitudes(self._h, _dptr(out), out.size), "ccd_nm_get_amplitudes")
        return out

    def set_amplitudes(self, t):
        t = np.ascontiguousarray(t, dtype=np.float64)
        _check(_lib.ccd_nm_set_amplitudes(self._h, _dptr(t), t.size), "ccd_nm_set_amplitudes")


def canonical_index(ctx: Context, p=0):
    """(i, j, a, b) state indices of every element of the canonical amplitude
    vector of problem p, from the exported maps."""
    ch = ctx.export_map(CCD_MAP_CHANNELS, p).reshape(-1, 6)
    hh = ctx.export_map(CCD_MAP_HH, p).reshape(-1, 2)
    pp = ctx.export_map(CCD_MAP_PP, p).reshape(-1, 2)
    out = []
    ho = po = 0
    for kx, ky, kz, sz, nhh, npp in ch:
        H = hh[ho:ho + nhh]
        Pp = pp[po:po + npp]
        ii = np.repeat(Pp, nhh, axis=0)
        jj = np.tile(H, (npp, 1))
        out.append(np.concatenate([jj, ii], axis=1))
        ho += nhh
        po += npp
    return np.concatenate(out, axis=0) if out else np.zeros((0, 4), dtype=np.int32)


def version():
    return _lib.ccd_version().decode()
