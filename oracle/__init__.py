"""ORACLE — test infrastructure, not product code.

Python binding of the plain FP64 CPU implementation in ``mhd_oracle.cpp``
(one step of the finite-volume ideal-MHD scheme: primitive recovery, PLM,
HLL/HLLD, upwind constrained-transport EMF, SSP-RK2, CFL time step), plus the
exact Euler Riemann solver used to pin it (``exact_euler``).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this package. It shares no code with the GPU library.

Arrays follow the state layout of the method: one float64 array of shape
``(8, nz, ny, nx)`` holding (rho, m_x, m_y, m_z, E, b_x, b_y, b_z); b_d lives
on the lower d-face of each cell; in 2D field 7 is the cell-centred B_z.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhd_oracle.cpp")
_SO = os.path.join(_HERE, "libmhd_oracle.so")

LIMITERS = {"minmod": 0, "vanleer": 1, "wenoz": 2}
SOLVERS = {"hlld": 0, "hll": 1}
PRECISIONS = {"fp64": 0, "mixed": 1}
INTEGRATORS = {"rk2": 0, "rk3": 1}
EMFS = {"uct_hll": 0, "uct_hlld": 1}


class OCfg(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("xmin", ctypes.c_double), ("xmax", ctypes.c_double),
        ("ymin", ctypes.c_double), ("ymax", ctypes.c_double),
        ("zmin", ctypes.c_double), ("zmax", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("riemann", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("nthreads", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("emf", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        cp = P(OCfg)
        for name, args, res in [
            ("oracle_rhs", [cp, dp, dp], ctypes.c_int),
            ("oracle_step", [cp, dp, ctypes.c_double], ctypes.c_int),
            ("oracle_dt", [cp, dp, dp], ctypes.c_int),
            ("oracle_run", [cp, dp, ctypes.c_int, dp], ctypes.c_int),
            ("oracle_run_dts", [cp, dp, ctypes.c_int, dp], ctypes.c_int),
            ("oracle_step_jvp", [cp, dp, dp, ctypes.c_double, ctypes.c_double], ctypes.c_int),
            ("oracle_divb", [cp, dp, dp], ctypes.c_int),
            ("oracle_glm_dt", [cp, dp, dp], ctypes.c_int),
            ("oracle_count_degenerate", [cp, dp, ctypes.POINTER(ctypes.c_longlong)],
             ctypes.c_int),
            ("oracle_glm_run", [cp, dp, ctypes.c_int, dp], ctypes.c_int),
            ("oracle_glm_run_dts", [cp, dp, ctypes.c_int, dp], ctypes.c_int),
            ("oracle_glm_rhs", [cp, dp, dp, ctypes.c_double], ctypes.c_int),
            ("oracle_glm_face", [ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, dp], ctypes.c_int),
            ("oracle_prim", [cp, dp, dp], ctypes.c_int),
            ("oracle_riemann", [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp,
                                ctypes.c_double, dp], ctypes.c_int),
            ("oracle_flux", [ctypes.c_double, dp, ctypes.c_double, dp, dp], ctypes.c_int),
            ("oracle_slope", [ctypes.c_int, ctypes.c_double, ctypes.c_double], ctypes.c_double),
            ("oracle_wenoz", [ctypes.POINTER(ctypes.c_double)], ctypes.c_double),
            ("oracle_fast_speed", [ctypes.c_double] * 6, ctypes.c_double),
            ("oracle_uct", [dp], ctypes.c_double),
            ("oracle_count_ops", [cp, dp, P(ctypes.c_longlong)], ctypes.c_int),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


class Unphysical(OracleError):
    pass


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int):
    if rc == -1:
        raise OracleError("oracle: invalid argument")
    if rc == -4:
        raise Unphysical("oracle: unphysical state (rho <= 0, p <= 0 or non-finite)")


def cfg_from(setup: dict, nthreads: int = 0, **over) -> OCfg:
    """Build the oracle configuration from a workload description dict."""
    s = dict(setup)
    s.update(over)
    box = s["box"]
    return OCfg(int(s["dim"]), int(s["nx"]), int(s["ny"]), int(s["nz"]),
                box[0], box[1], box[2], box[3], box[4], box[5],
                float(s["gamma"]), float(s["cfl"]),
                LIMITERS[s["limiter"]], SOLVERS[s["riemann"]],
                PRECISIONS[s.get("precision", "fp64")], int(nthreads),
                INTEGRATORS[s.get("integrator", "rk2")], EMFS[s.get("emf", "uct_hll")])


def _shape(c: OCfg):
    return (8, c.nz, c.ny, c.nx)


def _state(c: OCfg, U) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.shape != _shape(c):
        raise OracleError("state shape %s, expected %s" % (U.shape, _shape(c)))
    return U


def rhs(c: OCfg, U, allow_unphysical=False) -> np.ndarray:
    U = _state(c, U)
    L = np.empty_like(U)
    rc = _load().oracle_rhs(ctypes.byref(c), _ptr(U), _ptr(L))
    if not (allow_unphysical and rc == -4):
        _check(rc)
    return L


def step(c: OCfg, U, dt: float) -> np.ndarray:
    """One SSP-RK2 (or, with integrator "rk3", SSP-RK3) step with the given
    dt; returns the new state (copy)."""
    U = _state(c, U).copy()
    _check(_load().oracle_step(ctypes.byref(c), _ptr(U), float(dt)))
    return U


def dt(c: OCfg, U) -> float:
    U = _state(c, U)
    out = np.zeros(1)
    _check(_load().oracle_dt(ctypes.byref(c), _ptr(U), _ptr(out)))
    return float(out[0])


def run(c: OCfg, U, nsteps: int):
    """nsteps CFL-limited steps. Returns (new state, array of dts used)."""
    U = _state(c, U).copy()
    dts = np.zeros(max(nsteps, 1))
    _check(_load().oracle_run(ctypes.byref(c), _ptr(U), int(nsteps), _ptr(dts)))
    return U, dts[:nsteps]


def run_dts(c: OCfg, U, dts, allow_unphysical=False) -> np.ndarray:
    """Steps with the given time steps. With ``allow_unphysical`` the state is
    returned even where some cell lost positivity (the oracle computes on)."""
    U = _state(c, U).copy()
    d = np.ascontiguousarray(dts, dtype=np.float64)
    rc = _load().oracle_run_dts(ctypes.byref(c), _ptr(U), len(d), _ptr(d))
    if not (allow_unphysical and rc == -4):
        _check(rc)
    return U


def step_jvp(c: OCfg, U, dU, dt: float, ddt: float = 0.0):
    """Forward-mode tangent of one step: returns (Phi(U), dPhi.(dU, ddt))."""
    U = _state(c, U).copy()
    dU = _state(c, dU).copy()
    _check(_load().oracle_step_jvp(ctypes.byref(c), _ptr(U), _ptr(dU), float(dt), float(ddt)))
    return U, dU


def divb(c: OCfg, U) -> np.ndarray:
    U = _state(c, U)
    out = np.empty(U.shape[1:])
    _check(_load().oracle_divb(ctypes.byref(c), _ptr(U), _ptr(out)))
    return out


def prim(c: OCfg, U, allow_unphysical=False) -> np.ndarray:
    U = _state(c, U)
    V = np.empty_like(U)
    rc = _load().oracle_prim(ctypes.byref(c), _ptr(U), _ptr(V))
    if not (allow_unphysical and rc == -4):
        _check(rc)
    return V


def riemann(wl, wr, bn, gamma=5.0 / 3.0, solver="hlld", precision="fp64") -> np.ndarray:
    """Single face problem. w = (rho, u, v, w, B_t1, B_t2, p).
    Returns 16 values: flux of (rho, m_n, m_t1, m_t2, B_t1, B_t2, E),
    alpha+, alpha-, the HLL-weighted vt1, vt2, then the UCT-HLLD coefficients
    om, d^L, d^R and the om-weighted vt1, vt2."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    out = np.zeros(16)
    _check(_load().oracle_riemann(SOLVERS[solver], PRECISIONS[precision], float(gamma),
                                  _ptr(wl), _ptr(wr), float(bn), _ptr(out)))
    return out


def flux(w, bn, gamma=5.0 / 3.0):
    """Physical flux of one face-frame primitive state: returns (U7, F7)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    U7 = np.zeros(7)
    F7 = np.zeros(7)
    _check(_load().oracle_flux(float(gamma), _ptr(w), float(bn), _ptr(U7), _ptr(F7)))
    return U7, F7


def slope(limiter: str, dm: float, dp: float) -> float:
    return float(_load().oracle_slope(LIMITERS[limiter], float(dm), float(dp)))


def wenoz(v) -> float:
    """WENO-Z value at the upper interface of the middle of five cell values."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (5,)
    return float(_load().oracle_wenoz(_ptr(v)))


def fast_speed(gamma, rho, p, bn, bt1, bt2) -> float:
    return float(_load().oracle_fast_speed(gamma, rho, p, bn, bt1, bt2))


def uct(apa, ama, vW, bW, vE, bE, apb, amb, vS, bS, vN, bN) -> float:
    a = np.array([apa, ama, vW, bW, vE, bE, apb, amb, vS, bS, vN, bN], dtype=np.float64)
    return float(_load().oracle_uct(_ptr(a)))


def count_ops(c: OCfg, U) -> dict:
    """Floating-point operations of one right-hand side per phase
    (prims, faces, emf, update), each {add, mul, div, sqrt} totals."""
    U = _state(c, U)
    out = (ctypes.c_longlong * 16)()
    _check(_load().oracle_count_ops(ctypes.byref(c), _ptr(U), out))
    names = ("prims", "faces", "emf", "update")
    kinds = ("add", "mul", "div", "sqrt")
    return {names[p]: {kinds[k]: int(out[4 * p + k]) for k in range(4)} for p in range(4)}


# ------------------------------------------------------- GLM cleaning ----
GLM_ALPHA = 0.1  # damping of psi per step: exp(-GLM_ALPHA * c_h dt / min spacing)


def _glm_state(c: OCfg, U) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    assert U.shape == (9, c.nz, c.ny, c.nx), U.shape
    return U


def glm_dt(c: OCfg, U) -> float:
    out = ctypes.c_double(0.0)
    _check(_load().oracle_glm_dt(ctypes.byref(c), _ptr(_glm_state(c, U)), ctypes.byref(out)))
    return out.value


def glm_run(c: OCfg, U, nsteps: int):
    """nsteps GLM steps (CFL dt each); returns (state, dts)."""
    U = _glm_state(c, U).copy()
    dts = np.zeros(max(nsteps, 1))
    _check(_load().oracle_glm_run(ctypes.byref(c), _ptr(U), int(nsteps), _ptr(dts)))
    return U, dts[:nsteps]


def glm_run_dts(c: OCfg, U, dts) -> np.ndarray:
    U = _glm_state(c, U).copy()
    d = np.ascontiguousarray(dts, dtype=np.float64)
    _check(_load().oracle_glm_run_dts(ctypes.byref(c), _ptr(U), len(d), _ptr(d)))
    return U


def glm_rhs(c: OCfg, U, ch: float) -> np.ndarray:
    U = _glm_state(c, U)
    L = np.zeros_like(U)
    _check(_load().oracle_glm_rhs(ctypes.byref(c), _ptr(U), _ptr(L), float(ch)))
    return L


def glm_face(wl, wr, bnl, bnr, psil, psir, ch, gamma=5.0 / 3.0, solver="hlld") -> np.ndarray:
    """One GLM face: fluxes of (rho, m_n, m_t1, m_t2, B_t1, B_t2, E, B_n, psi)."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    out = np.zeros(9)
    _check(_load().oracle_glm_face(SOLVERS[solver], float(gamma), _ptr(wl), _ptr(wr), float(bnl),
                                   float(bnr), float(psil), float(psir), float(ch), _ptr(out)))
    return out


def divb_centred(c: OCfg, U) -> np.ndarray:
    """Central-difference div B of a GLM state (cell-centred B), test-side."""
    U = _glm_state(c, U)
    dx = (c.xmax - c.xmin) / c.nx
    dy = (c.ymax - c.ymin) / c.ny
    dz = (c.zmax - c.zmin) / c.nz
    d = (np.roll(U[5], -1, 2) - np.roll(U[5], 1, 2)) / (2 * dx) + \
        (np.roll(U[6], -1, 1) - np.roll(U[6], 1, 1)) / (2 * dy)
    if c.dim == 3:
        d = d + (np.roll(U[7], -1, 0) - np.roll(U[7], 1, 0)) / (2 * dz)
    return d


def count_degenerate(c: OCfg, U) -> dict:
    """HLLD star sides evaluated and found degenerate in one right-hand side
    of U, in FP64 and in the mixed (FP32) variant."""
    U = _state(c, U)
    out = (ctypes.c_longlong * 4)()
    _check(_load().oracle_count_degenerate(ctypes.byref(c), _ptr(U), out))
    return {"fp64": (int(out[0]), int(out[1])), "fp32": (int(out[2]), int(out[3]))}
