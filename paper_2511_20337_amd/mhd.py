"""Thin ctypes binding of libmhd.so (C ABI in include/mhd.h).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch supplies device memory (the state, adjoint arrays and workspace are
torch tensors) and the stream (torch's current stream). The functions keep the
C names; ``Context`` bundles a context handle with its workspace.

The library must be built (``python -m paper_2511_20337_amd.build``); if it is
missing every call raises — there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhd.so")

MHD_OK = 0
MHD_ERR_INVALID = -1
MHD_ERR_UNSUPPORTED = -2
MHD_ERR_DEVICE = -3
MHD_ERR_UNPHYSICAL = -4
MHD_ERR_WORKSPACE = -5

LIMITERS = {"minmod": 0, "vanleer": 1, "wenoz": 2}
SOLVERS = {"hlld": 0, "hll": 1}
PRECISIONS = {"fp64": 0, "mixed": 1}
INTEGRATORS = {"rk2": 0, "rk3": 1}
EMFS = {"uct_hll": 0, "uct_hlld": 1}
DIVB = {"ct": 0, "glm": 1}

# Every symbol include/mhd.h declares.
SYMBOLS = ("mhd_init", "mhd_destroy", "mhd_workspace_bytes", "mhd_dt", "mhd_dt_device",
           "mhd_dt_device_noalloc", "mhd_step", "mhd_step_device_dt", "mhd_step_cfl", "mhd_rhs",
           "mhd_adjoint_step",
           "mhd_adjoint_step_device", "mhd_check",
           "mhd_timing", "mhd_timing_read", "mhd_strerror", "mhd_last_error")


class mhd_config(ctypes.Structure):  # noqa: N801 — C name
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("xmin", ctypes.c_double), ("xmax", ctypes.c_double),
        ("ymin", ctypes.c_double), ("ymax", ctypes.c_double),
        ("zmin", ctypes.c_double), ("zmax", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("riemann", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("integrator", ctypes.c_int32),
        ("emf", ctypes.c_int32), ("divb", ctypes.c_int32),
    ]


class MHDError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s (%d)%s" % (strerror(status), status, (": " + msg) if msg else ""))


class Unphysical(MHDError):
    pass


_lib = None


def lib():
    """Load libmhd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmhd.so not built: run python -m paper_2511_20337_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
        st = ctypes.c_int
        sig = {
            "mhd_init": ([ctypes.POINTER(mhd_config), ctypes.POINTER(vp)], st),
            "mhd_destroy": ([vp], None),
            "mhd_workspace_bytes": ([vp, ctypes.c_int32], sz),
            "mhd_dt": ([vp, vp, vp, sz, dp, vp], st),
            "mhd_dt_device": ([vp, vp, vp, sz, vp, vp], st),
            "mhd_dt_device_noalloc": ([vp, vp, vp, vp, vp], st),
            "mhd_step": ([vp, vp, ctypes.c_double, vp, sz, vp], st),
            "mhd_step_device_dt": ([vp, vp, vp, vp, sz, vp], st),
            "mhd_step_cfl": ([vp, vp, vp, vp, sz, vp], st),
            "mhd_rhs": ([vp, vp, vp, vp, sz, vp], st),
            "mhd_adjoint_step": ([vp, vp, ctypes.c_double, vp, vp, dp, vp, sz, vp], st),
            "mhd_adjoint_step_device": ([vp, vp, ctypes.c_double, vp, vp, vp, vp, sz, vp], st),
            "mhd_check": ([vp, vp, sz, vp], st),
            "mhd_timing": ([vp, ctypes.c_int32], st),
            "mhd_timing_read": ([vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p),
                                 ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int64)], st),
            "mhd_strerror": ([st], ctypes.c_char_p),
            "mhd_last_error": ([vp], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def strerror(status: int) -> str:
    try:
        return lib().mhd_strerror(int(status)).decode()
    except ImportError:
        return "status"


def config_from(setup: dict) -> mhd_config:
    b = setup["box"]
    return mhd_config(int(setup["dim"]), int(setup["nx"]), int(setup["ny"]), int(setup["nz"]),
                      b[0], b[1], b[2], b[3], b[4], b[5], float(setup["gamma"]),
                      float(setup["cfl"]), LIMITERS[setup["limiter"]], SOLVERS[setup["riemann"]],
                      PRECISIONS[setup.get("precision", "fp64")],
                      INTEGRATORS[setup.get("integrator", "rk2")],
                      EMFS[setup.get("emf", "uct_hll")], DIVB[setup.get("divb", "ct")])


# ---------------------------------------------------------------- C names --
def mhd_init(cfg: mhd_config) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = lib().mhd_init(ctypes.byref(cfg), ctypes.byref(h))
    if rc != MHD_OK:
        raise MHDError(rc, "mhd_init")
    return h


def mhd_destroy(ctx) -> None:
    lib().mhd_destroy(ctx)


def mhd_workspace_bytes(ctx, with_adjoint: bool = False) -> int:
    return int(lib().mhd_workspace_bytes(ctx, 1 if with_adjoint else 0))


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _raise(ctx, rc, what):
    if rc == MHD_OK:
        return
    msg = lib().mhd_last_error(ctx).decode() if ctx else ""
    if rc == MHD_ERR_UNPHYSICAL:
        raise Unphysical(rc, what)
    raise MHDError(rc, "%s %s" % (what, msg))


def mhd_dt(ctx, U, ws) -> float:
    out = ctypes.c_double(0.0)
    rc = lib().mhd_dt(ctx, U.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.byref(out),
                      _stream(U.device))
    _raise(ctx, rc, "mhd_dt")
    return out.value


def mhd_dt_device(ctx, U, ws, dt_dev) -> None:
    rc = lib().mhd_dt_device(ctx, U.data_ptr(), ws.data_ptr(), ws.numel(), dt_dev.data_ptr(),
                             _stream(U.device))
    _raise(ctx, rc, "mhd_dt_device")


def mhd_dt_device_noalloc(ctx, U, dt_dev, flag_dev=None) -> None:
    """dt_dev: float64 device tensor; flag_dev: int32 device tensor or None."""
    rc = lib().mhd_dt_device_noalloc(ctx, U.data_ptr(), dt_dev.data_ptr(),
                                     None if flag_dev is None else flag_dev.data_ptr(),
                                     _stream(U.device))
    _raise(ctx, rc, "mhd_dt_device_noalloc")


def mhd_step(ctx, U, dt: float, ws) -> None:
    rc = lib().mhd_step(ctx, U.data_ptr(), float(dt), ws.data_ptr(), ws.numel(),
                        _stream(U.device))
    _raise(ctx, rc, "mhd_step")


def mhd_step_device_dt(ctx, U, dt_dev, ws) -> None:
    rc = lib().mhd_step_device_dt(ctx, U.data_ptr(), dt_dev.data_ptr(), ws.data_ptr(),
                                  ws.numel(), _stream(U.device))
    _raise(ctx, rc, "mhd_step_device_dt")


def mhd_step_cfl(ctx, U, dt_dev, ws) -> None:
    rc = lib().mhd_step_cfl(ctx, U.data_ptr(), dt_dev.data_ptr(), ws.data_ptr(), ws.numel(),
                            _stream(U.device))
    _raise(ctx, rc, "mhd_step_cfl")


def mhd_rhs(ctx, U, L, ws) -> None:
    rc = lib().mhd_rhs(ctx, U.data_ptr(), L.data_ptr(), ws.data_ptr(), ws.numel(),
                       _stream(U.device))
    _raise(ctx, rc, "mhd_rhs")


def mhd_adjoint_step(ctx, U_n, dt: float, Ubar_np1, Ubar_n, ws, want_dtbar=False):
    dtbar = ctypes.c_double(0.0)
    rc = lib().mhd_adjoint_step(ctx, U_n.data_ptr(), float(dt), Ubar_np1.data_ptr(),
                                Ubar_n.data_ptr(), ctypes.byref(dtbar) if want_dtbar else None,
                                ws.data_ptr(), ws.numel(), _stream(U_n.device))
    _raise(ctx, rc, "mhd_adjoint_step")
    return dtbar.value if want_dtbar else None


def mhd_adjoint_step_device(ctx, U_n, dt: float, Ubar_np1, Ubar_n, ws, dtbar_dev=None):
    """dtbar_dev: a float64 device tensor of at least one element (or None)."""
    ptr = None if dtbar_dev is None else dtbar_dev.data_ptr()
    rc = lib().mhd_adjoint_step_device(ctx, U_n.data_ptr(), float(dt), Ubar_np1.data_ptr(),
                                       Ubar_n.data_ptr(), ptr, ws.data_ptr(), ws.numel(),
                                       _stream(U_n.device))
    _raise(ctx, rc, "mhd_adjoint_step_device")


def mhd_check(ctx, ws, device=None) -> None:
    rc = lib().mhd_check(ctx, ws.data_ptr(), ws.numel(), _stream(device or ws.device))
    _raise(ctx, rc, "mhd_check")


def mhd_timing(ctx, enable: bool) -> None:
    _raise(ctx, lib().mhd_timing(ctx, 1 if enable else 0), "mhd_timing")


def mhd_timing_read(ctx) -> dict:
    """{kernel name: (total ms, launches)} for every kernel index."""
    out = {}
    k = 0
    while True:
        name = ctypes.c_char_p()
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        rc = lib().mhd_timing_read(ctx, k, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(cnt))
        if rc == MHD_ERR_INVALID:
            break
        _raise(ctx, rc, "mhd_timing_read")
        out[name.value.decode()] = (ms.value, cnt.value)
        k += 1
    return out


# ------------------------------------------------------------- Context ----
class Context:
    """A library context plus its device workspace (a torch uint8 tensor)."""

    def __init__(self, setup: dict, device="cuda", with_adjoint: bool = False):
        import torch
        self.setup = dict(setup)
        self.cfg = config_from(setup)
        self.device = torch.device(device)
        nf = 9 if setup.get("divb", "ct") == "glm" else 8  # GLM adds psi
        self.shape = (nf, int(setup["nz"]), int(setup["ny"]), int(setup["nx"]))
        self.ctx = mhd_init(self.cfg)
        nbytes = mhd_workspace_bytes(self.ctx, with_adjoint)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws = self.ws[off:off + nbytes]
        self.ws[:256].zero_()
        self.dt_dev = torch.zeros(1, dtype=torch.float64, device=self.device)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and _lib is not None:
            _lib.mhd_destroy(ctx)
            self.ctx = None

    def _state(self, U):
        import torch
        if not (isinstance(U, torch.Tensor) and U.dtype == torch.float64 and U.is_cuda and
                U.is_contiguous() and tuple(U.shape) == self.shape):
            raise MHDError(MHD_ERR_INVALID, "state must be a contiguous float64 CUDA tensor "
                           "of shape %s" % (self.shape,))
        return U

    def dt(self, U) -> float:
        return mhd_dt(self.ctx, self._state(U), self.ws)

    def dt_device(self, U, out=None):
        out = self.dt_dev if out is None else out
        mhd_dt_device(self.ctx, self._state(U), self.ws, out)
        return out

    def step(self, U, dt: float):
        mhd_step(self.ctx, self._state(U), dt, self.ws)
        return U

    def step_device_dt(self, U, dt_dev=None):
        mhd_step_device_dt(self.ctx, self._state(U), self.dt_dev if dt_dev is None else dt_dev,
                           self.ws)
        return U

    def step_cfl(self, U, dt_dev=None):
        """One step with dt = the CFL step of U, left in dt_dev (default:
        self.dt_dev); no host synchronisation."""
        import torch
        dt_dev = self.dt_dev if dt_dev is None else dt_dev
        if dt_dev.dtype != torch.float64 or dt_dev.device != self.device or dt_dev.numel() < 1:
            raise MHDError(MHD_ERR_INVALID, "dt_dev: a float64 tensor on the device")
        mhd_step_cfl(self.ctx, self._state(U), dt_dev, self.ws)
        return U

    def rhs(self, U, out=None):
        import torch
        out = torch.empty_like(U) if out is None else out
        mhd_rhs(self.ctx, self._state(U), self._state(out), self.ws)
        return out

    def adjoint_step(self, U_n, dt: float, Ubar_np1, want_dtbar=False, out=None,
                     dtbar_out=None):
        """Ubar_n (and dt-bar as a host float with want_dtbar). With dtbar_out
        (a float64 device tensor), dt-bar is written there without a host
        synchronisation."""
        import torch
        out = torch.empty_like(Ubar_np1) if out is None else out
        if dtbar_out is not None:
            if dtbar_out.dtype != torch.float64 or dtbar_out.device != self.device or \
                    dtbar_out.numel() < 1:
                raise MHDError(MHD_ERR_INVALID, "dtbar_out: a float64 tensor on the device")
            mhd_adjoint_step_device(self.ctx, self._state(U_n), dt, self._state(Ubar_np1),
                                    self._state(out), self.ws, dtbar_out)
            return out
        dtbar = mhd_adjoint_step(self.ctx, self._state(U_n), dt, self._state(Ubar_np1),
                                 self._state(out), self.ws, want_dtbar)
        return (out, dtbar) if want_dtbar else out

    def check(self):
        mhd_check(self.ctx, self.ws, self.device)

    def run(self, U, nsteps: int):
        """nsteps CFL-limited steps, dt computed on the device each step."""
        for _ in range(nsteps):
            self.step_cfl(U)
        return U
