"""ctypes binding of libhotrg.so (include/hotrg.h), argument marshalling only.

Every step of a solve runs in the library's HIP kernels on the device; this
module only converts Python values to C arguments and takes device memory and
streams from PyTorch.  There is no CPU fallback: if the built library is
missing the import of any entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads torch's HIP runtime first; the library then binds to it)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhotrg.so")

# status codes
OK, EINVAL, ENOMEM, EHIP, EEIG, ENONFINITE, ESTATE, ENODEV = 0, -1, -2, -3, -4, -5, -6, -7
# models and precisions
ISING, POTTS, CUSTOM, QCHAIN = 0, 1, 2, 3
FP64, FP32, BF16X3, BF16X6, FP16X3 = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6, "fp16x3": FP16X3}
MODELS = {"ising": ISING, "potts": POTTS, "custom": CUSTOM, "qchain": QCHAIN}
MAX_STEPS = 60
# how a step's eigensolve ended (hotrg_eig_info)
EIG_CONVERGED, EIG_STAGNATED, EIG_PASS_CAP = 0, 1, 2
EIG_MAX_PASSES = 60
# host-polled stepping (hotrg_step_poll)
POLL_IDLE, POLL_RUNNING, POLL_PASSES, POLL_STEPPED = 0, 1, 2, 3
STAGES = ["permute", "env", "eig", "x", "y", "tp", "norm", "obs"]
# observable slots (hotrg_observables): order parameter per site, energy of one y bond
OBS_MAGNETIZATION, OBS_BOND_ENERGY = 1, 2
OBSERVABLES = {"m": OBS_MAGNETIZATION, "e": OBS_BOND_ENERGY}

EXPORTS = [
    "hotrg_workspace_bytes", "hotrg_init_tensor", "hotrg_reset", "hotrg_coarse_grain",
    "hotrg_coarse_grain_batch", "hotrg_coarse_grain_axis", "hotrg_step_begin", "hotrg_step_poll",
    "hotrg_coarse_grain_async", "hotrg_async_busy",
    "hotrg_log_z", "hotrg_log_z_chain",
    "hotrg_step_info", "hotrg_step_sides", "hotrg_observables", "hotrg_eig_info", "hotrg_set_eig_limits",
    "hotrg_copy_tensor", "hotrg_copy_environment", "hotrg_copy_isometry", "hotrg_set_timing", "hotrg_stage_times", "hotrg_step_stage_times",
    "hotrg_gemm_y_time", "hotrg_destroy", "hotrg_strerror", "hotrg_device_count",
    "hotrg_runtime_version", "hotrg_gemm_scratch_bytes", "hotrg_gemm_nt", "hotrg_gemm_nt_role",
    "hotrg_gemm_nt_noalloc",
    "itebd_state_len", "itebd_workspace_bytes", "itebd_init", "itebd_evolve", "itebd_energy",
    "itebd_copy_states", "itebd_info", "itebd_work", "itebd_status", "itebd_set_max_sweeps", "itebd_destroy",
]
ITEBD_MAX_CHI = 32
ITEBD_MAX_SWEEPS = 40
# bits of an iTEBD chain's status word (itebd_status)
ITEBD_CHAIN_SWEEP_CAP, ITEBD_CHAIN_NONFINITE = 1, 2


class HotrgError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_strerror(status)} ({status})")


class Params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int),
        ("q", ctypes.c_int),
        ("coupling", ctypes.c_double),
        ("temperature", ctypes.c_double),
        ("dmax", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("custom_tensor", ctypes.POINTER(ctypes.c_double)),
        ("custom_dx", ctypes.c_int),
        ("custom_dy", ctypes.c_int),
        ("max_steps", ctypes.c_int),
        ("field", ctypes.c_double),
        ("two_sided", ctypes.c_int),
        ("observables", ctypes.c_int),
        ("custom_impurity", ctypes.POINTER(ctypes.c_double) * 2),
        ("bond_h", ctypes.POINTER(ctypes.c_double)),
        ("tau", ctypes.c_double),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libhotrg.so (built by paper_2602_05900_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_05900_amd.build` "
                          "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_size_t, c_long, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_long, ctypes.c_void_p
    P = ctypes.POINTER
    lib.hotrg_workspace_bytes.argtypes = [P(Params)]
    lib.hotrg_workspace_bytes.restype = c_size_t
    lib.hotrg_init_tensor.argtypes = [P(Params), c_void_p, c_size_t, c_void_p, P(c_void_p)]
    lib.hotrg_reset.argtypes = [c_void_p, P(Params)]
    lib.hotrg_coarse_grain.argtypes = [c_void_p, c_int]
    lib.hotrg_coarse_grain_batch.argtypes = [P(c_void_p), c_int, c_int]
    lib.hotrg_coarse_grain_axis.argtypes = [c_void_p, c_int, c_int]
    lib.hotrg_step_begin.argtypes = [c_void_p, c_int, c_int, P(c_int)]
    lib.hotrg_step_poll.argtypes = [c_void_p, P(c_int)]
    lib.hotrg_coarse_grain_async.argtypes = [c_void_p, c_int, c_int, c_int]
    lib.hotrg_async_busy.argtypes = [c_void_p, P(c_int)]
    lib.hotrg_log_z_chain.argtypes = [c_void_p, P(c_double)]
    lib.hotrg_log_z.argtypes = [c_void_p, P(c_double), P(c_int)]
    lib.hotrg_step_info.argtypes = [c_void_p, c_int, P(c_double), P(c_double), P(c_double)]
    lib.hotrg_eig_info.argtypes = [c_void_p, c_int, P(c_int), P(c_int), P(c_double), P(c_int)]
    lib.hotrg_set_eig_limits.argtypes = [c_void_p, c_int, c_double]
    lib.hotrg_step_sides.argtypes = [c_void_p, c_int, P(c_double), P(c_double), P(c_int)]
    lib.hotrg_observables.argtypes = [c_void_p, P(c_double)]
    lib.hotrg_copy_tensor.argtypes = [c_void_p, P(c_double), c_size_t, P(c_int)]
    lib.hotrg_copy_environment.argtypes = [c_void_p, P(c_double), c_size_t, P(c_int)]
    lib.hotrg_copy_isometry.argtypes = [c_void_p, P(c_double), c_size_t, P(c_int)]
    lib.hotrg_set_timing.argtypes = [c_void_p, c_int]
    lib.hotrg_stage_times.argtypes = [c_void_p, P(c_double), P(c_int)]
    lib.hotrg_step_stage_times.argtypes = [c_void_p, c_int, P(c_double), P(c_int)]
    lib.hotrg_gemm_y_time.argtypes = [c_void_p, P(c_double), P(c_int)]
    lib.hotrg_destroy.argtypes = [c_void_p]
    lib.hotrg_destroy.restype = None
    lib.hotrg_strerror.argtypes = [c_int]
    lib.hotrg_strerror.restype = ctypes.c_char_p
    lib.hotrg_device_count.argtypes = [P(c_int)]
    lib.hotrg_runtime_version.argtypes = [P(c_int)]
    lib.hotrg_gemm_scratch_bytes.argtypes = [c_int, c_int, c_int, c_int]
    lib.hotrg_gemm_scratch_bytes.restype = c_size_t
    lib.hotrg_gemm_nt.argtypes = [c_int, c_int, c_int, c_int, c_void_p, c_long, c_void_p, c_long,
                                  c_void_p, c_double, c_long, c_long, c_long, c_long, c_long, c_long,
                                  c_void_p, c_void_p]
    lib.hotrg_gemm_nt_noalloc.argtypes = [c_int, c_int, c_int, c_int, c_int, c_int, c_void_p, c_long, c_void_p,
                                          c_long, c_void_p, c_double, c_long, c_long, c_long, c_long, c_long,
                                          c_long, c_void_p]
    lib.hotrg_gemm_nt_role.argtypes = [c_int, c_int, c_int, c_int, c_int, c_int, c_void_p, c_long, c_void_p, c_long,
                                       c_void_p, c_double, c_long, c_long, c_long, c_long, c_long, c_long,
                                       c_void_p, c_void_p]
    lib.itebd_state_len.argtypes = [c_int]
    lib.itebd_state_len.restype = c_size_t
    lib.itebd_workspace_bytes.argtypes = [c_int, c_int]
    lib.itebd_workspace_bytes.restype = c_size_t
    lib.itebd_init.argtypes = [c_int, c_int, P(c_double), P(c_double), c_void_p, c_size_t, c_void_p, P(c_void_p)]
    lib.itebd_evolve.argtypes = [c_void_p, c_double, c_int]
    lib.itebd_energy.argtypes = [c_void_p, P(c_double)]
    lib.itebd_copy_states.argtypes = [c_void_p, P(c_double), c_size_t]
    lib.itebd_info.argtypes = [c_void_p, P(ctypes.c_long), P(c_int)]
    lib.itebd_work.argtypes = [c_void_p, P(c_double), P(c_double)]
    lib.itebd_status.argtypes = [c_void_p, P(c_int)]
    lib.itebd_set_max_sweeps.argtypes = [c_void_p, c_int]
    lib.itebd_destroy.argtypes = [c_void_p]
    lib.itebd_destroy.restype = None
    for name in EXPORTS:
        getattr(lib, name)  # every declared entry point must resolve
    _lib = lib
    return lib


def _strerror(status: int) -> str:
    try:
        return load().hotrg_strerror(status).decode()
    except ImportError:
        return "unknown"


def _check(status: int, what: str):
    if status != OK:
        raise HotrgError(status, what)


def device_count() -> int:
    n = ctypes.c_int(0)
    _check(load().hotrg_device_count(ctypes.byref(n)), "hotrg_device_count")
    return n.value


def runtime_version() -> int:
    v = ctypes.c_int(0)
    _check(load().hotrg_runtime_version(ctypes.byref(v)), "hotrg_runtime_version")
    return v.value


def make_params(model: str = "ising", q: int = 2, temperature: float = 2.0, dmax: int = 8,
                precision: str = "fp64", coupling: float = 1.0, tensor=None, max_steps: int = 0,
                field: float = 0.0, two_sided: bool = False, observables=(), impurities=None,
                bond_h=None, tau: float = 0.0) -> tuple:
    """hotrg_params plus the host arrays it points to (kept alive by the caller).

    observables: names from OBSERVABLES ("m", "e"); for the custom model,
    impurities maps each of them to a tensor of the custom tensor's dims."""
    p = Params()
    p.model = MODELS[model]
    p.q = q
    p.coupling = coupling
    p.temperature = temperature
    p.dmax = dmax
    p.precision = PRECISIONS[precision]
    p.max_steps = max_steps
    p.field = field
    p.two_sided = 1 if two_sided else 0
    mask = 0
    for o in observables:
        mask |= OBSERVABLES[o]
    p.observables = mask
    keep = []
    if model == "qchain":
        import numpy as np
        hb = np.ascontiguousarray(bond_h, dtype=np.float64).reshape(16)
        keep.append(hb)
        p.bond_h = hb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.tau = tau
    if model == "custom":
        import numpy as np
        t = np.ascontiguousarray(tensor, dtype=np.float64)
        if t.ndim != 4 or t.shape[0] != t.shape[1] or t.shape[2] != t.shape[3]:
            raise ValueError("custom tensor must have dims [Dx, Dx, Dy, Dy]")
        keep.append(t)
        p.custom_tensor = t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.custom_dx, p.custom_dy = t.shape[0], t.shape[2]
        for o in observables:
            imp = np.ascontiguousarray((impurities or {})[o], dtype=np.float64)
            if imp.shape != t.shape:
                raise ValueError("impurity tensors must have the custom tensor's dims")
            keep.append(imp)
            p.custom_impurity[OBSERVABLES[o] - 1] = imp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return p, keep


def workspace_bytes(**kw) -> int:
    p, _keep = make_params(**kw)
    return int(load().hotrg_workspace_bytes(ctypes.byref(p)))


class Solve:
    """One HOTRG solve on the device.  Workspace: a torch uint8 tensor of
    hotrg_workspace_bytes(); stream: a torch.cuda.Stream (default: current)."""

    def __init__(self, model: str = "ising", q: int = 2, temperature: float = 2.0, dmax: int = 8,
                 precision: str = "fp64", coupling: float = 1.0, tensor=None, stream=None,
                 workspace=None, device="cuda", max_steps: int = 0, field: float = 0.0,
                 two_sided: bool = False, observables=(), impurities=None, bond_h=None, tau: float = 0.0):
        lib = load()
        self._lib = lib
        p, keep = make_params(model, q, temperature, dmax, precision, coupling, tensor, max_steps,
                              field, two_sided, observables, impurities, bond_h, tau)
        self.tau = tau
        nbytes = lib.hotrg_workspace_bytes(ctypes.byref(p))
        if nbytes == 0:
            raise HotrgError(EINVAL, "hotrg_workspace_bytes")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.workspace = workspace
        self.temperature = temperature
        h = ctypes.c_void_p()
        _check(lib.hotrg_init_tensor(ctypes.byref(p), ctypes.c_void_p(workspace.data_ptr()),
                                     ctypes.c_size_t(workspace.numel()),
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "hotrg_init_tensor")
        del keep
        self._h = h

    def reset(self, model: str = "ising", q: int = 2, temperature: float = 2.0, dmax: int = 8,
              precision: str = "fp64", coupling: float = 1.0, tensor=None, max_steps: int = 0,
              field: float = 0.0, two_sided: bool = False, observables=(), impurities=None,
              bond_h=None, tau: float = 0.0) -> "Solve":
        """Restart this handle (same workspace, stream and eigensolver context)."""
        p, keep = make_params(model, q, temperature, dmax, precision, coupling, tensor, max_steps,
                              field, two_sided, observables, impurities, bond_h, tau)
        self.tau = tau
        _check(self._lib.hotrg_reset(self._h, ctypes.byref(p)), "hotrg_reset")
        del keep
        self.temperature = temperature
        return self

    def coarse_grain(self, nsteps: int, exchange: bool = True) -> "Solve":
        if exchange:
            _check(self._lib.hotrg_coarse_grain(self._h, int(nsteps)), "hotrg_coarse_grain")
        else:
            _check(self._lib.hotrg_coarse_grain_axis(self._h, int(nsteps), 0), "hotrg_coarse_grain_axis")
        return self

    def step_begin(self, exchange: bool = True, extra: int = 0) -> bool:
        """Begin one host-polled step (hotrg_step_begin) with `extra` passes
        beyond the handle's history; True if it waits for step_poll, False
        if the whole step was enqueued."""
        pending = ctypes.c_int()
        _check(self._lib.hotrg_step_begin(self._h, 1 if exchange else 0, int(extra), ctypes.byref(pending)),
               "hotrg_step_begin")
        return bool(pending.value)

    def step_poll(self) -> int:
        """One non-waiting poll of the pending step (hotrg_step_poll): one of
        POLL_IDLE, POLL_RUNNING, POLL_PASSES, POLL_STEPPED."""
        state = ctypes.c_int()
        _check(self._lib.hotrg_step_poll(self._h, ctypes.byref(state)), "hotrg_step_poll")
        return state.value

    def coarse_grain_async(self, nsteps: int, exchange: bool = True, extra: int = 0) -> "Solve":
        """Hand nsteps host-polled steps to the library's progress thread
        (hotrg_coarse_grain_async); returns at once."""
        _check(self._lib.hotrg_coarse_grain_async(self._h, int(nsteps), 1 if exchange else 0, int(extra)),
               "hotrg_coarse_grain_async")
        return self

    def async_busy(self) -> bool:
        """True while the progress thread still has steps of this solve to
        enqueue (hotrg_async_busy); never waits."""
        busy = ctypes.c_int()
        _check(self._lib.hotrg_async_busy(self._h, ctypes.byref(busy)), "hotrg_async_busy")
        return bool(busy.value)

    def log_z_chain(self) -> float:
        """ln Z per tensor with x infinite and y closed (hotrg_log_z_chain)."""
        v = ctypes.c_double()
        _check(self._lib.hotrg_log_z_chain(self._h, ctypes.byref(v)), "hotrg_log_z_chain")
        return v.value

    def log_z(self) -> float:
        v = ctypes.c_double()
        n = ctypes.c_int()
        _check(self._lib.hotrg_log_z(self._h, ctypes.byref(v), ctypes.byref(n)), "hotrg_log_z")
        return v.value

    def free_energy(self) -> float:
        return -self.temperature * self.log_z()

    def step_info(self, n: int):
        c, e, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self._lib.hotrg_step_info(self._h, int(n), ctypes.byref(c), ctypes.byref(e), ctypes.byref(g)),
               "hotrg_step_info")
        return c.value, e.value, g.value

    def step_sides(self, n: int):
        """(eps_left, eps_right, side) of step n (two-sided truncation)."""
        el, er, sd = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(self._lib.hotrg_step_sides(self._h, int(n), ctypes.byref(el), ctypes.byref(er), ctypes.byref(sd)),
               "hotrg_step_sides")
        return el.value, er.value, sd.value

    def observables(self):
        """{"m": <m>, "e": <e_b>} of the carried impurity tensors (NaN when not carried)."""
        v = (ctypes.c_double * 2)()
        _check(self._lib.hotrg_observables(self._h, v), "hotrg_observables")
        return {"m": v[0], "e": v[1]}

    def _eig_info(self, n: int):
        it, sw, r, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
        _check(self._lib.hotrg_eig_info(self._h, int(n), ctypes.byref(it), ctypes.byref(sw), ctypes.byref(r),
                                        ctypes.byref(st)), "hotrg_eig_info")
        return it.value, sw.value, r.value, st.value

    def eig_info(self, n: int):
        """(subspace passes, Jacobi sweeps, relative residual) of step n's eigensolve."""
        return self._eig_info(n)[:3]

    def eig_stop(self, n: int) -> int:
        """How step n's eigensolve ended: EIG_CONVERGED, EIG_STAGNATED or EIG_PASS_CAP."""
        return self._eig_info(n)[3]

    def set_eig_limits(self, max_passes: int = 30, fail_residual: float = 5e-2) -> "Solve":
        """Pass cap and failure bound of the eigensolves enqueued from now on."""
        _check(self._lib.hotrg_set_eig_limits(self._h, int(max_passes), float(fail_residual)),
               "hotrg_set_eig_limits")
        return self

    def tensor(self):
        import numpy as np
        dims = (ctypes.c_int * 2)()
        self._lib.hotrg_copy_tensor(self._h, None, 0, dims)
        dx, dy = dims[0], dims[1]
        out = np.empty((dx, dx, dy, dy), dtype=np.float64)
        _check(self._lib.hotrg_copy_tensor(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           out.size, dims), "hotrg_copy_tensor")
        return out

    def environment(self):
        """The last step's symmetrised left environment E (n x n, FP64)."""
        import numpy as np
        n = ctypes.c_int()
        self._lib.hotrg_copy_environment(self._h, None, 0, ctypes.byref(n))
        out = np.empty((n.value, n.value), dtype=np.float64)
        _check(self._lib.hotrg_copy_environment(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                out.size, ctypes.byref(n)), "hotrg_copy_environment")
        return out

    def isometry(self):
        """The isometry the last step applied (n x D', as the products used it)."""
        import numpy as np
        dims = (ctypes.c_int * 2)()
        self._lib.hotrg_copy_isometry(self._h, None, 0, dims)
        out = np.empty((dims[0], dims[1]), dtype=np.float64)
        _check(self._lib.hotrg_copy_isometry(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             out.size, dims), "hotrg_copy_isometry")
        return out

    def set_timing(self, enable: bool = True):
        _check(self._lib.hotrg_set_timing(self._h, 1 if enable else 0), "hotrg_set_timing")

    def stage_times(self):
        ms = (ctypes.c_double * len(STAGES))()
        n = ctypes.c_int()
        _check(self._lib.hotrg_stage_times(self._h, ms, ctypes.byref(n)), "hotrg_stage_times")
        return dict(zip(STAGES, list(ms))), n.value

    def step_stage_times(self):
        """Per recorded step: ((Dx, Dy, D'), {stage: ms})."""
        _, n = self.stage_times()
        out = []
        for k in range(n):
            ms = (ctypes.c_double * len(STAGES))()
            dims = (ctypes.c_int * 3)()
            _check(self._lib.hotrg_step_stage_times(self._h, k, ms, dims), "hotrg_step_stage_times")
            out.append(((dims[0], dims[1], dims[2]), dict(zip(STAGES, list(ms)))))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hotrg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Chains:
    """A batch of infinite chains evolved in imaginary time on the device
    (include/itebd.h).  h: the two-site term (4 x 4); states: rows of
    itebd_state_len(chi) doubles (B1, B2, lambda_1, lambda_2)."""

    def __init__(self, h, states, chi: int, stream=None, device="cuda"):
        import numpy as np
        lib = load()
        self._lib = lib
        self.chi = chi
        st = np.ascontiguousarray(states, dtype=np.float64)
        self.batch = st.shape[0]
        if st.ndim != 2 or st.shape[1] != lib.itebd_state_len(chi):
            raise ValueError("states must have itebd_state_len(chi) columns")
        hh = np.ascontiguousarray(h, dtype=np.float64).reshape(16)
        nbytes = lib.itebd_workspace_bytes(self.batch, chi)
        if nbytes == 0:
            raise HotrgError(EINVAL, "itebd_workspace_bytes")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        dp = ctypes.POINTER(ctypes.c_double)
        h_ = ctypes.c_void_p()
        _check(lib.itebd_init(self.batch, chi, hh.ctypes.data_as(dp), st.ctypes.data_as(dp),
                              ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_size_t(nbytes),
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h_)), "itebd_init")
        self._h = h_

    def evolve(self, tau: float, nupdates: int) -> "Chains":
        _check(self._lib.itebd_evolve(self._h, float(tau), int(nupdates)), "itebd_evolve")
        return self

    def energies(self):
        import numpy as np
        out = np.empty(self.batch)
        _check(self._lib.itebd_energy(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "itebd_energy")
        return out

    def states(self):
        import numpy as np
        out = np.empty((self.batch, self._lib.itebd_state_len(self.chi)))
        _check(self._lib.itebd_copy_states(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size),
               "itebd_copy_states")
        return out

    def info(self):
        u, m = ctypes.c_long(), ctypes.c_int()
        _check(self._lib.itebd_info(self._h, ctypes.byref(u), ctypes.byref(m)), "itebd_info")
        return u.value, m.value

    def status(self):
        """Per-chain status words (ITEBD_CHAIN_* bits; 0 = no failure)."""
        import numpy as np
        out = np.zeros(self.batch, dtype=np.int32)
        _check(self._lib.itebd_status(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), "itebd_status")
        return out

    def set_max_sweeps(self, max_sweeps: int) -> "Chains":
        _check(self._lib.itebd_set_max_sweeps(self._h, int(max_sweeps)), "itebd_set_max_sweeps")
        return self

    def work(self):
        """(Jacobi sweeps, pair rotations) summed over the chains so far."""
        sw, rot = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.itebd_work(self._h, ctypes.byref(sw), ctypes.byref(rot)), "itebd_work")
        return sw.value, rot.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.itebd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def coarse_grain_batch(solves, nsteps: int) -> None:
    """Advance every Solve in `solves` by nsteps, step by step across the
    group, each on its own stream (hotrg_coarse_grain_batch)."""
    lib = load()
    handles = (ctypes.c_void_p * max(len(solves), 1))(*[s._h.value for s in solves])
    _check(lib.hotrg_coarse_grain_batch(handles, len(solves), int(nsteps)), "hotrg_coarse_grain_batch")


ROLES = {"generic": 0, "x": 1, "y": 2, "tp": 3}
NOALLOC_SCRATCH_BYTES = 64 << 20


def gemm_nt_noalloc(A, B, C, M, N, K, lda, ldb, out_map, precision: str = "fp64", alpha: float = 1.0,
                    stream=None, role: str = "generic", panel: bool = False) -> int:
    """hotrg_gemm_nt_noalloc: the stand-alone product with the library's own
    device scratch array (no allocation).  Returns the status code."""
    lib = load()
    st = stream if stream is not None else torch.cuda.current_stream(C.device)
    sm, rs_hi, rs_lo, sn, cs_hi, cs_lo = out_map
    return lib.hotrg_gemm_nt_noalloc(PRECISIONS[precision], ROLES[role], 1 if panel else 0, M, N, K,
                                     ctypes.c_void_p(A.data_ptr()), lda, ctypes.c_void_p(B.data_ptr()), ldb,
                                     ctypes.c_void_p(C.data_ptr()), alpha, sm, rs_hi, rs_lo, sn, cs_hi, cs_lo,
                                     ctypes.c_void_p(st.cuda_stream))


def gemm_nt(A, B, C, M, N, K, lda, ldb, out_map, precision: str = "fp64", alpha: float = 1.0, stream=None,
            role: str | None = None, panel: bool = False):
    """Index-mapped product on the device (torch float64 CUDA tensors):
    C[map(m,n)] = alpha * sum_k A[m*lda+k] B[n*ldb+k],
    out_map = (sm, rs_hi, rs_lo, sn, cs_hi, cs_lo).  role / panel select the
    tile choice of one contraction of a step (hotrg_gemm_nt_role)."""
    lib = load()
    prec = PRECISIONS[precision]
    st = stream if stream is not None else torch.cuda.current_stream(C.device)
    nbytes = lib.hotrg_gemm_scratch_bytes(prec, M, N, K)
    scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=C.device) if nbytes else None
    sm, rs_hi, rs_lo, sn, cs_hi, cs_lo = out_map
    sp = ctypes.c_void_p(scratch.data_ptr() if scratch is not None else 0)
    if role is None and not panel:
        _check(lib.hotrg_gemm_nt(prec, M, N, K, ctypes.c_void_p(A.data_ptr()), lda, ctypes.c_void_p(B.data_ptr()),
                                 ldb, ctypes.c_void_p(C.data_ptr()), alpha, sm, rs_hi, rs_lo, sn, cs_hi, cs_lo,
                                 sp, ctypes.c_void_p(st.cuda_stream)), "hotrg_gemm_nt")
    else:
        _check(lib.hotrg_gemm_nt_role(prec, ROLES[role or "generic"], 1 if panel else 0, M, N, K,
                                      ctypes.c_void_p(A.data_ptr()), lda, ctypes.c_void_p(B.data_ptr()), ldb,
                                      ctypes.c_void_p(C.data_ptr()), alpha, sm, rs_hi, rs_lo, sn, cs_hi, cs_lo,
                                      sp, ctypes.c_void_p(st.cuda_stream)), "hotrg_gemm_nt_role")
    return scratch
