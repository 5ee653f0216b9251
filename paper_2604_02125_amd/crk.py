"""ctypes binding of ``libcrk.so`` (C ABI in ``include/crk.h``).

Argument marshalling only: every step of the method runs in the HIP
kernels behind the C ABI.  PyTorch provides the device memory (the state,
the workspace, the traces) and the stream.  The library must be built
(``__graft_entry__.build()`` or ``python -m paper_2604_02125_amd.build``);
there is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrk.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "crk.h")

CRK_EULER, CRK_GLM_MHD = 0, 1
VOL_CENTRAL, VOL_KG, VOL_RANOCHA, VOL_DERIGS = 0, 1, 2, 3
FP64, FP32 = 0, 1
LIM_NONE, LIM_BLEND = 0, 1
BC_PERIODIC, BC_WALL = 0, 1
NC_REDUCED, NC_STAGEWISE = 0, 1
SURF_RUSANOV, SURF_EC = 0, 1
OK, ERR_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NONPHYSICAL, ERR_NOT_FINITE, ERR_STATE = 0, -1, -2, -3, -4, -5, -6
STEP_COMPUTE_DT = 1
PHASE_LOCAL, PHASE_INTERFACE, PHASE_LOCAL_PLAIN, PHASE_LOCAL_BLEND = 1, 2, 4, 8


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("degree", C.c_int), ("equation", C.c_int), ("gamma", C.c_double), ("precision", C.c_int),
                ("boundary", C.c_int * 2)]


class SchemeDesc(C.Structure):
    _fields_ = [("stages", C.c_int), ("A", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)),
                ("volume_flux", C.c_int), ("cfl", C.c_double), ("limiter", C.c_int),
                ("alpha_max", C.c_double), ("alpha_min", C.c_double), ("nc_interface", C.c_int)]


class CrkError(RuntimeError):
    pass


_lib = None
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)


def header_functions():
    """Names of the functions declared in include/crk.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:crk_status|const char \*)\s*(crk_\w+)\s*\(", text, re.M)))


def lib():
    """Load libcrk.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CrkError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        sig = {
            "crk_create": (st, [C.POINTER(MeshDesc), C.POINTER(SchemeDesc), C.POINTER(_vp)]),
            "crk_destroy": (st, [_vp]),
            "crk_state_layout": (st, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_size_t)]),
            "crk_trace_bytes": (st, [_vp, C.POINTER(C.c_size_t)]),
            "crk_workspace_bytes": (st, [_vp, C.POINTER(C.c_size_t)]),
            "crk_set_workspace": (st, [_vp, _vp, C.c_size_t]),
            "crk_reference_element": (st, [C.c_int, _dp, _dp, _dp]),
            "crk_compute_dt": (st, [_vp, _vp, _vp, _vp]),
            "crk_indicator": (st, [_vp, _vp, _vp, _vp, _vp]),
            "crk_fr_rhs": (st, [_vp, _vp, _vp, C.c_int, _vp, _vp]),
            "crk_local_stages": (st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "crk_interface_update": (st, [_vp, _vp, _vp, _vp, _vp, _vp]),
            "crk_run": (st, [_vp, _vp, _vp, _vp, C.c_int, _vp]),
            "crk_step": (st, [_vp, _vp, _vp, _vp, _vp, C.c_int, _vp]),
            "crk_diagnostics": (st, [_vp, _vp, _vp, _vp]),
            "crk_check": (st, [_vp, _vp, C.POINTER(C.c_int64), _dp, _vp]),
            "crk_rkfr_workspace_bytes": (st, [_vp, C.POINTER(C.c_size_t)]),
            "crk_rkfr_step": (st, [_vp, _vp, _vp, _vp, C.c_int, _vp, C.c_size_t, _vp]),
            "crk_prepare": (st, [_vp, _vp, _vp, _vp]),
            "crk_advance": (st, [_vp, _vp, _vp, _vp, C.c_int, _vp]),
            "crk_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().crk_last_error().decode()
        raise CrkError(f"{what} failed ({rc}): {msg}")


def reference_element(degree: int):
    """(xi, w, D) of the library's reference element (host computation)."""
    import numpy as np
    xi, w = np.zeros(degree + 1), np.zeros(degree + 1)
    D = np.zeros((degree + 1, degree + 1))
    _check(lib().crk_reference_element(degree, xi.ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                                       D.ctypes.data_as(_dp)), "crk_reference_element")
    return xi, w, D


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Solver:
    """One mesh + scheme.  Owns the solver handle and a device workspace."""

    def __init__(self, dim=2, nx=4, ny=4, x0=0.0, x1=1.0, y0=0.0, y1=1.0, degree=3, equation=CRK_EULER,
                 gamma=1.4, precision=FP64, A=None, b=None, volume_flux=VOL_RANOCHA, cfl=0.4,
                 limiter=LIM_NONE, alpha_max=0.008, alpha_min=1e-3, boundary=(BC_PERIODIC, BC_PERIODIC),
                 nc_interface=NC_REDUCED, device="cuda"):
        import torch
        self.device = torch.device(device)
        # the constructor's arguments (checkpoints record them to rebuild the solver)
        self.config = dict(dim=dim, nx=nx, ny=ny, x0=x0, x1=x1, y0=y0, y1=y1, degree=degree, equation=equation,
                           gamma=gamma, precision=precision, A=None if A is None else [list(map(float, r)) for r in A],
                           b=None if b is None else list(map(float, b)), volume_flux=volume_flux, cfl=cfl,
                           limiter=limiter, alpha_max=alpha_max, alpha_min=alpha_min,
                           boundary=[int(boundary[0]), int(boundary[1])], nc_interface=int(nc_interface))
        m = MeshDesc(dim, nx, ny, x0, x1, y0, y1, degree, equation, gamma, precision)
        m.boundary[0], m.boundary[1] = int(boundary[0]), int(boundary[1])
        sc = SchemeDesc()
        if A is not None:
            s = len(b)
            self._A = (C.c_double * (s * s))(*[float(A[i][j]) for i in range(s) for j in range(s)])
            self._b = (C.c_double * s)(*[float(x) for x in b])
            sc.stages, sc.A, sc.b = s, C.cast(self._A, _dp), C.cast(self._b, _dp)
        sc.volume_flux, sc.cfl, sc.limiter = volume_flux, cfl, limiter
        sc.alpha_max, sc.alpha_min = alpha_max, alpha_min
        sc.nc_interface = int(nc_interface)
        h = _vp()
        _check(lib().crk_create(C.byref(m), C.byref(sc), C.byref(h)), "crk_create")
        self._h = h
        nv, ne, nn, nb = C.c_int64(), C.c_int64(), C.c_int64(), C.c_size_t()
        _check(lib().crk_state_layout(h, C.byref(nv), C.byref(ne), C.byref(nn), C.byref(nb)), "crk_state_layout")
        self.shape = (nv.value, ne.value, nn.value)
        self.nelem = ne.value
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        tb, wb = C.c_size_t(), C.c_size_t()
        _check(lib().crk_trace_bytes(h, C.byref(tb)), "crk_trace_bytes")
        _check(lib().crk_workspace_bytes(h, C.byref(wb)), "crk_workspace_bytes")
        self.trace_bytes, self.workspace_bytes = tb.value, wb.value
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        _check(lib().crk_set_workspace(h, _ptr(self.workspace), self.workspace_bytes), "crk_set_workspace")
        self.dim, self.nx, self.ny, self.degree, self.equation = dim, nx, ny, degree, equation

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.crk_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- buffers
    def new_state(self):
        import torch
        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    def new_traces(self):
        import torch
        n = self.trace_bytes // (8 if self.dtype == torch.float64 else 4)
        return torch.empty(n, dtype=self.dtype, device=self.device)

    def new_dt(self):
        import torch
        return torch.zeros(2, dtype=torch.float64, device=self.device)

    def trace_view(self, traces):
        """[face, c, e, k] view of a face-data buffer: c < nvar the element's
        share of the interface flux; MHD: c = nvar, nvar + 1 the time-averaged
        normal field and psi; last c: the face wave speed of the step's
        initial state."""
        nf = self.degree + 1 if self.dim == 2 else 1
        nc = self.shape[0] + (2 if self.equation == CRK_GLM_MHD else 0) + 1
        return traces.view(2 * self.dim, nc, self.nelem, nf)

    def _check_state(self, u):
        if u.dtype != self.dtype or tuple(u.shape) != self.shape or not u.is_contiguous() or u.device.type != "cuda":
            raise CrkError(f"state must be a contiguous {self.dtype} cuda tensor of shape {self.shape}")

    # ---------------------------------------------------------------- calls
    def compute_dt(self, u, dt=None, stream=None):
        self._check_state(u)
        dt = self.new_dt() if dt is None else dt
        _check(lib().crk_compute_dt(self._h, _ptr(u), _ptr(dt), _stream(stream)), "crk_compute_dt")
        return dt

    def indicator(self, u, stream=None):
        import torch
        self._check_state(u)
        araw = torch.empty(self.nelem, dtype=torch.float64, device=self.device)
        a = torch.empty_like(araw)
        _check(lib().crk_indicator(self._h, _ptr(u), _ptr(araw), _ptr(a), _stream(stream)), "crk_indicator")
        return araw, a

    def fr_rhs(self, u, surface=SURF_RUSANOV, dt=None, stream=None):
        """Semi-discrete FR right-hand side du/dt (test operator); dt = [dt, c_h] on the device (MHD)."""
        self._check_state(u)
        out = self.new_state()
        _check(lib().crk_fr_rhs(self._h, _ptr(u), _ptr(dt), int(surface), _ptr(out), _stream(stream)),
               "crk_fr_rhs")
        return out

    def local_stages(self, u_in, dt, u_out, traces, alpha=None, stream=None):
        self._check_state(u_in)
        self._check_state(u_out)
        _check(lib().crk_local_stages(self._h, _ptr(u_in), _ptr(dt), _ptr(alpha), _ptr(u_out), _ptr(traces),
                                      _stream(stream)), "crk_local_stages")

    def interface_update(self, u_in, traces, dt, u, stream=None):
        self._check_state(u_in)
        self._check_state(u)
        _check(lib().crk_interface_update(self._h, _ptr(u_in), _ptr(traces), _ptr(dt), _ptr(u), _stream(stream)),
               "crk_interface_update")

    def step(self, u_in, u_out, dt, alpha=None, compute_dt=True, stream=None):
        self._check_state(u_in)
        self._check_state(u_out)
        _check(lib().crk_step(self._h, _ptr(u_in), _ptr(u_out), _ptr(dt), _ptr(alpha),
                              STEP_COMPUTE_DT if compute_dt else 0, _stream(stream)), "crk_step")

    def rkfr_step(self, u_in, u_out, dt, compute_dt=True, stream=None):
        """One standard s-stage RKFR step (s interface exchanges); the stage
        scratch is allocated on first use and kept."""
        import torch
        self._check_state(u_in)
        self._check_state(u_out)
        if getattr(self, "_rk_ws", None) is None:
            nb = C.c_size_t()
            _check(lib().crk_rkfr_workspace_bytes(self._h, C.byref(nb)), "crk_rkfr_workspace_bytes")
            self._rk_ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        _check(lib().crk_rkfr_step(self._h, _ptr(u_in), _ptr(u_out), _ptr(dt), STEP_COMPUTE_DT if compute_dt else 0,
                                   _ptr(self._rk_ws), self._rk_ws.numel(), _stream(stream)), "crk_rkfr_step")

    def prepare(self, u, dt, stream=None):
        self._check_state(u)
        _check(lib().crk_prepare(self._h, _ptr(u), _ptr(dt), _stream(stream)), "crk_prepare")

    def advance(self, u_in, u_out, dt, phases=PHASE_LOCAL | PHASE_INTERFACE, stream=None):
        self._check_state(u_in)
        self._check_state(u_out)
        _check(lib().crk_advance(self._h, _ptr(u_in), _ptr(u_out), _ptr(dt), int(phases), _stream(stream)),
               "crk_advance")

    def run(self, u0, u1, dt, nsteps, stream=None):
        """nsteps pipelined steps alternating u0 -> u1 -> u0 ...; returns the
        tensor that holds the final state."""
        self._check_state(u0)
        self._check_state(u1)
        _check(lib().crk_run(self._h, _ptr(u0), _ptr(u1), _ptr(dt), int(nsteps), _stream(stream)), "crk_run")
        return u1 if nsteps % 2 else u0

    def diagnostics(self, u, stream=None):
        import torch
        self._check_state(u)
        out = torch.empty(self.shape[0] + 5, dtype=torch.float64, device=self.device)
        _check(lib().crk_diagnostics(self._h, _ptr(u), _ptr(out), _stream(stream)), "crk_diagnostics")
        return out


    def check(self, u, stream=None):
        """Crash detection (crk_check): (status, first bad element, FP64
        diagnostics as a host array).  status is OK, ERR_NOT_FINITE or
        ERR_NONPHYSICAL; other statuses raise.  Waits for the stream."""
        import numpy as np
        self._check_state(u)
        fb = C.c_int64()
        d = np.zeros(self.shape[0] + 5)
        rc = lib().crk_check(self._h, _ptr(u), C.byref(fb), d.ctypes.data_as(_dp), _stream(stream))
        if rc not in (OK, ERR_NOT_FINITE, ERR_NONPHYSICAL):
            _check(rc, "crk_check")
        return rc, fb.value, d


class BatchTuning(C.Structure):
    _fields_ = [("block", C.c_int), ("grid_per_cu", C.c_int), ("merged", C.c_int)]


TUNING_PATH = os.path.join(HERE, "tuning.json")


def load_tuning(precision: int, volume_flux: int):
    """Tile shape chosen by the autotuner for (precision, flux), or None."""
    import json
    if not os.path.exists(TUNING_PATH):
        return None
    with open(TUNING_PATH) as fh:
        tab = json.load(fh)
    key = f"{'fp64' if precision == FP64 else 'fp32'}/{ {VOL_KG: 'kg', VOL_RANOCHA: 'ranocha'}.get(volume_flux, '?') }"
    rec = tab.get("batch", {}).get(key)
    return None if rec is None else (int(rec["block"]), int(rec["grid_per_cu"]), int(rec.get("merged", 0)))


def _bind_batch_functions(L):
    st = C.c_int
    sig = {
        "crk_batch_create": (st, [C.POINTER(MeshDesc), C.c_int, C.POINTER(SchemeDesc), C.POINTER(BatchTuning),
                                  C.POINTER(_vp)]),
        "crk_batch_destroy": (st, [_vp]),
        "crk_batch_layout": (st, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_size_t),
                                  C.POINTER(C.c_size_t), C.POINTER(C.c_int64)]),
        "crk_batch_bind": (st, [_vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]),
        "crk_batch_prepare": (st, [_vp, C.c_int, _vp]),
        "crk_batch_advance": (st, [_vp, C.c_int, C.c_int, _vp]),
        "crk_batch_graph_capture": (st, [_vp, _vp]),
        "crk_batch_graph_launch": (st, [_vp, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


class Batch:
    """Independent periodic 2D Euler problems on [0,1]^2, problem i with
    n_i x n_i elements of degree N_i in {3, 4}, advanced together.

    Owns two flat state buffers (u0, u1), the per-problem time steps
    dt[2*nprob] and the workspace, all bound to the library at creation."""

    def __init__(self, specs, precision=FP64, volume_flux=VOL_RANOCHA, cfl=0.4, gamma=1.4, tuning=None,
                 device="cuda", stream=None):
        import numpy as np
        import torch
        L = lib()
        _bind_batch_functions(L)
        self.device = torch.device(device)
        self.specs = [(int(n), int(N)) for n, N in specs]
        self.nprob = len(self.specs)
        meshes = (MeshDesc * self.nprob)()
        for i, (n, N) in enumerate(self.specs):
            meshes[i] = MeshDesc(2, n, n, 0.0, 1.0, 0.0, 1.0, N, CRK_EULER, gamma, precision)
        sc = SchemeDesc()
        sc.volume_flux, sc.cfl, sc.limiter = volume_flux, cfl, LIM_NONE
        if tuning is None:
            tuning = load_tuning(precision, volume_flux)
        tn = BatchTuning(*(tuning if tuning is not None else (256, 4, 0)))
        self.tuning = (tn.block, tn.grid_per_cu, tn.merged)
        h = _vp()
        _check(L.crk_batch_create(meshes, self.nprob, C.byref(sc), C.byref(tn), C.byref(h)), "crk_batch_create")
        self._h = h
        offs = (C.c_int64 * (self.nprob + 1))()
        degs = (C.c_int * self.nprob)()
        sb, wb, nt = C.c_size_t(), C.c_size_t(), C.c_int64()
        _check(L.crk_batch_layout(h, offs, degs, C.byref(sb), C.byref(wb), C.byref(nt)), "crk_batch_layout")
        self.offsets = np.array(offs[:], dtype=np.int64)
        self.ntiles = nt.value
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        n = int(self.offsets[-1])
        self.u = [torch.zeros(n, dtype=self.dtype, device=self.device) for _ in range(2)]
        self.dt = torch.zeros(2 * self.nprob, dtype=torch.float64, device=self.device)
        self.workspace = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        _check(L.crk_batch_bind(h, _ptr(self.u[0]), _ptr(self.u[1]), _ptr(self.dt), _ptr(self.workspace),
                                wb.value, C.c_void_p(self.stream.cuda_stream)), "crk_batch_bind")
        self.ndof = sum(n * n * (N + 1) ** 2 for n, N in self.specs)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.crk_batch_destroy(h)
            self._h = None

    def view(self, buf: int, i: int):
        """State of problem i in buffer buf (0/1) as a [v, e, node] view."""
        n, N = self.specs[i]
        return self.u[buf][self.offsets[i]:self.offsets[i + 1]].view(4, n * n, (N + 1) ** 2)

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def prepare(self, src=0):
        _check(lib().crk_batch_prepare(self._h, src, self._s()), "crk_batch_prepare")

    def advance(self, src, phases=PHASE_LOCAL | PHASE_INTERFACE):
        _check(lib().crk_batch_advance(self._h, src, phases, self._s()), "crk_batch_advance")

    def capture_graph(self):
        _check(lib().crk_batch_graph_capture(self._h, self._s()), "crk_batch_graph_capture")

    def launch_graph(self):
        _check(lib().crk_batch_graph_launch(self._h, self._s()), "crk_batch_graph_launch")


def _bind_mlp_functions(L):
    st = C.c_int
    sig = {
        "crk_mlp_param_count": (st, [C.c_int, C.c_int, C.POINTER(C.c_int64)]),
        "crk_mlp_forward": (st, [C.c_int, C.c_int, _vp, _vp, C.c_int64, C.c_double, _vp, _vp, _vp]),
        "crk_mlp_grad_workspace_bytes": (st, [C.c_int, C.c_int, C.c_int64, C.POINTER(C.c_size_t)]),
        "crk_mlp_loss_grad": (st, [C.c_int, C.c_int, _vp, _vp, _vp, C.c_int64, _vp, _vp, _vp, C.c_size_t, _vp]),
        "crk_mlp_adam": (st, [C.c_int64, _vp, _vp, _vp, _vp, C.c_double, C.c_double, C.c_double, C.c_double,
                              C.c_int, _vp, _vp]),
        "crk_mlp_to_bf16": (st, [C.c_int64, _vp, _vp, _vp]),
        "crk_features": (st, [_vp, _vp, _vp, _vp]),
        "crk_labels": (st, [_vp, _vp, _vp, C.c_double, _vp, _vp]),
        "crk_set_mlp": (st, [_vp, _vp, _vp, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


class MLP:
    """Learned troubled-cell indicator 16 -> 64 -> 64 -> 1 on the GPU: FP32
    master parameters, their BF16 copy used by the network, Adam moments, and
    the feature range of the training set (outside it the modal indicator is
    kept).  All arithmetic runs in the library's kernels."""

    NIN, HID = 16, 64

    def __init__(self, theta=None, lo=None, hi=None, seed=0, device="cuda"):
        import numpy as np
        import torch
        L = lib()
        _bind_mlp_functions(L)
        cnt = C.c_int64()
        _check(L.crk_mlp_param_count(self.NIN, self.HID, C.byref(cnt)), "crk_mlp_param_count")
        self.count = cnt.value
        self.device = torch.device(device)
        if theta is None:
            # He-style initialisation, seeded
            rng = np.random.default_rng(seed)
            parts = [rng.normal(0, np.sqrt(2.0 / self.NIN), self.HID * self.NIN), np.zeros(self.HID),
                     rng.normal(0, np.sqrt(2.0 / self.HID), self.HID * self.HID), np.zeros(self.HID),
                     rng.normal(0, np.sqrt(1.0 / self.HID), self.HID), np.zeros(1)]
            theta = np.concatenate(parts)
        self.theta = torch.tensor(np.asarray(theta, dtype=np.float32), device=self.device)
        self.theta_bf16 = torch.empty(self.count, dtype=torch.int16, device=self.device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.t = 0
        self.lo = torch.zeros(self.NIN, dtype=torch.float32, device=self.device) if lo is None else \
            torch.tensor(np.asarray(lo, dtype=np.float32), device=self.device)
        self.hi = torch.ones(self.NIN, dtype=torch.float32, device=self.device) if hi is None else \
            torch.tensor(np.asarray(hi, dtype=np.float32), device=self.device)
        self.sync_bf16()

    def sync_bf16(self, stream=None):
        _check(lib().crk_mlp_to_bf16(self.count, _ptr(self.theta), _ptr(self.theta_bf16), _stream(stream)),
               "crk_mlp_to_bf16")

    def forward(self, x, alpha_max=0.008, stream=None):
        import torch
        n = x.shape[0]
        z = torch.empty(n, dtype=torch.float32, device=self.device)
        a = torch.empty(n, dtype=torch.float64, device=self.device)
        _check(lib().crk_mlp_forward(self.NIN, self.HID, _ptr(self.theta_bf16), _ptr(x), n, alpha_max, _ptr(z),
                                     _ptr(a), _stream(stream)), "crk_mlp_forward")
        return z, a

    def loss_grad(self, x, y, ws=None, stream=None):
        import torch
        n = x.shape[0]
        nb = C.c_size_t()
        _check(lib().crk_mlp_grad_workspace_bytes(self.NIN, self.HID, n, C.byref(nb)), "workspace bytes")
        if ws is None or ws.numel() < nb.value:
            ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        g = torch.empty(self.count, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(lib().crk_mlp_loss_grad(self.NIN, self.HID, _ptr(self.theta_bf16), _ptr(x), _ptr(y), n, _ptr(g),
                                       _ptr(loss), _ptr(ws), ws.numel(), _stream(stream)), "crk_mlp_loss_grad")
        return loss, g, ws

    def adam(self, grad, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.t += 1
        _check(lib().crk_mlp_adam(self.count, _ptr(self.theta), _ptr(self.m), _ptr(self.v), _ptr(grad), lr, b1, b2,
                                  eps, self.t, _ptr(self.theta_bf16), _stream(stream)), "crk_mlp_adam")

    def bind(self, solver):
        """Use this network for solver's blending coefficient."""
        _check(lib().crk_set_mlp(solver._h, _ptr(self.theta_bf16), _ptr(self.lo), _ptr(self.hi)), "crk_set_mlp")
        solver._mlp = self

    def save(self, path):
        import numpy as np
        np.savez(path, theta=self.theta.cpu().numpy(), lo=self.lo.cpu().numpy(), hi=self.hi.cpu().numpy())

    @classmethod
    def load(cls, path, device="cuda"):
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            return cls(theta=z["theta"], lo=z["lo"], hi=z["hi"], device=device)


def features(solver, u, stream=None):
    import torch
    _bind_mlp_functions(lib())
    f = torch.empty((solver.nelem, solver.shape[2]), dtype=torch.float32, device=solver.device)
    _check(lib().crk_features(solver._h, _ptr(u), _ptr(f), _stream(stream)), "crk_features")
    return f


def labels(solver, u_n, u_high, tol=1e-3, stream=None):
    import torch
    _bind_mlp_functions(lib())
    out = torch.empty(solver.nelem, dtype=torch.float32, device=solver.device)
    _check(lib().crk_labels(solver._h, _ptr(u_n), _ptr(u_high), tol, _ptr(out), _stream(stream)), "crk_labels")
    return out
