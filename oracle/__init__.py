"""FP64 CPU oracle of one cRKFR step with EC/KEP volume fluxes.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py`` -- never by the product path.
It shares no code with the HIP library; ``crk_oracle.c`` holds all of the
arithmetic and this module only marshals numpy arrays through ctypes.

State layout of every array: ``u[v, e, node]`` (conserved variable, element
``e = ey*nx + ex``, node ``j*(N+1) + i``), float64.

Citations refer to Babbar, Chen, Ranocha, "Compact Runge-Kutta flux
reconstruction methods with entropy- and/or kinetic energy-preserving fluxes"
(arXiv 2604.02125): Section 2 (eq:diff.matrix, eq:crkfr.inner,
eq:crkfr.non.cons.final, eq:disc.avg.flux, eq:numflux.cons) and Section 3
(eq:entropy.cons.flux.dev, eq:entropy.cons.noncons.dev).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXS = 8
EULER, MHD = 0, 1
VOL_CENTRAL, VOL_KG, VOL_RANOCHA, VOL_DERIGS = 0, 1, 2, 3
LIM_NONE, LIM_BLEND_MODAL, LIM_BLEND_GIVEN = 0, 1, 2
SURF_RUSANOV, SURF_EC = 0, 1
BC_PERIODIC, BC_WALL = 0, 1


def build(force: bool = True) -> str:
    """Compile ``crk_oracle.c`` with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("N", C.c_int), ("eq", C.c_int),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("gamma", C.c_double), ("stages", C.c_int),
                ("A", C.c_double * (MAXS * MAXS)), ("b", C.c_double * MAXS),
                ("vol_flux", C.c_int), ("limiter", C.c_int),
                ("alpha_max", C.c_double), ("alpha_min", C.c_double), ("cfl", C.c_double),
                ("ch", C.c_double), ("nthreads", C.c_int), ("bc", C.c_int * 2), ("nc_stagewise", C.c_int)]


# Butcher tableaus (eq:butcher).  The paper does not list the tableau it uses
# per degree; classical RK4 for N <= 3 and Butcher's six-stage fifth-order
# method for N >= 4 are this oracle's defaults.
RK4_A = [[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1, 0]]
RK4_B = [1 / 6, 1 / 3, 1 / 3, 1 / 6]
RK5_A = [[0, 0, 0, 0, 0, 0],
         [1 / 4, 0, 0, 0, 0, 0],
         [1 / 8, 1 / 8, 0, 0, 0, 0],
         [0, -1 / 2, 1, 0, 0, 0],
         [3 / 16, 0, 0, 9 / 16, 0, 0],
         [-3 / 7, 2 / 7, 12 / 7, -12 / 7, 8 / 7, 0]]
RK5_B = [7 / 90, 0, 32 / 90, 12 / 90, 32 / 90, 7 / 90]
EULER1_A = [[0]]
EULER1_B = [1.0]


def default_tableau(N: int):
    return (RK5_A, RK5_B) if N >= 4 else (RK4_A, RK4_B)


@dataclass
class Problem:
    dim: int = 2
    nx: int = 4
    ny: int = 4
    N: int = 3
    eq: int = EULER
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    gamma: float = 1.4
    A: list = field(default=None)
    b: list = field(default=None)
    vol_flux: int = VOL_RANOCHA
    limiter: int = LIM_NONE
    alpha_max: float = 0.008
    alpha_min: float = 1e-3
    cfl: float = 0.4
    ch: float = 0.0
    nthreads: int = 1
    bc: tuple = (BC_PERIODIC, BC_PERIODIC)   # per direction: periodic or reflective wall
    nc_stagewise: int = 0                    # MHD interface flux: 0 reduced form, 1 stage-wise

    def __post_init__(self):
        if self.A is None or self.b is None:
            self.A, self.b = default_tableau(self.N)

    @property
    def nvar(self) -> int:
        return 9 if self.eq == MHD else self.dim + 2

    @property
    def nnode(self) -> int:
        return (self.N + 1) ** self.dim

    @property
    def nelem(self) -> int:
        return self.nx * self.ny if self.dim == 2 else self.nx

    @property
    def shape(self):
        return (self.nvar, self.nelem, self.nnode)

    def to_c(self) -> _Problem:
        p = _Problem()
        for k in ("dim", "nx", "ny", "N", "eq", "vol_flux", "limiter", "nthreads", "nc_stagewise"):
            setattr(p, k, int(getattr(self, k)))
        p.bc[0], p.bc[1] = int(self.bc[0]), int(self.bc[1])
        for k in ("x0", "x1", "y0", "y1", "gamma", "alpha_max", "alpha_min", "cfl", "ch"):
            setattr(p, k, float(getattr(self, k)))
        s = len(self.b)
        if s > MAXS:
            raise ValueError("too many stages")
        p.stages = s
        for i in range(s):
            p.b[i] = float(self.b[i])
            for j in range(s):
                p.A[i * MAXS + j] = float(self.A[i][j])
        return p


_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER(_Problem)
        sig = {
            "orc_gll": (C.c_int, [C.c_int, _dp, _dp]),
            "orc_diffmat": (None, [C.c_int, _dp, _dp]),
            "orc_g2_derivatives": (None, [C.c_int, _dp, _dp, _dp]),
            "orc_nvar": (C.c_int, [P]),
            "orc_pressure": (C.c_double, [P, _dp]),
            "orc_phys_flux": (None, [P, C.c_int, _dp, _dp]),
            "orc_wave_speed": (C.c_double, [P, C.c_int, _dp]),
            "orc_nc_two_point": (None, [P, C.c_int, _dp, _dp, _dp]),
            "orc_lnmean": (C.c_double, [C.c_double, C.c_double]),
            "orc_two_point": (None, [P, C.c_int, _dp, _dp, _dp]),
            "orc_entropy": (C.c_double, [P, _dp]),
            "orc_entropy_vars": (None, [P, _dp, _dp]),
            "orc_entropy_flux": (C.c_double, [P, C.c_int, _dp]),
            "orc_flux_potential": (C.c_double, [P, C.c_int, _dp]),
            "orc_volume_residual": (None, [P, _dp, _dp]),
            "orc_compute_ch": (C.c_double, [P, _dp]),
            "orc_compute_dt": (C.c_double, [P, _dp]),
            "orc_indicator": (C.c_int, [P, _dp, _dp, _dp, _dp]),
            "orc_smooth_alpha": (None, [P, _dp, _dp]),
            "orc_crk_step": (C.c_int, [P, _dp, C.c_double, _dp, _dp, _dp]),
            "orc_local_phase": (C.c_int, [P, _dp, C.c_double, _dp, _dp, _dp, _dp]),
            "orc_face_fluxes": (C.c_int, [P, _dp, C.c_double, _dp, _dp]),
            "orc_fr_rhs": (C.c_int, [P, _dp, C.c_int, _dp]),
            "orc_rkfr_step": (C.c_int, [P, _dp, C.c_double, _dp]),
            "orc_diagnostics": (C.c_int, [P, _dp, _dp]),
            "orc_labels": (C.c_int, [P, _dp, _dp, C.c_double, _dp]),
            "orc_feature_transform": (None, [C.c_long, _dp, _dp]),
            "orc_mlp_nparams": (C.c_long, [C.c_int, C.c_int]),
            "orc_mlp_forward": (C.c_int, [C.c_int, C.c_int, _dp, C.c_long, _dp, C.c_double, _dp, _dp]),
            "orc_mlp_loss_grad": (C.c_double, [C.c_int, C.c_int, _dp, C.c_long, _dp, _dp, _dp]),
            "orc_adam_step": (None, [C.c_long, _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- layer 0
def gll(N: int):
    """GLL nodes and weights on [0, 1] (Section 2)."""
    xi, w = np.zeros(N + 1), np.zeros(N + 1)
    if lib().orc_gll(N, _ptr(xi), _ptr(w)) != 0:
        raise ValueError("unsupported degree")
    return xi, w


def diffmat(N: int, xi=None):
    """D_pq = l_q'(xi_p) (eq:diff.matrix)."""
    if xi is None:
        xi = gll(N)[0]
    D = np.zeros((N + 1, N + 1))
    lib().orc_diffmat(N, _ptr(_f64(xi)), _ptr(D))
    return D


def g2_derivatives(N: int, xi=None):
    if xi is None:
        xi = gll(N)[0]
    gl, gr = np.zeros(N + 1), np.zeros(N + 1)
    lib().orc_g2_derivatives(N, _ptr(_f64(xi)), _ptr(gl), _ptr(gr))
    return gl, gr


# ---------------------------------------------------------------- layers 1-2
def pressure(prob: Problem, u):
    return lib().orc_pressure(C.byref(prob.to_c()), _ptr(_f64(u)))


def phys_flux(prob: Problem, d: int, u):
    f = np.zeros(prob.nvar)
    lib().orc_phys_flux(C.byref(prob.to_c()), d, _ptr(_f64(u)), _ptr(f))
    return f


def wave_speed(prob: Problem, d: int, u):
    return lib().orc_wave_speed(C.byref(prob.to_c()), d, _ptr(_f64(u)))


def two_point(prob: Problem, d: int, uL, uR):
    f = np.zeros(prob.nvar)
    lib().orc_two_point(C.byref(prob.to_c()), d, _ptr(_f64(uL)), _ptr(_f64(uR)), _ptr(f))
    return f


def nc_two_point(prob: Problem, d: int, up, uq):
    f = np.zeros(prob.nvar)
    lib().orc_nc_two_point(C.byref(prob.to_c()), d, _ptr(_f64(up)), _ptr(_f64(uq)), _ptr(f))
    return f


def lnmean(x: float, y: float) -> float:
    return lib().orc_lnmean(float(x), float(y))


def entropy(prob: Problem, u) -> float:
    return lib().orc_entropy(C.byref(prob.to_c()), _ptr(_f64(u)))


def entropy_vars(prob: Problem, u):
    w = np.zeros(prob.nvar)
    lib().orc_entropy_vars(C.byref(prob.to_c()), _ptr(_f64(u)), _ptr(w))
    return w


def entropy_flux(prob: Problem, d: int, u) -> float:
    return lib().orc_entropy_flux(C.byref(prob.to_c()), d, _ptr(_f64(u)))


def flux_potential(prob: Problem, d: int, u) -> float:
    return lib().orc_flux_potential(C.byref(prob.to_c()), d, _ptr(_f64(u)))


def volume_residual(prob: Problem, ue):
    """Flux-differencing volume term of one element; ue, R as [node, v]."""
    ue = _f64(ue)
    R = np.zeros_like(ue)
    lib().orc_volume_residual(C.byref(prob.to_c()), _ptr(ue), _ptr(R))
    return R


# ---------------------------------------------------------------- step
def compute_ch(prob: Problem, u) -> float:
    return lib().orc_compute_ch(C.byref(prob.to_c()), _ptr(_f64(u)))


def compute_dt(prob: Problem, u) -> float:
    return lib().orc_compute_dt(C.byref(prob.to_c()), _ptr(_f64(u)))


def indicator(prob: Problem, u):
    """(alpha_raw, alpha_smoothed, features[e, node])."""
    u = _f64(u)
    E = prob.nelem
    araw, a, feat = np.zeros(E), np.zeros(E), np.zeros((E, prob.nnode))
    lib().orc_indicator(C.byref(prob.to_c()), _ptr(u), _ptr(araw), _ptr(a), _ptr(feat))
    return araw, a, feat


def smooth_alpha(prob: Problem, alpha_raw):
    """alpha_e = max(alpha_raw_e, max over face neighbours of alpha_raw / 2)."""
    araw = np.ascontiguousarray(alpha_raw, dtype=np.float64)
    if araw.shape != (prob.nelem,):
        raise ValueError("one coefficient per element")
    a = np.zeros(prob.nelem)
    lib().orc_smooth_alpha(C.byref(prob.to_c()), _ptr(araw), _ptr(a))
    return a


def crk_step(prob: Problem, u, dt: float, alpha=None):
    """One cRKFR step; returns (u_new, alpha_used)."""
    u = _f64(u)
    out = np.empty_like(u)
    aout = np.zeros(prob.nelem)
    ain = None if alpha is None else _f64(alpha)
    rc = lib().orc_crk_step(C.byref(prob.to_c()), _ptr(u), float(dt), _ptr(ain), _ptr(out), _ptr(aout))
    if rc != 0:
        raise ValueError(f"orc_crk_step failed ({rc})")
    return out, aout


def local_phase(prob: Problem, u, dt: float):
    """(V, Ut, Ft, Fnct): V in the state layout, traces as [e, face, k, v]."""
    u = _f64(u)
    V = np.zeros_like(u)
    nf = prob.N + 1 if prob.dim == 2 else 1
    shp = (prob.nelem, 2 * prob.dim, nf, prob.nvar)
    Ut, Ft, Fnct = np.zeros(shp), np.zeros(shp), np.zeros(shp)
    lib().orc_local_phase(C.byref(prob.to_c()), _ptr(u), float(dt), _ptr(V), _ptr(Ut), _ptr(Ft), _ptr(Fnct))
    return V, Ut, Ft, Fnct


def face_fluxes(prob: Problem, u, dt: float, alpha=None):
    """Interface flux F* of every face node of one cRKFR step (eq:numflux.cons,
    blended with the first-order flux of u^n when alpha is given), as
    [e, face, k, v]."""
    u = _f64(u)
    nf = prob.N + 1 if prob.dim == 2 else 1
    out = np.zeros((prob.nelem, 2 * prob.dim, nf, prob.nvar))
    a = None if alpha is None else _f64(alpha)
    lib().orc_face_fluxes(C.byref(prob.to_c()), _ptr(u), float(dt), None if a is None else _ptr(a), _ptr(out))
    return out


def fr_rhs(prob: Problem, u, surface: int = SURF_RUSANOV):
    u = _f64(u)
    r = np.empty_like(u)
    if lib().orc_fr_rhs(C.byref(prob.to_c()), _ptr(u), int(surface), _ptr(r)) != 0:
        raise ValueError("orc_fr_rhs: unsupported configuration")
    return r


def rkfr_step(prob: Problem, u, dt: float):
    u = _f64(u)
    out = np.empty_like(u)
    lib().orc_rkfr_step(C.byref(prob.to_c()), _ptr(u), float(dt), _ptr(out))
    return out


def diagnostics(prob: Problem, u) -> dict:
    M = prob.nvar
    out = np.zeros(M + 5)
    lib().orc_diagnostics(C.byref(prob.to_c()), _ptr(_f64(u)), _ptr(out))
    return {"totals": out[:M].copy(), "entropy": out[M], "min_rho": out[M + 1], "min_p": out[M + 2],
            "nonfinite": int(out[M + 3]), "first_bad": int(out[M + 4])}


def labels(prob: Problem, un, uH, tol: float = 1e-3):
    """A-posteriori troubled-element flags (1.0/0.0) of the unlimited update uH from un."""
    out = np.zeros(prob.nelem)
    lib().orc_labels(C.byref(prob.to_c()), _ptr(_f64(un)), _ptr(_f64(uH)), float(tol), _ptr(out))
    return out


def feature_transform(f):
    """Learned-indicator input from modal energy fractions: 1 + log10(max(f, 1e-16))/16."""
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_feature_transform(f.size, _ptr(f), _ptr(out))
    return out


# ---------------------------------------------------------------- MLP
def mlp_nparams(nin: int, H: int) -> int:
    return int(lib().orc_mlp_nparams(nin, H))


def mlp_forward(nin: int, H: int, theta, x, alpha_max: float):
    x = _f64(x)
    n = x.shape[0]
    z, a = np.zeros(n), np.zeros(n)
    lib().orc_mlp_forward(nin, H, _ptr(_f64(theta)), n, _ptr(x), float(alpha_max), _ptr(z), _ptr(a))
    return z, a


def mlp_loss_grad(nin: int, H: int, theta, x, y):
    x, y = _f64(x), _f64(y)
    g = np.zeros(mlp_nparams(nin, H))
    loss = lib().orc_mlp_loss_grad(nin, H, _ptr(_f64(theta)), x.shape[0], _ptr(x), _ptr(y), _ptr(g))
    return loss, g


def adam_step(theta, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays theta, m, v."""
    lib().orc_adam_step(theta.size, _ptr(theta), _ptr(m), _ptr(v), _ptr(_f64(g)), float(lr), float(b1),
                        float(b2), float(eps), int(t))
