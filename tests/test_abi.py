"""Host-side checks of the C ABI: the library loads, exports every function
that include/crk.h declares, validates arguments, and builds the same
reference element (GLL nodes, weights, differentiation matrix) as the
oracle.  No GPU needed."""
import ctypes as C

import numpy as np
import pytest

from paper_2604_02125_amd import crk


def test_exports_every_declared_function():
    names = crk.header_functions()
    assert len(names) >= 14
    L = crk.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_reference_element_matches_oracle(orc, N):
    xi, w, D = crk.reference_element(N)
    oxi, ow = orc.gll(N)
    assert np.max(np.abs(xi - oxi)) < 1e-15
    assert np.max(np.abs(w - ow)) < 1e-15
    assert np.max(np.abs(D - orc.diffmat(N))) < 1e-12


def _create(**kw):
    m = crk.MeshDesc(2, 4, 4, 0.0, 1.0, 0.0, 1.0, 3, crk.CRK_EULER, 1.4, crk.FP64)
    sc = crk.SchemeDesc()
    sc.volume_flux, sc.cfl, sc.limiter, sc.alpha_max, sc.alpha_min = crk.VOL_KG, 0.4, 0, 0.008, 1e-3
    for k, v in kw.items():
        setattr(m if hasattr(m, k) else sc, k, v)
    h = C.c_void_p()
    rc = crk.lib().crk_create(C.byref(m), C.byref(sc), C.byref(h))
    if rc == 0:
        crk.lib().crk_destroy(h)
    return rc


def test_argument_validation():
    assert _create() == 0
    assert _create(degree=0) == -2
    assert _create(degree=5) == -2
    assert _create(dim=3) == -1
    assert _create(nx=0) == -1
    assert _create(gamma=1.0) == -1
    assert _create(cfl=0.0) == -1
    assert _create(equation=crk.CRK_GLM_MHD) == -2             # KG is not an MHD flux
    assert _create(equation=crk.CRK_GLM_MHD, volume_flux=crk.VOL_DERIGS) == 0
    assert _create(volume_flux=crk.VOL_DERIGS) == -2           # Derigs is not an Euler flux
    assert _create(equation=crk.CRK_GLM_MHD, volume_flux=crk.VOL_DERIGS, limiter=1) == -2
    assert "Euler" in crk.lib().crk_last_error().decode()
    assert _create(precision=7) == -1


def _tableau(A, b):
    s = len(b)
    Ac = (C.c_double * (s * s))(*[float(x) for row in A for x in row])
    bc = (C.c_double * s)(*[float(x) for x in b])
    return dict(stages=s, A=C.cast(Ac, C.POINTER(C.c_double)), b=C.cast(bc, C.POINTER(C.c_double))), (Ac, bc)


def test_limits_and_tableau_validation():
    # node count beyond 32-bit indexing: rejected before anything is sized
    assert _create(nx=16384, ny=16384) == -1
    assert "too large" in crk.lib().crk_last_error().decode()
    # tableaus: 1..6 stages, strictly lower-triangular A
    kw, keep = _tableau([[0, 0, 0], [1, 0, 0], [0.25, 0.25, 0]], [1 / 6, 1 / 6, 2 / 3])
    assert _create(**kw) == 0
    kw, keep = _tableau([[0, 0], [1, 0.5]], [0.5, 0.5])
    assert _create(**kw) == -1
    kw, keep = _tableau([[0] * 7 for _ in range(7)], [1 / 7] * 7)
    assert _create(**kw) == -2


def test_calls_without_workspace_fail_cleanly():
    m = crk.MeshDesc(2, 4, 4, 0.0, 1.0, 0.0, 1.0, 3, crk.CRK_EULER, 1.4, crk.FP64)
    sc = crk.SchemeDesc()
    sc.volume_flux, sc.cfl = crk.VOL_KG, 0.4
    h = C.c_void_p()
    assert crk.lib().crk_create(C.byref(m), C.byref(sc), C.byref(h)) == 0
    # no workspace bound: state error, nothing launched
    assert crk.lib().crk_step(h, C.c_void_p(256), C.c_void_p(512), C.c_void_p(768), None, 1, None) == -6
    # aliasing / alignment are rejected before any launch
    assert crk.lib().crk_local_stages(h, C.c_void_p(256), C.c_void_p(768), None, C.c_void_p(256),
                                      C.c_void_p(1024), None) == -1
    assert crk.lib().crk_local_stages(h, C.c_void_p(256), C.c_void_p(768), None, C.c_void_p(300),
                                      C.c_void_p(1024), None) == -1
    assert crk.lib().crk_set_workspace(h, C.c_void_p(256), 16) == -1      # too small
    nb = C.c_size_t()
    assert crk.lib().crk_workspace_bytes(h, C.byref(nb)) == 0 and nb.value > 0
    # a (never dereferenced) workspace address: pipelined steps still need crk_prepare first
    assert crk.lib().crk_set_workspace(h, C.c_void_p(1 << 20), nb.value) == 0
    assert crk.lib().crk_advance(h, C.c_void_p(256), C.c_void_p(4096), C.c_void_p(768), 3, None) == -6
    assert crk.lib().crk_run(h, C.c_void_p(256), C.c_void_p(4096), C.c_void_p(768), 5, None) == -6
    assert crk.lib().crk_advance(h, C.c_void_p(256), C.c_void_p(4096), C.c_void_p(768), 16, None) == -1
    crk.lib().crk_destroy(h)


def test_check_validation():
    """crk_check (crash detection) validates before it launches or reads back:
    a null solver, no workspace, a null or misaligned state."""
    L = crk.lib()
    fb = C.c_int64(123)
    assert L.crk_check(None, C.c_void_p(256), C.byref(fb), None, None) == crk.ERR_ARG
    assert fb.value == -1
    m = crk.MeshDesc(2, 4, 4, 0.0, 1.0, 0.0, 1.0, 3, crk.CRK_EULER, 1.4, crk.FP64)
    sc = crk.SchemeDesc()
    sc.volume_flux, sc.cfl = crk.VOL_KG, 0.4
    h = C.c_void_p()
    assert L.crk_create(C.byref(m), C.byref(sc), C.byref(h)) == 0
    assert L.crk_check(h, C.c_void_p(256), C.byref(fb), None, None) == crk.ERR_STATE
    nb = C.c_size_t()
    assert L.crk_workspace_bytes(h, C.byref(nb)) == 0
    assert L.crk_set_workspace(h, C.c_void_p(1 << 20), nb.value) == 0
    assert L.crk_check(h, None, C.byref(fb), None, None) == crk.ERR_ARG
    assert L.crk_check(h, C.c_void_p(264), C.byref(fb), None, None) == crk.ERR_ARG
    assert "aligned" in L.crk_last_error().decode()
    L.crk_destroy(h)


def test_fr_rhs_validation():
    # the semi-discrete test operator validates its arguments before any launch
    L = crk.lib()
    for eq, vol in ((crk.CRK_EULER, crk.VOL_KG), (crk.CRK_GLM_MHD, crk.VOL_DERIGS)):
        m = crk.MeshDesc(2, 4, 4, 0.0, 1.0, 0.0, 1.0, 3, eq, 1.4, crk.FP64)
        sc = crk.SchemeDesc()
        sc.volume_flux, sc.cfl = vol, 0.4
        h = C.c_void_p()
        assert L.crk_create(C.byref(m), C.byref(sc), C.byref(h)) == 0
        u, r, dt = C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20)
        assert L.crk_fr_rhs(h, u, dt, 7, r, None) == -1                    # unknown surface flux
        assert L.crk_fr_rhs(h, u, dt, crk.SURF_EC, u, None) == -1          # aliasing
        assert L.crk_fr_rhs(h, C.c_void_p((1 << 20) + 8), dt, 0, r, None) == -1   # misaligned
        assert L.crk_fr_rhs(h, None, dt, 0, r, None) == -1
        if eq == crk.CRK_GLM_MHD:
            assert L.crk_fr_rhs(h, u, None, 0, r, None) == -1              # MHD needs c_h
            assert "c_h" in L.crk_last_error().decode()
        L.crk_destroy(h)


def test_rkfr_validation():
    """The standard RKFR step: scratch size, and argument checks before any launch."""
    L = crk.lib()
    m = crk.MeshDesc(2, 4, 4, 0.0, 1.0, 0.0, 1.0, 3, crk.CRK_EULER, 1.4, crk.FP64)
    sc = crk.SchemeDesc()
    sc.volume_flux, sc.cfl = crk.VOL_KG, 0.4
    h = C.c_void_p()
    assert L.crk_create(C.byref(m), C.byref(sc), C.byref(h)) == 0
    nb = C.c_size_t()
    assert L.crk_rkfr_workspace_bytes(h, C.byref(nb)) == 0
    state = 4 * 16 * 16 * 8
    assert nb.value == (4 + 2) * ((state + 255) // 256 * 256)        # RK4: two stage states + four K
    u, o, dt, ws = (C.c_void_p(x << 20) for x in (1, 2, 3, 8))
    assert L.crk_rkfr_step(h, u, u, dt, 0, ws, nb.value, None) == crk.ERR_ARG           # aliasing
    assert L.crk_rkfr_step(h, u, o, dt, 0, ws, nb.value - 1, None) == crk.ERR_ARG       # scratch too small
    assert L.crk_rkfr_step(h, u, C.c_void_p((8 << 20) + 256), dt, 0, ws, nb.value, None) == crk.ERR_ARG
    assert L.crk_rkfr_step(h, u, o, dt, 0, C.c_void_p((8 << 20) + 8), nb.value, None) == crk.ERR_ARG
    assert L.crk_rkfr_step(h, u, o, None, 0, ws, nb.value, None) == crk.ERR_ARG
    L.crk_destroy(h)
    sc.limiter = crk.LIM_BLEND
    assert L.crk_create(C.byref(m), C.byref(sc), C.byref(h)) == 0
    assert L.crk_rkfr_step(h, u, o, dt, 0, ws, nb.value, None) == crk.ERR_UNSUPPORTED
    L.crk_destroy(h)
