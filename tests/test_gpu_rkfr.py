"""GPU standard multi-stage RKFR step (crk_rkfr_step, eq:rkfr.non.cons: one
interface exchange per stage) against the oracle's orc_rkfr_step, stepped
from the same u^n with the same dt: per conserved variable
max|u_gpu - u_orc| / max|u_orc| <= 1e-12, at small sizes (several
workgroups, ragged last one), for every degree, both systems, several
tableau classes, and at the full 256^2 Kelvin-Helmholtz size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_02125_amd import crk, inputs  # noqa: E402

SSPRK3_A = [[0, 0, 0], [1, 0, 0], [0.25, 0.25, 0]]
SSPRK3_B = [1 / 6, 1 / 6, 2 / 3]
DENSE6_A = [[0] * 6, [0.2, 0, 0, 0, 0, 0], [0.1, 0.15, 0, 0, 0, 0], [0.3, -0.1, 0.4, 0, 0, 0],
            [0.05, 0.1, 0.2, 0.25, 0, 0], [0.1, 0.2, -0.05, 0.3, 0.15, 0]]
DENSE6_B = [0.1, 0.15, 0.2, 0.25, 0.2, 0.1]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    crk.lib()


def _pair(orc, **kw):
    p = orc.Problem(**kw)
    s = crk.Solver(dim=p.dim, nx=p.nx, ny=p.ny, x0=p.x0, x1=p.x1, y0=p.y0, y1=p.y1, degree=p.N, equation=p.eq,
                   gamma=p.gamma, precision=crk.FP64, A=p.A, b=p.b, volume_flux=p.vol_flux, cfl=p.cfl, limiter=0)
    return p, s


def _rel(a, b):
    return max(np.max(np.abs(a[v] - b[v])) / max(np.max(np.abs(b[v])), 1e-300) for v in range(b.shape[0]))


CASES = {
    "khi_kg_N3": dict(dim=2, nx=13, ny=11, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=3, vol_flux=1),
    "ranocha_N4": dict(dim=2, nx=7, ny=6, N=4, vol_flux=2),
    "central_N2": dict(dim=2, nx=9, ny=14, N=2, vol_flux=0),
    "kg_N1": dict(dim=2, nx=29, ny=17, N=1, vol_flux=1),
    "wave1d_ranocha": dict(dim=1, nx=37, N=3, vol_flux=2),
    "mhd_N3": dict(dim=2, nx=10, ny=9, N=3, eq=1, gamma=5.0 / 3.0, vol_flux=3),
    "mhd_N4": dict(dim=2, nx=6, ny=5, N=4, eq=1, gamma=5.0 / 3.0, vol_flux=3),
    "ssprk3_N3": dict(dim=2, nx=8, ny=7, N=3, vol_flux=2, A=SSPRK3_A, b=SSPRK3_B),
    "dense6_N3": dict(dim=2, nx=8, ny=7, N=3, vol_flux=1, A=DENSE6_A, b=DENSE6_B),
}


def _state(orc, p, seed):
    xi, _ = orc.gll(p.N)
    if p.eq == orc.MHD:
        return inputs.perturb(inputs.orszag_tang(p.nx, p.ny, xi), seed, 1e-3)
    if p.dim == 1:
        return inputs.perturb(inputs.density_wave_1d(p.nx, xi), seed, 1e-3)
    if p.x0 == -1.0:
        return inputs.perturb(inputs.kelvin_helmholtz(p.nx, p.ny, xi), seed, 1e-3)
    return inputs.random_smooth_euler(p.nx, p.ny, xi, seed=seed, amp=0.25)


@pytest.mark.parametrize("case", sorted(CASES))
def test_rkfr_step_parity(orc, case):
    kw = dict(CASES[case])
    if kw.get("eq") == 1:
        kw["eq"] = orc.MHD
    p, s = _pair(orc, **kw)
    u = _state(orc, p, seed=71)
    if p.eq == orc.MHD:
        p.ch = orc.compute_ch(p, u)
    dt = orc.compute_dt(p, u)
    ref = u
    got = torch.tensor(u, device="cuda")
    dtt = torch.tensor([dt, p.ch], dtype=torch.float64, device="cuda")
    for _ in range(2):          # two steps: the scratch of the first must not leak into the second
        ref = orc.rkfr_step(p, ref, dt)
        out = s.new_state()
        s.rkfr_step(got, out, dtt, compute_dt=False)
        got = out
    torch.cuda.synchronize()
    rel = _rel(got.cpu().numpy(), ref)
    print(f"rkfr {case}: rel {rel:.2e}")
    assert rel <= 1e-12


def test_rkfr_full_size_khi(orc):
    """KHI 256^2, N=3, Kennedy-Gruber, RK4 (the benchmarked RKFR variant),
    with the GPU's own dt against the oracle's."""
    n = 256
    p, s = _pair(orc, dim=2, nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=3, vol_flux=1)
    p.nthreads = 16
    xi, _ = orc.gll(3)
    u = inputs.kelvin_helmholtz(n, n, xi)
    ug = torch.tensor(u, device="cuda")
    out, dt = s.new_state(), s.new_dt()
    s.rkfr_step(ug, out, dt, compute_dt=True)
    torch.cuda.synchronize()
    dref = orc.compute_dt(p, u)
    assert abs(dt[0].item() - dref) <= 1e-14 * dref
    ref = orc.rkfr_step(p, u, dt[0].item())
    rel = _rel(out.cpu().numpy(), ref)
    print(f"rkfr khi256: rel {rel:.2e}")
    assert rel <= 1e-12
    # conservative: totals of the new state equal those of the old one
    d0, d1 = s.diagnostics(ug).cpu().numpy(), s.diagnostics(out).cpu().numpy()
    assert np.max(np.abs(d1[:4] - d0[:4]) / np.maximum(np.abs(d0[:4]), 1.0)) < 1e-13


def test_rkfr_argument_checks():
    s = crk.Solver(dim=2, nx=4, ny=4, degree=3, volume_flux=crk.VOL_KG, limiter=crk.LIM_BLEND)
    u, o, dt = s.new_state(), s.new_state(), s.new_dt()
    with pytest.raises(crk.CrkError, match="limiter"):
        s.rkfr_step(u, o, dt)
    s = crk.Solver(dim=2, nx=4, ny=4, degree=3, volume_flux=crk.VOL_KG)
    with pytest.raises(crk.CrkError, match="alias"):
        s.rkfr_step(u, u, dt)
    import ctypes as C
    L = crk.lib()
    nb = C.c_size_t()
    assert L.crk_rkfr_workspace_bytes(s._h, C.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    P = lambda t: C.c_void_p(t.data_ptr())
    assert L.crk_rkfr_step(s._h, P(u), P(o), P(dt), 0, P(ws), nb.value - 1, None) == crk.ERR_ARG   # too small
    assert L.crk_rkfr_step(s._h, P(u), P(ws), P(dt), 0, P(ws), nb.value, None) == crk.ERR_ARG      # u_out in ws
    assert L.crk_rkfr_step(s._h, P(u), P(o), P(dt), 8, P(ws), nb.value, None) == crk.ERR_ARG       # flag bits
