"""GPU MHD step with the stage-wise non-conservative interface flux of
eq:bad.numflux.non.cons (the local phase leaves every stage's state at the
face nodes; the interface phase forms sum_j b_j 1/2 B(u^(j)_own) g(u^(j)_nb))
against the oracle's stage-wise form, per conserved variable to 1e-12 (FP64)
or 2e-5 (FP32 against the FP64 oracle from the FP32-rounded input), for
classical RK4 (N = 3) and Butcher's six-stage method (N = 4), and at the
Orszag-Tang 192^2 size in the benchmark's launch configuration."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_02125_amd import crk, inputs  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    crk.lib()


def _pair(orc, n, N, precision=crk.FP64, nthreads=1):
    p = orc.Problem(dim=2, nx=n, ny=n, N=N, eq=orc.MHD, gamma=5.0 / 3.0, vol_flux=orc.VOL_DERIGS, nc_stagewise=1,
                    nthreads=nthreads)
    s = crk.Solver(dim=2, nx=n, ny=n, degree=N, equation=crk.CRK_GLM_MHD, gamma=5.0 / 3.0, precision=precision,
                   volume_flux=crk.VOL_DERIGS, nc_interface=crk.NC_STAGEWISE)
    return p, s


def _rel(a, b, psi_scale=None):
    a = np.asarray(a, dtype=np.float64)
    out = []
    for v in range(b.shape[0]):
        sc = np.max(np.abs(b[v]))
        if v == 8 and psi_scale is not None:
            sc = max(sc, psi_scale)     # psi starts at zero: measured on the field's scale
        out.append(np.max(np.abs(a[v] - b[v])) / max(sc, 1e-300))
    return max(out)


@pytest.mark.parametrize("N,n", [(3, 10), (4, 9), (2, 11)])
def test_stagewise_step_parity(orc, N, n):
    p, s = _pair(orc, n, N)
    xi, _ = orc.gll(N)
    u = inputs.perturb(inputs.orszag_tang(n, n, xi), 91, 1e-3)
    nsteps = 3
    ref = u.copy()
    for _ in range(nsteps):
        p.ch = orc.compute_ch(p, ref)
        ref, _ = orc.crk_step(p, ref, orc.compute_dt(p, ref))
    ug = torch.tensor(u, device="cuda")
    buf, dt = [ug.clone(), s.new_state()], s.new_dt()
    s.prepare(buf[0], dt)
    for k in range(nsteps):
        s.advance(buf[k % 2], buf[(k + 1) % 2], dt)
    b2, d2 = [ug.clone(), s.new_state()], s.new_dt()
    for k in range(nsteps):
        s.step(b2[k % 2], b2[(k + 1) % 2], d2)
    torch.cuda.synchronize()
    bscale = np.max(np.abs(u[5:8]))
    r1, r2 = _rel(buf[nsteps % 2].cpu().numpy(), ref, bscale), _rel(b2[nsteps % 2].cpu().numpy(), ref, bscale)
    print(f"stage-wise N={N}: pipelined {r1:.2e}, step {r2:.2e}")
    assert r1 <= 1e-12 and r2 <= 1e-12
    # and it is not the reduced form
    pr = orc.Problem(dim=2, nx=n, ny=n, N=N, eq=orc.MHD, gamma=5.0 / 3.0, vol_flux=orc.VOL_DERIGS)
    pr.ch = orc.compute_ch(pr, u)
    red, _ = orc.crk_step(pr, u, orc.compute_dt(pr, u))
    o = s.new_state()
    s.step(ug, o, s.new_dt())
    torch.cuda.synchronize()
    assert _rel(o.cpu().numpy(), red, bscale) > 1e-9


def test_stagewise_fp32(orc):
    N, n = 4, 8
    p, _ = _pair(orc, n, N)
    s = crk.Solver(dim=2, nx=n, ny=n, degree=N, equation=crk.CRK_GLM_MHD, gamma=5.0 / 3.0, precision=crk.FP32,
                   volume_flux=crk.VOL_DERIGS, nc_interface=crk.NC_STAGEWISE)
    xi, _ = orc.gll(N)
    u = inputs.perturb(inputs.orszag_tang(n, n, xi), 92, 1e-3).astype(np.float32).astype(np.float64)
    p.ch = orc.compute_ch(p, u)
    ref, _ = orc.crk_step(p, u, orc.compute_dt(p, u))
    o = s.new_state()
    s.step(torch.tensor(u, dtype=torch.float32, device="cuda"), o, s.new_dt())
    torch.cuda.synchronize()
    assert _rel(o.cpu().numpy(), ref, np.max(np.abs(u[5:8]))) <= 2e-5


def test_stagewise_full_size(orc):
    """Orszag-Tang 192^2, N = 4, Butcher RK5: two pipelined steps."""
    n, N = 192, 4
    p, s = _pair(orc, n, N, nthreads=16)
    xi, _ = orc.gll(N)
    u = inputs.orszag_tang(n, n, xi)
    ref = u.copy()
    for _ in range(2):
        p.ch = orc.compute_ch(p, ref)
        ref, _ = orc.crk_step(p, ref, orc.compute_dt(p, ref))
    ug = torch.tensor(u, device="cuda")
    buf, dt = [ug.clone(), s.new_state()], s.new_dt()
    s.prepare(buf[0], dt)
    for k in range(2):
        s.advance(buf[k % 2], buf[(k + 1) % 2], dt)
    torch.cuda.synchronize()
    r = _rel(buf[0].cpu().numpy(), ref, np.max(np.abs(u[5:8])))
    print(f"stage-wise OT192: {r:.2e}")
    assert r <= 1e-12


def test_stagewise_needs_a_default_tableau():
    A = [[0, 0, 0], [1, 0, 0], [0.25, 0.25, 0]]
    b = [1 / 6, 1 / 6, 2 / 3]
    with pytest.raises(crk.CrkError, match="stage-wise"):
        crk.Solver(dim=2, nx=4, ny=4, degree=3, equation=crk.CRK_GLM_MHD, gamma=5.0 / 3.0, A=A, b=b,
                   volume_flux=crk.VOL_DERIGS, nc_interface=crk.NC_STAGEWISE)
    with pytest.raises(crk.CrkError, match="MHD option"):
        crk.Solver(dim=2, nx=4, ny=4, degree=3, volume_flux=crk.VOL_KG, nc_interface=crk.NC_STAGEWISE)
