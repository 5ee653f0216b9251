"""GPU semi-discrete FR operator (crk_fr_rhs, a test operator beside the time
step) against the oracle's, and the entropy property it exists for: with the
entropy-conservative Ranocha volume flux and the same flux at the element
faces, the total entropy rate sum_e sum_p w_p v(u_p) . du_p/dt vanishes on a
periodic mesh (the semi-discrete statement behind the EC scheme of Section 3),
while Rusanov faces dissipate.  The rate is formed on the CPU from the GPU's
right-hand side with the oracle's entropy variables."""
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


def _pair(orc, **kw):
    p = orc.Problem(**kw)
    s = crk.Solver(dim=p.dim, nx=p.nx, ny=p.ny, x0=p.x0, x1=p.x1, y0=p.y0, y1=p.y1, degree=p.N,
                   equation=p.eq, gamma=p.gamma, precision=crk.FP64, A=p.A, b=p.b, volume_flux=p.vol_flux,
                   cfl=p.cfl, limiter=0, alpha_max=p.alpha_max, alpha_min=p.alpha_min)
    return p, s


def _rel(a, b):
    return max(np.max(np.abs(a[v] - b[v])) / max(np.max(np.abs(b[v])), 1e-300) for v in range(b.shape[0]))


def _term_scale(orc, p, u):
    """Per variable, the size of the terms a right-hand side value sums:
    max|2 D_pq / dx_d| times max over nodes and directions of |f_d(u)|.
    A value is a sum of at most 2 (N+1) dim + 2 such terms, so rounding moves
    it by a few ulps of this size whatever the size of the sum; where the
    terms cancel (a state near uniform pressure) the relative difference
    against max|rhs| grows accordingly."""
    D = orc.diffmat(p.N)
    dxs = [(p.x1 - p.x0) / p.nx] + ([(p.y1 - p.y0) / p.ny] if p.dim == 2 else [])
    cmax = 2.0 * np.max(np.abs(D)) / min(dxs)
    fmax = np.zeros(u.shape[0])
    for e in range(u.shape[1]):
        for q in range(u.shape[2]):
            for d in range(p.dim):
                fmax = np.maximum(fmax, np.abs(orc.phys_flux(p, d, u[:, e, q])))
    return cmax * fmax


# (dim, N, equation, volume flux, surface flux, nx, ny)
CASES = [
    (2, 3, 0, 1, 0, 13, 11),   # KG, Rusanov
    (2, 3, 0, 2, 1, 13, 11),   # Ranocha, EC faces
    (2, 2, 0, 0, 0, 9, 14),    # central, Rusanov
    (2, 4, 0, 2, 1, 7, 6),     # Ranocha, EC faces, degree 4 (256-lane workgroups)
    (1, 3, 0, 2, 1, 37, 1),    # 1D Ranocha, EC faces
    (1, 1, 0, 1, 0, 29, 1),    # 1D KG, Rusanov
    (2, 3, 1, 3, 1, 10, 9),    # MHD Derigs, EC faces
    (2, 2, 1, 3, 0, 8, 7),     # MHD Derigs, Rusanov
]


@pytest.mark.parametrize("dim,N,eq,vol,surf,nx,ny", CASES)
def test_fr_rhs_parity(orc, dim, N, eq, vol, surf, nx, ny):
    kw = dict(dim=dim, N=N, nx=nx, ny=ny, vol_flux=vol)
    if eq == 1:
        kw.update(eq=orc.MHD, gamma=5.0 / 3.0)
    p, s = _pair(orc, **kw)
    xi, _ = orc.gll(N)
    if eq == 1:
        u = inputs.perturb(inputs.orszag_tang(nx, ny, xi), 31, 1e-3)
        p.ch = orc.compute_ch(p, u)
    elif dim == 1:
        u = inputs.perturb(inputs.density_wave_1d(nx, xi), 32, 1e-3)
    else:
        u = inputs.random_smooth_euler(nx, ny, xi, seed=33, amp=0.25)
    ref = orc.fr_rhs(p, u, orc.SURF_EC if surf else orc.SURF_RUSANOV)
    dt = torch.tensor([0.0, p.ch], dtype=torch.float64, device="cuda")
    got = s.fr_rhs(torch.tensor(u, device="cuda"), surface=surf, dt=dt).cpu().numpy()
    T = _term_scale(orc, p, u)
    err = np.array([np.max(np.abs(got[v] - ref[v])) for v in range(ref.shape[0])])
    scale = np.maximum(T, np.array([np.max(np.abs(ref[v])) for v in range(ref.shape[0])]))
    # components that vanish identically (v_3, B_3, psi of Orszag-Tang) are held
    # to the scale of the others
    scale = np.maximum(scale, 1e-3 * np.max(scale))
    print(f"fr_rhs dim={dim} N={N} eq={eq} vol={vol} surf={surf}: rel={_rel(got, ref):.2e} "
          f"err/term scale={np.max(err / scale):.2e}")
    assert np.all(err <= 1e-13 * scale)


@pytest.mark.parametrize("dim,eq", [(1, 0), (2, 0), (2, 1)])
def test_fr_rhs_entropy_rate(orc, dim, eq):
    """Euler with the Ranocha flux, GLM-MHD with the Derigs-form flux and the
    local Powell/GLM term (faces: the same flux plus 1/2 B(u)(g^- + g^+))."""
    N, nx, ny = 3, 5, 4
    xi, w = orc.gll(N)
    if eq == 1:
        p, s = _pair(orc, dim=2, N=N, nx=nx, ny=ny, eq=orc.MHD, gamma=5.0 / 3.0, vol_flux=orc.VOL_DERIGS)
        u = inputs.perturb(inputs.random_smooth_mhd(nx, ny, xi, seed=21, amp=0.25), 22, 1e-2)
        p.ch = orc.compute_ch(p, u)
    else:
        p, s = _pair(orc, dim=dim, N=N, nx=nx, ny=ny, vol_flux=orc.VOL_RANOCHA)
        # nodal noise makes the traces of neighbouring elements differ
        u = inputs.perturb(inputs.random_smooth_euler(nx, ny, xi, seed=7, dim=dim, amp=0.3), 8, 1e-2)
    wq = w if dim == 1 else np.outer(w, w).ravel()
    ug = torch.tensor(u, device="cuda")
    dt = torch.tensor([0.0, p.ch], dtype=torch.float64, device="cuda")
    for surf, conservative in ((crk.SURF_EC, True), (crk.SURF_RUSANOV, False)):
        r = s.fr_rhs(ug, surface=surf, dt=dt).cpu().numpy()
        rate, scale = 0.0, 0.0
        for e in range(p.nelem):
            for q in range(p.nnode):
                wv = orc.entropy_vars(p, u[:, e, q])
                rate += wq[q] * wv @ r[:, e, q]
                scale += wq[q] * np.abs(wv) @ np.abs(r[:, e, q])
        print(f"dim={dim} eq={eq} surface={surf}: rate={rate:.3e} scale={scale:.3e}")
        if conservative:
            assert abs(rate) < 1e-13 * scale
        else:
            assert rate < -1e-6 * scale


def test_fr_rhs_rejects_bad_arguments():
    s = crk.Solver(dim=2, nx=4, ny=4, degree=3, volume_flux=crk.VOL_KG)
    u = s.new_state()
    with pytest.raises(crk.CrkError):
        s.fr_rhs(u, surface=7)
    L = crk.lib()
    import ctypes as C
    assert L.crk_fr_rhs(s._h, C.c_void_p(u.data_ptr()), None, 0, C.c_void_p(u.data_ptr()), None) == -1
