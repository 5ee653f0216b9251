"""Resume from a checkpoint is bit for bit: a run of 2k pipelined steps
equals k steps, a checkpoint written to disk, a solver rebuilt from it,
crk_prepare and k more steps (state and dt), for the Kelvin-Helmholtz
setting with the blending limiter and tile flags and for GLM-MHD (where dt
carries the cleaning speed)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_02125_amd import checkpoint, crk, inputs  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    crk.lib()


def _run(s, u0, n):
    buf, dt = [u0.clone(), s.new_state()], s.new_dt()
    s.prepare(buf[0], dt)
    t = 0.0
    for k in range(n):
        t += float(dt[0].item())
        s.advance(buf[k % 2], buf[(k + 1) % 2], dt)
    torch.cuda.synchronize()
    return buf[n % 2], dt, t


@pytest.mark.parametrize("case", ["khi_blend", "mhd"])
def test_resume_is_bitwise(tmp_path, case):
    if case == "mhd":
        n, N = 12, 4
        s = crk.Solver(dim=2, nx=n, ny=n, degree=N, equation=crk.CRK_GLM_MHD, gamma=5.0 / 3.0,
                       volume_flux=crk.VOL_DERIGS)
        xi, _, _ = crk.reference_element(N)
        u0 = inputs.orszag_tang(n, n, xi)
    else:
        n = 24
        s = crk.Solver(nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, degree=3, volume_flux=crk.VOL_KG,
                       limiter=crk.LIM_BLEND, alpha_max=0.008)
        xi, _, _ = crk.reference_element(3)
        u0 = inputs.perturb(inputs.kelvin_helmholtz(n, n, xi), 11, 0.05)
    ug = torch.tensor(u0, device="cuda")
    k = 7
    full, dt_full, t_full = _run(s, ug, 2 * k)
    half, dt_half, t_half = _run(s, ug, k)
    path = str(tmp_path / f"{case}.ckpt")
    checkpoint.save(path, s, half, t=t_half, step=k, dt=dt_half)
    s2, u2, head = checkpoint.load(path)
    assert head["step"] == k and head["t"] == t_half and s2.shape == s.shape
    assert torch.equal(u2, half)
    rest, dt_rest, t_rest = _run(s2, u2, k)
    assert torch.equal(rest, full), case
    assert torch.equal(dt_rest, dt_full), case
    assert abs(t_half + t_rest - t_full) <= 1e-15 * t_full
