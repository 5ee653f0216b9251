"""Section 4.2's robustness claim on the GPU: the Kelvin-Helmholtz run
(64 x 64 elements, N = 3, the paper's density 1/4 + 3B/4, blending with
alpha_max = 0.008, CFL 0.4) lasts to t = 15 with the Kennedy-Gruber (KEP)
and Ranocha (EC) volume fluxes, while the central flux, which recovers the
plain FR derivative, becomes non-physical first (the paper: at about t = 4).
Crash detection is crk_check every 100 steps."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_02125_amd import crk, robustness  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    crk.lib()


def test_khi_crash_study():
    res = robustness.khi_crash_study()
    for k, r in res.items():
        print(f"{k}: t = {r['t']:.3f} after {r['steps']} steps, {r['status']}, min rho {r['min_rho']:.3f}, "
              f"min p {r['min_p']:.3f}")
    assert not res["kennedy_gruber"]["failed"] and res["kennedy_gruber"]["t"] >= 15.0
    assert not res["ranocha"]["failed"] and res["ranocha"]["t"] >= 15.0
    assert res["central"]["failed"] and res["central"]["t"] < 15.0
