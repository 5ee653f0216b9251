"""The largest meshes the library accepts: fewer than 2^31 node values per
conserved variable (2D Euler, degree 3: 11584^2 elements in FP32, 8192^2 in
FP64, where a 32-bit offset would already wrap several times over).  The
state is a uniform flow with four rough patches (3 x 3 elements of 10 %
node noise, so that the blending limiter acts there), centred at the last
element (its neighbours wrap around both periodic directions), mid-mesh,
and next to the left and the bottom edge.  One pipelined step
(crk_prepare + crk_advance, the launch configuration of the benchmark) is
checked against the oracle: every element of a patch depends only on
elements at most two faces away (the smoothed blending coefficient looks
one face further than the interface flux), so the oracle steps a 9 x 9
periodic copy of the neighbourhood with the same dt, and the inner 5 x 5
elements must agree.  Away from the patches the uniform flow must stay
uniform, the FP64 totals must be those of the input and stay conserved,
and the dt of the input and of the new state must be the oracle's over the
patches and the uniform flow."""
import gc
import traceback

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_02125_amd import crk  # noqa: E402

GAMMA = 1.4
H = 2.0 / 256           # element width (that of the 256^2 Kelvin-Helmholtz mesh)
R_PATCH = 4             # oracle patch radius in elements
NOISE = 0.1


def _background(dtype):
    rho, vx, vy, p = 1.0, 0.3, -0.2, 1.0
    u = np.array([rho, rho * vx, rho * vy, p / (GAMMA - 1) + 0.5 * rho * (vx * vx + vy * vy)])
    return u.astype(dtype).astype(np.float64)


def _sites(n):
    return [(n - 1, n - 1), (n // 2, n // 2), (2, n // 4), (n // 4, 1)]


def _patch_ids(n, cx, cy, r):
    ids = np.empty((2 * r + 1, 2 * r + 1), dtype=np.int64)
    for j in range(-r, r + 1):
        for i in range(-r, r + 1):
            ids[j + r, i + r] = ((cy + j) % n) * n + (cx + i) % n
    return ids.ravel()                      # patch order: x fastest, as the oracle numbers elements


def _problem(orc, nx):
    return orc.Problem(dim=2, nx=nx, ny=nx, x0=0.0, x1=nx * H, y0=0.0, y1=nx * H, N=3, vol_flux=orc.VOL_KG,
                       limiter=orc.LIM_BLEND_MODAL, alpha_max=0.008, alpha_min=1e-3, cfl=0.4)


@pytest.mark.parametrize("precision,n", [(crk.FP32, 11584), (crk.FP64, 8192)], ids=["fp32_11584", "fp64_8192"])
def test_largest_mesh_step(orc, precision, n):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    npdt = np.float32 if precision == crk.FP32 else np.float64
    tdt = torch.float32 if precision == crk.FP32 else torch.float64
    M, NP, E = 4, 16, n * n
    assert E * NP < 2 ** 31
    esz = 4 if precision == crk.FP32 else 8
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = 2 * M * E * NP * esz + 4 * 5 * E * 4 * esz + 64 * E    # two states, face data, coefficients
    print(f"largest mesh {n}^2 {'fp32' if esz == 4 else 'fp64'}: {free / 2**30:.0f} GiB free, "
          f"{need / 2**30:.0f} GiB needed", flush=True)
    if free < 1.1 * need:
        pytest.skip("not enough device memory for the largest mesh")
    # a failure is reported as text, so that no traceback keeps the device
    # buffers alive for the tests that follow
    held, err = {}, None
    try:
        _largest_step(orc, precision, n, npdt, tdt, M, NP, E, esz, held)
    except AssertionError as ex:
        err = "".join(traceback.format_exception(type(ex), ex, ex.__traceback__))
    held.clear()
    gc.collect()
    torch.cuda.empty_cache()
    if err is not None:
        pytest.fail(err, pytrace=False)


def _largest_step(orc, precision, n, npdt, tdt, M, NP, E, esz, held):
    s = crk.Solver(nx=n, ny=n, x0=0.0, x1=n * H, y0=0.0, y1=n * H, degree=3, precision=precision,
                   volume_flux=crk.VOL_KG, cfl=0.4, limiter=crk.LIM_BLEND, alpha_max=0.008, alpha_min=1e-3)
    held["solver"] = s
    assert s.shape == (M, E, NP)
    bg = _background(npdt)
    u0 = held["u0"] = torch.empty(s.shape, dtype=tdt, device="cuda")
    for v in range(M):
        u0[v].fill_(float(bg[v]))
    rng = np.random.default_rng(2604)
    noisy = {}
    for (cx, cy) in _sites(n):
        ids = _patch_ids(n, cx, cy, 1)
        val = (bg[:, None, None] * (1.0 + NOISE * rng.uniform(-1.0, 1.0, size=(M, ids.size, NP)))).astype(npdt)
        u0[:, torch.from_numpy(ids).cuda(), :] = torch.from_numpy(val).cuda()
        for k, e in enumerate(ids):
            noisy[int(e)] = val[:, k, :].astype(np.float64)

    u1 = held["u1"] = s.new_state()
    dt = s.new_dt()
    d0 = s.diagnostics(u0).cpu().numpy()
    s.prepare(u0, dt)
    dt0 = dt.cpu().numpy().copy()
    s.advance(u0, u1, dt)
    dt1 = dt.cpu().numpy().copy()
    d1 = s.diagnostics(u1).cpu().numpy()
    torch.cuda.synchronize()

    # FP64 totals: the input's, exactly up to the reduction's rounding; conserved by the step
    w = orc.gll(3)[1]                                          # GLL weights on [0, 1]
    w2 = np.outer(w, w).ravel()
    area = (n * H) ** 2
    expect = bg * area
    for e, val in noisy.items():
        expect += ((val - bg[:, None]) * w2[None, :]).sum(axis=1) * H * H
    for v in range(M):
        assert abs(d0[v] - expect[v]) <= 1e-10 * max(abs(expect[v]), area)
    for v in (0, 3):                                           # mass and energy
        assert abs(d1[v] - d0[v]) <= (1e-12 if esz == 8 else 1e-5) * abs(d0[v])

    # each rough patch against the oracle on its 9 x 9 periodic neighbourhood, with the same dt
    p = _problem(orc, 2 * R_PATCH + 1)
    inner = _patch_ids(2 * R_PATCH + 1, R_PATCH, R_PATCH, 2)
    worst, dts, dts0 = 0.0, [], []
    for (cx, cy) in _sites(n):
        ids = _patch_ids(n, cx, cy, R_PATCH)
        up = np.empty((M, ids.size, NP))
        for k, e in enumerate(ids):
            up[:, k, :] = noisy.get(int(e), np.broadcast_to(bg[:, None], (M, NP)))
        dts0.append(orc.compute_dt(p, up))
        ref, alpha = orc.crk_step(p, up, float(dt0[0]))
        assert alpha.max() > 0.0                               # the limiter acts in the patch
        got = u1[:, torch.from_numpy(ids[inner]).cuda(), :].double().cpu().numpy()
        r = ref[:, inner, :]
        scale = np.array([np.max(np.abs(r[v])) for v in range(M)])
        err = max(np.max(np.abs(got[v] - r[v])) / scale[v] for v in range(M))
        worst = max(worst, err)
        # dt of the new state over this neighbourhood (the oracle's CFL rule on the GPU's state)
        full = u1[:, torch.from_numpy(ids).cuda(), :].double().cpu().numpy()
        dts.append(orc.compute_dt(p, full))
    print(f"largest mesh {n}^2: worst patch difference {worst:.2e}, dt {dt0[0]:.6e} -> {dt1[0]:.6e}", flush=True)
    assert worst <= (1e-12 if esz == 8 else 2e-5)
    for got_dt, ref_dt in ((dt0[0], min(dts0)), (dt1[0], min(dts))):
        assert abs(got_dt - ref_dt) <= (1e-14 if esz == 8 else 1e-6) * ref_dt

    # the uniform flow away from the patches stays uniform
    far = rng.integers(0, E, size=4096)
    ex, ey = far % n, far // n
    near = np.zeros(far.size, dtype=bool)
    for (cx, cy) in _sites(n):
        dx = np.minimum((ex - cx) % n, (cx - ex) % n)
        dy = np.minimum((ey - cy) % n, (cy - ey) % n)
        near |= (dx <= 3) & (dy <= 3)
    far = far[~near]
    uf = u1[:, torch.from_numpy(far).cuda(), :].double().cpu().numpy()
    dev = max(np.max(np.abs(uf[v] - bg[v])) / abs(bg[v]) for v in range(M))
    assert dev <= (1e-13 if esz == 8 else 1e-5)
