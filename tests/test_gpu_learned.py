"""GPU tests of the learned troubled-cell indicator against the FP64 oracle:
forward pass, loss gradient, Adam step, features, labels, inference with
fallback to the modal indicator, training progress, and what the trained
network gains over the modal indicator on a Kelvin-Helmholtz run."""
import os

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


def _bf16_round(x):
    """float -> nearest-even BF16 -> float64 (numpy, independent of the kernels)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _net(seed=0):
    net = crk.MLP(seed=seed)
    theta64 = _bf16_round(net.theta.cpu().numpy())
    return net, theta64


def test_mlp_forward_parity(orc):
    net, th = _net(1)
    rng = np.random.default_rng(2)
    x = rng.dirichlet(np.ones(16), size=1000).astype(np.float32)
    z, a = net.forward(torch.tensor(x, device="cuda"), alpha_max=0.008)
    zo, ao = orc.mlp_forward(16, 64, th, x.astype(np.float64), 0.008)
    assert np.max(np.abs(z.cpu().numpy() - zo)) <= 1e-5 * max(1.0, np.max(np.abs(zo)))
    assert np.max(np.abs(a.cpu().numpy() - ao)) <= 1e-7


def test_mlp_gradient_parity(orc):
    net, th = _net(3)
    rng = np.random.default_rng(4)
    n = 1000                                      # several workgroups and a ragged last one
    x = rng.dirichlet(np.ones(16), size=n).astype(np.float32)
    y = (rng.uniform(size=n) < 0.3).astype(np.float32)
    loss, g, _ = net.loss_grad(torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"))
    lo, go = orc.mlp_loss_grad(16, 64, th, x.astype(np.float64), y.astype(np.float64))
    gg = g.cpu().numpy()
    assert abs(loss.item() - lo) <= 1e-5 * abs(lo)
    assert np.linalg.norm(gg - go) <= 1e-4 * np.linalg.norm(go)
    assert np.max(np.abs(gg - go)) <= 1e-4 * np.max(np.abs(go))


def test_adam_parity(orc):
    net, _ = _net(5)
    rng = np.random.default_rng(6)
    th = net.theta.cpu().numpy().astype(np.float64)
    m, v = np.zeros_like(th), np.zeros_like(th)
    for t in range(1, 4):
        g = rng.normal(size=th.size).astype(np.float32)
        net.adam(torch.tensor(g, device="cuda"), lr=1e-2)
        orc.adam_step(th, m, v, g.astype(np.float64), 1e-2, t)
    assert np.max(np.abs(net.theta.cpu().numpy() - th)) <= 1e-5
    # the BF16 copy is the nearest-even rounding of the FP32 master
    assert np.array_equal(net.theta_bf16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16,
                          (_bf16_round(net.theta.cpu().numpy()).astype(np.float32)).view(np.uint32))


def _khi_pair(orc, n=24):
    p = orc.Problem(dim=2, nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=3, vol_flux=orc.VOL_KG,
                    limiter=orc.LIM_BLEND_MODAL)
    s = crk.Solver(dim=2, nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, degree=3, volume_flux=crk.VOL_KG,
                   limiter=crk.LIM_BLEND)
    xi, _ = orc.gll(3)
    u = inputs.perturb(inputs.kelvin_helmholtz(n, n, xi, v2_modes=inputs.khi_modes(3)), 5, 1e-2)
    return p, s, u


def test_features_parity(orc):
    p, s, u = _khi_pair(orc)
    f = crk.features(s, torch.tensor(u, device="cuda")).cpu().numpy()
    _, _, fo = orc.indicator(p, u)
    assert np.max(np.abs(f - orc.feature_transform(fo))) <= 1e-6


def test_labels_parity(orc):
    """Labels of the unlimited update: identical decisions on both sides."""
    p, s, u = _khi_pair(orc, n=32)
    dt = orc.compute_dt(p, u)
    q = orc.Problem(**{**p.__dict__, "limiter": orc.LIM_NONE})
    uh, _ = orc.crk_step(q, u, 2.5 * dt)            # a larger step makes some elements troubled
    lo = orc.labels(p, u, uh)
    lg = crk.labels(s, torch.tensor(u, device="cuda"), torch.tensor(uh, device="cuda")).cpu().numpy()
    assert 0 < lo.sum() < p.nelem
    assert np.array_equal(lg.astype(np.float64), lo)


def test_inference_and_fallback(orc):
    """The bound network replaces the modal coefficient except where a
    feature lies outside the training range; alpha < alpha_min is cut."""
    p, s, u = _khi_pair(orc)
    ug = torch.tensor(u, device="cuda")
    araw_modal, _ = s.indicator(ug)
    f = crk.features(s, ug)
    net, th = _net(7)
    # training range that excludes the elements whose first feature is large
    cut = float(torch.quantile(f[:, 0], 0.7))
    net.lo = torch.zeros(16, device="cuda")
    net.hi = torch.ones(16, device="cuda")
    net.hi[0] = cut
    net.bind(s)
    araw, alpha = s.indicator(ug)
    _, a_net = orc.mlp_forward(16, 64, th, f.cpu().numpy().astype(np.float64), 0.008)
    a_net = np.where(a_net < 1e-3, 0.0, a_net)
    inside = f[:, 0].cpu().numpy() <= cut
    got = araw.cpu().numpy()
    assert np.max(np.abs(got[inside] - a_net[inside])) <= 1e-7
    assert np.array_equal(got[~inside], araw_modal.cpu().numpy()[~inside])
    # unbinding restores the modal indicator
    crk.lib().crk_set_mlp(s._h, None, None, None)
    assert torch.equal(s.indicator(ug)[0], araw_modal)


def test_training_reduces_loss(orc):
    """A few Adam steps on labelled snapshots of a small run lower the loss."""
    from paper_2604_02125_amd import learned
    X, Y = learned.generate([11], n=32, t_snaps=(1.0, 1.5), log=lambda *a: None)
    assert 0.0 < Y.mean().item() < 1.0
    net = crk.MLP(seed=0)
    l0, _, _ = net.loss_grad(X, Y)
    for _ in range(60):
        _, g, _ = net.loss_grad(X, Y)
        net.adam(g, lr=3e-3)
    l1, _, _ = net.loss_grad(X, Y)
    assert l1.item() < 0.8 * l0.item()


WEIGHTS = os.path.join(os.path.dirname(crk.HERE), "paper_2604_02125_amd", "mlp_indicator.npz")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_gain_over_modal_indicator(orc):
    """Kelvin-Helmholtz 128x128 to t ~ 3 (6000 pipelined steps) with the
    trained network and with the modal indicator: both stay admissible; the
    network blends in less low-order dissipation (smaller sum of alpha over
    the run); the per-element disagreement of alpha > 0 on the final state
    is reported."""
    from paper_2604_02125_amd import learned
    n, steps = 128, 6000
    xi, _, _ = crk.reference_element(3)
    u0 = inputs.kelvin_helmholtz(n, n, xi)
    res = {}
    for kind in ("modal", "mlp"):
        s = learned.khi_solver(n)
        if kind == "mlp":
            crk.MLP.load(WEIGHTS).bind(s)
        u = [torch.tensor(u0, device="cuda"), s.new_state()]
        dt = s.new_dt()
        s.prepare(u[0], dt)
        asum = 0.0
        for k in range(steps):
            s.advance(u[k % 2], u[(k + 1) % 2], dt)
            if k % 100 == 0:
                asum += float(s.indicator(u[(k + 1) % 2])[1].sum())
        torch.cuda.synchronize()
        d = s.diagnostics(u[steps % 2]).cpu().numpy()
        res[kind] = dict(min_p=d[6], nonfinite=d[7], first_bad=d[8], asum=asum, state=u[steps % 2],
                         alpha=s.indicator(u[steps % 2])[1].cpu().numpy())
    for kind in res:
        assert res[kind]["nonfinite"] == 0 and res[kind]["first_bad"] == -1 and res[kind]["min_p"] > 0
    disagree = np.mean((res["mlp"]["alpha"] > 0) != (res["modal"]["alpha"] > 0))
    print(f"sum alpha: modal {res['modal']['asum']:.3f}, learned {res['mlp']['asum']:.3f}; "
          f"alpha>0 disagreement on the final state {disagree:.4f}")
    assert res["mlp"]["asum"] < res["modal"]["asum"]


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_gain_on_held_out_labels():
    """The modal indicator as judge, on runs the network never saw (seeds 101
    and 102, snapshots at t = 1.5 and 2.5, KHI 128^2): against the
    a-posteriori troubled-element labels the network must flag at least as
    many labelled elements as the modal indicator (a bounded miss rate: not
    above the modal one) while flagging fewer elements in all."""
    from paper_2604_02125_amd import learned
    st = learned.held_out(crk.MLP.load(WEIGHTS))
    net, mod = st["network"], st["modal"]
    print(f"held-out labels: network tp {net['tp']} fn {net['fn']} fp {net['fp']} (flagged "
          f"{net['flagged_fraction']:.4f}); modal tp {mod['tp']} fn {mod['fn']} fp {mod['fp']} "
          f"(flagged {mod['flagged_fraction']:.4f})")
    assert net["tp"] + net["fn"] > 100                      # enough troubled elements to judge
    assert net["miss_rate"] <= mod["miss_rate"]
    assert net["flagged_fraction"] < mod["flagged_fraction"]


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_gain_closer_to_unlimited_solution():
    """KHI 128^2 to t = 2 with one fixed time step for all runs: the unlimited
    high-order run (no blending) is the reference, since every blended
    element adds first-order dissipation to it.  With the network the run
    stays closer to it than with the modal indicator, and blends less."""
    from paper_2604_02125_amd import learned
    n = 128
    xi, _, _ = crk.reference_element(3)
    u0 = torch.tensor(inputs.kelvin_helmholtz(n, n, xi), device="cuda")
    h = 0.8 * learned.khi_solver(n).compute_dt(u0)[0].item()
    nsteps = int(round(2.0 / h))
    net = crk.MLP.load(WEIGHTS)
    res = {}
    for kind in ("none", "modal", "mlp"):
        s = learned.khi_solver(n, limiter=kind != "none")
        if kind == "mlp":
            net.bind(s)
        u = [u0.clone(), s.new_state()]
        dtt = torch.tensor([h, 0.0], dtype=torch.float64, device="cuda")
        asum = 0.0
        for k in range(nsteps):
            s.step(u[k % 2], u[(k + 1) % 2], dtt, compute_dt=False)
            if kind != "none" and k % 50 == 0:
                asum += float(s.indicator(u[(k + 1) % 2])[1].sum())
        rc, fb, _ = s.check(u[nsteps % 2])
        assert rc == crk.OK, kind
        res[kind] = (u[nsteps % 2].cpu().numpy(), asum)
    ref = res["none"][0]
    err = {k: float(np.sqrt(np.sum((res[k][0] - ref) ** 2) / np.sum(ref ** 2))) for k in ("modal", "mlp")}
    print(f"t = 2 ({nsteps} steps): rel L2 to the unlimited run: modal {err['modal']:.3e}, network {err['mlp']:.3e}; "
          f"sum alpha: modal {res['modal'][1]:.2f}, network {res['mlp'][1]:.2f}")
    assert err["mlp"] < err["modal"]
    assert res["mlp"][1] < res["modal"][1]


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_pipelined_learned_tile_flags(orc):
    """Pipelined steps with the trained network bound, where the network's
    own coefficients flag the local-phase tiles that may blend, against
    crk_step with the same network, which runs the blending code on every
    tile.  A tile left unflagged would skip its blending (an O(alpha)
    difference)."""
    p, s, u = _khi_pair(orc, n=32)
    crk.MLP.load(WEIGHTS).bind(s)
    ug = torch.tensor(u, device="cuda")
    araw, _ = s.indicator(ug)
    npos = int((araw > 0).sum())
    print(f"elements with alpha > 0: {npos} of {s.nelem}")
    assert 0 < npos < s.nelem // 2
    nsteps = 4
    a = [ug.clone(), s.new_state()]
    da = s.new_dt()
    s.prepare(a[0], da)
    for n in range(nsteps):
        s.advance(a[n % 2], a[(n + 1) % 2], da)
    b = [ug.clone(), s.new_state()]
    db = s.new_dt()
    for n in range(nsteps):
        s.step(b[n % 2], b[(n + 1) % 2], db)
    torch.cuda.synchronize()
    got, ref = a[nsteps % 2].cpu().numpy(), b[nsteps % 2].cpu().numpy()
    rel = max(np.max(np.abs(got[v] - ref[v])) / np.max(np.abs(ref[v])) for v in range(ref.shape[0]))
    print(f"pipelined vs crk_step with the network: {rel:.2e}")
    assert rel <= 1e-13


def _oracle_learned_alpha(orc, p, u, th, lo, hi):
    """The learned blending coefficients composed from the oracle's parts:
    modal energy fractions -> log features -> the FP64 network with the
    BF16-rounded parameters -> alpha_max sigmoid, cut below alpha_min, where
    every feature lies in the training range [lo, hi] (compared in FP32, as
    the features are stored), else the modal coefficient; then smoothing over
    face neighbours.  Also returns the network's uncut coefficient."""
    araw_modal, _, fo = orc.indicator(p, u)
    x32 = orc.feature_transform(fo).astype(np.float32)
    z, a = orc.mlp_forward(16, 64, th, x32.astype(np.float64), p.alpha_max)
    inside = np.all((x32 >= lo) & (x32 <= hi), axis=1) & np.isfinite(z)
    araw = np.where(inside, np.where(a < p.alpha_min, 0.0, a), araw_modal)
    return araw, orc.smooth_alpha(p, araw), a, inside


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
@pytest.mark.parametrize("fallback", [False, True], ids=["trained_range", "narrowed_range"])
def test_pipelined_learned_step_against_oracle(orc, fallback):
    """End to end: one pipelined step with the trained network bound (the
    features of u^n from the interface tail of crk_prepare, inference on the
    matrix cores, smoothing and tile flags in the local phase) against the
    oracle's step with the coefficients composed from the oracle's own
    indicator, network and smoothing.  The network runs in FP32 on the GPU
    and in FP64 in the oracle, so the coefficients agree to ~1e-8; the input
    is checked to have no element within 1e-7 of the alpha_min cut, where
    the two could decide differently.  narrowed_range: the first feature's
    range is cut at its 70th percentile, so that a third of the elements
    fall back to the modal coefficient."""
    p, s, u = _khi_pair(orc, n=32)
    pg = orc.Problem(dim=2, nx=32, ny=32, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=3, vol_flux=orc.VOL_KG,
                     limiter=orc.LIM_BLEND_GIVEN)
    net = crk.MLP.load(WEIGHTS)
    th = _bf16_round(net.theta.cpu().numpy())
    lo, hi = net.lo.cpu().numpy().copy(), net.hi.cpu().numpy().copy()
    if fallback:
        _, _, fo = orc.indicator(p, u)
        hi[0] = np.float32(np.quantile(orc.feature_transform(fo)[:, 0], 0.7))
        net.hi = torch.tensor(hi, device="cuda")
    net.bind(s)
    araw, alpha, a_net, inside = _oracle_learned_alpha(orc, p, u, th, lo, hi)
    assert np.min(np.abs(a_net[inside] - p.alpha_min)) > 1e-7
    assert (araw[inside] > 0).sum() > 50
    assert (not fallback) or (0 < (~inside).sum() < p.nelem)
    ug = torch.tensor(u, device="cuda")
    ga, gs = s.indicator(ug)
    assert np.max(np.abs(ga.cpu().numpy() - araw)) <= 1e-7
    assert np.max(np.abs(gs.cpu().numpy() - alpha)) <= 1e-7
    dt = orc.compute_dt(p, u)
    ref, _ = orc.crk_step(pg, u, dt, alpha)
    buf, dtg = [ug.clone(), s.new_state()], s.new_dt()
    s.prepare(buf[0], dtg)
    assert abs(dtg[0].item() - dt) <= 1e-14 * dt
    s.advance(buf[0], buf[1], dtg)
    torch.cuda.synchronize()
    got = buf[1].cpu().numpy()
    rel = max(np.max(np.abs(got[v] - ref[v])) / np.max(np.abs(ref[v])) for v in range(ref.shape[0]))
    print(f"learned step against the oracle ({'narrowed' if fallback else 'trained'} range): {rel:.2e}, "
          f"{int((araw > 0).sum())} elements with alpha > 0, {int((~inside).sum())} on the modal fallback")
    assert rel <= 1e-8
