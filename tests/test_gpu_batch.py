"""GPU tests of the batched path: mixed degrees in one persistent launch,
per-problem time steps, equivalence with single-problem runs and with the
oracle, and HIP-graph replays against eager steps."""
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


def _rel(a, b):
    return max(np.max(np.abs(a[v] - b[v])) / np.max(np.abs(b[v])) for v in range(b.shape[0]))


SPECS = [(5, 3), (7, 4), (3, 3), (9, 4), (4, 3), (6, 4), (11, 3)]


def _fill(orc, batch, seed):
    rng = np.random.default_rng(seed)
    states = []
    for i, (n, N) in enumerate(batch.specs):
        xi, _ = orc.gll(N)
        u = inputs.random_fourier_state(rng, n, xi)
        batch.view(0, i).copy_(torch.tensor(u, dtype=batch.dtype))
        states.append(u)
    torch.cuda.synchronize()
    return states


@pytest.mark.parametrize("tuning", [(256, 4), (128, 0), (64, 2), (128, 0, 1), (64, 32, 1)])
def test_batch_matches_oracle_per_problem(orc, tuning):
    b = crk.Batch(SPECS, tuning=tuning)
    u0 = _fill(orc, b, seed=1)
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        b.advance(0)
        b.advance(1)
    b.stream.synchronize()
    for i, (n, N) in enumerate(SPECS):
        p = orc.Problem(dim=2, nx=n, ny=n, N=N, vol_flux=orc.VOL_RANOCHA)
        ref = u0[i]
        for _ in range(2):
            ref, _ = orc.crk_step(p, ref, orc.compute_dt(p, ref))
        got = b.view(0, i).cpu().numpy()
        assert _rel(got, ref) <= 1e-12, (i, n, N)
        # dt left behind belongs to the final state of problem i
        assert abs(b.dt[2 * i].item() - orc.compute_dt(p, ref)) <= 1e-14 * b.dt[2 * i].item()


EDGE_SPECS = {
    "one_element_deg3": [(1, 3)],
    "deg4_only_tiny": [(1, 4), (2, 4)],
    "deg4_only": [(6, 4), (3, 4)],
    "deg3_only": [(5, 3)],
    "mixed_tiny": [(2, 3), (1, 4)],
}


@pytest.mark.parametrize("tuning", [(128, 0, 0), (64, 2, 0), (128, 0, 1)], ids=["tile", "persistent", "merged"])
@pytest.mark.parametrize("case", sorted(EDGE_SPECS))
def test_batch_edge_shapes(orc, case, tuning):
    """Batches with a single degree (the other degree's launch has no
    tiles), single-element problems (every neighbour is the element itself)
    and fewer tiles than a persistent grid, in every launch shape."""
    specs = EDGE_SPECS[case]
    b = crk.Batch(specs, tuning=tuning)
    u0 = _fill(orc, b, seed=5)
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        b.advance(0)
        b.advance(1)
    b.stream.synchronize()
    for i, (n, N) in enumerate(specs):
        p = orc.Problem(dim=2, nx=n, ny=n, N=N, vol_flux=orc.VOL_RANOCHA)
        ref = u0[i]
        for _ in range(2):
            ref, _ = orc.crk_step(p, ref, orc.compute_dt(p, ref))
        assert _rel(b.view(0, i).cpu().numpy(), ref) <= 1e-12, (case, i)
        assert abs(b.dt[2 * i].item() - orc.compute_dt(p, ref)) <= 1e-14 * b.dt[2 * i].item()


def test_batch_equals_single_problem_runs(orc):
    b = crk.Batch(SPECS)
    u0 = _fill(orc, b, seed=2)
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        for k in range(3):
            b.advance(k % 2)
    b.stream.synchronize()
    for i, (n, N) in enumerate(SPECS):
        s = crk.Solver(dim=2, nx=n, ny=n, degree=N, volume_flux=crk.VOL_RANOCHA)
        buf = [torch.tensor(u0[i], device="cuda"), s.new_state()]
        dt = s.new_dt()
        s.prepare(buf[0], dt)
        for k in range(3):
            s.advance(buf[k % 2], buf[(k + 1) % 2], dt)
        torch.cuda.synchronize()
        assert _rel(b.view(1, i).cpu().numpy(), buf[1].cpu().numpy()) <= 1e-13


def test_graph_replay_equals_eager(orc):
    """Two steps captured once; each replay checked against eager steps from
    the same state, with eager work and synchronisations in between."""
    b = crk.Batch(SPECS)
    _fill(orc, b, seed=3)
    ref = crk.Batch(SPECS)
    ref.u[0].copy_(b.u[0])
    torch.cuda.synchronize()
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        b.capture_graph()
    with torch.cuda.stream(ref.stream):
        ref.prepare(0)
    for rep in range(3):
        with torch.cuda.stream(b.stream):
            b.launch_graph()
        with torch.cuda.stream(ref.stream):
            ref.advance(0)
            ref.advance(1)
        b.stream.synchronize()
        ref.stream.synchronize()
        assert torch.equal(b.u[0], ref.u[0]), rep
        assert torch.equal(b.dt, ref.dt), rep
        # eager work on the graph's buffers between replays
        x = b.u[0].clone() * 1.0
        torch.cuda.synchronize()
        assert torch.equal(x, ref.u[0])


def test_batch_fp32(orc):
    b = crk.Batch(SPECS[:4], precision=crk.FP32)
    u0 = _fill(orc, b, seed=4)
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        b.advance(0)
    b.stream.synchronize()
    for i, (n, N) in enumerate(SPECS[:4]):
        p = orc.Problem(dim=2, nx=n, ny=n, N=N, vol_flux=orc.VOL_RANOCHA)
        u32 = u0[i].astype(np.float32).astype(np.float64)
        ref, _ = orc.crk_step(p, u32, b.dt[2 * i].item() if False else orc.compute_dt(p, u32))
        assert _rel(b.view(1, i).cpu().numpy().astype(np.float64), ref) <= 2e-5


def test_batch_rejects_bad_input():
    with pytest.raises(crk.CrkError):
        crk.Batch([])                 # no problems
    with pytest.raises(crk.CrkError):
        crk.Batch([(4, 2)])           # degree 2 not in a batch
    with pytest.raises(crk.CrkError):
        crk.Batch([(4, 3)], volume_flux=crk.VOL_CENTRAL)


def test_full_size_batch_sampled(orc):
    """The benchmarked batch (512 problems, n ~ U{16..96}, N in {3, 4}, seed
    20260402) in the benchmark's launch configuration (default tile shape,
    two pipelined steps replayed from a HIP graph): sampled problems (the
    largest of each degree, the smallest, and a seeded random few) against
    the oracle after the two steps, state and dt."""
    specs, rng = inputs.random_fourier_problems(512, seed=20260402)
    b = crk.Batch(specs, volume_flux=crk.VOL_RANOCHA)
    pick = set(np.random.default_rng(7).choice(len(specs), 6, replace=False).tolist())
    for deg in (3, 4):
        idx = [i for i, (n, N) in enumerate(specs) if N == deg]
        pick.add(max(idx, key=lambda i: specs[i][0]))
    pick.add(min(range(len(specs)), key=lambda i: specs[i][0]))
    keep = {}
    for i, (n, N) in enumerate(specs):
        xi, _ = orc.gll(N)
        u = inputs.random_fourier_state(rng, n, xi)
        b.view(0, i).copy_(torch.tensor(u, dtype=b.dtype))
        if i in pick:
            keep[i] = u
    torch.cuda.synchronize()
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        b.capture_graph()
        b.launch_graph()
    b.stream.synchronize()
    for i, u in sorted(keep.items()):
        n, N = specs[i]
        p = orc.Problem(dim=2, nx=n, ny=n, N=N, vol_flux=orc.VOL_RANOCHA, nthreads=16)
        ref = u
        for _ in range(2):
            ref, _ = orc.crk_step(p, ref, orc.compute_dt(p, ref))
        assert _rel(b.view(0, i).cpu().numpy(), ref) <= 1e-12, (i, n, N)
        assert abs(b.dt[2 * i].item() - orc.compute_dt(p, ref)) <= 1e-14 * b.dt[2 * i].item(), (i, n, N)
