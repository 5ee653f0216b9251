"""Throughput benchmark of the cRKFR hot path on one MI355X.

Headline workload: 2D compressible Euler, Kelvin-Helmholtz initial data on
[-1,1]^2 periodic, 256 x 256 elements, degree N = 3 on Gauss-Lobatto nodes
(1,048,576 nodal DOFs), Kennedy-Gruber volume flux, Rusanov interfaces,
classical RK4 inner stages, CFL 0.4, subcell-FV blending limiter with
alpha_max = 0.008, FP64.  One step = local stages + interface exchange and
final update + CFL time-step reduction + blending indicator of the new state
(the pipelined step; crk_prepare seeds dt and the indicator of u0), with the
state resident in HBM.  Metric: DOF-updates/s (one DOF = one solution node).

The same JSON line carries the variants (FP32; the batch of 512 uneven
problems replayed as a HIP graph; Kelvin-Helmholtz 512^2 with the learned
indicator; GLM-MHD Orszag-Tang; the 1D density wave), each with its relative
L2 error against the FP64 CPU oracle stepped from the same initial state.
``--gpus`` above 1 is rejected: the path is measured on a single GPU (it is not sharded).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3

# Per local phase of the KHI 256^2 FP64 workload (with the Kennedy-Gruber flux
# both k_local instances, the one for flagged tiles and the one for the rest),
# from rocprofv3 --pmc:
# HBM bytes = FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB, scaled by the plain-copy
# calibration) and FP64 FLOPs = SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes; valid only
# for the kernel sources whose digest is recorded with them.
MEASURED_TRAFFIC = {
    ("khi256", "fp64"): {"sources_sha256": "8008dc124bbbdf6eb170a2289eefd6911f4b04ef836f339e2a0b7349b76002d8",
                         "bytes": (2.0 * 22854.4 + 1.0 * 66112.0) * 1024,
                         "fp64_flops": 15433728.0 * 64},
    ("khi256_ranocha", "fp64"): {"sources_sha256": "8008dc124bbbdf6eb170a2289eefd6911f4b04ef836f339e2a0b7349b76002d8",
                                 "bytes": (2.0 * 23608.1 + 1.0 * 66048.0) * 1024,
                                 "fp64_flops": 38551552.0 * 64},
}
KERNEL_SOURCES = ("paper_2604_02125_amd/csrc/crk_kernels.hpp", "paper_2604_02125_amd/csrc/crk_physics.hpp")


def sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


KHI = dict(dim=2, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, degree=3, volume_flux=1, cfl=0.4, limiter=1,
           alpha_max=0.008, alpha_min=1e-3)


def k2_bytes_per_dof(M: int, dim: int, N: int, elem: int) -> float:
    """Algorithmic (unique) HBM bytes of the local-stage kernel per DOF: read
    u^n and write the provisional state (M values per node); per face node
    (2*dim faces of (N+1)^(dim-1) nodes per element) write the element's
    share of the interface flux (M values) and read one wave speed: each
    face node's two speeds are read by both elements of the face, so one
    value per element and face node is unique."""
    npe = (N + 1) ** dim
    face_nodes = 2 * dim * (N + 1) ** (dim - 1)
    return elem * (2 * M + (M + 1) * face_nodes / npe)


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def rel_linf(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


class Pipelined:
    """Pipelined stepping of one crk.Solver on torch's current stream."""

    def __init__(self, solver, u0):
        import torch

        from paper_2604_02125_amd import crk
        self.s, self.crk = solver, crk
        self.u0 = torch.tensor(u0, dtype=solver.dtype, device="cuda")
        self.buf = [self.u0.clone(), solver.new_state()]
        self.dt = solver.new_dt()
        self.stream = torch.cuda.current_stream()
        self.sp = crk._stream(self.stream)
        self.reset()

    def reset(self):
        """Back to the initial state (prepared)."""
        crk = self.crk
        self.buf[0].copy_(self.u0)
        self.n = 0
        crk._check(crk.lib().crk_prepare(self.s._h, crk._ptr(self.buf[0]), crk._ptr(self.dt), self.sp), "prepare")

    def step(self):
        crk, L = self.crk, self.crk.lib()
        ui, uo = self.buf[self.n % 2], self.buf[(self.n + 1) % 2]
        p = crk._ptr
        crk._check(L.crk_advance(self.s._h, p(ui), p(uo), p(self.dt), crk.PHASE_LOCAL, self.sp), "advance/local")
        crk._check(L.crk_advance(self.s._h, p(ui), p(uo), p(self.dt), crk.PHASE_INTERFACE, self.sp), "advance/iface")
        self.n += 1

    def local_phase(self):
        """The local phase of the next step alone (leaves the step undone)."""
        crk, L = self.crk, self.crk.lib()
        ui, uo = self.buf[self.n % 2], self.buf[(self.n + 1) % 2]
        p = crk._ptr
        crk._check(L.crk_advance(self.s._h, p(ui), p(uo), p(self.dt), crk.PHASE_LOCAL, self.sp), "advance/local")

    @property
    def state(self):
        return self.buf[self.n % 2]


def timed(pipe, steps, warmup, events=False, reps=20, settle=0.3):
    """Wall time of `steps` pipelined steps; with events, then the mean
    duration of the local-stage kernel from HIP events on the launch stream
    around `reps` back-to-back local phases of the current state (the local
    phase only reads u_in, so repeating it is the same launch each time;
    events around single launches would add their own cost to each)."""
    import torch
    # settle: keep the GPU busy with the same steps for a few tenths of a
    # second first, so that the timed steps see the clocks of a running
    # simulation, then start again from the initial state
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < settle:
        for _ in range(8):
            pipe.step()
        torch.cuda.synchronize()
    pipe.reset()
    for _ in range(warmup):
        pipe.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    k2 = None
    if events:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pipe.local_phase()
        a.record(pipe.stream)
        for _ in range(reps):
            pipe.local_phase()
        b.record(pipe.stream)
        b.synchronize()
        k2 = a.elapsed_time(b) / reps
    return el, k2


def check_admissible(solver, u, what):
    import numpy as np
    d = solver.diagnostics(u).cpu().numpy()
    M = solver.shape[0]
    if not np.isfinite(d[:M]).all() or d[M + 3] > 0 or d[M + 4] >= 0:
        print(f"bench: non-physical state after {what}", file=sys.stderr)
        sys.exit(3)


def conservation(pipe):
    """FP64 diagnostics of the pipelined run so far against its initial state:
    the relative drift of the total mass and the largest drift of any total
    (relative to that total, or to the total mass where the total itself
    vanishes; for MHD the Powell/GLM non-conservative terms move momentum,
    energy, B and psi by design) and the relative change of the total
    entropy (negative: Rusanov interfaces and blending dissipate)."""
    d0 = pipe.s.diagnostics(pipe.u0).cpu().numpy()
    d1 = pipe.s.diagnostics(pipe.state).cpu().numpy()
    M = pipe.s.shape[0]
    drift = max(abs(d1[v] - d0[v]) / max(abs(d0[v]), abs(d0[0])) for v in range(M))
    return {"after_steps": pipe.n, "mass_rel_drift": float(abs(d1[0] - d0[0]) / abs(d0[0])),
            "totals_max_rel_drift": float(drift), "entropy_rel_change": float((d1[M] - d0[M]) / abs(d0[M]))}


def oracle_steps(prob, u0, nsteps):
    import oracle as orc
    u = u0
    for _ in range(nsteps):
        if prob.eq == orc.MHD:
            prob.ch = orc.compute_ch(prob, u)
        u, _ = orc.crk_step(prob, u, orc.compute_dt(prob, u))
    return u


def gpu_steps(solver, u0, nsteps):
    pipe = Pipelined(solver, u0)
    for _ in range(nsteps):
        pipe.step()
    return pipe.state.double().cpu().numpy()


def variant_khi(crk, inputs, orc, n, precision, steps, warmup, err_steps, threads, learned=False, flux=None,
                rough=0.0, half=False):
    import numpy as np
    cfg = dict(KHI)
    if flux is not None:
        cfg["volume_flux"] = flux
    s = crk.Solver(nx=n, ny=n, precision=precision, **cfg)
    if learned:
        net = crk.MLP.load(os.path.join(ROOT, "paper_2604_02125_amd", "mlp_indicator.npz"))
        net.bind(s)
    xi, _, _ = crk.reference_element(3)
    # rough > 0: multiplicative noise of that size on the KHI state, so that
    # the indicator blends (almost) every element; half: in the lower half of
    # the mesh only
    def start(x):
        u = inputs.kelvin_helmholtz(n, n, x)
        if rough:
            r = inputs.perturb(u, 17, rough)
            if half:
                r[:, (n // 2) * n:, :] = u[:, (n // 2) * n:, :]
            u = r
        return u
    u0 = start(xi)
    pipe = Pipelined(s, u0)
    el, k2_ms = timed(pipe, steps, warmup, events=True)
    check_admissible(s, pipe.state, f"khi{n}")
    cons = conservation(pipe)
    ndof = s.nelem * s.shape[2]
    out = {"value": ndof * steps / el, "unit": "DOF-updates/s", "ms_per_step": el / steps * 1e3, "steps": steps,
           "k_local_ms": k2_ms}
    out["conservation"] = cons
    out["blended_element_fraction"] = float((s.indicator(pipe.state)[1] > 0).double().mean().item())
    key = (f"khi{n}" + ("_ranocha" if flux == crk.VOL_RANOCHA else ""), "fp64" if precision == crk.FP64 else "fp32")
    rec = MEASURED_TRAFFIC.get(key)
    if rec and rec["sources_sha256"] == sources_digest() and flux is not None:
        out["k_local_fp64_tflops"] = rec["fp64_flops"] / (k2_ms * 1e-3) / 1e12
        out["k_local_fp64_frac"] = out["k_local_fp64_tflops"] / PEAK_FP64_TFLOPS
    if err_steps:
        p = orc.Problem(dim=2, nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=3,
                        vol_flux=orc.VOL_KG if flux is None else flux, limiter=orc.LIM_BLEND_MODAL, nthreads=threads)
        oxi, _ = orc.gll(3)
        ref = oracle_steps(p, start(oxi), err_steps)
        got = gpu_steps(s, u0, err_steps)
        out["l2_rel_error_vs_fp64_oracle"] = rel_l2(got, ref)
        out["linf_rel_error_vs_fp64_oracle"] = rel_linf(got, ref)
        out["error_after_steps"] = err_steps
        if learned:
            s2 = crk.Solver(nx=n, ny=n, precision=precision, **KHI)
            pa = Pipelined(s2, u0)
            for _ in range(err_steps):
                pa.step()
            a_modal = s2.indicator(pa.state)[1].cpu().numpy()
            a_net = s.indicator(pa.state)[1].cpu().numpy()
            out["alpha_positive_disagreement_vs_modal"] = float(np.mean((a_modal > 0) != (a_net > 0)))
    return out


def variant_batch(crk, inputs, orc, precision, reps, err_sample=4):
    import numpy as np
    import torch
    specs, rng = inputs.random_fourier_problems(512, seed=20260402)
    b = crk.Batch(specs, precision=precision, volume_flux=crk.VOL_RANOCHA)
    states = []
    for i, (n, N) in enumerate(specs):
        xi, _, _ = crk.reference_element(N)
        u = inputs.random_fourier_state(rng, n, xi)
        if i < err_sample:
            states.append(u)
        b.view(0, i).copy_(torch.tensor(u, dtype=b.dtype))
    u_init = b.u[0].clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        b.capture_graph()
        b.launch_graph()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        for _ in range(reps):
            b.launch_graph()
        e1.record(b.stream)
    b.stream.synchronize()
    ms = e0.elapsed_time(e1) / (2 * reps)
    # error: two eager steps from the initial states against the oracle
    b.u[0].copy_(u_init)
    torch.cuda.synchronize()
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        b.advance(0)
        b.advance(1)
    b.stream.synchronize()
    num = den = dmax = rmax = 0.0
    for i in range(err_sample):
        n, N = specs[i]
        p = orc.Problem(dim=2, nx=n, ny=n, N=N, vol_flux=orc.VOL_RANOCHA)
        ref = oracle_steps(p, states[i], 2)
        got = b.view(0, i).double().cpu().numpy()
        num += float(np.sum((got - ref) ** 2))
        den += float(np.sum(ref ** 2))
        dmax = max(dmax, float(np.max(np.abs(got - ref))))
        rmax = max(rmax, float(np.max(np.abs(ref))))
    return {"value": b.ndof / (ms * 1e-3), "unit": "DOF-updates/s", "ms_per_step": ms, "steps": 2 * reps,
            "problems": len(specs), "dofs": b.ndof, "tuning": {"block": b.tuning[0], "grid_per_cu": b.tuning[1]},
            "graph": "2 pipelined steps per replay",
            "l2_rel_error_vs_fp64_oracle": float(np.sqrt(num / den)), "linf_rel_error_vs_fp64_oracle": dmax / rmax,
            "error_after_steps": 2, "error_sample": f"first {err_sample} problems"}


def variant_mhd(crk, inputs, orc, precision, steps, warmup, threads):
    n = 192
    s = crk.Solver(dim=2, nx=n, ny=n, degree=4, equation=crk.CRK_GLM_MHD, gamma=5.0 / 3.0, precision=precision,
                   volume_flux=crk.VOL_DERIGS, cfl=0.4)
    xi, _, _ = crk.reference_element(4)
    u0 = inputs.orszag_tang(n, n, xi)
    pipe = Pipelined(s, u0)
    el, _ = timed(pipe, steps, warmup)
    check_admissible(s, pipe.state, "mhd")
    cons = conservation(pipe)
    p = orc.Problem(dim=2, nx=n, ny=n, N=4, eq=orc.MHD, gamma=5.0 / 3.0, vol_flux=orc.VOL_DERIGS, nthreads=threads)
    oxi, _ = orc.gll(4)
    ref = oracle_steps(p, inputs.orszag_tang(n, n, oxi), 1)
    got1 = gpu_steps(s, u0, 1)
    ndof = s.nelem * s.shape[2]
    return {"value": ndof * steps / el, "unit": "DOF-updates/s", "ms_per_step": el / steps * 1e3, "steps": steps,
            "l2_rel_error_vs_fp64_oracle": rel_l2(got1, ref), "linf_rel_error_vs_fp64_oracle": rel_linf(got1, ref),
            "error_after_steps": 1, "conservation": cons}


def variant_wave1d(crk, inputs, orc):
    import numpy as np
    import torch
    s = crk.Solver(dim=1, nx=64, degree=3, volume_flux=crk.VOL_RANOCHA, cfl=0.4)
    xi, _, _ = crk.reference_element(3)
    u0 = inputs.density_wave_1d(64, xi)
    # all 200 steps in one launch (crk_run: one workgroup holds the 256 nodes)
    ug = torch.tensor(u0, device="cuda")
    buf, dt = [ug.clone(), s.new_state()], s.new_dt()
    for _ in range(3):                       # warm-up runs
        buf[0].copy_(ug)
        s.prepare(buf[0], dt)
        s.run(buf[0], buf[1], dt, 200)
    buf[0].copy_(ug)
    s.prepare(buf[0], dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got_t = s.run(buf[0], buf[1], dt, 200)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    p = orc.Problem(dim=1, nx=64, N=3, vol_flux=orc.VOL_RANOCHA)
    oxi, _ = orc.gll(3)
    ref = oracle_steps(p, inputs.density_wave_1d(64, oxi), 200)
    got = got_t.cpu().numpy()
    return {"value": 256 * 200 / el, "unit": "DOF-updates/s", "us_per_step": el / 200 * 1e6, "steps": 200,
            "launch": "one crk_run launch for the 200 steps",
            "l2_rel_error_vs_fp64_oracle": rel_l2(got, ref), "linf_rel_error_vs_fp64_oracle": rel_linf(got, ref),
            "error_after_steps": 200,
            "max_velocity_deviation": float(np.max(np.abs(got[1] / got[0] - 0.1)))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)   # the configuration's run length
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    # the blended variant launches the headline's local-stage kernel on the same
    # grid: profiler runs skip it so that per-kernel averages cover the headline
    ap.add_argument("--no-blended", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--err-steps", type=int, default=3)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path is not sharded across GPUs; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8, "copies": 5}))
        return

    from paper_2604_02125_amd import crk, inputs
    torch.cuda.set_device(0)
    threads = min(16, os.cpu_count() or 1)

    # ------------------------------------------------------------ headline
    s = crk.Solver(nx=256, ny=256, precision=crk.FP64, **KHI)
    xi, _, _ = crk.reference_element(3)
    u0 = inputs.kelvin_helmholtz(256, 256, xi)
    M, E, NP = s.shape
    ndof = E * NP
    pipe = Pipelined(s, u0)
    elapsed, k2_ms = timed(pipe, args.steps, args.warmup, events=True)
    check_admissible(s, pipe.state, "the timed steps")
    value = ndof * args.steps / elapsed
    kb = k2_bytes_per_dof(M, 2, 3, 8) * ndof
    achieved = kb / (k2_ms * 1e-3) / 1e9
    rec = MEASURED_TRAFFIC.get(("khi256", "fp64"))
    fresh = bool(rec) and rec["sources_sha256"] == sources_digest()
    traffic = rec["bytes"] if fresh else None
    fp64 = rec["fp64_flops"] / (k2_ms * 1e-3) / 1e12 if fresh else None
    out = {
        "metric": "DOF-updates/s at 1 GPU",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic Kelvin-Helmholtz initial condition)",
        "config": {"workload": "2D Euler Kelvin-Helmholtz 256x256, N=3, Kennedy-Gruber, blending alpha_max=0.008",
                   "elements": E, "degree": 3, "dofs": ndof, "precision": "fp64", "parallelism": "single GPU"},
        # a DOF is a node; the same rate counted per conserved variable (x M = 4)
        "variable_dof_updates_per_s": value * 4,
        "roofline": {"bound": "hbm", "kernel": "k_local (local stages)", "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "kernel_ms": k2_ms, "algorithmic_bytes_per_launch": kb,
                     # counter FP64 FLOPs of the same kernel over its live duration
                     "fp64_tflops": fp64, "fp64_peak_tflops": PEAK_FP64_TFLOPS,
                     "fp64_frac": fp64 / PEAK_FP64_TFLOPS if fp64 is not None else None},
    }
    import oracle as orc
    if not args.no_cpu_baseline:
        p = orc.Problem(dim=2, nx=256, ny=256, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=3, vol_flux=orc.VOL_KG,
                        limiter=orc.LIM_BLEND_MODAL, nthreads=threads)
        oxi, _ = orc.gll(3)
        uc = inputs.kelvin_helmholtz(256, 256, oxi)
        c0 = time.perf_counter()
        for _ in range(args.cpu_steps):
            uc, _ = orc.crk_step(p, uc, orc.compute_dt(p, uc))
        c1 = time.perf_counter()
        out["cpu_baseline"] = {"value": ndof * args.cpu_steps / (c1 - c0), "unit": "DOF-updates/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{args.cpu_steps} full steps of the same workload (FP64 C oracle, "
                                         f"OpenMP over elements, {threads} threads)"}
    if not args.no_variants:
        v = {}
        v["khi256_fp64"] = variant_khi(crk, inputs, orc, 256, crk.FP64, 20, 2, args.err_steps, threads)
        v["khi256_fp32"] = variant_khi(crk, inputs, orc, 256, crk.FP32, 20, 2, args.err_steps, threads)
        # the same workload with the entropy-conservative Ranocha flux (log means)
        v["khi256_ranocha_fp64"] = variant_khi(crk, inputs, orc, 256, crk.FP64, 20, 2, args.err_steps, threads,
                                               flux=crk.VOL_RANOCHA)
        if not args.no_blended:
            v["khi256_blended_fp64"] = variant_khi(crk, inputs, orc, 256, crk.FP64, 20, 2, args.err_steps,
                                                   threads, rough=0.05)
            v["khi256_half_blended_fp64"] = variant_khi(crk, inputs, orc, 256, crk.FP64, 20, 2, args.err_steps,
                                                        threads, rough=0.05, half=True)
        v["batch512_fp64"] = variant_batch(crk, inputs, orc, crk.FP64, 5)
        v["batch512_fp32"] = variant_batch(crk, inputs, orc, crk.FP32, 5)
        v["khi512_learned_fp64"] = variant_khi(crk, inputs, orc, 512, crk.FP64, 10, 2, args.err_steps, threads,
                                               learned=True)
        v["mhd_ot192_fp64"] = variant_mhd(crk, inputs, orc, crk.FP64, 10, 2, threads)
        v["mhd_ot192_fp32"] = variant_mhd(crk, inputs, orc, crk.FP32, 10, 2, threads)
        v["density_wave_1d_fp64"] = variant_wave1d(crk, inputs, orc)
        v["_note"] = ("l2_rel_error_vs_fp64_oracle = ||u_gpu - u_oracle||_2 / ||u_oracle||_2 and "
                      "linf_rel_error_vs_fp64_oracle = max|u_gpu - u_oracle| / max|u_oracle| over all values "
                      "after error_after_steps steps from the same initial state (the FP64 rows are a "
                      "round-off check)")
        out["variants"] = v
    print(json.dumps(out))


if __name__ == "__main__":
    main()
