"""Throughput benchmark of the cRKFR hot path on one MI355X.

Headline workload: 2D compressible Euler, Kelvin-Helmholtz initial data on
[-1,1]^2 periodic, 256 x 256 elements, degree N = 3 on Gauss-Lobatto nodes
(1,048,576 nodal DOFs), Kennedy-Gruber volume flux, Rusanov interfaces,
classical RK4 inner stages, CFL 0.4, subcell-FV blending limiter with
alpha_max = 0.008, FP64.  One step = local stages + interface exchange and
final update + CFL time-step reduction + blending indicator of the new state
(the pipelined step; crk_prepare seeds dt and the indicator of u0), with the
state resident in HBM.  Metric: DOF-updates/s (one DOF = one solution node).

The same JSON line carries the variants (FP32; the Ranocha EC flux; rough
states that blend everywhere or on one half; the batch of 512 uneven problems
replayed as a HIP graph; Kelvin-Helmholtz 512^2 with the learned indicator;
GLM-MHD Orszag-Tang in FP64 and FP32 and with the stage-wise non-conservative
interface flux; the 1D density wave; cRKFR against the standard multi-stage
RKFR step; the Kelvin-Helmholtz and Richtmyer-Meshkov robustness runs), each
throughput variant with its relative L2 error against the FP64 CPU oracle
stepped from the same initial state.
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

# Counter figures (HBM bytes from FETCH_SIZE/WRITE_SIZE, executed FLOPs from
# SQ_INSTS_VALU_FLOPS_FP64/FP32) are not measured by this script: they come
# from the rocprofv3 summaries under profiles/, each of which carries one
# machine-readable "counters:" line per profiled workload and the digest of
# the kernel sources it was taken with.  A figure is used only when that
# digest matches the sources of this checkout; otherwise it is null.
KERNEL_SOURCES = ("paper_2604_02125_amd/csrc/crk_kernels.hpp", "paper_2604_02125_amd/csrc/crk_physics.hpp")


def profiled_counters(workload: str):
    """The counters line of profiles/*.md for `workload` taken with the
    current kernel sources, or None."""
    import glob
    dig = sources_digest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(f) as fh:
            for line in fh:
                if line.startswith("counters: "):
                    rec = json.loads(line[len("counters: "):])
                    if rec.get("workload") == workload and rec.get("sources_sha256") == dig:
                        rec["profile"] = os.path.relpath(f, ROOT)
                        return rec
    return None


# Formula (algorithmic) FLOPs of the local-stage kernel per DOF-update:
# add/mul/div = 1, FMA = 2, log/sqrt = 1, each unordered node pair counted
# once.  Per stage and node: dim*N/2 unordered pairs (two-point flux plus
# accumulation into the M residual components), the per-node fields, and
# the stage update (4 M).  The executed count is higher (reciprocal and log
# sequences, mirrored pairs); the counters give that one.
PAIR_FLOPS = {0: 24, 1: 33, 2: 60, 3: 136}      # central, Kennedy-Gruber, Ranocha, Derigs MHD
NODE_FLOPS = {0: 20, 1: 10, 2: 12, 3: 183}


def k2_formula_flops_per_dof(flux: int, N: int, dim: int, stages: int, M: int) -> float:
    return stages * (dim * N / 2.0 * PAIR_FLOPS[flux] + NODE_FLOPS[flux] + 4 * M)


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
    """Algorithmic HBM bytes of the local-stage phase per DOF for the general
    trace design: read u^n, write the provisional state (M values per node),
    and per face node (2*dim faces of (N+1)^(dim-1) nodes per element) write
    three traces of M values (U, F and u^n), written once and read once by
    the interface phase.  For the KHI workload: 64 + 96 = 160 B/DOF."""
    npe = (N + 1) ** dim
    face_nodes = 2 * dim * (N + 1) ** (dim - 1)
    return elem * (2 * M + 3 * M * face_nodes / npe)


def k2_design_bytes_per_dof(M: int, dim: int, N: int, elem: int) -> float:
    """Algorithmic (unique) HBM bytes of this library's local-stage kernel per
    DOF: read u^n and write the provisional state (M values per node); per
    face node write the element's share of the interface flux (M values) and
    read one wave speed (each face node's two speeds are read by both
    elements of the face, so one value per element and face node is
    unique).  For the KHI workload: 104 B/DOF."""
    npe = (N + 1) ** dim
    face_nodes = 2 * dim * (N + 1) ** (dim - 1)
    return elem * (2 * M + (M + 1) * face_nodes / npe)


def step_bytes_per_dof(M: int, dim: int, N: int, elem: int) -> float:
    """Algorithmic HBM bytes of one whole step per DOF: state read and
    written once (2 M values per node) plus the three M-value traces of
    every face node written once and read once.  KHI: 64 + 192 = 256 B/DOF."""
    npe = (N + 1) ** dim
    face_nodes = 2 * dim * (N + 1) ** (dim - 1)
    return elem * (2 * M + 2 * 3 * M * face_nodes / npe)


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

    def step(self, events=None):
        """One pipelined step; with events (four torch.cuda.Event), record
        them around the local phase's two launches and the interface phase."""
        crk, L = self.crk, self.crk.lib()
        ui, uo = self.buf[self.n % 2], self.buf[(self.n + 1) % 2]
        p = crk._ptr
        h, a, b, d = self.s._h, p(ui), p(uo), p(self.dt)
        if events is None:
            crk._check(L.crk_advance(h, a, b, d, crk.PHASE_LOCAL, self.sp), "advance/local")
            crk._check(L.crk_advance(h, a, b, d, crk.PHASE_INTERFACE, self.sp), "advance/iface")
        else:
            events[0].record(self.stream)
            crk._check(L.crk_advance(h, a, b, d, crk.PHASE_LOCAL_PLAIN, self.sp), "advance/local plain")
            events[1].record(self.stream)
            crk._check(L.crk_advance(h, a, b, d, crk.PHASE_LOCAL_BLEND, self.sp), "advance/local blend")
            events[2].record(self.stream)
            crk._check(L.crk_advance(h, a, b, d, crk.PHASE_INTERFACE, self.sp), "advance/iface")
            events[3].record(self.stream)
        self.n += 1

    @property
    def state(self):
        return self.buf[self.n % 2]


def timed(pipe, steps, warmup, events=False, settle=0.3):
    """Wall time of `steps` pipelined steps (no events inside).  With events,
    the same steps are then run again from the initial state with HIP events
    on the launch stream between the launches of every step, which gives the
    average duration of the local phase's instance without the blending code
    (the dominant kernel: every tile of a state where no coefficient is
    positive), of the instance with it, and of the interface phase (its
    kernel and the dt slots kernel), in milliseconds."""
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
    if not events:
        return el, None
    n = pipe.n
    pipe.reset()
    for _ in range(warmup):
        pipe.step()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for k in range(steps):
        pipe.step(ev[k])
    torch.cuda.synchronize()
    assert pipe.n == n
    mean = lambda i, j: sum(e[i].elapsed_time(e[j]) for e in ev) / steps
    return el, {"k_local_plain_ms": mean(0, 1), "k_local_blend_ms": mean(1, 2), "interface_ms": mean(2, 3),
                "local_phase_ms": mean(0, 2)}


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


def kernel_report(workload, kt, ndof, M, dim, N, stages, flux, precision, ms_step):
    """Roofline figures of a single-mesh workload from the live kernel times
    kt (timed()): the dominant kernel is the local phase's instance without
    the blending code.  Bytes and FLOPs are algorithmic (per DOF x DOFs per
    launch) over that kernel's average duration; counter figures come from
    the profile summary taken with the same kernel sources (else null)."""
    elem = 8 if precision == "fp64" else 4
    # the instance that did the work: without tile flags (Ranocha, or no
    # limiter) one of the two launches is empty
    plain = kt["k_local_plain_ms"] >= kt["k_local_blend_ms"]
    t_ms = kt["k_local_plain_ms"] if plain else kt["k_local_blend_ms"]
    t = t_ms * 1e-3
    kb = k2_bytes_per_dof(M, dim, N, elem) * ndof
    db = k2_design_bytes_per_dof(M, dim, N, elem) * ndof
    sb = step_bytes_per_dof(M, dim, N, elem) * ndof
    ff = k2_formula_flops_per_dof(flux, N, dim, stages, M) * ndof
    peak_f = PEAK_FP64_TFLOPS if precision == "fp64" else PEAK_FP32_TFLOPS
    r = {"bound": "hbm",
         "kernel": "k_local (local stages, instance " + ("without" if plain else "with") + " the blending code)",
         "achieved": kb / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": kb / t / 1e9 / PEAK_HBM_GBS,
         "traffic": None, "kernel_ms": t_ms,
         "algorithmic_bytes_per_dof": kb / ndof, "algorithmic_bytes_per_launch": kb,
         # this library's own traces (flux shares instead of U, F and u^n)
         "design_bytes_per_dof": db / ndof, "design_frac": db / t / 1e9 / PEAK_HBM_GBS,
         "local_phase_ms": kt["local_phase_ms"],
         "other_instance_ms": kt["k_local_blend_ms"] if plain else kt["k_local_plain_ms"],
         "interface_ms": kt["interface_ms"],
         # the whole step against its own algorithmic bytes
         "step_bytes_per_dof": sb / ndof, "step_achieved_gbs": sb / (ms_step * 1e-3) / 1e9,
         "step_frac": sb / (ms_step * 1e-3) / 1e9 / PEAK_HBM_GBS,
         "formula_flops_per_dof": ff / ndof, "formula_tflops": ff / t / 1e12, "vector_peak_tflops": peak_f,
         "formula_frac": ff / t / 1e12 / peak_f,
         "counter_tflops": None, "counter_frac": None, "counter_profile": None}
    rec = profiled_counters(workload)
    if rec is not None and rec.get("kernel_instance") != ("plain" if plain else "blend"):
        rec = None
    if rec is not None:
        r["traffic"] = rec["hbm_bytes"]
        fl = rec.get("fp64_flops" if precision == "fp64" else "fp32_flops")
        if fl is not None:
            r["counter_tflops"] = fl / t / 1e12
            r["counter_frac"] = r["counter_tflops"] / peak_f
        r["counter_profile"] = rec["profile"]
    return r


def variant_khi(crk, inputs, orc, n, precision, steps, warmup, err_steps, threads, learned=False, flux=None,
                rough=0.0, half=False, workload=None):
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
    el, kt = timed(pipe, steps, warmup, events=True)
    check_admissible(s, pipe.state, f"khi{n}")
    cons = conservation(pipe)
    M, E, NP = s.shape
    ndof = E * NP
    prec = "fp64" if precision == crk.FP64 else "fp32"
    out = {"value": ndof * steps / el, "unit": "DOF-updates/s", "ms_per_step": el / steps * 1e3, "steps": steps,
           "kernels_ms": kt}
    if workload is not None:
        out["roofline"] = kernel_report(workload, kt, ndof, M, 2, 3, 4, cfg["volume_flux"], prec, el / steps * 1e3)
    out["conservation"] = cons
    out["blended_element_fraction"] = float((s.indicator(pipe.state)[1] > 0).double().mean().item())
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
    out = {"value": b.ndof / (ms * 1e-3), "unit": "DOF-updates/s", "ms_per_step": ms, "steps": 2 * reps,
           "problems": len(specs), "dofs": b.ndof, "tuning": {"block": b.tuning[0], "grid_per_cu": b.tuning[1], "merged": b.tuning[2]},
           "graph": "2 pipelined steps per replay"}
    if err_sample:
        out.update({"l2_rel_error_vs_fp64_oracle": float(np.sqrt(num / den)),
                    "linf_rel_error_vs_fp64_oracle": dmax / rmax,
                    "error_after_steps": 2, "error_sample": f"first {err_sample} problems"})
    return out


def variant_mhd(crk, inputs, orc, precision, steps, warmup, threads):
    n = 192
    s = crk.Solver(dim=2, nx=n, ny=n, degree=4, equation=crk.CRK_GLM_MHD, gamma=5.0 / 3.0, precision=precision,
                   volume_flux=crk.VOL_DERIGS, cfl=0.4)
    xi, _, _ = crk.reference_element(4)
    u0 = inputs.orszag_tang(n, n, xi)
    pipe = Pipelined(s, u0)
    el, kt = timed(pipe, steps, warmup, events=True)
    check_admissible(s, pipe.state, "mhd")
    cons = conservation(pipe)
    p = orc.Problem(dim=2, nx=n, ny=n, N=4, eq=orc.MHD, gamma=5.0 / 3.0, vol_flux=orc.VOL_DERIGS, nthreads=threads)
    oxi, _ = orc.gll(4)
    ref = oracle_steps(p, inputs.orszag_tang(n, n, oxi), 1)
    got1 = gpu_steps(s, u0, 1)
    M, E, NP = s.shape
    ndof = E * NP
    prec = "fp64" if precision == crk.FP64 else "fp32"
    rl = kernel_report(f"mhd_ot192_{prec}", kt, ndof, M, 2, 4, 6, crk.VOL_DERIGS, prec, el / steps * 1e3)
    # by the formula counts this kernel is balanced between FP64 issue and HBM
    rl["bound"] = "balanced (vector FLOPs and HBM)"
    return {"value": ndof * steps / el, "unit": "DOF-updates/s", "ms_per_step": el / steps * 1e3, "steps": steps,
            "kernels_ms": kt, "roofline": rl,
            "l2_rel_error_vs_fp64_oracle": rel_l2(got1, ref), "linf_rel_error_vs_fp64_oracle": rel_linf(got1, ref),
            "error_after_steps": 1, "conservation": cons}


def variant_mhd_stagewise(crk, inputs, steps, warmup, compare_steps=100):
    """Orszag-Tang 192^2 FP64 with the stage-wise non-conservative interface
    flux of eq:bad.numflux.non.cons against the reduced form the paper uses:
    throughput, the extra face-node data per step, and how far the two
    trajectories are apart after compare_steps steps from the same start."""
    import numpy as np
    n = 192
    mk = lambda nc: crk.Solver(dim=2, nx=n, ny=n, degree=4, equation=crk.CRK_GLM_MHD, gamma=5.0 / 3.0,
                               precision=crk.FP64, volume_flux=crk.VOL_DERIGS, cfl=0.4, nc_interface=nc)
    xi, _, _ = crk.reference_element(4)
    u0 = inputs.orszag_tang(n, n, xi)
    s = mk(crk.NC_STAGEWISE)
    pipe = Pipelined(s, u0)
    el, kt = timed(pipe, steps, warmup, events=True)
    check_admissible(s, pipe.state, "mhd stage-wise")
    M, E, NP = s.shape
    ndof = E * NP
    S = 6
    face_nodes_per_dof = 2 * 2 * (4 + 1) / NP
    a = gpu_steps(s, u0, compare_steps)
    b = gpu_steps(mk(crk.NC_REDUCED), u0, compare_steps)
    return {"value": ndof * steps / el, "unit": "DOF-updates/s", "ms_per_step": el / steps * 1e3, "steps": steps,
            "kernels_ms": kt, "interface_exchanges_per_step": 1,
            # per face node: every stage's state written once and read once
            # (the own side reads all of it, the neighbour B_d and psi of it),
            # against the reduced form's time-averaged B_d and psi
            "extra_face_bytes_per_dof": face_nodes_per_dof * 8.0 * (2 * S * M - 2 * 2),
            "face_values_exchanged_per_face_node": {"stagewise": 2 * S, "reduced": 2},
            "rel_l2_difference_from_reduced_form": rel_l2(a, b),
            "rel_linf_difference_from_reduced_form": rel_linf(a, b),
            "after_steps": compare_steps}


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


def variant_rkfr(crk, inputs, orc, steps, warmup, threads, err=True):
    """cRKFR against the standard multi-stage RKFR step on the same mesh,
    fluxes and tableau (KHI 256^2, N=3, Kennedy-Gruber, RK4, no limiter):
    one interface exchange per step against one per stage."""
    import numpy as np
    import torch
    n = 256
    cfg = dict(KHI)
    cfg["limiter"] = 0
    s = crk.Solver(nx=n, ny=n, precision=crk.FP64, **cfg)
    xi, _, _ = crk.reference_element(3)
    u0 = inputs.kelvin_helmholtz(n, n, xi)
    M, E, NP = s.shape
    ndof = E * NP
    pipe = Pipelined(s, u0)
    el_c, kt = timed(pipe, steps, warmup, events=True)
    # RKFR: dt of the state, then the s stages, every step
    ug = torch.tensor(u0, device="cuda")
    buf, dt = [ug.clone(), s.new_state()], s.new_dt()
    for k in range(warmup):
        s.rkfr_step(buf[k % 2], buf[(k + 1) % 2], dt, compute_dt=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        s.rkfr_step(buf[(warmup + k) % 2], buf[(warmup + k + 1) % 2], dt, compute_dt=True)
    torch.cuda.synchronize()
    el_r = time.perf_counter() - t0
    check_admissible(s, buf[(warmup + steps) % 2], "rkfr")
    S = 4
    out = {"workload": "2D Euler Kelvin-Helmholtz 256x256, N=3, Kennedy-Gruber, RK4, Rusanov faces, no limiter, FP64",
           "crkfr": {"value": ndof * steps / el_c, "ms_per_step": el_c / steps * 1e3, "interface_exchanges_per_step": 1,
                     "algorithmic_bytes_per_dof": step_bytes_per_dof(M, 2, 3, 8), "kernels_ms": kt},
           "rkfr": {"value": ndof * steps / el_r, "ms_per_step": el_r / steps * 1e3, "interface_exchanges_per_step": S,
                    # per stage: stage state in, u^n in, next stage state and K_i out; last stage:
                    # stage state, u^n and K_0..K_2 in, u^{n+1} out; plus the dt pass over u^n
                    "algorithmic_bytes_per_dof": 8.0 * M * (4 * (S - 1) + (2 + S) + 1)},
           "steps": steps}
    out["crkfr_over_rkfr"] = out["crkfr"]["value"] / out["rkfr"]["value"]
    if err:
        p = orc.Problem(dim=2, nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=3, vol_flux=orc.VOL_KG,
                        nthreads=threads)
        oxi, _ = orc.gll(3)
        uo = inputs.kelvin_helmholtz(n, n, oxi)
        dto = orc.compute_dt(p, uo)
        ref = orc.rkfr_step(p, uo, dto)
        o1 = s.new_state()
        s.rkfr_step(ug, o1, torch.tensor([dto, 0.0], dtype=torch.float64, device="cuda"), compute_dt=False)
        got = o1.cpu().numpy()
        out["rkfr"]["l2_rel_error_vs_fp64_oracle"] = rel_l2(got, ref)
        out["rkfr"]["linf_rel_error_vs_fp64_oracle"] = rel_linf(got, ref)
        # one step of each scheme from the same state and dt: how far the
        # single-exchange scheme lands from the s-exchange one
        ref_c, _ = orc.crk_step(p, uo, dto)
        out["crkfr_vs_rkfr_one_step_rel_l2"] = rel_l2(ref_c, ref)
    return out


def variant_sizes(crk, inputs, sizes=(128, 256, 512, 1024, 2048)):
    """The headline workload's pipelined step against mesh size, FP64 and
    FP32 (run only when asked for by name: the 2048^2 meshes take a while)."""
    import torch
    xi, _, _ = crk.reference_element(3)
    rows = {}
    for prec in (crk.FP64, crk.FP32):
        for n in sizes:
            s = crk.Solver(nx=n, ny=n, precision=prec, **KHI)
            pipe = Pipelined(s, inputs.kelvin_helmholtz(n, n, xi))
            steps = max(10, min(200, int(200 * (256 / n) ** 2)))
            _, kt = timed(pipe, steps, 3, events=True)
            el = min(timed(pipe, steps, 2)[0] for _ in range(2))
            dofs = n * n * 16
            rows[f"{'fp64' if prec == crk.FP64 else 'fp32'}_{n}x{n}"] = {
                "value": dofs * steps / el, "unit": "DOF-updates/s", "ms_per_step": el / steps * 1e3,
                "k_local_plain_ms": kt["k_local_plain_ms"], "interface_ms": kt.get("interface_ms"),
                "state_bytes": 4 * dofs * (8 if prec == crk.FP64 else 4)}
            del pipe, s
            torch.cuda.empty_cache()
    return {"workload": "2D Euler Kelvin-Helmholtz, N=3, Kennedy-Gruber, blending, pipelined step", "sizes": rows}


def variant_crash_study(crk):
    """Section 4.2's robustness claim on the paper's own mesh: KHI 64^2, N=3,
    blending with alpha_max = 0.008, to t = 15, for the central (plain FR
    derivative), Kennedy-Gruber and Ranocha volume fluxes."""
    from paper_2604_02125_amd import robustness
    t0 = time.perf_counter()
    res = robustness.khi_crash_study()
    return {"workload": "2D Euler Kelvin-Helmholtz 64x64, N=3, rho = 1/4 + 3B/4, blending alpha_max=0.008, "
                        "CFL 0.4, to t=15",
            "runs": res, "wall_s": time.perf_counter() - t0,
            "paper_context": "paper (Section 4.2, unstated hardware): stable to t=15 with the EC or KEP flux, "
                             "crash at about t=4 without"}


def host_cpu():
    """Host CPU model and the logical CPU count of the machine."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(orc, inputs, threads, steps_all, steps_one):
    """The FP64 CPU oracle on the headline workload (KHI 256^2), timed on the
    host: `steps_all` full steps with OpenMP over elements on `threads`
    threads, and `steps_one` steps on one thread."""
    oxi, _ = orc.gll(3)
    u0 = inputs.kelvin_helmholtz(256, 256, oxi)
    ndof = 256 * 256 * 16
    rates = {}
    for nth, nsteps in ((threads, steps_all), (1, steps_one)):
        p = orc.Problem(dim=2, nx=256, ny=256, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=3, vol_flux=orc.VOL_KG,
                        limiter=orc.LIM_BLEND_MODAL, nthreads=nth)
        uc = u0
        c0 = time.perf_counter()
        for _ in range(nsteps):
            uc, _ = orc.crk_step(p, uc, orc.compute_dt(p, uc))
        rates[nth] = ndof * nsteps / (time.perf_counter() - c0)
    model, ncpu = host_cpu()
    return {"value": rates[threads], "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps_all} full steps of the headline workload (KHI 256x256, N=3, KG, blending; FP64 C "
                      f"oracle, OpenMP over elements on {threads} threads) and {steps_one} steps on one thread",
            "single_thread_value": rates[1], "host_cpu_model": model, "host_logical_cpus": ncpu,
            "threads_note": "threads = the host CPU share of one GPU (OMP_NUM_THREADS on the GPU host)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)   # the configuration's run length
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    # the blended variants launch the headline's local-stage kernels on the same
    # grid: profiler runs skip them so that per-kernel averages cover the headline
    ap.add_argument("--no-blended", action="store_true")
    ap.add_argument("--only", default=None, help="comma-separated variant names to run (profiling)")
    ap.add_argument("--sizes", default="128,256,512,1024,2048",
                    help="mesh sizes of the khi_size_sweep variant (comma-separated n for n x n)")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--cpu-steps-single", type=int, default=2)
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

    import oracle as orc
    from paper_2604_02125_amd import crk, inputs
    torch.cuda.set_device(0)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)

    # ------------------------------------------------------------ headline
    head = variant_khi(crk, inputs, orc, 256, crk.FP64, args.steps, args.warmup, 0, threads,
                       workload="khi256_fp64")
    value = head["value"]
    out = {
        "metric": "DOF-updates/s at 1 GPU",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic Kelvin-Helmholtz initial condition)",
        "config": {"workload": "2D Euler Kelvin-Helmholtz 256x256, N=3, Kennedy-Gruber, blending alpha_max=0.008",
                   "elements": 65536, "degree": 3, "dofs": 1048576, "precision": "fp64",
                   "parallelism": "single GPU"},
        # a DOF is a node; the same rate counted per conserved variable (x M = 4)
        "variable_dof_updates_per_s": value * 4,
        "roofline": head["roofline"],
        "kernels_ms": head["kernels_ms"],
        "conservation": head["conservation"],
        "blended_element_fraction": head["blended_element_fraction"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(orc, inputs, threads, args.cpu_steps, args.cpu_steps_single)
    if not args.no_variants:
        only = set(args.only.split(",")) if args.only else None
        want = lambda k: only is None or k in only
        v = {}
        if want("khi256_fp64_check"):
            v["khi256_fp64_check"] = variant_khi(crk, inputs, orc, 256, crk.FP64, 20, 2, args.err_steps, threads)
        if want("khi256_fp32"):
            v["khi256_fp32"] = variant_khi(crk, inputs, orc, 256, crk.FP32, 20, 2, args.err_steps, threads,
                                           workload="khi256_fp32")
        if want("khi256_ranocha_fp64"):
            # the same workload with the entropy-conservative Ranocha flux (log means)
            v["khi256_ranocha_fp64"] = variant_khi(crk, inputs, orc, 256, crk.FP64, 20, 2, args.err_steps, threads,
                                                   flux=crk.VOL_RANOCHA, workload="khi256_ranocha_fp64")
        if not args.no_blended:
            if want("khi256_blended_fp64"):
                v["khi256_blended_fp64"] = variant_khi(crk, inputs, orc, 256, crk.FP64, 20, 2, args.err_steps,
                                                       threads, rough=0.05)
            if want("khi256_half_blended_fp64"):
                v["khi256_half_blended_fp64"] = variant_khi(crk, inputs, orc, 256, crk.FP64, 20, 2, args.err_steps,
                                                            threads, rough=0.05, half=True)
        if want("batch512_fp64"):
            v["batch512_fp64"] = variant_batch(crk, inputs, orc, crk.FP64, 5)
        if want("batch512_fp32"):
            v["batch512_fp32"] = variant_batch(crk, inputs, orc, crk.FP32, 5)
        if want("khi512_learned_fp64"):
            v["khi512_learned_fp64"] = variant_khi(crk, inputs, orc, 512, crk.FP64, 10, 2, args.err_steps, threads,
                                                   learned=True)
        if want("mhd_ot192_fp64"):
            v["mhd_ot192_fp64"] = variant_mhd(crk, inputs, orc, crk.FP64, 10, 2, threads)
        if want("mhd_ot192_fp32"):
            v["mhd_ot192_fp32"] = variant_mhd(crk, inputs, orc, crk.FP32, 10, 2, threads)
        if want("density_wave_1d_fp64"):
            v["density_wave_1d_fp64"] = variant_wave1d(crk, inputs, orc)
        if want("mhd_ot192_stagewise_fp64"):
            v["mhd_ot192_stagewise_fp64"] = variant_mhd_stagewise(crk, inputs, 10, 2)
        if want("rmi_crash_study"):
            from paper_2604_02125_amd import robustness
            t0 = time.perf_counter()
            v["rmi_crash_study"] = {
                "workload": "2D Euler Richtmyer-Meshkov 32x96 on [0,40/3]x[0,40], N=3, reflective walls, blending "
                            "alpha_max=0.001, CFL 0.4, to t=30",
                "runs": robustness.rmi_crash_study(), "wall_s": None,
                "paper_context": "paper (Section 4.3, unstated hardware): stable to t=30 with the EC or KEP flux, "
                                 "crash at about t=8.7 without"}
            v["rmi_crash_study"]["wall_s"] = time.perf_counter() - t0
        if want("khi256_crkfr_vs_rkfr"):
            v["khi256_crkfr_vs_rkfr"] = variant_rkfr(crk, inputs, orc, 20, 2, threads, err=args.err_steps > 0)
        if want("khi64_crash_study"):
            v["khi64_crash_study"] = variant_crash_study(crk)
        if only is not None and "khi_size_sweep" in only:
            v["khi_size_sweep"] = variant_sizes(crk, inputs, tuple(int(x) for x in args.sizes.split(",")))
        v["_note"] = ("l2_rel_error_vs_fp64_oracle = ||u_gpu - u_oracle||_2 / ||u_oracle||_2 and "
                      "linf_rel_error_vs_fp64_oracle = max|u_gpu - u_oracle| / max|u_oracle| over all values "
                      "after error_after_steps steps from the same initial state (the FP64 rows are a "
                      "round-off check); roofline.achieved = algorithmic bytes per launch / the dominant "
                      "kernel's live duration (HIP events)")
        out["variants"] = v
    print(json.dumps(out))


if __name__ == "__main__":
    main()
