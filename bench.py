"""Throughput benchmark of the cRKFR hot path on one MI355X.

Workload (default): 2D compressible Euler, Kelvin-Helmholtz initial data on
[-1,1]^2 periodic, 256 x 256 elements, degree N = 3 on Gauss-Lobatto nodes
(1,048,576 nodal DOFs), Kennedy-Gruber volume flux, Rusanov interfaces,
classical RK4 inner stages, CFL 0.4, subcell-FV blending limiter with
alpha_max = 0.008, FP64.  One step = CFL time step reduction + blending
indicator + local stages + interface exchange and final update, with the
state resident in HBM; the time-step reduction and the indicator of the
new state run inside the interface phase (pipelined step).  Metric: DOF-updates/s (one DOF = one solution node).

Prints one JSON line.  ``--gpus`` above 1 is rejected: this build runs on a
single GPU.
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

# HBM bytes per launch of k_local measured by rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE, scaled by the plain-copy calibration (read x2.0, write x1.0);
# valid only for the kernel sources whose digest is recorded with it.
MEASURED_TRAFFIC = {
    ("khi256", "fp64"): {"sources_sha256": "e9752acc560995176e5fd6f9f738a68afc7257adb1bf16f0633f4e15363ca0f9",
                         "bytes": (2.0 * 17253.9 + 1.0 * 98816.1) * 1024},
}
KERNEL_SOURCES = ("paper_2604_02125_amd/csrc/crk_kernels.hpp", "paper_2604_02125_amd/csrc/crk_physics.hpp")


def sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


WORKLOADS = {
    "khi256": dict(nx=256, ny=256, degree=3, flux=1, limiter=1,
                   desc="2D Euler Kelvin-Helmholtz 256x256, N=3, Kennedy-Gruber, blending alpha_max=0.008"),
    "khi512": dict(nx=512, ny=512, degree=3, flux=1, limiter=1,
                   desc="2D Euler Kelvin-Helmholtz 512x512, N=3, Kennedy-Gruber, blending alpha_max=0.008"),
}


def k2_bytes_per_dof(M: int, dim: int, N: int, elem: int) -> float:
    """Algorithmic HBM bytes of the local-stage kernel per DOF: read u^n, write
    the provisional state, write the face traces (U, F: 2M values per face
    node, 2*dim faces of (N+1)^(dim-1) nodes per element)."""
    npe = (N + 1) ** dim
    traces = 2 * dim * (N + 1) ** (dim - 1) * 2 * M
    return elem * (2 * M + traces / npe)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="khi256", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (no multi-GPU path in this build); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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

    w = WORKLOADS[args.workload]
    prec = crk.FP64 if args.precision == "fp64" else crk.FP32
    elem = 8 if prec == crk.FP64 else 4
    torch.cuda.set_device(0)
    s = crk.Solver(dim=2, nx=w["nx"], ny=w["ny"], x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, degree=w["degree"],
                   precision=prec, volume_flux=w["flux"], cfl=0.4, limiter=w["limiter"], alpha_max=0.008,
                   alpha_min=1e-3)
    xi, _, _ = crk.reference_element(w["degree"])
    u0 = inputs.kelvin_helmholtz(w["nx"], w["ny"], xi)
    M, E, NP = s.shape
    ndof = E * NP
    buf = [torch.tensor(u0, dtype=s.dtype, device="cuda"), s.new_state()]
    dt = s.new_dt()
    stream = torch.cuda.current_stream()
    L = crk.lib()
    h = s._h
    ptr = crk._ptr
    sp = crk._stream(stream)

    def step(n, ev=None):
        # pipelined step: dt and the blending indicator of the new state are
        # computed by the interface phase (crk_prepare seeded them for u0)
        ui, uo = buf[n % 2], buf[(n + 1) % 2]
        if ev is not None:
            ev[0].record(stream)
        crk._check(L.crk_advance(h, ptr(ui), ptr(uo), ptr(dt), crk.PHASE_LOCAL, sp), "advance/local")
        if ev is not None:
            ev[1].record(stream)
        crk._check(L.crk_advance(h, ptr(ui), ptr(uo), ptr(dt), crk.PHASE_INTERFACE, sp), "advance/interface")

    crk._check(L.crk_prepare(h, ptr(buf[0]), ptr(dt), sp), "prepare")
    for n in range(args.warmup):
        step(n)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for n in range(args.steps):
        step(args.warmup + n, evs[n])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    k2_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    diag = s.diagnostics(buf[(args.warmup + args.steps) % 2]).cpu().numpy()
    if not np.isfinite(diag).all() or diag[M + 4] >= 0:
        print("bench: non-physical state after the timed steps", file=sys.stderr)
        sys.exit(3)

    value = ndof * args.steps / elapsed
    kb = k2_bytes_per_dof(M, 2, w["degree"], elem) * ndof
    achieved = kb / (k2_ms * 1e-3) / 1e9
    rec = MEASURED_TRAFFIC.get((args.workload, args.precision))
    traffic = rec["bytes"] if rec and rec["sources_sha256"] == sources_digest() else None
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
        "dtype": "f64" if prec == crk.FP64 else "f32",
        "data": "synthetic (analytic Kelvin-Helmholtz initial condition)",
        "config": {"workload": w["desc"], "elements": E, "degree": w["degree"], "dofs": ndof,
                   "precision": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "k_local (local stages)", "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "kernel_ms": k2_ms,
                     "algorithmic_bytes_per_launch": kb},
    }
    if not args.no_cpu_baseline:
        import oracle as orc
        nthreads = min(16, os.cpu_count() or 1)
        p = orc.Problem(dim=2, nx=w["nx"], ny=w["ny"], x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, N=w["degree"],
                        vol_flux=w["flux"], limiter=orc.LIM_BLEND_MODAL if w["limiter"] else 0, nthreads=nthreads)
        oxi, _ = orc.gll(w["degree"])
        uc = inputs.kelvin_helmholtz(w["nx"], w["ny"], oxi)
        c0 = time.perf_counter()
        for _ in range(args.cpu_steps):
            uc, _ = orc.crk_step(p, uc, orc.compute_dt(p, uc))
        c1 = time.perf_counter()
        out["cpu_baseline"] = {"value": ndof * args.cpu_steps / (c1 - c0), "unit": "DOF-updates/s",
                               "cores": nthreads, "kind": "oracle",
                               "sample": f"{args.cpu_steps} full steps of the same workload (FP64 C oracle, "
                                         f"OpenMP over elements, {nthreads} threads)"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
