"""Autotuner of the batched path's tile shape.

For each precision and volume flux it builds the batch of 512 independent
periodic 2D Euler problems (sizes n ~ U{16..96}, degrees N in {3, 4}, seeded
random Fourier initial data), captures two pipelined steps into a HIP graph
for every candidate tile shape (lanes per workgroup 64/128/256 x persistent
workgroups per compute unit 0/1/2/4/8/16/32/64, 0 meaning one workgroup per
tile, x one launch per degree or one over both),
times graph replays with HIP events on the batch's stream, and writes the
fastest shape per (precision, flux) to tuning.json next to this file, which
crk.Batch reads by default.

    python -m paper_2604_02125_amd.autotune [--nprob 512] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

BLOCKS = (64, 128, 256)
# 0: one workgroup per tile; otherwise persistent workgroups per compute
# unit, up to the most that can be resident at once (64-lane workgroups of
# the degree-3 path fit 8 per SIMD)
GRID_PER_CU = (0, 1, 2, 4, 8, 16, 32, 64)
MERGED = (0, 1)   # one launch per degree and phase, or one over both degrees


def fill_batch(batch, seed_rng):
    import torch
    from paper_2604_02125_amd import crk, inputs
    for i, (n, N) in enumerate(batch.specs):
        xi, _, _ = crk.reference_element(N)
        batch.view(0, i).copy_(torch.tensor(inputs.random_fourier_state(seed_rng, n, xi), dtype=batch.dtype))


_initial = {}


def time_shape(specs, precision, flux, tuning, reps, seed=20260402):
    import torch
    from paper_2604_02125_amd import crk, inputs
    b = crk.Batch(specs, precision=precision, volume_flux=flux, tuning=tuning)
    key = (len(specs), seed, precision)
    if key not in _initial:
        # the flat initial state depends only on the problems, not on the
        # tile shape: sampled once per precision and reused
        _, rng = inputs.random_fourier_problems(len(specs), seed=seed)
        fill_batch(b, rng)
        _initial[key] = b.u[0].clone()
    else:
        b.u[0].copy_(_initial[key])
    torch.cuda.synchronize()
    with torch.cuda.stream(b.stream):
        b.prepare(0)
        b.capture_graph()
        b.launch_graph()                      # warm-up replay
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        for _ in range(reps):
            b.launch_graph()
        e1.record(b.stream)
    b.stream.synchronize()
    ms_per_step = e0.elapsed_time(e1) / (2 * reps)
    return ms_per_step, b.ndof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nprob", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    args = ap.parse_args()
    from paper_2604_02125_amd import crk, inputs
    specs, _ = inputs.random_fourier_problems(args.nprob, seed=20260402)
    result = {"workload": f"{args.nprob} periodic 2D Euler problems, n ~ U{{16..96}}, N in {{3,4}}, seed 20260402",
              "batch": {}}
    for prec, pname in ((crk.FP64, "fp64"), (crk.FP32, "fp32")):
        for flux, fname in ((crk.VOL_RANOCHA, "ranocha"), (crk.VOL_KG, "kg")):
            sweep = []
            for blk in BLOCKS:
                for gpc in GRID_PER_CU:
                    for mg in MERGED:
                        t0 = time.time()
                        ms, ndof = time_shape(specs, prec, flux, (blk, gpc, mg), args.reps)
                        sweep.append({"block": blk, "grid_per_cu": gpc, "merged": mg, "ms_per_step": ms,
                                      "dof_updates_per_s": ndof / (ms * 1e-3)})
                        print(f"{pname}/{fname} block={blk} grid_per_cu={gpc} merged={mg}: {ms:.3f} ms/step "
                              f"({ndof / (ms * 1e-3):.3e} DOF/s) [{time.time() - t0:.1f}s]", flush=True)
            best = min(sweep, key=lambda r: r["ms_per_step"])
            result["batch"][f"{pname}/{fname}"] = dict(best, sweep=sweep)
    with open(args.out, "w") as fh:
        json.dump(result, fh, indent=1)
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
