"""Training and evaluation of the learned troubled-cell indicator.

Snapshots come from the method itself: Kelvin-Helmholtz runs (2D Euler,
128 x 128 elements, N = 3, Kennedy-Gruber volume flux, blending with the
modal indicator, alpha_max = 0.008) whose v2 perturbation is a seeded sum of
four modes, taken once the instability has developed (t = 1, 1.5, ..., 3;
before t ~ 1 the flow is smooth and no element is troubled).  Each element
contributes its 16 modal energy fractions of rho*p (features) and the
a-posteriori label of the unlimited (alpha = 0) update from that state
(crk_labels) with a relative tolerance of 1e-5: at 1e-3 almost no element
of these runs is troubled (a few in a million), at 1e-5 about 1-2 % are,
while the modal indicator blends in 3-16 % of them.  The network is trained with the
library's gradient and Adam kernels on binary cross-entropy; the weights and
the feature range of the training set are written to mlp_indicator.npz.

    python -m paper_2604_02125_amd.learned train [--seeds 16] [--n 128]
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
WEIGHTS = os.path.join(HERE, "mlp_indicator.npz")


def khi_solver(n, limiter=True, precision=None):
    from paper_2604_02125_amd import crk
    return crk.Solver(dim=2, nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, degree=3, volume_flux=crk.VOL_KG,
                      limiter=crk.LIM_BLEND if limiter else crk.LIM_NONE, alpha_max=0.008, alpha_min=1e-3,
                      precision=crk.FP64 if precision is None else precision)


def generate(seeds, n=128, t_snaps=(1.0, 1.5, 2.0, 2.5, 3.0), frac=1.0, sample_seed=7, tol=1e-5, log=print):
    """Features X [m, 16] and labels Y [m] (float32, on the GPU) from the
    snapshots of Kelvin-Helmholtz runs at the times t_snaps."""
    import numpy as np
    import torch

    from paper_2604_02125_amd import crk, inputs
    s = khi_solver(n)
    xi, _, _ = crk.reference_element(3)
    zero_alpha = torch.zeros(s.nelem, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(sample_seed)
    X, Y = [], []
    for seed in seeds:
        t0 = time.time()
        u = [torch.tensor(inputs.kelvin_helmholtz(n, n, xi, v2_modes=inputs.khi_modes(seed)), device="cuda"),
             s.new_state()]
        uh = s.new_state()
        dt, dt_h = s.new_dt(), s.new_dt()
        s.prepare(u[0], dt)
        t, k, nsnap = 0.0, 0, 0
        for ts in t_snaps:
            while t < ts:
                t += dt[0].item()
                s.advance(u[k % 2], u[(k + 1) % 2], dt)
                k += 1
            cur = u[k % 2]
            f = crk.features(s, cur)
            s.step(cur, uh, dt_h, alpha=zero_alpha, compute_dt=True)
            lab = crk.labels(s, cur, uh, tol=tol)
            s.prepare(cur, dt)              # the full step used the pipeline's workspace
            keep = torch.tensor(rng.permutation(s.nelem)[: int(frac * s.nelem)], device="cuda")
            X.append(f[keep])
            Y.append(lab[keep])
            nsnap += 1
        torch.cuda.synchronize()
        d = s.diagnostics(u[k % 2]).cpu().numpy()
        log(f"seed {seed}: {k} steps to t={t:.3f} in {time.time() - t0:.2f}s, min p {d[6]:.3e}, "
            f"troubled fraction at snapshots {torch.cat(Y[-nsnap:]).mean().item():.4f}")
    return torch.cat(X), torch.cat(Y)


def train(X, Y, epochs=8, batch=8192, lr=2e-3, seed=0, log=print):
    """Adam on binary cross-entropy with class-balanced minibatches (half
    troubled, half untroubled samples, drawn with replacement), since only
    about 1 % of the elements are troubled."""
    import torch

    from paper_2604_02125_amd import crk
    lo = X.min(0).values.cpu().numpy()
    hi = X.max(0).values.cpu().numpy()
    net = crk.MLP(seed=seed, lo=lo, hi=hi)
    pos = torch.nonzero(Y > 0.5).flatten()
    neg = torch.nonzero(Y <= 0.5).flatten()
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps = max(1, epochs * X.shape[0] // batch)
    ws = None
    tot, nb = 0.0, 0
    for it in range(steps):
        ip = pos[torch.randint(len(pos), (batch // 2,), generator=g).to(pos.device)]
        ineg = neg[torch.randint(len(neg), (batch - batch // 2,), generator=g).to(neg.device)]
        idx = torch.cat([ip, ineg])
        loss, grad, ws = net.loss_grad(X[idx].contiguous(), Y[idx].contiguous(), ws)
        net.adam(grad, lr=lr)
        if it % 32 == 0:
            tot += loss.item()
            nb += 1
        if (it + 1) % (steps // epochs) == 0:
            log(f"step {it + 1}/{steps}: mean sampled balanced loss {tot / max(nb, 1):.5f}")
            tot, nb = 0.0, 0
    # balanced batches estimate the odds under a 50 % prior; shifting the
    # output bias by the log prior odds of the data gives calibrated
    # probabilities, so alpha = alpha_max P(troubled)
    prior = float(Y.mean())
    net.theta[-1] += math.log(prior / (1.0 - prior))
    net.sync_bf16()
    return net


def confusion(net, X, Y, alpha_max=0.008, alpha_min=1e-3):
    """Agreement of the network's alpha > 0 with the labels."""
    z, a = net.forward(X, alpha_max)
    pred = (a >= alpha_min).float()
    tp = float(((pred == 1) & (Y == 1)).sum())
    tn = float(((pred == 0) & (Y == 0)).sum())
    fp = float(((pred == 1) & (Y == 0)).sum())
    fn = float(((pred == 0) & (Y == 1)).sum())
    return {"tp": tp, "tn": tn, "fp": fp, "fn": fn, "accuracy": (tp + tn) / max(tp + tn + fp + fn, 1.0)}


def held_out(net, seeds=(101, 102), n=128, t_snaps=(1.5, 2.5), tol=1e-5):
    """The troubled-cell labels of snapshots from runs the network was not
    trained on (seeds outside 1..16) against the raw blending coefficients of
    the network and of the modal indicator on the same states: per
    indicator, how many labelled elements it flags (tp), misses (fn), and
    how many unlabelled ones it flags (fp)."""
    import numpy as np
    import torch

    from paper_2604_02125_amd import crk, inputs
    s = khi_solver(n)
    sn = khi_solver(n)
    net.bind(sn)
    xi, _, _ = crk.reference_element(3)
    zero_alpha = torch.zeros(s.nelem, dtype=torch.float64, device="cuda")
    stats = {k: {"tp": 0, "fn": 0, "fp": 0, "tn": 0} for k in ("network", "modal")}
    for seed in seeds:
        u = [torch.tensor(inputs.kelvin_helmholtz(n, n, xi, v2_modes=inputs.khi_modes(seed)), device="cuda"),
             s.new_state()]
        uh = s.new_state()
        dt, dt_h = s.new_dt(), s.new_dt()
        s.prepare(u[0], dt)
        t, k = 0.0, 0
        for ts in t_snaps:
            while t < ts:
                t += dt[0].item()
                s.advance(u[k % 2], u[(k + 1) % 2], dt)
                k += 1
            cur = u[k % 2]
            s.step(cur, uh, dt_h, alpha=zero_alpha, compute_dt=True)
            lab = crk.labels(s, cur, uh, tol=tol).cpu().numpy() > 0.5
            s.prepare(cur, dt)
            for name, solver in (("network", sn), ("modal", s)):
                pred = solver.indicator(cur)[0].cpu().numpy() > 0.0
                st = stats[name]
                st["tp"] += int(np.sum(pred & lab))
                st["fn"] += int(np.sum(~pred & lab))
                st["fp"] += int(np.sum(pred & ~lab))
                st["tn"] += int(np.sum(~pred & ~lab))
            s.prepare(cur, dt)
    for st in stats.values():
        st["miss_rate"] = st["fn"] / max(st["tp"] + st["fn"], 1)
        st["flagged_fraction"] = (st["tp"] + st["fp"]) / max(sum(st[k] for k in ("tp", "fn", "fp", "tn")), 1)
    return stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--seeds", type=int, default=16)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    import torch
    t0 = time.time()
    X, Y = generate(range(1, args.seeds + 1), n=args.n, tol=args.tol)
    print(f"dataset: {X.shape[0]} samples, troubled fraction {Y.mean().item():.4f} ({time.time() - t0:.1f}s)",
          flush=True)
    net = train(X, Y, epochs=args.epochs)
    torch.cuda.synchronize()
    print("confusion on the training set (network alpha > 0 vs label):", confusion(net, X, Y), flush=True)
    net.save(args.out)
    print(f"wrote {args.out} ({time.time() - t0:.1f}s total)")


if __name__ == "__main__":
    main()
