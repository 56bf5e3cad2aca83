"""Training set and GPU training loop of the sketch-rank predictor.

One sample is a pair of neighbouring updates of a sweep: the input is the
feature row of the previous bond's kept spectrum (computed on the GPU by
``tci_sketch_features``), the target is log2 chi*(eps) of the current bond,
where chi* is the bond dimension that the truncation rule keeps when it is
not capped.  The network predicts the 0.9-quantile of that target (pinball
loss), and the library turns a prediction y into the sketch rank
k = 32 ceil((1.5 2^y + 32) / 32), or into the plain truncated SVD when
y > log2 chi_max or k > n / 4.

Spectra of three families, each with a drifting parameter along a sweep of
``length`` bonds (n singular values, normalised to unit 2-norm):
  * power law   s_k ~ k^-alpha,  alpha ~ U[a_lo, a_hi], drift N(0, 0.05^2),
    clipped to [a_lo, a_hi] (the learned-sketch workload uses alpha in [1, 3]);
  * exponential s_k ~ exp(-k / kappa), log10 kappa ~ U[1, 3.5], drift N(0, 0.05^2);
  * quarter circle: singular values of a square Gaussian matrix (the dense
    workload with Gaussian site tensors), whose empirical distribution
    follows the density sqrt(4 - x^2) / pi on [0, 2]; no drift.
The spectra are the exact singular values of the matrices these workloads
build (theta = U diag(s) V^T with orthogonal U, V); a GPU test checks the
library's truncated SVD against them.

Spectra from the method's own updates (``make_update_pairs``): the library
runs two-site updates at chi = 1024, d = 2 whose input bond carries a known
spectrum (A = U diag(s), B = V^dagger with Haar isometries U, V drawn from a
pool, s a power law with alpha ~ U[1, 3] or an exponential decay), followed by
a Haar-random two-site gate; the input is the features of s (the bond's
spectrum before the update) and the target is log2 of the bond dimension the
truncation rule keeps for eps at the cap chi_max = chi: below the cap that
is chi* itself; where the cap binds (eps missed at chi) the target is
log2(d chi), a value beyond the cap, so that the network learns to send
such bonds to the plain SVD (its rank would exceed n / 4 either way).  The
gate spreads the spectrum, so chi* after the update is two to four times the
chi* of s; this is the workload of the two-site update benchmark.

The shipped weights are trained on 50k pairs: 8192 from the library's
updates and the rest from the closed-form sweeps above.

Training: Adam (lr 1e-3), batch 256, 30 epochs, 90/10 train/validation
split, all on the GPU through ``tci_sketch_train_step`` (hand-written
forward, backward and Adam kernels).
"""
from __future__ import annotations

import argparse
import math
import os

import numpy as np

from . import tci

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sketch_mlp.bin")


def power_law(n: int, alpha: float) -> np.ndarray:
    s = np.arange(1, n + 1, dtype=np.float64) ** (-alpha)
    return s / np.linalg.norm(s)


def exp_decay(n: int, kappa: float) -> np.ndarray:
    s = np.exp(-np.arange(n, dtype=np.float64) / kappa)
    return s / np.linalg.norm(s)


def quarter_circle(n: int) -> np.ndarray:
    """Descending quantiles x_j = F^-1(1 - (j + 1/2) / n) of the density
    sqrt(4 - x^2) / pi on [0, 2], with F(x) = (x sqrt(4 - x^2) / 2 + 2 asin(x / 2)) / pi
    inverted by bisection."""
    p = 1.0 - (np.arange(n, dtype=np.float64) + 0.5) / n
    lo, hi = np.zeros(n), np.full(n, 2.0)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        f = (mid * np.sqrt(np.maximum(4.0 - mid * mid, 0.0)) / 2.0 + 2.0 * np.arcsin(mid / 2.0)) / math.pi
        below = f < p
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    s = 0.5 * (lo + hi)
    return s / np.linalg.norm(s)


def chi_star(s: np.ndarray, eps: float) -> int:
    """Smallest chi >= 1 with sum_{k >= chi} s_k^2 <= eps * sum s_k^2 (no cap)."""
    w = s * s
    tail = np.concatenate([np.cumsum(w[::-1])[::-1], [0.0]])
    ok = np.nonzero(tail[1:] <= eps * tail[0])[0]
    return int(ok[0]) + 1 if len(ok) else len(s)


def sweep_spectra(rng: np.random.Generator, family: str, n: int, length: int, alpha_range=(1.0, 3.0)):
    if family == "power":
        lo, hi = alpha_range
        a = rng.uniform(lo, hi)
        out = []
        for _ in range(length):
            out.append(power_law(n, a))
            a = float(np.clip(a + rng.normal(0.0, 0.05), lo, hi))
        return out
    if family == "exp":
        lk = rng.uniform(1.0, 3.5)
        out = []
        for _ in range(length):
            out.append(exp_decay(n, 10.0 ** lk))
            lk = float(np.clip(lk + rng.normal(0.0, 0.05), 1.0, 3.5))
        return out
    if family == "qc":
        return [quarter_circle(n)] * length
    raise ValueError(family)


def make_pairs(n_samples: int, seed: int, n: int = 2048, chi_max: int = 1024, eps: float = 1e-8,
               mix=(0.8, 0.15, 0.05), length: int = 8, alpha_range=(1.0, 3.0)):
    """Returns (prev kept spectra list, targets log2 chi*) for n_samples pairs."""
    rng = np.random.default_rng(seed)
    fams = ["power", "exp", "qc"]
    prev, targ = [], []
    qc_cache = None
    while len(prev) < n_samples:
        fam = fams[rng.choice(3, p=np.asarray(mix) / np.sum(mix))]
        if fam == "qc":
            if qc_cache is None:
                qc_cache = sweep_spectra(rng, "qc", n, length)
            seq = qc_cache
        else:
            seq = sweep_spectra(rng, fam, n, length, alpha_range)
        chis = [chi_star(s, eps) for s in seq]
        for t in range(1, length):
            if len(prev) >= n_samples:
                break
            keep = min(chis[t - 1], chi_max)
            sp = seq[t - 1][:keep]
            prev.append(sp / np.linalg.norm(sp))
            targ.append(math.log2(chis[t]))
    return prev, np.asarray(targ)


def update_input(rng: np.random.Generator, chi: int, alpha_range=(1.0, 3.0), exp_frac: float = 0.2) -> np.ndarray:
    """Spectrum of the input bond of one sampled update (unit 2-norm)."""
    if rng.random() < exp_frac:
        return exp_decay(chi, 10.0 ** rng.uniform(1.0, 3.0))
    return power_law(chi, rng.uniform(*alpha_range))


def make_update_pairs(ctx, n_samples: int, seed: int, chi: int = 1024, d: int = 2, eps: float = 1e-8,
                      batch: int = 32, pool: int = 8, alpha_range=(1.0, 3.0), exp_frac: float = 0.2,
                      log=None):
    """(input spectra, targets log2 chi*) from the library's own two-site
    updates: A = U diag(s) (chi, d, chi), B = V^dagger (chi, d, chi), a Haar
    gate, complex64 storage with split-BF16x3 products and the plain FP64
    truncated SVD at eps with chi_max = chi: info.chi = chi* below the cap,
    and the target is log2(chi d) where the cap binds.  U, V come from a
    pool of `pool` Haar isometries each (generated on the host), combined at
    random per update."""
    import torch
    from . import synth
    rng = np.random.default_rng(seed)
    dev = ctx.torch_device
    us = [torch.from_numpy(synth.haar(rng, chi * d, chi)).to(dev, torch.complex64) for _ in range(pool)]
    vhs = [torch.from_numpy(synth.haar(rng, d * chi, chi).conj().T.copy()).to(dev, torch.complex64)
           for _ in range(pool)]
    p = tci.update_params(chi_min=1, chi_max=chi, target_trunc_err=eps, direction=tci.DIR_RIGHT,
                          precision=tci.PREC_BF16X3)
    prev, targ = [], []
    while len(targ) < n_samples:
        nb = min(batch, n_samples - len(targ))
        A, B, G, sp = [], [], [], []
        for _ in range(nb):
            s = update_input(rng, chi, alpha_range, exp_frac)
            i, j = rng.integers(pool, size=2)
            sd = torch.as_tensor(s, dtype=torch.float32, device=dev)
            A.append(tci.Tensor(ctx, (us[i] * sd[None, :]).contiguous(), (chi, d, chi)))
            B.append(tci.Tensor(ctx, vhs[j], (chi, d, chi)))
            G.append(tci.Tensor.from_numpy(ctx, synth.haar_gate(rng).astype(np.complex64), tci.C64))
            sp.append(s)
        _, _, _, infos = tci.two_site_update_batched(ctx, A, B, G, p)
        for s, inf in zip(sp, infos):
            prev.append(s)
            capped = inf.chi >= chi and inf.trunc_err > eps
            targ.append(math.log2(chi * d) if capped else math.log2(inf.chi))
        if log is not None:
            log(f"  update pairs {len(targ)}/{n_samples}")
    return prev, np.asarray(targ)


def features(ctx, spectra, chi_max: int, d: int, eps: float, chunk: int = 2048):
    import torch
    rows = [tci.sketch_features(ctx, spectra[i:i + chunk], chi_max, d, eps) for i in range(0, len(spectra), chunk)]
    return torch.cat(rows, 0)


def make_dataset(ctx, n_samples: int, seed: int, n: int = 2048, chi_max: int = 1024, d: int = 2, eps: float = 1e-8,
                 **kw):
    import torch
    prev, targ = make_pairs(n_samples, seed, n, chi_max, eps, **kw)
    X = features(ctx, prev, chi_max, d, eps)
    T = torch.as_tensor(targ, dtype=torch.float32, device=ctx.torch_device)
    return X, T


def pinball(y, t, tau: float = 0.9) -> float:
    import torch
    u = t.double() - y.double()
    return float(torch.maximum(tau * u, (tau - 1.0) * u).mean())


def train(ctx, X, T, epochs: int = 30, batch: int = 256, lr: float = 1e-3, seed: int = 0, val_frac: float = 0.1,
          model=None):
    """Trains on the GPU; returns (model, history) with per-epoch mean train
    loss and validation pinball loss."""
    import torch
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    nval = int(round(val_frac * X.shape[0]))
    perm = torch.randperm(X.shape[0], generator=g).to(X.device)
    Xv, Tv = X[perm[:nval]].contiguous(), T[perm[:nval]].contiguous()
    Xt, Tt = X[perm[nval:]].contiguous(), T[perm[nval:]].contiguous()
    m = model if model is not None else tci.SketchModel(ctx, seed=seed)
    hist = {"train": [], "val": []}
    for _ in range(epochs):
        order = torch.randperm(Xt.shape[0], generator=g).to(X.device)
        tot, cnt = 0.0, 0
        for i in range(0, Xt.shape[0] - batch + 1, batch):
            idx = order[i:i + batch]
            xb, tb = Xt[idx].contiguous(), Tt[idx].contiguous()
            tot += m.train_step(xb, tb, lr)
            cnt += 1
        hist["train"].append(tot / max(cnt, 1))
        hist["val"].append(pinball(m.predict(Xv), Tv) if nval else float("nan"))
    return m, hist


def make_mixed_dataset(ctx, n_samples: int, n_updates: int, seed: int, chi_max: int = 1024, d: int = 2,
                       eps: float = 1e-8, log=None):
    """n_updates pairs from the library's updates plus closed-form sweep
    pairs up to n_samples; features on the GPU."""
    import torch
    prev_u, targ_u = make_update_pairs(ctx, n_updates, seed + 1, chi=chi_max, d=d, eps=eps, log=log)
    X_u = features(ctx, prev_u, chi_max, d, eps)
    X_c, T_c = make_dataset(ctx, n_samples - n_updates, seed, chi_max=chi_max, d=d, eps=eps)
    T_u = torch.as_tensor(targ_u, dtype=torch.float32, device=ctx.torch_device)
    return torch.cat([X_u, X_c], 0), torch.cat([T_u, T_c], 0)


def main(argv=None):
    ap = argparse.ArgumentParser(description="Train the sketch-rank predictor on the GPU")
    ap.add_argument("--samples", type=int, default=50000)
    ap.add_argument("--update-samples", type=int, default=8192,
                    help="pairs generated by the library's own two-site updates (the rest: closed-form sweeps)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    import time
    ctx = tci.Context(0)
    t0 = time.time()
    log = lambda m: print(m, flush=True)
    X, T = make_mixed_dataset(ctx, args.samples, args.update_samples, args.seed, log=log)
    log(f"dataset {X.shape[0]} pairs in {time.time() - t0:.1f}s")
    m, hist = train(ctx, X, T, epochs=args.epochs, seed=args.seed)
    m.save(args.out)
    # held-out pairs from the library's updates: coverage of chi* by the prediction
    prev, targ = make_update_pairs(ctx, 512, args.seed + 977)
    y = m.predict(features(ctx, prev, 1024, 2, 1e-8)).cpu().numpy().astype(np.float64)
    cover = float(np.mean(y >= targ))
    sketchable = targ <= math.log2(1024)
    print(f"samples {X.shape[0]}  epochs {args.epochs}  final train {hist['train'][-1]:.4f}  "
          f"val {hist['val'][-1]:.4f}  held-out update pairs: coverage {cover:.3f}, "
          f"chi* <= 1024 on {np.mean(sketchable):.3f}, predicted plain on "
          f"{np.mean(y[~sketchable] > math.log2(1024)) if (~sketchable).any() else float('nan'):.3f} of the rest "
          f"-> {args.out}", flush=True)


if __name__ == "__main__":
    main()
