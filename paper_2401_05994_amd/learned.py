"""Training and evaluation driver for the learned per-level bin-width allocation.

Every numeric step runs in the HIP library: decomposition, level statistics,
quantization, recomposition and the L-infinity check for the labels, and the
network's forward, loss, backward and Adam kernels for training.  This module
only orders the calls and keeps the data set.

Labels.  For one field and tolerance, theta* is found greedily from the finest
level to the coarsest: theta_l is raised by bisection on [0, theta_max] while
the recomposed error stays at or below `target` * tau, with the other levels
kept at their current values.  Starting from theta = 0 (the plain allocation,
which meets the bound a priori) every accepted step keeps the bound.

Features (one row per level, as the device computes them): log(rms/tau),
log(max|c|/tau), log(count / stream length), l/L.

Usage:
    python -m paper_2401_05994_amd.learned train --count 2000 --n 257 --out <file.npz>
    python -m paper_2401_05994_amd.learned evaluate --model <file.npz> --n 1025
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "models", "alloc_mlp.npz")


def _lib():
    import paper_2401_05994_amd as m

    return m


def plain_bins(u, tol, coords=None):
    """The library's plain widths and tau for u under a relative tol (computed on the device)."""
    return _lib().mgard_bin_widths(u, tol, coords)


def features(coeff, shape, tau):
    """The network's raw input rows, from the device kernels the learned compression runs."""
    return _lib().mgard_level_features(coeff, shape, tau).astype(np.float64)


class BoundCheck:
    """Recomposed L-infinity error of a bin allocation for one decomposed field."""

    def __init__(self, u, coords=None, dict_size=8192):
        m = _lib()
        self.u = u
        self.shape = tuple(u.shape)
        self.coords = coords
        self.dict_size = dict_size
        self.coeff = m.mgard_decompose(u, coords)
        self.calls = 0

    def error(self, bins):
        m = _lib()
        self.calls += 1
        sym, qside = m.mgard_quantize(self.coeff, self.shape, list(bins), self.dict_size)
        c = m.mgard_dequantize(sym, qside, self.shape, list(bins), self.u.dtype, self.dict_size)
        r = m.mgard_recompose(c, self.shape, self.coords)
        return m.mgard_linf_error(r, self.u)


def label(u, tol, theta_max=5.0, iters=6, target=0.95, coords=None):
    """(features, theta*) rows for one field and tolerance."""
    plain, tau = plain_bins(u, tol, coords)
    check = BoundCheck(u, coords)
    feats = features(check.coeff, tuple(u.shape), tau)
    nlev = len(plain)
    theta = np.zeros(nlev)
    limit = target * tau
    for l in range(nlev - 1, -1, -1):
        lo, hi = 0.0, theta_max
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            trial = theta.copy()
            trial[l] = mid
            err = check.error([b * math.exp(t) for b, t in zip(plain, trial)])
            if err <= limit:
                lo = mid
            else:
                hi = mid
        theta[l] = lo
    return feats, theta, {"tau": tau, "check_calls": check.calls}


def training_field(n, seed, beta):
    import torch

    import fieldgen

    return fieldgen.spectral((n, n, n), beta, seed, device="cuda", noise="torch").to(torch.float32).contiguous()


def build_dataset(count, n, seed0=10000, tol_lo=1e-5, tol_hi=1e-2, log=print):
    rng = np.random.default_rng(seed0)
    X, Y = [], []
    t0 = time.time()
    for i in range(count):
        beta = float(rng.uniform(-4.0, -5.0 / 3.0))
        tol = float(math.exp(rng.uniform(math.log(tol_lo), math.log(tol_hi))))
        u = training_field(n, seed0 + i, beta)
        f, th, _ = label(u, tol)
        X.append(f)
        Y.append(th)
        if (i + 1) % max(1, count // 20) == 0:
            log(f"[learned] labelled {i + 1}/{count} fields ({time.time() - t0:.0f} s)")
    return np.concatenate(X).astype(np.float32), np.concatenate(Y).astype(np.float32)


def init_params(seed, mean, std):
    """He-normal weights from a seeded generator, zero biases; flat layout of the library."""
    rng = np.random.default_rng(seed)
    sizes = (4, 64, 64, 1)
    parts = [np.asarray(mean, dtype=np.float64), np.asarray(std, dtype=np.float64)]
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        parts.append((rng.standard_normal((fo, fi)) * math.sqrt(2.0 / fi)).ravel())
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def train(X, Y, epochs=200, batch=512, lr=2e-3, seed=0, log=print):
    """Adam on mean squared error with the library's kernels; returns flat float32 parameters."""
    import torch

    m = _lib()
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std < 1e-6] = 1.0
    params = torch.from_numpy(init_params(seed, mean, std)).cuda()
    mom = torch.zeros_like(params)
    vel = torch.zeros_like(params)
    dx = torch.from_numpy(X).cuda()
    dy = torch.from_numpy(Y).cuda()
    n = X.shape[0]
    rng = np.random.default_rng(seed + 1)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        tot = 0.0
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            xb = dx.index_select(0, idx).contiguous()
            yb = dy.index_select(0, idx).contiguous()
            out, cache = m.mgard_mlp_forward(params, xb)
            dout, loss = m.mgard_mlp_mse(out, yb)
            g = m.mgard_mlp_backward(params, cache, dout, xb.shape[0])
            step += 1
            m.mgard_mlp_adam(params, g, mom, vel, step, lr=lr)
            tot += loss * xb.shape[0]
        hist.append(tot / n)
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            log(f"[learned] epoch {ep} loss {hist[-1]:.5f}")
    return params.cpu().numpy(), hist


def save(path, params, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), meta=json.dumps(meta))


def load(path=DEFAULT_MODEL):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(str(z["meta"]))


def evaluate(model_params, u, tols, coords=None, log=print):
    """Plain versus learned ratio and error at each tolerance (device compression, host-side sizes)."""
    m = _lib()
    model = m.Model(model_params)
    nbytes_in = u.numel() * u.element_size()
    rows = []
    for tol in tols:
        log(f"[learned] evaluating tol {tol:g}")
        _, nb_p, info_p = m.mgard_compress(u, tol, coords)
        _, nb_c, info_c = m.mgard_compress(u, tol, coords, alloc="count")
        buf, nb_l, info_l = m.mgard_compress_learned(u, tol, model, coords)
        rows.append({
            "tol": tol, "ratio_plain": nbytes_in / nb_p, "ratio_count": nbytes_in / nb_c,
            "ratio_learned": nbytes_in / nb_l, "linf_learned": info_l["linf_err"], "tau": info_l["tau_abs"],
            "fallback": info_l["fallback_used"],
        })
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--count", type=int, default=2000)
    t.add_argument("--n", type=int, default=257)
    t.add_argument("--epochs", type=int, default=200)
    t.add_argument("--out", default=DEFAULT_MODEL)
    t.add_argument("--dataset", default=None, help="optional .npz to save/load the labelled rows")
    t.add_argument("--seed0", type=int, default=10000, help="seed of the first training field")
    t.add_argument("--merge", default=None,
                   help="comma-separated labelled-row files (.npz) to train on instead of labelling")
    t.add_argument("--label-only", action="store_true", help="write the labelled rows (--dataset) and stop")
    e = sub.add_parser("evaluate")
    e.add_argument("--model", default=DEFAULT_MODEL)
    e.add_argument("--n", type=int, default=1025)
    e.add_argument("--seed", type=int, default=5)
    e.add_argument("--tols", default="1e-2,1e-3,1e-4,1e-5")
    args = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    if args.cmd == "train":
        fields = args.count
        if args.merge:
            parts = []
            for f in args.merge.split(","):
                with np.load(f, allow_pickle=False) as z:
                    parts.append((z["X"], z["Y"], int(z["fields"]) if "fields" in z else 0))
            X = np.concatenate([p[0] for p in parts])
            Y = np.concatenate([p[1] for p in parts])
            fields = sum(p[2] for p in parts)
        elif args.dataset and os.path.exists(args.dataset):
            with np.load(args.dataset, allow_pickle=False) as z:
                X, Y = z["X"], z["Y"]
        else:
            X, Y = build_dataset(args.count, args.n, seed0=args.seed0, log=log)
            if args.dataset:
                np.savez(args.dataset, X=X, Y=Y, fields=args.count, seed0=args.seed0, n=args.n)
            if args.label_only:
                print(json.dumps({"rows": int(X.shape[0]), "dataset": args.dataset}))
                return
        params, hist = train(X, Y, epochs=args.epochs, log=log)
        save(args.out, params, {"fields": fields, "n": args.n, "rows": int(X.shape[0]),
                                "final_loss": hist[-1], "theta_mean": float(Y.mean())})
        print(json.dumps({"rows": int(X.shape[0]), "final_loss": hist[-1], "out": args.out}))
    else:
        import torch

        params, meta = load(args.model)
        log(f"[learned] generating the {args.n}^3 evaluation field (seed {args.seed})")
        u = training_field(args.n, args.seed, -5.0 / 3.0)
        torch.cuda.synchronize()
        rows = evaluate(params, u, [float(x) for x in args.tols.split(",")], log=log)
        print(json.dumps({"model": meta, "n": args.n, "rows": rows}))


if __name__ == "__main__":
    main()
