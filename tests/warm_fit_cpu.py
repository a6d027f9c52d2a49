"""Fit of the warm-start network by the float64 CPU twin (oracle/mlp.py) on
labels written by ``python -m paper_2608_25376_amd.warmstart --save-labels``:
does a plain float64 fit of the same architecture bring the cross-entropy of
the labelled visiting steps below the uniform level log m, on the fitted
fields and on fields it did not see?  (A GPU-trained network that stays at
the uniform level while this fit does not would point at the training
kernels; both staying there means the labels carry no per-cell signal.)

Usage: python tests/warm_fit_cpu.py LABELS.npz [--fit 300] [--val 100] [--epochs 30]
       [--params GPU_PARAMS.npy]   (also report the GPU-trained network on the same fields)
Test infrastructure: imports the oracle."""
import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import mlp  # noqa: E402


def load(path):
    z = np.load(path)
    m, side, nofly, labels = z["m"], z["side"], z["nofly"], z["labels"]
    fields, off = [], 0
    for i in range(len(m)):
        s = int(side[i])
        X = mlp.features(s, s, 0, nofly[i][:s * s])
        assert X.shape[0] == m[i]
        fields.append((X.astype(np.float64), labels[off:off + m[i]], int(m[i])))
        off += int(m[i])
    return fields


def stack(fields):
    X = np.concatenate([f[0] for f in fields])
    y = np.concatenate([f[1] for f in fields])
    ms = np.concatenate([np.full(f[2], f[2]) for f in fields])
    return X, y, ms


def ce(theta, fields):
    X, y, ms = stack(fields)
    loss, _ = mlp.loss_grad(theta, X, ms, y, bf16_ops=False)
    uni = float(np.sum(np.log(ms)))
    return loss / len(y), uni / len(y)


def init(seed):
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, (16, 128)) * np.sqrt(6 / 144), np.zeros(128),
             rng.uniform(-1, 1, (128, 128)) * np.sqrt(6 / 256), np.zeros(128),
             rng.uniform(-1, 1, (128, 128)) * np.sqrt(6 / 256), np.zeros(128)]
    return np.concatenate([p.reshape(-1) for p in parts])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("labels")
    ap.add_argument("--fit", type=int, default=300)
    ap.add_argument("--val", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--params", default="")
    args = ap.parse_args()
    fields = load(args.labels)
    fit, val = fields[:args.fit], fields[args.fit:args.fit + args.val]
    theta = init(1)
    m1, m2 = np.zeros_like(theta), np.zeros_like(theta)
    rng = np.random.default_rng(1)
    step = 0
    print(f"fields: fit {len(fit)}, validation {len(val)}")
    print(f"epoch -1: fit CE {ce(theta, fit)[0]:.4f}  validation CE {ce(theta, val)[0]:.4f}  "
          f"(uniform {ce(theta, fit)[1]:.4f} / {ce(theta, val)[1]:.4f})", flush=True)
    for ep in range(args.epochs):
        idx = rng.permutation(len(fit))
        for b in range(0, len(idx), args.batch):
            X, y, ms = stack([fit[i] for i in idx[b:b + args.batch]])
            _, g = mlp.loss_grad(theta, X, ms, y, bf16_ops=False)
            step += 1
            theta, m1, m2 = mlp.adam(theta, m1, m2, g, step, args.lr)
        if ep % 5 == 4 or ep == args.epochs - 1:
            print(f"epoch {ep}: fit CE {ce(theta, fit)[0]:.4f}  validation CE {ce(theta, val)[0]:.4f}", flush=True)
    if args.params:
        gp = np.load(args.params).astype(np.float64)
        print(f"GPU-trained network: fit-set CE {ce(gp, fit)[0]:.4f}  validation CE {ce(gp, val)[0]:.4f}")


if __name__ == "__main__":
    main()
