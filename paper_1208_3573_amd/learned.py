"""Training and use of the learned W-pattern proposer (host driver).

Every numerical step runs in libdiaf's kernels through the C ABI: the plain
factorization that produces the labels (W pattern pattern(A^2), numerical
dropping by a per-mode tolerance of |w_j(i)| ||A(:,i)||), the pair features, and
the MLP forward/backward/Adam updates.  The host only generates the seeded
training matrices and loops over them.

Training set: seeded 3D convection-diffusion problems on 48^3 grids
(seeds 5000, 5001, ...), V = diagonal + top-4 lower rows, both norm modes.
One Adam step per instance (the gradient over all its candidate pairs).
The residual gate is 1.25 x the 99th percentile of the plain method's
normalised residual r_j / s_j over the training set; the stability gate
rejects a proposal whose V column has |v_jj| below gate_dom times the sum of
its off-diagonal magnitudes, with gate_dom half the 0.1 % quantile of that
ratio for the plain method over the training set.

    python -m paper_1208_3573_amd.learned --mode unit_v --out weights.npz
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import diaf

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_DIR = os.path.join(_HERE, "weights")
TRAIN_N = 48
TRAIN_SEED0 = 5000
# dropping tolerance of the labels, per norm mode (unit-norm w concentrates w
# on fewer entries, so it keeps entries down to a smaller fraction)
LABEL_TAU = {"unit_v": 0.03, "unit_w": 0.01}


def weights_path(mode: str, vrule: str = "topk_lower") -> str:
    sfx = "" if vrule == "topk_lower" else f"_{vrule}"
    return os.path.join(WEIGHTS_DIR, f"mlp_convdiff48_{mode}{sfx}.npz")


def plain_spec(vrule: str, n: int, N: int):
    """The plain factorization's spec on an N^3 grid problem: W =
    pattern(A^2) and V = diagonal + top-4 lower rows (topk_lower), or the
    block diagonal V whose blocks are the grid's x-lines (block: the pattern
    of D, Section 5's splitting)."""
    if vrule == "block":
        import torch
        vb = torch.arange(0, n + 1, N, dtype=torch.int32, device="cuda")
        return diaf.make_spec(w="A2", v="block", v_blocks=vb), vb
    return diaf.make_spec(w="A2", v=vrule, v_count=5), None


def init_params(seed: int) -> np.ndarray:
    """He initialisation of the 16-64-64-1 network (host random numbers)."""
    rng = np.random.default_rng(seed)
    nf, nh = diaf.MLP_NFEAT, diaf.MLP_HIDDEN
    W1 = rng.standard_normal((nh, nf)) * np.sqrt(2.0 / nf)
    W2 = rng.standard_normal((nh, nh)) * np.sqrt(2.0 / nh)
    w3 = rng.standard_normal(nh) * np.sqrt(1.0 / nh)
    return np.concatenate([W1.ravel(), np.zeros(nh), W2.ravel(), np.zeros(nh), w3,
                           [0.0]]).astype(np.float32)


def _block_fro(A, Jcp, Jri):
    cn2 = np.zeros(A.n)
    np.add.at(cn2, np.repeat(np.arange(A.n), np.diff(A.colptr)), np.abs(A.val) ** 2)
    out = np.zeros(A.n)
    np.add.at(out, np.repeat(np.arange(A.n), np.diff(Jcp)), cn2[Jri])
    return np.sqrt(out)


def _dominance(H):
    """|v_jj| / sum_{i != j} |v_ij| per column of V (host arrays)."""
    n = len(H["Vcp"]) - 1
    cp, ri, vv = H["Vcp"], H["Vri"], H["Vval"]
    col = np.repeat(np.arange(n), np.diff(cp))
    isd = ri == col
    d = np.zeros(n)
    d[col[isd]] = np.abs(vv[isd])
    off = np.zeros(n)
    np.add.at(off, col[~isd], np.abs(vv[~isd]))
    return np.where(off > 0, d / np.maximum(off, 1e-300), np.inf)


def gates_from(qs, doms):
    """Residual and stability gates from the plain method's statistics."""
    gate = 1.25 * float(np.percentile(np.concatenate(qs), 99))
    gate_dom = 0.5 * float(np.quantile(np.concatenate(doms), 0.001))
    return gate, gate_dom


def build_training_set(ctx, mode: str, n_instances: int, N: int = TRAIN_N, log=print,
                       with_data: bool = True, label_tau: float | None = None,
                       vrule: str = "topk_lower"):
    """Features and labels of n_instances seeded problems, kept on the GPU,
    and the gates calibrated on the plain factorizations."""
    import torch

    import synth
    data = []
    qs = []
    doms = []
    for t in range(n_instances):
        A = synth.convdiff(N, 3, TRAIN_SEED0 + t)
        dA = diaf.DeviceCSC.from_host(A)
        spec, _vb = plain_spec(vrule, A.n, N)
        F = diaf.diaf_factor(ctx, dA, spec, mode)
        H = F.to_host()
        s = np.ones(A.n) if mode == "unit_v" else _block_fro(A, H["Wcp"], H["Wri"])
        qs.append(H["r"] / s)
        doms.append(_dominance(H))
        if with_data:
            C = diaf.DevicePattern.from_host(H["Wcp"], H["Wri"])
            npairs = len(H["Wri"])
            feat = torch.empty(npairs * diaf.MLP_NFEAT, dtype=torch.float32, device="cuda")
            diaf.diaf_features(ctx, dA, C, feat)
            lab = torch.empty(npairs, dtype=torch.float32, device="cuda")
            diaf.diaf_labels(ctx, dA, F, LABEL_TAU[mode] if label_tau is None else label_tau,
                             lab)
            data.append((feat, lab, npairs))
        F.close()
        if (t + 1) % 10 == 0:
            log(f"  training data: {t + 1}/{n_instances} instances")
    gate, gate_dom = gates_from(qs, doms)
    return data, gate, gate_dom


def train(ctx, mode: str, n_instances: int = 100, epochs: int = 8, lr: float = 3e-3,
          seed: int = 0, log=print, label_tau: float | None = None, vrule: str = "topk_lower"):
    data, gate, gate_dom = build_training_set(ctx, mode, n_instances, log=log,
                                              label_tau=label_tau, vrule=vrule)
    model = diaf.Model(ctx, init_params(seed))
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(data))
        losses = []
        for i in order:
            feat, lab, npairs = data[i]
            step_lr = lr * (0.5 ** (ep // 3))
            losses.append(diaf.diaf_mlp_train_step(ctx, model, feat, lab, npairs, step_lr))
        hist.append(float(np.mean(losses)))
        log(f"  epoch {ep}: mean loss {hist[-1]:.5f}")
    log(f"  training: {time.perf_counter() - t0:.1f} s, gate {gate:.3e}, gate_dom {gate_dom:.3f}")
    return model, gate, gate_dom, hist


def save(model, gate, gate_dom, mode, path, hist=(), label_tau=None, vrule="topk_lower"):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    np.savez(path, params=model.params(), gate_tau=np.float64(gate),
             gate_dom=np.float64(gate_dom), mode=mode,
             loss_history=np.asarray(hist, dtype=np.float64),
             label_tau=np.float64(LABEL_TAU[mode] if label_tau is None else label_tau),
             vrule=vrule)


def load(ctx, path):
    """(model, gate_tau, gate_dom) from a weights file."""
    z = np.load(path, allow_pickle=False)
    return diaf.Model(ctx, z["params"]), float(z["gate_tau"]), float(z["gate_dom"])


def load_or_train(ctx, mode: str, log=print, n_instances: int = 100, vrule: str = "topk_lower",
                  label_tau: float | None = None):
    path = weights_path(mode, vrule)
    if os.path.exists(path):
        log(f"  loading {path}")
        return load(ctx, path)
    model, gate, gate_dom, hist = train(ctx, mode, n_instances=n_instances, log=log,
                                        vrule=vrule, label_tau=label_tau)
    save(model, gate, gate_dom, mode, path, hist, label_tau, vrule)
    return model, gate, gate_dom


def recalibrate(ctx, mode: str, path: str, n_instances: int = 100, log=print):
    """Recompute both gates of a weights file from the plain method on the
    training instances (the network is left as it is)."""
    z = dict(np.load(path, allow_pickle=False))
    _, gate, gate_dom = build_training_set(ctx, mode, n_instances, log=log, with_data=False)
    z["gate_tau"] = np.float64(gate)
    z["gate_dom"] = np.float64(gate_dom)
    np.savez(path, **z)
    log(f"  {path}: gate {gate:.4e}, gate_dom {gate_dom:.4f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", default="unit_v", choices=["unit_v", "unit_w"])
    ap.add_argument("--instances", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--out", default=None)
    ap.add_argument("--label-tau", type=float, default=None,
                    help="dropping tolerance of the labels (default: per mode)")
    ap.add_argument("--recalibrate", action="store_true",
                    help="only recompute the gates of an existing weights file")
    ap.add_argument("--vrule", default="topk_lower", choices=["topk_lower", "block"],
                    help="V rule of the plain factorizations that give the labels")
    args = ap.parse_args()
    ctx = diaf.Context(0)
    path = args.out or weights_path(args.mode, args.vrule)
    if args.recalibrate:
        recalibrate(ctx, args.mode, path, args.instances)
        return
    model, gate, gate_dom, hist = train(ctx, args.mode, args.instances, args.epochs,
                                        label_tau=args.label_tau, vrule=args.vrule)
    save(model, gate, gate_dom, args.mode, path, hist, args.label_tau, args.vrule)


if __name__ == "__main__":
    main()
