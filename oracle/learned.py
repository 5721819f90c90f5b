"""FP64 reference of the learned W-pattern proposer.  TEST INFRASTRUCTURE ONLY.

Plain NumPy / Python loops (small cases only):
* features of (column j, candidate i) pairs of a candidate pattern C,
  defined from column access to A only (the definitions are listed in
  ``features``);
* labels from a plain factorization by numerical dropping by tolerance
  (Section 4.1: keep the entries that are relatively large, never drop the
  diagonal): label = 1 iff |w_j(i)| ||A(:,i)|| >= tau * max over the column;
* the MLP 16 -> 64 -> 64 -> 1 (ReLU), its mean binary cross-entropy loss
  on logits, the gradient by back-propagation, and one Adam step.

Parameter vector layout: W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

NF, NH = 16, 64
NPARAM = NH * NF + NH + NH * NH + NH + NH + 1


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = t[o:o + NH * NF].reshape(NH, NF); o += NH * NF
    b1 = t[o:o + NH]; o += NH
    W2 = t[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = t[o:o + NH]; o += NH
    w3 = t[o:o + NH]; o += NH
    b3 = t[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation (host-side random numbers, passed to the GPU)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((NH, NF)) * np.sqrt(2.0 / NF)
    W2 = rng.standard_normal((NH, NH)) * np.sqrt(2.0 / NH)
    w3 = rng.standard_normal(NH) * np.sqrt(1.0 / NH)
    return pack(W1, np.zeros(NH), W2, np.zeros(NH), w3, 0.0).astype(np.float32)


def forward(theta, X):
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.maximum(X @ W1.T + b1, 0.0)
    H2 = np.maximum(H1 @ W2.T + b2, 0.0)
    return H2 @ w3 + b3


def loss_grad(theta, X, y):
    """Mean BCE-with-logits loss and its gradient (back-propagation)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    N = X.shape[0]
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    s = H2 @ w3 + b3
    loss = np.mean(np.maximum(s, 0) - s * y + np.log1p(np.exp(-np.abs(s))))
    d3 = (1.0 / (1.0 + np.exp(-s)) - y) / N
    gw3 = H2.T @ d3
    gb3 = d3.sum()
    D2 = np.outer(d3, w3) * (Z2 > 0)
    gW2 = D2.T @ H1
    gb2 = D2.sum(axis=0)
    D1 = (D2 @ W2) * (Z1 > 0)
    gW1 = D1.T @ X
    gb1 = D1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def loss_only(theta, X, y):
    s = forward(theta, X)
    y = np.asarray(y, dtype=np.float64)
    return np.mean(np.maximum(s, 0) - s * y + np.log1p(np.exp(-np.abs(s))))


def adam_step(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def _col(A, c):
    sl = slice(A.colptr[c], A.colptr[c + 1])
    return A.rowidx[sl], np.abs(A.val[sl])


def features(A, Ccp, Cri) -> np.ndarray:
    """16 features per candidate pair (plain loops; small n only).

    With d_c = |a_cc|, s_c = sum_{r != c} |a_rc|, nrm_c = ||A(:,c)||,
    deg_c = nnz(A(:,c)) and, over c in rows(A(:,j)),
    pw = sum |a_ic||a_cj|, cnt = #{c : a_ic a_cj != 0}, mx = max |a_ic||a_cj|:
      f0 [i==j], f1 [a_ij != 0], f2 pw/max_col pw, f3 cnt/max_col cnt,
      f4 |a_ij|/d_j, f5 deg_j/8, f6 deg_i/8, f7 d_j/(d_j+s_j),
      f8 d_i/(d_i+s_i), f9 sign(i-j), f10 log2(1+|i-j|)/24, f11 nrm_i/nrm_j,
      f12 mx/pw, f13 pw/(d_i d_j), f14 |C_j|/32,
      f15 fraction of the column's other candidates with a larger pw.
    """
    n = A.n
    cols = [dict(zip(*_col(A, c))) for c in range(n)]
    d = np.array([cols[c].get(c, 0.0) for c in range(n)])
    s = np.array([sum(v for r, v in cols[c].items() if r != c) for c in range(n)])
    nrm = np.array([np.sqrt(sum(v * v for v in cols[c].values())) for c in range(n)])
    deg = np.diff(A.colptr)
    F = np.zeros((int(Ccp[-1]), NF))
    for j in range(n):
        cand = Cri[Ccp[j]:Ccp[j + 1]]
        rows_j = sorted(cols[j].items())
        stats = []
        for i in cand:
            pw, cnt, mx = 0.0, 0, 0.0
            for c, acj in rows_j:
                pr = cols[c].get(i, 0.0) * acj
                pw += pr
                cnt += pr != 0.0
                mx = max(mx, pr)
            stats.append((pw, cnt, mx))
        pwmax = max(st[0] for st in stats)
        cntmax = max(st[1] for st in stats)
        nc = len(cand)
        for t, i in enumerate(cand):
            pw, cnt, mx = stats[t]
            larger = sum(1 for u in range(nc) if u != t and stats[u][0] > pw)
            aij = cols[j].get(i, 0.0)
            f = F[Ccp[j] + t]
            f[0] = float(i == j)
            f[1] = float(i in cols[j])
            f[2] = pw / pwmax if pwmax > 0 else 0.0
            f[3] = cnt / cntmax if cntmax > 0 else 0.0
            f[4] = aij / d[j] if d[j] > 0 else 0.0
            f[5] = deg[j] / 8.0
            f[6] = deg[i] / 8.0
            f[7] = d[j] / (d[j] + s[j]) if d[j] + s[j] > 0 else 0.0
            f[8] = d[i] / (d[i] + s[i]) if d[i] + s[i] > 0 else 0.0
            f[9] = float(np.sign(i - j))
            f[10] = np.log2(1.0 + abs(int(i) - j)) / 24.0
            f[11] = nrm[i] / nrm[j] if nrm[j] > 0 else 0.0
            f[12] = mx / pw if pw > 0 else 0.0
            f[13] = pw / (d[i] * d[j]) if d[i] > 0 and d[j] > 0 else 0.0
            f[14] = nc / 32.0
            f[15] = larger / (nc - 1) if nc > 1 else 0.0
    return F


def labels(A, Jcp, Jri, Wval, tau: float = 0.1) -> np.ndarray:
    """label(i) = 1 iff |w_j(i)| ||A(:,i)|| >= tau max_i' |w_j(i')| ||A(:,i')||,
    and always for i = j."""
    n = A.n
    nrm = np.array([np.linalg.norm(A.val[A.colptr[c]:A.colptr[c + 1]]) for c in range(n)])
    out = np.zeros(int(Jcp[-1]))
    for j in range(n):
        sl = slice(Jcp[j], Jcp[j + 1])
        c = np.abs(Wval[sl]) * nrm[Jri[sl]]
        out[sl] = (c >= tau * c.max()) | (Jri[sl] == j)
    return out
