"""Pins of the learned proposer's FP64 reference (oracle/learned.py)."""
import numpy as np
import scipy.sparse as sp

import synth
from oracle import learned as L


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = L.init_params(3).astype(np.float64)
    X = rng.standard_normal((40, L.NF))
    y = (rng.random(40) < 0.4).astype(float)
    loss, g = L.loss_grad(theta, X, y)
    assert abs(loss - L.loss_only(theta, X, y)) < 1e-14
    idx = rng.choice(L.NPARAM, 60, replace=False)
    h = 1e-6
    for q in list(idx) + [L.NPARAM - 1, 0]:
        e = np.zeros(L.NPARAM)
        e[q] = h
        fd = (L.loss_only(theta + e, X, y) - L.loss_only(theta - e, X, y)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 * max(1.0, abs(g[q])), q


def test_loss_closed_form_at_zero_logits():
    """All-zero output layer: every logit is 0 and the loss is log 2."""
    theta = L.init_params(1).astype(np.float64)
    W1, b1, W2, b2, w3, b3 = L.unpack(theta)
    theta0 = L.pack(W1, b1, W2, b2, np.zeros_like(w3), 0.0)
    X = np.random.default_rng(2).standard_normal((17, L.NF))
    y = np.arange(17) % 2
    loss, g = L.loss_grad(theta0, X, y)
    assert abs(loss - np.log(2)) < 1e-15
    # d loss / d b3 = mean(sigmoid(0) - y)
    assert abs(g[-1] - np.mean(0.5 - y)) < 1e-15


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = L.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(th[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert th[3] == 0.0


def test_features_on_a_hand_checked_matrix():
    # A = [[4, -1, 0], [-2, 5, -1], [0, -1, 3]] (column j sees rows of A(:,j))
    Ad = np.array([[4.0, -1.0, 0.0], [-2.0, 5.0, -1.0], [0.0, -1.0, 3.0]])
    A = synth.CSC.from_scipy(sp.csc_matrix(Ad))
    P = sp.csc_matrix((np.abs(Ad) > 0).astype(float))
    C = (P @ P).tocsc()
    C.sort_indices()
    F = L.features(A, C.indptr, C.indices)
    # column 0 candidates: rows 0,1,2; pw_i = sum_c |a_ic||a_c0|, c in {0,1}
    # pw0 = 4*4 + 1*2 = 18, pw1 = 2*4 + 5*2 = 18, pw2 = 0*4 + 1*2 = 2
    f = F[C.indptr[0]:C.indptr[1]]
    assert list(f[:, 0]) == [1, 0, 0]
    assert list(f[:, 1]) == [1, 1, 0]
    assert np.allclose(f[:, 2], [1, 1, 2 / 18])
    assert np.allclose(f[:, 3], [1, 1, 0.5])          # path counts 2, 2, 1
    assert np.allclose(f[:, 4], [1, 2 / 4, 0])         # |a_i0| / |a_00|
    assert np.allclose(f[:, 9], [0, 1, 1])
    assert np.allclose(f[:, 12], [16 / 18, 10 / 18, 1.0])
    assert np.allclose(f[:, 15], [0, 0, 1.0])          # two candidates beat pw2
    # degrees 2, 3, 2; diagonals 4, 5, 3; off-diagonal column sums 2, 2, 1;
    # column norms sqrt(20), sqrt(27), sqrt(10)
    assert np.allclose(f[:, 5], [2 / 8] * 3)           # deg_j / 8
    assert np.allclose(f[:, 6], [2 / 8, 3 / 8, 2 / 8])  # deg_i / 8
    assert np.allclose(f[:, 7], [4 / 6] * 3)           # d_j / (d_j + s_j)
    assert np.allclose(f[:, 8], [4 / 6, 5 / 7, 3 / 4])  # d_i / (d_i + s_i)
    assert np.allclose(f[:, 10], [0, 1 / 24, np.log2(3) / 24])
    assert np.allclose(f[:, 11], [1, np.sqrt(27 / 20), np.sqrt(10 / 20)])
    assert np.allclose(f[:, 13], [18 / 16, 18 / 20, 2 / 12])  # pw / (d_i d_j)
    assert np.allclose(f[:, 14], [3 / 32] * 3)
    f2 = F[C.indptr[2]:C.indptr[3]]
    assert np.allclose(f2[:, 5], 2 / 8) and np.allclose(f2[:, 7], 3 / 4)
    assert np.allclose(f2[:, 10], [np.log2(3) / 24, 1 / 24, 0])


def test_labels_keep_diagonal_and_large_entries():
    Ad = np.diag([2.0, 2.0, 2.0])
    A = synth.CSC.from_scipy(sp.csc_matrix(Ad))
    Jcp = np.array([0, 3, 4, 5])
    Jri = np.array([0, 1, 2, 1, 2])
    W = np.array([0.001, 1.0, 0.2, 0.5, 0.5])
    lab = L.labels(A, Jcp, Jri, W, tau=0.1)
    assert list(lab) == [1, 1, 1, 1, 1]
    W = np.array([1e-3, 1.0, 0.05, 0.5, 0.5])
    lab = L.labels(A, Jcp, Jri, W, tau=0.1)
    assert list(lab[:3]) == [1, 1, 0]
