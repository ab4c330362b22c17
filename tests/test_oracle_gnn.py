"""Pins of the network reference: gradients against central finite
differences, the parameter layout, and pooling/normalisation invariants."""
import numpy as np

from oracle import gnn
import sdpgen


def _graphs():
    probs = [sdpgen.maxcut_er(12, 0.4, 1, "pm1"), sdpgen.maxcut_er(9, 0.5, 2, "pm1")]
    rows, cols, w, n_of, g_of = [], [], [], [], []
    off = 0
    for gi, p in enumerate(probs):
        ei, ej, ww = p.meta["edges"]
        rows += [ei + off, ej + off]; cols += [ej + off, ei + off]; w += [ww, ww]
        n_of += [np.full(p.n, p.n)]; g_of += [np.full(p.n, gi)]
        off += p.n
    return (off, np.concatenate(rows), np.concatenate(cols), np.concatenate(w),
            np.concatenate(n_of), np.concatenate(g_of), len(probs))


def test_gradient_finite_differences():
    N, rows, cols, w, n_of, g_of, G = _graphs()
    x, A = gnn.graph_inputs(N, rows, cols, w, n_of)
    H, L = 8, 3
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(gnn.n_params(H, L)) * 0.3
    y = rng.standard_normal(N)
    r = rng.standard_normal(G)
    loss, grad, _, _ = gnn.loss_and_grad(theta, H, L, x, A, g_of, G, y, r, 0.5)
    h = 1e-6
    for idx in rng.choice(theta.size, 40, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[idx] += h; tm[idx] -= h
        fd = (gnn.loss_and_grad(tp, H, L, x, A, g_of, G, y, r, 0.5)[0] -
              gnn.loss_and_grad(tm, H, L, x, A, g_of, G, y, r, 0.5)[0]) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), idx


def test_parameter_count_and_layout():
    assert gnn.n_params(64, 3) == 64 * 5 + 64 + 3 * (2 * 64 * 64 + 64) + 2 * 64 + 2
    theta = np.arange(gnn.n_params(4, 2), dtype=float)
    P = gnn.unpack(theta, 4, 2)
    assert P["W_in"][0, 0] == 0 and P["b_in"][0] == 20 and P["c_r"][0] == theta[-1]


def test_normalisation_and_pooling():
    N, rows, cols, w, n_of, g_of, G = _graphs()
    x, A = gnn.graph_inputs(N, rows, cols, w, n_of)
    # |A| row sums stay below one; features of graph 0 see n = 12
    assert np.all(np.abs(A).sum(axis=1) < 1.0)
    assert np.allclose(x[:12, 4], np.log(12) / 10)
    H, L = 6, 1
    theta = np.random.default_rng(1).standard_normal(gnn.n_params(H, L))
    yhat, rhat, c = gnn.forward(theta, H, L, x, A, g_of, G)
    assert np.allclose(c["pool"][1], c["H"][-1][12:].mean(axis=0))
