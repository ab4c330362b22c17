"""FP64 reference of the learned warm start's network (test infrastructure).

A message-passing network over a weighted graph (for MaxCut, the graph itself)
predicts a per-node dual multiplier and a graph-level rank factor.  Layout and
maths (the GPU library implements the same definitions independently):

  node features x_j (5): [deg_j, sum_k w_jk, sum_k |w_jk|, sum_k w_jk^2, ln n] / 10
  normalised adjacency   A_jk = w_jk / (1 + sum_k |w_jk|)
  H0 = relu(x W_in^T + b_in)
  H_l = relu(H_{l-1} W_s^T + (A H_{l-1}) W_n^T + b_l),  l = 1..L
  yhat_j = <H_L[j], v_y> + c_y
  rhat_g = <mean_{j in g} H_L[j], v_r> + c_r
  loss = mean_j (yhat_j - y_j)^2 + omega * mean_g (rhat_g - r_g)^2

Flat parameter vector: W_in (H x 5), b_in (H), then per layer W_s (H x H),
W_n (H x H), b (H), then v_y (H), c_y, v_r (H), c_r; matrices row-major.
"""
from __future__ import annotations

import numpy as np

F_IN = 5


def n_params(hidden: int, layers: int) -> int:
    H = hidden
    return H * F_IN + H + layers * (2 * H * H + H) + 2 * H + 2


def unpack(theta, hidden, layers):
    H = hidden
    o = 0
    def take(k, shape):
        nonlocal o
        a = theta[o:o + k].reshape(shape)
        o += k
        return a
    P = {"W_in": take(H * F_IN, (H, F_IN)), "b_in": take(H, (H,))}
    P["layers"] = []
    for _ in range(layers):
        P["layers"].append((take(H * H, (H, H)), take(H * H, (H, H)), take(H, (H,))))
    P["v_y"] = take(H, (H,)); P["c_y"] = take(1, (1,))
    P["v_r"] = take(H, (H,)); P["c_r"] = take(1, (1,))
    assert o == theta.size
    return P


def graph_inputs(n_nodes: int, rows, cols, w, n_of_node):
    """Features and normalised adjacency (dense) of a block-diagonal union of
    graphs given as symmetric COO (both directions listed)."""
    deg = np.bincount(rows, minlength=n_nodes).astype(np.float64)
    sw = np.bincount(rows, weights=w, minlength=n_nodes)
    sa = np.bincount(rows, weights=np.abs(w), minlength=n_nodes)
    s2 = np.bincount(rows, weights=w * w, minlength=n_nodes)
    x = np.stack([deg, sw, sa, s2, np.log(n_of_node)], axis=1) / 10.0
    A = np.zeros((n_nodes, n_nodes))
    np.add.at(A, (rows, cols), w / (1.0 + sa[rows]))
    return x, A


def forward(theta, hidden, layers, x, A, graph_of_node, n_graphs):
    P = unpack(theta, hidden, layers)
    cache = {}
    Z0 = x @ P["W_in"].T + P["b_in"]
    H = np.maximum(Z0, 0.0)
    cache["Z"] = [Z0]
    cache["H"] = [H]
    cache["M"] = []
    for Ws, Wn, b in P["layers"]:
        M = A @ H
        Z = H @ Ws.T + M @ Wn.T + b
        H = np.maximum(Z, 0.0)
        cache["M"].append(M); cache["Z"].append(Z); cache["H"].append(H)
    yhat = H @ P["v_y"] + P["c_y"][0]
    counts = np.bincount(graph_of_node, minlength=n_graphs).astype(np.float64)
    pool = np.zeros((n_graphs, hidden))
    np.add.at(pool, graph_of_node, H)
    pool /= counts[:, None]
    rhat = pool @ P["v_r"] + P["c_r"][0]
    cache.update(pool=pool, counts=counts, P=P)
    return yhat, rhat, cache


def loss_and_grad(theta, hidden, layers, x, A, graph_of_node, n_graphs, y, r, omega):
    yhat, rhat, c = forward(theta, hidden, layers, x, A, graph_of_node, n_graphs)
    P = c["P"]
    N = x.shape[0]
    ey, er = yhat - y, rhat - r
    loss = float(np.mean(ey ** 2) + omega * np.mean(er ** 2))
    dy = 2.0 * ey / N
    dr = 2.0 * omega * er / n_graphs
    HL = c["H"][-1]
    g = {"v_y": HL.T @ dy, "c_y": np.array([dy.sum()]),
         "v_r": c["pool"].T @ dr, "c_r": np.array([dr.sum()])}
    dH = np.outer(dy, P["v_y"])
    dpool = np.outer(dr, P["v_r"])
    dH += dpool[graph_of_node] / c["counts"][graph_of_node][:, None]
    layer_grads = []
    for l in range(layers - 1, -1, -1):
        Ws, Wn, b = P["layers"][l]
        Z, Hprev, M = c["Z"][l + 1], c["H"][l], c["M"][l]
        dZ = dH * (Z > 0)
        gWs = dZ.T @ Hprev
        gWn = dZ.T @ M
        gb = dZ.sum(axis=0)
        layer_grads.append((gWs, gWn, gb))
        dM = dZ @ Wn
        dH = dZ @ Ws + A.T @ dM
    layer_grads.reverse()
    dZ0 = dH * (c["Z"][0] > 0)
    g["W_in"] = dZ0.T @ x
    g["b_in"] = dZ0.sum(axis=0)
    flat = [g["W_in"].ravel(), g["b_in"]]
    for gWs, gWn, gb in layer_grads:
        flat += [gWs.ravel(), gWn.ravel(), gb]
    flat += [g["v_y"], g["c_y"], g["v_r"], g["c_r"]]
    return loss, np.concatenate(flat), yhat, rhat
