"""Pins of the oracle's result measures and of its normal stream (CPU only).

Recovery error of a planted completion (the relative error of the off-diagonal
block of X = U U^T against M = L R^T):
  * closed form: U1 = (1 + d) L, U2 = R gives U1 U2^T = (1 + d) M, so the error
    is exactly |d|, for any d (a clamped or sign-flipped expansion fails at
    d = 1e-3 and d = -0.5);
  * exact recovery gives 0; the error is invariant under U -> U Q (Q orthogonal);
  * brute force: the dense n1 x n2 difference at small sizes.
Gram products: integer factors, whose products and sums are exact in FP64,
against the entry-by-entry triple loop.
Normals (Box-Muller on SplitMix64 uniforms): a Kolmogorov-Smirnov test against
the standard normal distribution function of scipy (independent code), and the
first element of a stream rebuilt from the published SplitMix64 outputs.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats

import oracle
import sdpgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _planted(n1=37, n2=29, k=3, seed=4):
    return sdpgen.mc_planted(n1, n2, k, seed, count=400)


@pytest.mark.parametrize("d", [0.0, 1e-3, -0.5, 2.0])
def test_recovery_error_closed_form(d):
    p = _planted()
    L, R = p.meta["L"], p.meta["R"]
    U = np.vstack([(1.0 + d) * L, R])
    e = oracle.metrics.mc_recovery_error(p, U, block=8)
    assert abs(e - abs(d)) <= 1e-14 * max(1.0, abs(d)) + 1e-15, (e, d)


def test_recovery_error_rotation_invariant():
    p = _planted()
    rng = np.random.default_rng(2)
    U = np.vstack([p.meta["L"], p.meta["R"]]) + 1e-2 * rng.standard_normal((p.n, 3))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    a = oracle.metrics.mc_recovery_error(p, U)
    b = oracle.metrics.mc_recovery_error(p, U @ Q)
    assert a > 1e-3 and abs(a - b) <= 1e-12 * a


@pytest.mark.parametrize("r", [3, 6])
def test_recovery_error_bruteforce(r):
    p = _planted()
    n1 = p.meta["n1"]
    rng = np.random.default_rng(r)
    U = rng.standard_normal((p.n, r))
    M = p.meta["L"] @ p.meta["R"].T
    ref = np.linalg.norm(U[:n1] @ U[n1:].T - M) / np.linalg.norm(M)
    for block in (1, 5, 1024):
        e = oracle.metrics.mc_recovery_error(p, U, block=block)
        assert abs(e - ref) <= 1e-13 * ref


def test_normals_kolmogorov_smirnov():
    x = oracle.rng.normals(2024, 3, 200_000)
    res = scipy.stats.kstest(x, "norm")
    assert res.pvalue > 1e-3, res


def test_normals_first_element_from_published_stream():
    # seed 0, event 0, element 0 takes SplitMix64 outputs k = 1 and k = 2
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_seed0.json")))
    o1, o2 = (int(h, 16) for h in g["outputs"][:2])
    u1 = ((o1 >> 11) + 1) * 2.0 ** -53
    u2 = (o2 >> 11) * 2.0 ** -53
    want = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
    assert oracle.rng.normals(0, 0, 1)[0] == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("n,ra,rb,block", [(37, 3, 5, 8), (9, 1, 1, 4096), (200, 6, 2, 7)])
def test_gram_integer_exact(n, ra, rb, block):
    rng = np.random.default_rng(n)
    A = rng.integers(-9, 10, (n, ra)).astype(np.float64)
    B = rng.integers(-9, 10, (n, rb)).astype(np.float64)
    want = np.zeros((ra, rb))
    for i in range(ra):
        for j in range(rb):
            want[i, j] = sum(A[t, i] * B[t, j] for t in range(n))
    assert np.array_equal(oracle.metrics.gram(A, B, block=block), want)
