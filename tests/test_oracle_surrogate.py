"""Pins of the oracle's plain network (oracle/surrogate.py), on the CPU.

A layer is checked against scipy's n-dimensional correlation (circular in x
and y, the thickness padded with zeros), equivariance under circular shifts
in x and y, and the back-propagated gradients against central finite
differences of the loss.
"""
import numpy as np
import scipy.ndimage as nd

from oracle import surrogate as S


def _params(rng, widths):
    ps = []
    for ci, co in zip(widths[:-1], widths[1:]):
        ps.append((rng.standard_normal((co, ci, 3, 3, 3)) / np.sqrt(27 * ci),
                   0.1 * rng.standard_normal(co)))
    return ps


def test_layer_is_a_wrapped_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 4, 6, 5))
    W = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    got = S.layer(x, W, b)
    for co in range(2):
        ref = np.full(x.shape[1:], b[co])
        for ci in range(3):
            padded = np.pad(x[ci], ((1, 1), (0, 0), (0, 0)))
            ref += nd.correlate(padded, W[co, ci], mode="wrap")[1:-1]
        assert np.abs(got[co] - ref).max() < 1e-12


def test_network_commutes_with_circular_shifts():
    rng = np.random.default_rng(2)
    ps = _params(rng, [1, 4, 4, 1])
    x = rng.standard_normal((1, 3, 8, 7))
    y, _ = S.forward(x, ps)
    ys, _ = S.forward(np.roll(x, (2, -3), axis=(2, 3)), ps)
    assert np.abs(np.roll(y, (2, -3), axis=(2, 3)) - ys).max() < 1e-12
    # no such symmetry across the thickness (zero padding there)
    yz, _ = S.forward(np.roll(x, 1, axis=1), ps)
    assert np.abs(np.roll(y, 1, axis=1) - yz).max() > 1e-3


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    ps = _params(rng, [1, 3, 2, 1])
    x = rng.standard_normal((1, 3, 5, 4))
    t = rng.standard_normal((1, 3, 5, 4))
    mask = np.zeros((3, 5, 4), dtype=bool)
    mask[:, 1:4, :] = True
    loss, grads = S.loss_and_grads(x, t, ps, mask)
    eps = 1e-6
    for li in range(len(ps)):
        W, b = ps[li]
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += eps
            Wm[idx] -= eps
            lp, _ = S.loss_and_grads(x, t, ps[:li] + [(Wp, b)] + ps[li + 1:], mask)
            lm, _ = S.loss_and_grads(x, t, ps[:li] + [(Wm, b)] + ps[li + 1:], mask)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grads[li][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (li, idx)
        k = int(rng.integers(0, b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[k] += eps
        bm[k] -= eps
        lp, _ = S.loss_and_grads(x, t, ps[:li] + [(W, bp)] + ps[li + 1:], mask)
        lm, _ = S.loss_and_grads(x, t, ps[:li] + [(W, bm)] + ps[li + 1:], mask)
        assert abs((lp - lm) / (2 * eps) - grads[li][1][k]) <= 1e-6 * max(1.0, abs(lp))
