"""Pins of the CPU oracle of the learned warm start (feature map, periodic
convolutional network, gradient, Adam) against brute force, adjoint
identities, finite differences and closed forms."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import cnn


def _tiny(n=(5, 6, 7), L=(3.0, 3.3, 3.6), n_atoms=2, seed=4):
    return W.tiny_system(n=n, L=L, n_atoms=n_atoms, with_nonlocal=False, seed=seed)


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(0)
    ci, co, nz, ny, nx = 2, 3, 4, 3, 5
    u = rng.standard_normal((ci, nz, ny, nx))
    Wt = rng.standard_normal((co, ci, 3, 3, 3))
    b = rng.standard_normal(co)
    out = cnn.conv(Wt, u, b)
    for o, z, y, x in itertools.product(range(co), range(nz), range(ny), range(nx)):
        acc = b[o]
        for i, kz, ky, kx in itertools.product(range(ci), range(3), range(3), range(3)):
            acc += Wt[o, i, kz, ky, kx] * u[i, (z + kz - 1) % nz, (y + ky - 1) % ny, (x + kx - 1) % nx]
        assert abs(out[o, z, y, x] - acc) < 1e-12


def test_conv_delta_taps():
    rng = np.random.default_rng(1)
    u = rng.standard_normal((1, 4, 5, 6))
    Wt = np.zeros((1, 1, 3, 3, 3))
    Wt[0, 0, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(cnn.conv(Wt, u), u)
    Wt[:] = 0.0
    Wt[0, 0, 1, 1, 2] = 1.0          # out[p] = u[p + e_x]
    out = cnn.conv(Wt, u)
    assert out[0, 2, 3, 5] == u[0, 2, 3, 0]
    assert out[0, 2, 3, 1] == u[0, 2, 3, 2]


def test_conv_transpose_and_weight_grad_are_adjoints():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3, 4, 5, 6))
    g = rng.standard_normal((2, 4, 5, 6))
    Wt = rng.standard_normal((2, 3, 3, 3, 3))
    lhs = np.sum(cnn.conv(Wt, u) * g)
    assert abs(lhs - np.sum(u * cnn.conv_transpose(Wt, g))) < 1e-10
    assert abs(lhs - np.sum(Wt * cnn.conv_weight_grad(u, g))) < 1e-10


def test_backward_matches_finite_differences():
    s = _tiny()
    rng = np.random.default_rng(3)
    w = W.cnn_initial_weights(5).astype(np.float64)
    w[-1] += 0.3
    f = cnn.features(s)
    target = rng.uniform(0.0, 1.0, f.shape[1:])
    target *= s.n_electrons / (s.dV * target.sum())
    rho, cache = cnn.forward(s, w, f)
    g = cnn.backward(s, w, rho, target, cache)

    def L(wv):
        return cnn.loss(cnn.forward(s, wv, f)[0], target)

    # coordinates from every parameter block, and a random direction
    idx = [0, 100, 1295, 1296 + 5, 1312, 1312 + 3000, 8224 + 7, 8240, 8240 + 200, 8672]
    for k in idx:
        e = np.zeros_like(w)
        e[k] = 1e-5
        fd = (L(w + e) - L(w - e)) / 2e-5
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-7 * np.max(np.abs(g)), (k, fd, g[k])
    d = rng.standard_normal(w.size)
    d /= np.linalg.norm(d)
    fd = (L(w + 1e-5 * d) - L(w - 1e-5 * d)) / 2e-5
    assert abs(fd - g @ d) <= 1e-6 * np.linalg.norm(g)


def test_forward_density_normalised_and_positive():
    s = _tiny()
    rho, _ = cnn.forward(s, W.cnn_initial_weights(0).astype(np.float64), cnn.features(s))
    assert np.all(rho > 0)
    assert abs(s.dV * rho.sum() - s.n_electrons) < 1e-12 * s.n_electrons


def test_softplus_stable_and_sigmoid_is_its_derivative():
    z = np.array([-800.0, -30.0, -1.0, 0.0, 2.0, 40.0, 800.0])
    sp = cnn.softplus(z)
    assert np.all(np.isfinite(sp))
    assert sp[-1] == 800.0 and sp[0] == 0.0 and abs(sp[3] - np.log(2.0)) < 1e-15
    zz = np.linspace(-5, 5, 11)
    np.testing.assert_allclose((cnn.softplus(zz + 1e-6) - cnn.softplus(zz - 1e-6)) / 2e-6, cnn.sigmoid(zz),
                               atol=1e-9)


def test_adam_first_step_and_constant_gradient():
    rng = np.random.default_rng(4)
    w = rng.standard_normal(20)
    g = rng.standard_normal(20)
    w1, m, v = cnn.adam(w, g, np.zeros(20), np.zeros(20), 1, lr=1e-2)
    # bias correction makes the first step lr * g / (|g| + eps)
    np.testing.assert_allclose(w1, w - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    ww, m, v = w.copy(), np.zeros(20), np.zeros(20)
    for t in range(1, 200):
        ww, m, v = cnn.adam(ww, g, m, v, t, lr=1e-3)
    # a constant gradient gives bias-corrected moments g and g^2 at every step
    np.testing.assert_allclose(ww, w - 199e-3 * g / (np.abs(g) + 1e-8), atol=1e-12)


def test_features_peak_integral_and_translation():
    s = W.config1(0)
    f = cnn.features(s)
    h = s.h[0]
    for c, w in enumerate(cnn.WIDTHS):
        # one Gaussian of std w integrates to (2 pi w^2)^{3/2}; the grid sum is
        # spectrally accurate for w / h >= 1.5 and the 6 w cut costs ~e^-18
        assert abs(s.dV * f[c].sum() / (s.n_atoms * (2 * np.pi * w * w) ** 1.5) - 1.0) < 1e-7
    # atom on a grid point: the narrow channel peaks at 1 there
    t = W.tiny_system(n=(16, 16, 16), L=(8.0, 8.0, 8.0), n_atoms=1, with_nonlocal=False)
    t.pos[:] = np.array([[2.0, 3.5, 5.0]])
    ft = cnn.features(t)
    assert abs(ft[0, 10, 7, 4] - 1.0) < 1e-12
    # translation by one grid spacing in x rolls the features
    t2 = W.tiny_system(n=(16, 16, 16), L=(8.0, 8.0, 8.0), n_atoms=1, with_nonlocal=False)
    t2.pos[:] = np.array([[2.5, 3.5, 5.0]])
    np.testing.assert_allclose(cnn.features(t2), np.roll(ft, 1, axis=3), atol=1e-12)


def test_parameter_count():
    assert cnn.n_params() == 8673
    assert W.cnn_initial_weights(0).size == 8673
