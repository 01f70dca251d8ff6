"""Pins of the learned-correction oracle (oracle/cnn.py) on the CPU: each
function against something other than itself -- a library routine, an
adjoint identity, finite differences, a closed form."""
import numpy as np
import pytest

from oracle import cnn


def _rand(rng, *shape):
    return rng.standard_normal(shape)


@pytest.mark.parametrize("bc,mode", [(cnn.PERIODIC, "wrap"), (cnn.OUTFLOW, "nearest")])
def test_conv3_is_a_sum_of_scipy_correlations(bc, mode):
    # scipy.ndimage.correlate with a 3x3x3 kernel computes
    # out[p] = sum_t k[t + 1] in[p + t], extending the array by wrapping
    # ("wrap") or by repeating the edge value ("nearest")
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(0)
    x = _rand(rng, 3, 5, 6, 7)
    w = _rand(rng, 4, 3, 3, 3, 3)
    b = _rand(rng, 4)
    y = cnn.conv3(x, w, b, bc)
    for o in range(4):
        ref = b[o] + sum(ndimage.correlate(x[i], w[o, i], mode=mode) for i in range(3))
        np.testing.assert_allclose(y[o], ref, rtol=1e-13, atol=1e-13)


def test_conv3_with_a_single_tap_is_a_shift():
    rng = np.random.default_rng(1)
    x = _rand(rng, 2, 4, 5, 6)
    w = np.zeros((2, 2, 3, 3, 3))
    w[0, 0, 2, 1, 0] = 1.0      # y0(z, y, x) = x0(z + 1, y, x - 1)
    w[1, 1, 1, 1, 1] = 1.0      # y1 = x1
    y = cnn.conv3(x, w, np.zeros(2), cnn.PERIODIC)
    assert np.array_equal(y[0], np.roll(np.roll(x[0], -1, axis=0), 1, axis=2))
    assert np.array_equal(y[1], x[1])


@pytest.mark.parametrize("bc", [cnn.PERIODIC, cnn.OUTFLOW])
def test_conv3_backward_input_is_the_adjoint(bc):
    # <conv3(x, w, 0), g> = <x, dx(g)> for every x, g: pins the scatter
    # through the boundary map
    rng = np.random.default_rng(2)
    x = _rand(rng, 3, 4, 5, 3)
    w = _rand(rng, 2, 3, 3, 3, 3)
    g = _rand(rng, 2, 4, 5, 3)
    y = cnn.conv3(x, w, np.zeros(2), bc)
    _, _, dx = cnn.conv3_backward(x, w, g, bc)
    assert abs(np.sum(y * g) - np.sum(x * dx)) <= 1e-12 * np.sum(np.abs(y * g))


@pytest.mark.parametrize("bc", [cnn.PERIODIC, cnn.OUTFLOW])
def test_network_gradients_match_finite_differences(bc):
    rng = np.random.default_rng(3)
    shape = (3, 4, 5)
    x = _rand(rng, 5, *shape)
    t = _rand(rng, 5, *shape)
    params = [(0.3 * _rand(rng, 6, 5, 3, 3, 3), 0.1 * _rand(rng, 6)),
              (0.2 * _rand(rng, 6, 6, 3, 3, 3), 0.1 * _rand(rng, 6)),
              (0.2 * _rand(rng, 5, 6, 3, 3, 3), 0.1 * _rand(rng, 5))]

    def loss(ps):
        y, _ = cnn.forward(x, ps, bc)
        return cnn.mse_loss(y, t)[0]

    y, cache = cnn.forward(x, params, bc)
    _, dy = cnn.mse_loss(y, t)
    grads = cnn.backward(x, params, cache, dy, bc)
    h = 1e-6
    for layer in range(3):
        for which in range(2):
            p = params[layer][which]
            g = grads[layer][which]
            for _ in range(6):
                idx = tuple(int(rng.integers(0, s)) for s in p.shape)
                old = p[idx]
                p[idx] = old + h
                lp = loss(params)
                p[idx] = old - h
                lm = loss(params)
                p[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (layer, which, idx, fd, g[idx])


def test_mse_gradient_is_exact():
    rng = np.random.default_rng(4)
    y, t = _rand(rng, 5, 2, 2, 2), _rand(rng, 5, 2, 2, 2)
    L, g = cnn.mse_loss(y, t)
    assert L == pytest.approx(np.sum((y - t) ** 2) / y.size, rel=1e-15)
    np.testing.assert_allclose(g, 2 * (y - t) / y.size, rtol=1e-15)


def test_adam_first_step_is_a_signed_step_of_the_learning_rate():
    # after one step both bias-corrected moments are g and g^2, so the update
    # is lr g / (|g| + eps)
    rng = np.random.default_rng(5)
    p, g = _rand(rng, 50), _rand(rng, 50)
    q, m, v = cnn.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    np.testing.assert_allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_with_a_constant_gradient_moves_by_the_learning_rate_every_step():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -4.0])
    m = v = np.zeros(2)
    for step in range(1, 30):
        p_new, m, v = cnn.adam(p, g, m, v, step, lr=0.1)
        np.testing.assert_allclose(p - p_new, 0.1 * np.sign(g), rtol=1e-6)
        p = p_new


def test_restriction_conserves_totals_and_is_exact_on_linear_data():
    rng = np.random.default_rng(6)
    U = rng.random((5, 8, 6, 4)) + 0.5
    C = cnn.restrict2(U)
    assert C.shape == (5, 4, 3, 2)
    np.testing.assert_allclose(8.0 * C.sum(axis=(1, 2, 3)), U.sum(axis=(1, 2, 3)), rtol=1e-14)
    # linear data: the mean over a coarse cell is the value at its centre
    z, y, x = np.meshgrid(np.arange(8) + 0.5, np.arange(6) + 0.5, np.arange(4) + 0.5, indexing="ij")
    L = (1.5 + 0.25 * x - 0.5 * y + 0.125 * z)[None]
    zc, yc, xc = np.meshgrid(2 * np.arange(4) + 1.0, 2 * np.arange(3) + 1.0, 2 * np.arange(2) + 1.0,
                             indexing="ij")
    np.testing.assert_allclose(cnn.restrict2(L)[0], 1.5 + 0.25 * xc - 0.5 * yc + 0.125 * zc,
                               rtol=1e-15)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-5, 5, 1000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(x), ref)


def test_features_and_scales_of_a_hand_computed_state():
    # rho = 2, v = (1, -2, 0.5), p = 3, gamma = 1.4: E = 3 / 0.4 + 0.5 * 2 * 5.25
    gamma = 1.4
    U = np.array([2.0, 2.0, -4.0, 1.0, 7.5 + 5.25]).reshape(5, 1, 1, 1)
    f = cnn.features(U, gamma)[:, 0, 0, 0]
    np.testing.assert_allclose(f, [np.log(2.0), 1.0, -2.0, 0.5, np.log(3.0)], rtol=1e-14)
    s = cnn.scales(U, gamma)[:, 0, 0, 0]
    c = np.sqrt(1.4 * 3.0 / 2.0)
    np.testing.assert_allclose(s, [2.0, 2.0 * c, 2.0 * c, 2.0 * c, 12.75], rtol=1e-14)


def test_features_shift_under_mass_scaling():
    # rho, m, E -> lambda (rho, m, E) leaves v unchanged and shifts both logs
    rng = np.random.default_rng(8)
    rho = 0.5 + rng.random((2, 3, 4))
    v = rng.standard_normal((3, 2, 3, 4))
    p = 0.5 + rng.random((2, 3, 4))
    U = np.concatenate([rho[None], rho * v, (p / 0.4 + 0.5 * rho * np.sum(v * v, 0))[None]])
    f1, f2 = cnn.features(U, 1.4), cnn.features(7.0 * U, 1.4)
    np.testing.assert_allclose(f2[1:4], f1[1:4], rtol=1e-13)
    np.testing.assert_allclose(f2[[0, 4]] - f1[[0, 4]], np.log(7.0), rtol=1e-12)
    np.testing.assert_allclose(cnn.scales(7.0 * U, 1.4), 7.0 * cnn.scales(U, 1.4), rtol=1e-13)
