"""Pins of the warm-start oracle (resampling, network, loss gradient, AdamW)
against closed forms and finite differences -- no GPU."""
import math

import numpy as np
import pytest

from oracle import warmstart as W


def test_resample_closed_forms():
    # values linear in the index: the resampled curve is the same line at t_b (clamped)
    for r in (1, 7, 300, 512, 2000):
        a, b = 1.25, -0.375
        vals = a + b * np.arange(r)
        t = np.clip((np.arange(512) + 0.5) * r / 512 - 0.5, 0, r - 1)
        np.testing.assert_allclose(W.resample(vals), a + b * t, rtol=0, atol=1e-12)
    v = np.random.default_rng(0).standard_normal(512)
    assert np.array_equal(W.resample(v), v)                  # r = B: bins are the indices


def test_features_of_an_exponential_spectrum():
    r_c, r_g = 100, 3000
    Ec = np.exp(5.0 - 0.01 * np.arange(r_c))
    Eg = np.exp(6.0 - 0.002 * np.arange(r_g))
    f = W.features(Ec, Eg, 1_000_000, 20_000)
    assert f.shape == (W.D_IN,) == (1028,)
    tc = np.clip((np.arange(512) + 0.5) * r_c / 512 - 0.5, 0, r_c - 1)
    tg = np.clip((np.arange(512) + 0.5) * r_g / 512 - 0.5, 0, r_g - 1)
    np.testing.assert_allclose(f[:512], 5.0 - 0.01 * tc - 6.0, atol=1e-12)
    np.testing.assert_allclose(f[512:1024], 6.0 - 0.002 * tg - 6.0, atol=1e-12)
    np.testing.assert_allclose(f[1024:], [math.log(100), math.log(3000), math.log(1e6), math.log(2e4)])


def test_targets_then_apply_round_trip():
    rng = np.random.default_rng(1)
    # r = B: exact for any eigenvalues
    Ec, Eg = rng.random(512) + 0.5, rng.random(512) + 0.5
    lc, lg = rng.random(512) + 0.1, rng.random(512) + 0.1
    ac, ag = W.apply(W.targets(Ec, lc, Eg, lg), Ec, Eg)
    np.testing.assert_allclose(ac, lc, rtol=1e-13)
    np.testing.assert_allclose(ag, lg, rtol=1e-13)
    # r = 2B with log(lambda E) linear in the index: exact away from the two ends
    r = 1024
    E = rng.random(r) + 0.5
    lam = np.exp(0.3 - 0.004 * np.arange(r)) / E
    a, _ = W.apply(W.targets(E, lam, E, lam), E, E)
    np.testing.assert_allclose(a[1:-1], lam[1:-1], rtol=1e-12)


def test_silu_gradient_finite_difference():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (W.silu(z + h) - W.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(W.silu_grad(z), fd, rtol=1e-7, atol=1e-9)


def _small_problem(seed, batch=5):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(W.N_PARAMS) * 0.05
    X = rng.standard_normal((batch, W.D_IN))
    T = rng.standard_normal((batch, W.D_OUT))
    M = (rng.random((batch, W.D_OUT)) < 0.8).astype(np.float64)
    return theta, X, T, M


def test_loss_gradient_matches_finite_differences():
    theta, X, T, M = _small_problem(2)
    L, g = W.loss_and_grad(theta, X, T, M)
    assert abs(L - W.loss(theta, X, T, M)) <= 1e-14 * L
    rng = np.random.default_rng(3)
    # directional derivatives along random directions and single coordinates of every block
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in W.SHAPES])
    dirs = [rng.standard_normal(W.N_PARAMS) for _ in range(3)]
    for lo, hi in zip(offs[:-1], offs[1:]):
        e = np.zeros(W.N_PARAMS)
        e[rng.integers(lo, hi)] = 1.0
        dirs.append(e)
    h = 1e-5
    for d in dirs:
        fd = (W.loss(theta + h * d, X, T, M) - W.loss(theta - h * d, X, T, M)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd)), (fd, g @ d)


def test_output_layer_only_network_is_affine():
    """With W3 = 0 the outputs are b3 whatever the input; with W1 = W2 = 0 the hidden
    units are silu(b)."""
    theta, X, _, _ = _small_problem(4)
    P = W.unpack(theta)
    P["W3"][:] = 0
    np.testing.assert_allclose(W.forward(W.pack(P), X), np.tile(P["b3"], (X.shape[0], 1)), atol=0)
    P = W.unpack(theta)
    P["W1"][:] = 0
    P["W2"][:] = 0
    h2 = W.silu(P["b2"] + 0 * P["b1"].sum())
    # W2 = 0: the second hidden layer is silu(b2) for every input
    np.testing.assert_allclose(W.forward(W.pack(P), X), np.tile(P["W3"] @ h2 + P["b3"], (X.shape[0], 1)),
                               rtol=1e-12)


def test_adamw_first_step_closed_form():
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, wd = 1e-3, 1e-2
    t1, m1, v1 = W.adamw_step(theta, np.zeros(50), np.zeros(50), g, 1, lr, wd)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.001 * g * g)
    np.testing.assert_allclose(t1, theta - lr * (g / (np.abs(g) + 1e-8) + wd * theta), rtol=1e-12)


def test_parameter_count():
    assert W.N_PARAMS == 1028 * 256 + 256 + 256 * 256 + 256 + 1024 * 256 + 1024 == 592384


@pytest.mark.parametrize("wd", [0.0, 1e-2])
def test_adamw_constant_gradient_every_step(wd):
    """A constant gradient g: m_t = (1 - 0.9^t) g and v_t = (1 - 0.999^t) g^2, so
    the bias-corrected moments are g and g^2 at every step t and each update is
    lr (g / (|g| + eps) + wd theta); a wrong correction at any t > 1 breaks it."""
    rng = np.random.default_rng(6)
    theta0 = rng.standard_normal(40)
    g = rng.standard_normal(40)
    lr = 1e-3
    theta, m, v = theta0.copy(), np.zeros(40), np.zeros(40)
    want = theta0.copy()
    for t in range(1, 8):
        theta, m, v = W.adamw_step(theta, m, v, g, t, lr, wd)
        want = want - lr * (g / (np.abs(g) + 1e-8) + wd * want)
        np.testing.assert_allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)
        np.testing.assert_allclose(theta, want, rtol=1e-12, atol=1e-15)


def test_adamw_alternating_gradient_closed_form():
    """g_t = (-1)^(t+1) g: m_t = 0.1 g (-1)^(t+1) (1 - (-0.9)^t) / 1.9 (a geometric
    sum), v_t = (1 - 0.999^t) g^2; the update uses m_t / (1 - 0.9^t) and |g|."""
    rng = np.random.default_rng(7)
    theta0 = rng.standard_normal(30)
    g = rng.standard_normal(30)
    lr, wd = 2e-3, 0.0
    theta, m, v = theta0.copy(), np.zeros(30), np.zeros(30)
    want = theta0.copy()
    for t in range(1, 7):
        gt = g if t % 2 == 1 else -g
        theta, m, v = W.adamw_step(theta, m, v, gt, t, lr, wd)
        m_t = 0.1 * g * (-1) ** (t + 1) * (1 - (-0.9) ** t) / 1.9
        np.testing.assert_allclose(m, m_t, rtol=1e-12, atol=1e-15)
        mh = m_t / (1 - 0.9 ** t)
        want = want - lr * mh / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(theta, want, rtol=1e-12, atol=1e-15)


def test_bf16_rounding_against_the_definition():
    """The BF16-weight mode's rounding: the nearest value with 8 significant bits
    (ties to even), from the FP32 value, brute force over a grid."""
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.standard_normal(500) * 10.0 ** rng.integers(-5, 5, 500),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 0.0, 1 + 2 ** -9]])
    got = W.bf16(x)
    for v, g in zip(x, got):
        f = float(np.float32(v))
        if f == 0.0:
            assert g == 0.0
            continue
        e = math.floor(math.log2(abs(f)))
        ulp = 2.0 ** (e - 7)
        lo = math.floor(f / ulp) * ulp
        cands = [lo, lo + ulp]
        d = [abs(c - f) for c in cands]
        if d[0] == d[1]:
            want = cands[0] if round(cands[0] / ulp) % 2 == 0 else cands[1]
        else:
            want = cands[int(np.argmin(d))]
        assert g == want, (v, g, want)


def test_bf16_mode_error_is_the_rounding_of_its_operands():
    """With the inputs and the output weights already BF16 values and the hidden
    weights zero, the only operand the BF16 mode rounds is the constant hidden
    row silu(b2): the outputs then differ from the full mode by at most one BF16
    rounding (2^-8 relative) of it, per output weight row, and do differ."""
    theta, X, T, _ = _small_problem(5)
    P = W.unpack(theta)
    P["W1"][:] = 0
    P["W2"][:] = 0
    P["W3"] = W.bf16(P["W3"])
    th = W.pack(P)
    Xb = W.bf16(X)
    h2 = W.silu(P["b2"])
    Y0 = W.forward(th, Xb)
    Y1 = W.forward(th, Xb, low=True)
    bound = 2.0 ** -8 * (np.abs(P["W3"]) @ np.abs(h2))
    assert np.all(np.abs(Y0 - Y1) <= bound[None, :] * (1 + 1e-12))
    assert np.max(np.abs(Y0 - Y1)) > 0
