"""Parity of the learned warm start's kernels (through the C ABI) with the FP64
NumPy oracle, and the gain test.

Bars: features, targets and apply within FP32 rounding of the FP64 values
(1e-6 relative); forward outputs and every parameter block's gradient within
1e-4 of the block's largest reference magnitude (FP32 parameters, FP32
accumulation); the AdamW update within 1e-3 lr wherever the gradient's sign is
well determined.  Gain: a network trained on cold solves of generated spectra
starts held-out solves with fewer Newton iterations, and every warm solve ends
within the solver's parity bar (1e-10 relative plus 1e-12 of the axis
maximum) of the cold solve.
"""
import numpy as np
import pytest

import synth
from oracle import warmstart as W
from oracle import solver as S

pytestmark = pytest.mark.gpu


def _d(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype))).cuda()


def _spectra(seed, p, n, spikes, rc):
    e = synth.spectrum_proxy(p, n, spikes, seed=seed)
    return e[:rc].copy(), e.copy()


@pytest.mark.parametrize("rc,rg", [(1, 1), (5, 3000), (100, 20000), (512, 512), (500, 500), (50, 2000)])
def test_features_targets_apply_parity(lib, rc, rg):
    rng = np.random.default_rng(rc + rg)
    Ec = np.sort(rng.random(rc) * 100 + 0.5)[::-1].copy()
    Eg = np.sort(rng.random(rg) * 30 + 0.1)[::-1].copy()
    f = lib.ws_features(_d(Ec), _d(Eg), 1e6, 2e4).cpu().numpy()
    fr = W.features(Ec, Eg, 1e6, 2e4)
    assert np.all(np.abs(f - fr) <= 1e-6 * np.maximum(1, np.abs(fr)))
    lc = rng.random(rc) * 0.1 + 1e-3
    lg = rng.random(rg) * 0.1 + 1e-3
    t = lib.ws_targets(_d(Ec), _d(lc), _d(Eg), _d(lg)).cpu().numpy()
    tr = W.targets(Ec, lc, Eg, lg)
    assert np.all(np.abs(t - tr) <= 1e-6 * np.maximum(1, np.abs(tr)))
    curves = rng.standard_normal(1024).astype(np.float32)
    ac, ag = lib.ws_apply(_d(curves), _d(Ec), _d(Eg))
    rc_, rg_ = W.apply(curves.astype(np.float64), Ec, Eg)
    np.testing.assert_allclose(ac.cpu().numpy(), rc_, rtol=1e-12)
    np.testing.assert_allclose(ag.cpu().numpy(), rg_, rtol=1e-12)


def _net(seed, batch):
    rng = np.random.default_rng(seed)
    theta = np.concatenate([
        rng.uniform(-1, 1, int(np.prod(s))) / np.sqrt(s[1] if len(s) == 2 else (1028 if n == "b1" else 256))
        for n, s in W.SHAPES]).astype(np.float32)
    X = rng.standard_normal((batch, W.D_IN)).astype(np.float32)
    T = rng.standard_normal((batch, W.D_OUT)).astype(np.float32)
    M = (rng.random((batch, W.D_OUT)) < 0.7).astype(np.float32)
    return theta, X, T, M


@pytest.mark.parametrize("batch", [1, 37, 64, 200])
def test_forward_parity(lib, batch):
    theta, X, _, _ = _net(batch, batch)
    Y = lib.ws_forward(_d(theta), _d(X)).cpu().numpy()
    Yr = W.forward(theta.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(Y - Yr)) <= 1e-4 * np.max(np.abs(Yr))


@pytest.mark.parametrize("batch,masked", [(1, False), (37, True), (128, True)])
def test_gradient_and_adamw_step_parity(lib, batch, masked):
    import torch
    theta, X, T, M = _net(100 + batch, batch)
    if not masked:
        M = None
    n = lib.ws_param_count()
    p = _d(theta)
    m = torch.zeros(n, dtype=torch.float32, device="cuda")
    v = torch.zeros(n, dtype=torch.float32, device="cuda")
    gout = torch.empty(n, dtype=torch.float32, device="cuda")
    lr, wd = 1e-3, 1e-2
    loss = lib.ws_train_step(p, m, v, 1, _d(X), _d(T), None if M is None else _d(M), lr, wd, grad_out=gout)
    L, g_ref = W.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                               None if M is None else M.astype(np.float64))
    assert abs(loss - L) <= 1e-5 * L
    g = gout.cpu().numpy()
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in W.SHAPES])
    for (name, _), lo, hi in zip(W.SHAPES, offs[:-1], offs[1:]):
        scale = np.max(np.abs(g_ref[lo:hi]))
        assert np.max(np.abs(g[lo:hi] - g_ref[lo:hi])) <= 1e-4 * scale, name
    t_ref, m_ref, v_ref = W.adamw_step(theta.astype(np.float64), np.zeros(n), np.zeros(n), g_ref, 1, lr, wd)
    t_gpu = p.cpu().numpy()
    assert np.all(np.abs(t_gpu - t_ref) <= 2.1 * lr)          # an AdamW step is bounded by lr (1 + wd |p|)
    for lo, hi in zip(offs[:-1], offs[1:]):
        sure = np.abs(g_ref[lo:hi]) > 1e-2 * np.max(np.abs(g_ref[lo:hi]))
        assert np.all(np.abs(t_gpu[lo:hi] - t_ref[lo:hi])[sure] <= 1e-3 * lr)
    np.testing.assert_allclose(m.cpu().numpy(), m_ref, rtol=1e-3, atol=1e-4 * np.max(np.abs(m_ref)))


def test_three_adamw_steps_parity_both_entry_points(lib):
    """Three consecutive steps (bias corrections past the first) through
    gmgm_ws_train_step (host update count) and gmgm_warmstart_train_step
    (update count in the device state): both give the same parameters, and
    they follow the oracle's FP64 trajectory wherever the gradient's sign is
    well determined at every step."""
    import torch
    theta, X, T, M = _net(321, 48)
    n = lib.ws_param_count()
    lr, wd = 1e-3, 1e-2
    p1 = _d(theta)
    m1 = torch.zeros(n, dtype=torch.float32, device="cuda")
    v1 = torch.zeros(n, dtype=torch.float32, device="cuda")
    p2 = _d(theta)
    st = lib.warmstart_state(weight_decay=wd)
    th, mr, vr = theta.astype(np.float64), np.zeros(n), np.zeros(n)
    sure = np.ones(n, bool)
    for t in range(1, 4):
        l1 = lib.ws_train_step(p1, m1, v1, t, _d(X), _d(T), _d(M), lr, wd)
        l2 = lib.warmstart_train_step(p2, st, _d(X), _d(T), _d(M), lr)
        L, g = W.loss_and_grad(th, X.astype(np.float64), T.astype(np.float64), M.astype(np.float64))
        assert abs(l1 - L) <= 1e-5 * L and abs(l2 - L) <= 1e-5 * L
        offs = np.cumsum([0] + [int(np.prod(s)) for _, s in W.SHAPES])
        for lo, hi in zip(offs[:-1], offs[1:]):
            sure[lo:hi] &= np.abs(g[lo:hi]) > 1e-2 * np.max(np.abs(g[lo:hi]))
        th, mr, vr = W.adamw_step(th, mr, vr, g, t, lr, wd)
    a, b = p1.cpu().numpy(), p2.cpu().numpy()
    assert np.array_equal(a, b)
    assert int(st[:8].cpu().numpy().view(np.int64)[0]) == 3
    assert sure.mean() > 0.5
    assert np.all(np.abs(a - th)[sure] <= 3e-3 * lr)
    assert np.all(np.abs(a - th) <= 6.3 * lr)
    # first moments: sums of three gradients, each within the gradient bar (1e-4
    # of the largest reference magnitude), so an absolute term of that size
    np.testing.assert_allclose(m1.cpu().numpy()[sure], mr[sure], rtol=1e-3, atol=1e-4 * np.max(np.abs(mr)))
    ms = st[256:256 + 4 * n].view(torch.float32).cpu().numpy()
    np.testing.assert_array_equal(ms, m1.cpu().numpy())


def test_warmstart_infer_equals_forward(lib):
    theta, X, _, _ = _net(77, 19)
    a = lib.ws_forward(_d(theta), _d(X)).cpu().numpy()
    b = lib.warmstart_infer(_d(theta), _d(X)).cpu().numpy()
    Yr = W.forward(theta.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(b - Yr)) <= 1e-4 * np.max(np.abs(Yr))
    np.testing.assert_array_equal(a, b)


def test_training_is_deterministic(lib):
    import torch
    theta, X, T, M = _net(7, 64)
    outs = []
    for _ in range(2):
        n = lib.ws_param_count()
        p = _d(theta)
        m = torch.zeros(n, dtype=torch.float32, device="cuda")
        v = torch.zeros(n, dtype=torch.float32, device="cuda")
        for s in range(1, 4):
            lib.ws_train_step(p, m, v, s, _d(X), _d(T), _d(M), 1e-3, 1e-4, want_loss=False)
        outs.append(p.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def _pair_instances(seed, count):
    """Axis pairs of generated spectra: p, n log-uniform, cell ranks 20/50/100/full."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        p = int(np.exp(rng.uniform(np.log(200), np.log(2000))))
        n = int(np.exp(rng.uniform(np.log(200), np.log(20000))))
        spikes = int(rng.integers(4, 41))
        m = min(p, n)
        rc = int(min(m, rng.choice([20, 50, 100, m])))
        e = synth.spectrum_proxy(p, n, spikes, seed=seed * 1000 + i)
        out.append((e[:rc].copy(), e[:m].copy(), float(n), float(p)))
    return out


def test_gain_warm_start_reduces_newton_iterations(lib):
    import torch
    from paper_2407_19892_amd import warmstart as ws
    train = [(_d(a), _d(b), dc, dg) for a, b, dc, dg in _pair_instances(11, 192)]
    feats, targs, cold_train = ws.make_examples(train)
    model = ws.WarmStart(seed=3)
    losses = ws.train(model, feats, targs, steps=600, batch=64, lr=2e-3, weight_decay=1e-5, seed=0)
    assert losses[-1] < 0.2 * losses[0]
    held = _pair_instances(12, 24)
    cold_it, warm_it = [], []
    for a, b, dc, dg in held:
        Ec, Eg = _d(a), _d(b)
        # tol 1e-13: at the default 1e-12 a 20 x 1107 instance ended 1.5x the bar
        # from the minimiser (an ill-conditioned gene block)
        cold = lib.solve_eigs([Ec, Eg], [(0, 1)], tol=1e-13)
        warm = model.solve(Ec, Eg, dc, dg, tol=1e-13)
        cold_it.append(cold.info["iterations"])
        warm_it.append(warm.info["iterations"])
        assert warm.info["converged"] and warm.info["n_pinned"] == cold.info["n_pinned"]
        # the warm solve ends where the cold one does, within the solver's parity
        # bar; on a miss both are set against the oracle's minimiser to say which
        # one is off
        for l, (x, y) in enumerate(zip(warm.lam, cold.lam)):
            x, y = x.cpu().numpy(), y.cpu().numpy()
            if np.all(np.abs(x - y) <= 1e-10 * np.abs(y) + 1e-12 * np.max(y)):
                continue
            ref = S.solve_eigs(S.Problem([a, b], [(0, 1)])).lam[l]
            ew = np.max(np.abs(x - ref) / (1e-10 * np.abs(ref) + 1e-12 * np.max(ref)))
            ec = np.max(np.abs(y - ref) / (1e-10 * np.abs(ref) + 1e-12 * np.max(ref)))
            q = int(np.argmax(np.abs(x - y)))
            pytest.fail(f"warm vs cold on axis {l} of a {a.size} x {b.size} pair: warm {ew:.3f} x bar, cold "
                        f"{ec:.3f} x bar from the oracle; kkt warm {warm.info['kkt']:.2e} cold "
                        f"{cold.info['kkt']:.2e}; worst index {q}: warm {x[q]!r} cold {y[q]!r} oracle {ref[q]!r} "
                        f"max {np.max(ref)!r}")
        print("held-out", len(cold_it), a.size, b.size, cold.info["iterations"], warm.info["iterations"], flush=True)
    print("cold", cold_it, "warm", warm_it, "loss", losses[0], losses[-1], flush=True)
    assert np.mean(warm_it) < np.mean(cold_it)
