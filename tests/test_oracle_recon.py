"""Pins of the oracle's lossy stage (Section 4.2: dequantization + inverse
DCT per window) and of its analytic backward (gradients of the MSE with
respect to the per-zone scales and the coefficients)."""
import numpy as np
import pytest
import scipy.fft as sfft

import synth


def _stream(O, domain, L, N=64, E=64, kind="amp", seed=0):
    p = O.QuantParams(kind, N, E) if kind == "amp" else O.QuantParams(kind, N, E, B1=2, B2=E // 2, A0=40.0, A1=10.0)
    x = synth.domain_signal(domain, L, synth.stream_rng(7, seed)).astype(np.float32)
    return p, x, O.quantize_stream(x, p)


@pytest.mark.parametrize("L,N,E,kind", [(64 * 40, 64, 64, "amp"), (64 * 40 + 13, 64, 64, "amp"),
                                        (32 * 50 + 31, 32, 16, "paper"), (128 * 9 + 1, 128, 96, "amp")])
def test_reconstruct_matches_scipy_idct(O, L, N, E, kind):
    p, x, sym = _stream(O, "eeg", L, N, E, kind)
    v, z = O.dequant_table(p)
    nw = O.n_windows(L, N)
    C = np.zeros((nw, N))
    C[:, :E] = v[np.arange(E)[None, :], sym.reshape(nw, E)]
    ref = sfft.idct(C, type=2, norm="ortho", axis=1).ravel()[:L]
    np.testing.assert_allclose(O.reconstruct(sym, L, p), ref, rtol=0, atol=1e-10)


def test_reconstruction_error_is_quantization_error(O):
    # Parseval: with E = N and L a multiple of N, the time-domain error energy
    # equals the coefficient-domain error energy.
    p, x, sym = _stream(O, "meteo", 64 * 64)
    xh = O.reconstruct(sym, x.size, p)
    X = O.dct_stream(x, 64, 64)
    v, _ = O.dequant_table(p)
    ch = v[np.tile(np.arange(64), 64), sym]
    e_t = np.sum((xh - x.astype(np.float64)) ** 2)
    assert abs(e_t - np.sum((X - ch) ** 2)) <= 1e-9 * max(1.0, e_t)
    assert O.prd(x, xh) == pytest.approx(100 * np.sqrt(e_t / np.sum(x.astype(np.float64) ** 2)), rel=1e-12)


def test_gamma_is_linear_per_zone(O):
    p, x, sym = _stream(O, "eeg", 64 * 30 + 5)
    g = np.array([0.7, 1.3, 0.9])
    parts = [O.reconstruct(sym, x.size, p, np.eye(3)[z]) for z in range(3)]
    np.testing.assert_allclose(O.reconstruct(sym, x.size, p, g), sum(g[z] * parts[z] for z in range(3)), atol=1e-10)
    np.testing.assert_allclose(parts[0], 0.0)  # the zero zone carries no value


def _loss(O, sym, x, p, gamma, M):
    d = O.reconstruct(sym, x.size, p, gamma) - x.astype(np.float64)
    return float(np.sum(d * d)) / M


@pytest.mark.parametrize("kind,domain", [("amp", "power"), ("amp", "meteo"), ("paper", "eeg")])
def test_gamma_gradient_matches_central_differences(O, kind, domain):
    p, x, sym = _stream(O, domain, 128 * 20 + 9, N=128, E=128 if kind == "amp" else 64, kind=kind)
    M = x.size
    gamma = np.array([1.1, 0.95, 1.05])
    d = O.reconstruct(sym, x.size, p, gamma) - x.astype(np.float64)
    _, gg = O.backward(sym, x.size, p, 2.0 * d / M)
    h = 1e-6
    for z in range(3):
        e = np.eye(3)[z] * h
        fd = (_loss(O, sym, x, p, gamma + e, M) - _loss(O, sym, x, p, gamma - e, M)) / (2 * h)
        assert abs(fd - gg[z]) <= 1e-6 * max(1.0, abs(gg[z])), (z, fd, gg[z])


def test_coefficient_gradient_matches_central_differences(O):
    p, x, sym = _stream(O, "eeg", 64 * 6 + 20)
    L, N, E = x.size, 64, 64
    v, _ = O.dequant_table(p)
    nw = O.n_windows(L, N)
    C = v[np.tile(np.arange(E), nw), sym].reshape(nw, E)

    def loss_of(Cm):
        xh = np.concatenate([O.idct_ortho(Cm[w], N, E) for w in range(nw)])[:L]
        return float(np.sum((xh - x.astype(np.float64)) ** 2)) / L

    xh = np.concatenate([O.idct_ortho(C[w], N, E) for w in range(nw)])[:L]
    gc, _ = O.backward(sym, L, p, 2.0 * (xh - x.astype(np.float64)) / L)
    gc = gc.reshape(nw, E)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(40):
        w, k = int(rng.integers(nw)), int(rng.integers(E))
        Cp, Cm = C.copy(), C.copy()
        Cp[w, k] += h
        Cm[w, k] -= h
        fd = (loss_of(Cp) - loss_of(Cm)) / (2 * h)
        assert abs(fd - gc[w, k]) <= 1e-6 * max(1.0, abs(gc[w, k])), (w, k)
    # the padded tail of the last window carries no gradient: gc of bins is still defined,
    # and zeroing the output gradient past L is what the backward does
    assert np.all(np.isfinite(gc))


def test_closed_form_optimal_gamma_zeroes_gradient(O):
    # Zones are disjoint and the basis orthonormal, so the MSE is a separable
    # quadratic in gamma: gamma*_z = sum_z v X / sum_z v^2 (L a multiple of N).
    p, x, sym = _stream(O, "power", 128 * 64, N=128, E=128)
    X = O.dct_stream(x, 128, 128)
    v, zt = O.dequant_table(p)
    kk = np.tile(np.arange(128), 64)
    vv, zz = v[kk, sym], zt[kk, sym]
    gstar = np.ones(3)
    for z in (1, 2):
        den = np.sum(vv[zz == z] ** 2)
        if den > 0:
            gstar[z] = np.sum(vv[zz == z] * X[zz == z]) / den
    d = O.reconstruct(sym, x.size, p, gstar) - x.astype(np.float64)
    _, gg = O.backward(sym, x.size, p, 2.0 * d / x.size)
    scale = np.sum(np.abs(vv * X)) / x.size
    assert np.all(np.abs(gg[1:]) <= 1e-10 * scale)
    assert gg[0] == 0.0  # zone 0 (the zero level) has v == 0 exactly


def test_adam_refit_lowers_loss(O):
    streams = []
    for i, dom in enumerate(["power", "meteo"]):
        p, x, sym = _stream(O, dom, 128 * 16, N=128, E=128, seed=i)
        streams.append((sym, x))
    gamma, losses = O.adam_refit(streams, p, steps=20)
    assert losses[-1] <= losses[0]
    assert gamma.shape == (2, 3)


def _refit_streams(O):
    streams = []
    for i, dom in enumerate(["power", "meteo", "power"]):
        p, x, sym = _stream(O, dom, 128 * 16, N=128, E=128, seed=i)
        streams.append((sym, x))
    return p, streams


def _gamma_star(O, p, sym, x):
    """Closed-form optimum of the separable quadratic loss of one stream
    (zones disjoint, basis orthonormal, L a multiple of N): per zone,
    sum v X / sum v^2 over that zone's coefficients; 1 where a zone is empty."""
    X = O.dct_stream(x, p.N, p.E)
    v, zt = O.dequant_table(p)
    kk = np.tile(np.arange(p.E), x.size // p.N)
    vv, zz = v[kk, sym], zt[kk, sym]
    g = np.ones(3)
    for z in range(3):
        den = np.sum(vv[zz == z] ** 2)
        if den > 0:
            g[z] = np.sum(vv[zz == z] * X[zz == z]) / den
    return g


def test_adam_first_step_closed_form(O):
    # At t = 1 both moment estimates are exact after bias correction
    # (m_hat = g, v_hat = g^2), so Adam moves every scale by exactly
    # lr * g / (|g| + eps): a step of about lr against the gradient's sign,
    # and none where the gradient is zero.
    p, streams = _refit_streams(O)
    M = sum(x.size for _, x in streams)
    lr, eps = 1e-2, 1e-8
    gamma, losses = O.adam_refit(streams, p, steps=1, lr=lr, eps=eps)
    for i, (sym, x) in enumerate(streams):
        d = O.reconstruct(sym, x.size, p, np.ones(3)) - x.astype(np.float64)
        _, g = O.backward(sym, x.size, p, 2.0 * d / M, want_coef=False)
        expect = 1.0 - lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(gamma[i], expect, rtol=0, atol=1e-15)
        assert gamma[i][0] == 1.0  # zone 0 is the zero level: v == 0, no gradient
    assert len(losses) == 2


def test_adam_refit_matches_torch_adam_fp64(O):
    # Same 20 full-batch steps with torch.optim.Adam (FP64, CPU) fed the
    # oracle's gradients: an independent implementation of the update rule
    # (bias corrections, beta1/beta2 roles, eps outside the square root).
    import torch
    p, streams = _refit_streams(O)
    M = sum(x.size for _, x in streams)
    gamma, losses = O.adam_refit(streams, p, steps=20)
    gt = torch.ones((len(streams), 3), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([gt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    tl = []
    for _ in range(20):
        opt.zero_grad()
        g = np.zeros((len(streams), 3))
        loss = 0.0
        cur = gt.detach().numpy().copy()
        for i, (sym, x) in enumerate(streams):
            d = O.reconstruct(sym, x.size, p, cur[i]) - x.astype(np.float64)
            loss += float(np.sum(d * d))
            g[i] = O.backward(sym, x.size, p, 2.0 * d / M, want_coef=False)[1]
        tl.append(loss / M)
        gt.grad = torch.from_numpy(g)
        opt.step()
    np.testing.assert_allclose(gamma, gt.detach().numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(losses[:20], tl, rtol=1e-12)


def test_adam_refit_bounded_by_closed_form_optimum(O):
    # The loss is a separable quadratic in gamma with a closed-form minimum
    # L(gamma*), so no iterate may go below it; 20 steps of lr 1e-2 from
    # gamma = 1 must also close part of the gap.
    p, streams = _refit_streams(O)
    M = sum(x.size for _, x in streams)
    gamma, losses = O.adam_refit(streams, p, steps=20)
    lstar = 0.0
    gs = []
    for sym, x in streams:
        g = _gamma_star(O, p, sym, x)
        gs.append(g)
        lstar += float(np.sum((O.reconstruct(sym, x.size, p, g) - x.astype(np.float64)) ** 2))
    lstar /= M
    assert all(l >= lstar * (1 - 1e-12) for l in losses)
    assert losses[-1] < losses[0]
    assert losses[-1] - lstar < losses[0] - lstar
    # a zone whose optimum lies far from 1 (beyond what the steps can overshoot)
    # has moved toward it
    gs = np.array(gs)
    far = np.abs(gs - 1.0) > 0.05
    assert far.any()
    assert np.all(np.sign(gamma - 1.0)[far] == np.sign(gs - 1.0)[far])
    assert np.all(np.abs(gamma - gs)[far] < np.abs(1.0 - gs)[far])
    print(f"L(gamma=1) {losses[0]:.6e}  L(after 20 Adam steps) {losses[-1]:.6e}  L(gamma*) {lstar:.6e}")
