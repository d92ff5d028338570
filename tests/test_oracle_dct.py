"""Pins of the oracle's transform (Section 3.1, Eq. 1) against scipy, closed
forms and invariants."""
import numpy as np
import pytest
import scipy.fft as sfft


@pytest.mark.parametrize("N", [4, 8, 16, 32, 64, 128, 256])
def test_dct_matches_scipy_ortho(O, N):
    x = np.random.default_rng(N).standard_normal(N) * 10
    np.testing.assert_allclose(O.dct_ortho(x), sfft.dct(x, type=2, norm="ortho"), rtol=0, atol=1e-11)
    X = np.random.default_rng(N + 1).standard_normal(N)
    np.testing.assert_allclose(O.idct_ortho(X, N), sfft.idct(X, type=2, norm="ortho"), rtol=0, atol=1e-11)


@pytest.mark.parametrize("N", [4, 32, 64, 256])
def test_eq1_scaling_is_unnormalised_dct_over_N(O, N):
    # scipy's unnormalised DCT-II is 2 * sum x cos(...); Eq. (1) is (2/N) * sum x cos(...).
    x = np.random.default_rng(3).standard_normal(N)
    np.testing.assert_allclose(O.dct_eq1(x), sfft.dct(x, type=2, norm=None) / N, atol=1e-12)


@pytest.mark.parametrize("N", [4, 64, 128, 256])
def test_round_trip_and_orthonormal_basis(O, N):
    x = np.random.default_rng(5).standard_normal(N) * 100
    assert np.max(np.abs(O.idct_ortho(O.dct_ortho(x), N) - x)) <= 1e-12 * np.max(np.abs(x)) * N
    B = np.stack([O.dct_ortho(np.eye(N)[n]) for n in range(N)], axis=1)  # B[k, n]
    np.testing.assert_allclose(B @ B.T, np.eye(N), atol=1e-13)
    # Parseval
    X = O.dct_ortho(x)
    assert abs(np.sum(x * x) - np.sum(X * X)) <= 1e-12 * np.sum(x * x)


@pytest.mark.parametrize("N,k0", [(8, 0), (8, 3), (64, 1), (64, 17), (256, 255)])
def test_cosine_at_bin_is_a_delta(O, N, k0):
    n = np.arange(N)
    x = np.cos(np.pi / N * (n + 0.5) * k0)
    X = O.dct_ortho(x)
    expect = np.zeros(N)
    expect[k0] = np.sqrt(N) if k0 == 0 else np.sqrt(N / 2.0)  # a_k * sum cos^2
    np.testing.assert_allclose(X, expect, atol=1e-11)


@pytest.mark.parametrize("N,E", [(32, 16), (64, 1), (64, 63)])
def test_truncated_inverse_zeroes_high_bins(O, N, E):
    X = np.random.default_rng(9).standard_normal(N)
    Xz = X.copy()
    Xz[E:] = 0.0
    np.testing.assert_allclose(O.idct_ortho(X[:E], N, E), sfft.idct(Xz, type=2, norm="ortho"), atol=1e-12)


def test_stream_windows_and_zero_padded_tail(O):
    N, E = 16, 16
    L = 5 * N + 7
    x = np.random.default_rng(1).standard_normal(L).astype(np.float32)
    coef = O.dct_stream(x, N, E).reshape(-1, E)
    assert coef.shape[0] == 6
    pad = np.zeros(6 * N)
    pad[:L] = x
    np.testing.assert_allclose(coef, sfft.dct(pad.reshape(6, N), type=2, norm="ortho", axis=1), atol=1e-12)


@pytest.mark.parametrize("N,E", [(4, 4), (64, 64), (64, 20), (256, 256)])
def test_table_transforms_equal_per_term_transforms_bitwise(O, N, E):
    # stream-level routines use a precomputed cosine table; it must change nothing
    rng = np.random.default_rng(N + E)
    for _ in range(5):
        x = rng.standard_normal(N) * 100
        assert np.array_equal(O.dct_ortho_tab(x), O.dct_ortho(x))
        X = rng.standard_normal(E) * 100
        assert np.array_equal(O.idct_ortho_tab(X, N, E), O.idct_ortho(X, N, E))
