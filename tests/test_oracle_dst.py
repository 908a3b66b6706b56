"""Pins for the oracle's naive DST-I (CPU): library routine, involution, Parseval."""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import dst


@pytest.mark.parametrize("N", [4, 6, 32, 96, 128, 384])
def test_naive_dst_matches_library(N):
    x = np.random.default_rng(N).standard_normal(N - 1)
    # scipy's DST-I of length N-1 is 2 * sum_m x_m sin(pi k m / N)
    ref = sfft.dst(x, type=1) / 2
    assert np.allclose(dst.dst1(x), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("N", [8, 64, 192])
def test_involution(N):
    S = dst.sine_matrix(N)
    assert np.abs(S @ S - (N / 2) * np.eye(N - 1)).max() < 1e-11 * N


@pytest.mark.parametrize("dim", [1, 2])
def test_parseval_corollary1(dim):
    # h^{d-1} sum |g|^2 = 2^{1-d} sum |g_hat|^2, g_hat = (2/N)^{d-1} S^{(x)} g (Corollary 1,
    # written for the (d-1)-dimensional face data; here d-1 = dim)
    N = 24
    h = 1.0 / N
    g = np.random.default_rng(3).standard_normal((N - 1,) * dim)
    gh = g
    for ax in range(dim):
        gh = dst.dst1(gh, axis=ax)
    gh = gh * (2.0 / N) ** dim
    lhs = h ** dim * np.sum(g ** 2)
    rhs = np.sum(gh ** 2) / 2 ** dim
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_single_mode():
    N = 16
    m = np.arange(1, N)
    for k in (1, 5, 15):
        X = dst.dst1(np.sin(np.pi * k * m / N))
        e = np.zeros(N - 1)
        e[k - 1] = N / 2
        assert np.abs(X - e).max() < 1e-13
