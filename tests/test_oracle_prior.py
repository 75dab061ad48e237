"""Pins for the oracle's lognormal prior construction (section 2.3:
S_L(r) = ln(1 + S(r)), mu = -sigma0^2 / 2, sigma0^2 = S_L(0))."""
import numpy as np
import pytest

from oracle import dft, prior
from paper_0911_1407_amd import synth


def _full_from_half(half, n):
    """Full spectrum of a real field from its half spectrum (Hermitian)."""
    full = np.zeros(n, dtype=np.complex128)
    h = n[2] // 2 + 1
    for kx in range(n[0]):
        for ky in range(n[1]):
            for kz in range(n[2]):
                if kz < h:
                    full[kx, ky, kz] = half[kx, ky, kz]
                else:
                    full[kx, ky, kz] = np.conj(half[(-kx) % n[0], (-ky) % n[1], n[2] - kz])
    return full


def test_white_spectrum_closed_form():
    # lambda_k = sigma^2 for every k: S(r) = sigma^2 at r = 0 and 0 elsewhere,
    # so S_L = ln(1 + sigma^2) at r = 0 and every lambda^L_k = ln(1 + sigma^2)
    n, box, sigma2 = (8, 12, 10), (16.0, 24.0, 20.0), 0.9
    N, V = np.prod(n), np.prod(box)
    pk = np.full((n[0], n[1], n[2] // 2 + 1), sigma2 * V / N)
    pl, mu, s0, nc = prior.lognormal_prior(n, box, pk, 1.0)
    assert np.allclose(pl * N / V, np.log1p(sigma2), rtol=1e-13, atol=0)
    assert s0 == pytest.approx(np.log1p(sigma2), rel=1e-14)
    assert mu == pytest.approx(-0.5 * np.log1p(sigma2), rel=1e-14)
    assert nc == 0


def test_correlation_function_is_the_dense_inverse_dft():
    n, box = (8, 8, 8), (40.0,) * 3
    pk = synth.power_shape_half(n, box)
    S = prior.correlation_function(n, box, pk, 3.0)
    lam_half = 3.0 * pk * np.prod(n) / np.prod(box)
    ref = dft.idftn(_full_from_half(lam_half, n))
    assert np.abs(ref.imag).max() <= 1e-14 * np.abs(ref.real).max()
    assert np.abs(S - ref.real).max() <= 1e-13 * np.abs(ref.real).max()
    # S(0) is the cell variance (1/V) sum over all modes of A pk
    assert S[0, 0, 0] == pytest.approx(np.sum(_full_from_half(3.0 * pk, n).real) / np.prod(box), rel=1e-13)


def test_second_order_expansion():
    # ln(1 + S) = S - S^2/2 + O(S^3): lambda^L = lambda - (1/2N) (lambda (*) lambda) + O(eps^3),
    # (*) the circular convolution over the full spectrum
    n, box = (8, 8, 8), (40.0,) * 3
    N, V = np.prod(n), np.prod(box)
    pk = synth.power_shape_half(n, box)
    errs = []
    for eps in (1e-2, 1e-3):
        amp = eps / (np.sum(_full_from_half(pk, n).real) / V)  # S(0) = eps
        pl, mu, s0, nc = prior.lognormal_prior(n, box, pk, amp)
        lam = _full_from_half(amp * pk * N / V, n).real
        conv = np.real(np.fft.ifftn(np.fft.fftn(lam) ** 2))  # sum_q lam_q lam_{k-q}
        pred = lam - 0.5 * conv / N
        got = _full_from_half(pl * N / V, n).real
        # k = 0: pk_0 = 0, and the log transform makes lambda^L_0 negative
        # (raised to the floor), so it is left out
        m = np.ones(n, dtype=bool)
        m[0, 0, 0] = False
        err2 = np.abs(got - pred)[m].max() / np.abs(lam).max()
        err1 = np.abs(got - lam)[m].max() / np.abs(lam).max()
        assert err2 <= 0.01 * err1  # the second-order term is the leading correction
        errs.append(err2)
        assert s0 == pytest.approx(np.log1p(eps), rel=1e-12)
    # relative third-order remainder: ~eps^2, so 100x smaller for a 10x smaller eps
    assert errs[1] <= errs[0] / 50.0
    assert errs[0] <= 1e-4


def test_domain_error_below_minus_one():
    n, box = (8, 8, 8), (8.0,) * 3
    pk = np.zeros((8, 8, 5))
    pk[4, 0, 0] = 1.0  # a single Nyquist mode: S(r) = +-A/N alternates in sign
    prior.lognormal_prior(n, box, pk, 256.0)  # |S| = 1/2: defined
    with pytest.raises(ValueError):
        prior.lognormal_prior(n, box, pk, 1024.0)  # S = -2 at odd x
