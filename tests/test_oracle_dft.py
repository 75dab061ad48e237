"""Pins for the oracle's Fourier conventions (section 2.2: S is a convolution,
so it is diagonal in Fourier space; section 2.3: the same for S_L)."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import dft, grid, model
from paper_0911_1407_amd import synth


@pytest.mark.parametrize("n", [(8, 8, 8), (12, 12, 12), (16, 8, 12), (24, 24, 24)])
def test_dense_dft_matches_library_fft(n, rng):
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = dft.dftn(x)
    ref = np.fft.fftn(x)
    assert np.abs(X - ref).max() <= 1e-12 * np.abs(ref).max()
    back = dft.idftn(X)
    assert np.abs(back - x).max() <= 1e-13 * np.abs(x).max() * 10


@pytest.mark.parametrize("n", [(8, 8, 8), (12, 12, 12)])
def test_plane_wave_closed_form(n):
    # cos(2 pi m.x/n) transforms to N/2 at +m and -m and zero elsewhere
    m = (1, 2, 3)
    ix = np.indices(n)
    phase = 2 * np.pi * sum(m[a] * ix[a] / n[a] for a in range(3))
    X = dft.dftn(np.cos(phase))
    N = np.prod(n)
    expect = np.zeros(n, complex)
    expect[m] = N / 2
    expect[tuple((-np.array(m)) % np.array(n))] += N / 2
    assert np.abs(X - expect).max() <= 1e-11 * N


def test_parseval_with_hermitian_weights(rng):
    n = (12, 8, 16)
    x = rng.standard_normal(n)
    y = rng.standard_normal(n)
    c = grid.hermitian_weights(n)
    X, Y = dft.rdftn(x), dft.rdftn(y)
    got = np.sum(c * (np.conj(X) * Y).real) / np.prod(n)
    assert abs(got - np.sum(x * y)) <= 1e-12 * np.sqrt(np.sum(x * x) * np.sum(y * y))


def test_folded_index_and_nyquist():
    assert list(grid.folded_index(8)) == [0, 1, 2, 3, -4, -3, -2, -1]


def _prob(n, box, seed=0, beta=1.0):
    inst = synth.make_instance(n, box, 1.0, 1.0, beta, seed=seed)
    return oracle_problem(inst)


def test_inverse_eigenvalues_follow_convention():
    # lambda_k = A pk(|k|) N / V; compare against a direct evaluation of the
    # generator's spectrum shape on the full grid
    n, box = (8, 12, 8), (20.0, 30.0, 20.0)
    p = _prob(n, box)
    full = grid.inv_lambda_full(p)
    mx = grid.folded_index(n[0]); my = grid.folded_index(n[1]); mz = grid.folded_index(n[2])
    k = np.sqrt((2 * np.pi * mx / box[0])[:, None, None] ** 2 + (2 * np.pi * my / box[1])[None, :, None] ** 2
                + (2 * np.pi * mz / box[2])[None, None, :] ** 2)
    with np.errstate(divide="ignore"):
        pk = np.where(k > 0, k ** -1.5 * np.exp(-(2 * k) ** 2), 0.0)
    lam = p.amp * pk * p.ncells / p.volume
    expect = np.where(k > 0, 1.0 / np.where(k > 0, lam, 1.0), p.inv_p0)
    assert np.allclose(full, expect, rtol=1e-13, atol=0)


@pytest.mark.parametrize("mvec", [(1, 0, 0), (1, 2, 3), (4, 4, 4), (0, 3, 4)])
def test_prior_on_plane_wave(mvec):
    # S_L^-1 cos(k.x) = cos(k.x) / lambda_k for the eigenvector cos(k.x);
    # a coarse box keeps 1/lambda within a few decades so that roundoff in
    # the other modes is not amplified past the tolerance
    n, box = (8, 8, 8), (64.0, 64.0, 64.0)
    p = _prob(n, box)
    ix = np.indices(n)
    phase = 2 * np.pi * sum(mvec[a] * ix[a] / n[a] for a in range(3))
    x = np.cos(phase)
    kk = np.sqrt(sum((2 * np.pi * grid.folded_index(n[a])[mvec[a]] / box[a]) ** 2 for a in range(3)))
    lam = p.amp * kk ** -1.5 * np.exp(-(2 * kk) ** 2) * p.ncells / p.volume
    for f in (model.prior_apply, model.prior_apply_dense_dft):
        y = f(p, x)
        assert np.abs(y - x / lam).max() <= 1e-12 * np.abs(x / lam).max()


def test_prior_matrix_matches_operator(rng):
    n, box = (8, 8, 8), (16.0, 16.0, 16.0)
    p = _prob(n, box).replace(inv_p0=0.37)
    M = model.prior_matrix(p)
    x = rng.standard_normal(n)
    y1 = (M @ x.ravel()).reshape(n)
    y2 = model.prior_apply(p, x)
    assert np.abs(y1 - y2).max() <= 1e-12 * np.abs(y2).max()
    assert np.allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())
