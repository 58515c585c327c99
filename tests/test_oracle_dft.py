"""Pins for the oracle's DFT (O1): brute force on tiny grids, a library cross-check,
Parseval and the inverse. The brute force forms the exponent from floats (no integer
index reduction), so it shares no arithmetic shortcut with the oracle's matrix."""

import cmath
import math

import numpy as np
import pytest

import oracle


def _brute_dft2(u):
    n = u.shape[0]
    out = np.zeros((n, n), dtype=complex)
    for ky in range(n):
        for kx in range(n):
            acc = 0j
            for y in range(n):
                for x in range(n):
                    acc += u[y, x] * cmath.exp(-2j * math.pi * (ky * y + kx * x) / n)
            out[ky, kx] = acc
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dft2_brute_force(n, rng):
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ref = _brute_dft2(u)
    got = oracle.dft2(u)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [12, 64, 96, 250])
def test_dft2_matches_library(n, rng):
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ref = np.fft.fft2(u)
    got = oracle.dft2(u)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    back = oracle.idft2(got)
    assert np.max(np.abs(back - u)) <= 1e-13 * np.max(np.abs(u))


def test_dft_rows_are_along_y_then_x():
    # a single bright pixel at (y=1, x=0) must give a phase ramp along ky only
    n = 8
    u = np.zeros((n, n), complex)
    u[1, 0] = 1.0
    f = oracle.dft2(u)
    ky = np.arange(n)[:, None]
    assert np.allclose(f, np.exp(-2j * np.pi * ky / n) * np.ones((1, n)), atol=1e-15)


@pytest.mark.parametrize("n", [16, 31, 128])
def test_parseval(n, rng):
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    e_in = np.sum(np.abs(u) ** 2)
    e_out = np.sum(np.abs(oracle.dft2(u)) ** 2)
    assert abs(e_out - n * n * e_in) <= 1e-12 * n * n * e_in


def test_signed_index_and_centring():
    assert list(oracle.signed_index(6)) == [0, 1, 2, -3, -2, -1]
    assert list(oracle.signed_index(5)) == [0, 1, 2, -2, -1]
    assert list(oracle.centred(6)) == [-3, -2, -1, 0, 1, 2]
