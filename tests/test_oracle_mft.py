"""Pins for the oracle's matrix Fourier transform (O4): brute force, the exact DFT special case,
the DC term, the adjoint identity, the Airy pattern of a circular aperture and the exact
angular-spectrum / MFT invariance on the padded-grid frequency lattice."""

import cmath
import math

import numpy as np
import pytest
from scipy.special import j1

import oracle
from paper_1806_06467_amd import synth


def _brute_mft(e, n_d, m, du):
    n = e.shape[0]
    out = np.zeros((m, m), complex)
    for ky in range(m):
        for kx in range(m):
            uy, ux = (ky - m // 2) * du, (kx - m // 2) * du
            acc = 0j
            for y in range(n):
                for x in range(n):
                    yy, xx = (y - n // 2) / n_d, (x - n // 2) / n_d
                    acc += e[y, x] * cmath.exp(-2j * math.pi * (uy * yy + ux * xx))
            out[ky, kx] = acc * du / n_d
    return out


@pytest.mark.parametrize("n,m,n_d,du", [(6, 5, 4.0, 0.37), (5, 8, 3.0, 0.91), (7, 3, 7.0, 1.3)])
def test_mft_brute_force(n, m, n_d, du, rng):
    e = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    got = oracle.mft(e, n_d, m, du)
    ref = _brute_mft(e, n_d, m, du)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,n_d", [(64, 16), (48, 24)])
def test_mft_reduces_to_centred_dft(n, n_d, rng):
    e = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    got = oracle.mft(e, n_d, n, n_d / n)
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(e))) / n
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # unitary in this case: Parseval holds and the adjoint is the inverse
    assert abs(np.sum(np.abs(got) ** 2) - np.sum(np.abs(e) ** 2)) <= 1e-12 * np.sum(np.abs(e) ** 2)
    back = oracle.mft_adjoint(got, n_d, n, n_d / n)
    assert np.max(np.abs(back - e)) <= 1e-13 * np.max(np.abs(e))


def test_mft_dc_term_256_aperture():
    # 256 px circular aperture (r < 128) in a 512 grid, 128^2 focal plane at 0.25 lambda/D
    ap = synth.circular_aperture(512, 128.0)
    assert ap.sum() == 51429
    eb = oracle.mft(ap, 256.0, 128, 0.25)
    assert abs(eb[64, 64] - 0.25 / 256 * 51429) <= 1e-12
    assert abs(eb[64, 64].real - 50.2236328125) <= 1e-12


@pytest.mark.parametrize("n,m,n_d,du", [(20, 12, 9.0, 0.41), (16, 16, 16.0, 1.0)])
def test_mft_adjoint_identity(n, m, n_d, du, rng):
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    lhs = np.vdot(oracle.mft(x, n_d, m, du), y)
    rhs = np.vdot(x, oracle.mft_adjoint(y, n_d, n, du))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_airy_pattern_256_aperture():
    ap = synth.circular_aperture(512, 128.0)
    eb = oracle.mft(ap, 256.0, 128, 0.25)
    peak = abs(eb[64, 64])
    rho = np.abs((np.arange(128) - 64) * 0.25)
    with np.errstate(invalid="ignore", divide="ignore"):
        airy = np.where(rho > 0, 2 * j1(np.pi * rho) / (np.pi * rho), 1.0)
    core = rho <= 3.0
    for cut in (np.abs(eb[64, :]), np.abs(eb[:, 64])):
        assert np.max(np.abs(cut / peak - np.abs(airy))[core]) <= 1.5e-3
    # first null: the axial minimum falls on the sample nearest 1.22 lambda/D (1.25)
    cut = np.abs(eb[64, 64:64 + 8])
    assert int(np.argmin(cut)) == 5 and cut[5] / peak < 0.02


def test_as_mft_lattice_invariance():
    # 256 px aperture on a 512 grid: z = 1 m, dx = 1e-4 m, lambda = 550 nm; padded-grid lattice = every 2nd sample
    n, n_d, lam, dx, z = 512, 256.0, 550e-9, 1e-4, 1.0
    ap = synth.circular_aperture(n, 128.0)
    e_z = oracle.as_propagate(ap, dx, lam, z)
    i0 = np.abs(oracle.mft(ap, n_d, 128, 0.25)) ** 2
    iz = np.abs(oracle.mft(e_z, n_d, 128, 0.25)) ** 2
    lat = (np.arange(128) - 64) % 2 == 0
    sel = np.ix_(lat, lat)
    assert np.max(np.abs(iz[sel] - i0[sel])) <= 1e-12 * i0.max()
    # off the lattice the Fresnel step does change the sampled spectrum
    off = np.ix_(~lat, ~lat)
    assert np.max(np.abs(iz[off] - i0[off])) > 1e-9 * i0.max()
