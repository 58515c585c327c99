"""Pins for the oracle's exact (non-paraxial) angular-spectrum step (O10): a grid plane wave is an
eigenfunction whose phase follows the propagation angle, cos(theta) = sqrt(1 - (lambda f)^2)
(written here from the angle, not from the oracle's cancellation-free form); agreement with the
pinned paraxial step within its fourth-order remainder; unitarity and the group law on
propagating fields; evanescent decay."""

import math

import numpy as np
import pytest

import oracle
from paper_1806_06467_amd import synth


@pytest.mark.parametrize("kx,ky", [(3, 0), (-5, 7), (20, -11), (31, 31)])
def test_plane_wave_is_an_eigenfunction_with_the_angle_phase(kx, ky):
    n, dx, lam, z = 64, 1.2e-6, 633e-9, 2.5e-3
    y, x = np.mgrid[0:n, 0:n]
    u = np.exp(2j * np.pi * (kx * x + ky * y) / n)
    got = oracle.as_propagate_exact(u, dx, lam, z)
    f = math.hypot(kx, ky) / (n * dx)
    cos_t = math.sqrt(1.0 - (lam * f) ** 2)
    phase = 2.0 * math.pi * z * (cos_t - 1.0) / lam
    assert np.max(np.abs(got - np.exp(1j * phase) * u)) <= 1e-9


def test_evanescent_plane_wave_decays():
    n, dx, lam, z = 32, 0.25e-6, 633e-9, 0.3e-6
    y, x = np.mgrid[0:n, 0:n]
    kx = 15   # f = 15 / (32 * 0.25 um) = 1.9 / um > 1 / lambda = 1.58 / um
    u = np.exp(2j * np.pi * kx * x / n)
    got = oracle.as_propagate_exact(u, dx, lam, z)
    f = kx / (n * dx)
    expect = math.exp(-2.0 * math.pi * z * math.sqrt(f * f - 1.0 / lam ** 2))
    assert abs(np.abs(got[0, 0]) - expect) <= 1e-12
    assert np.max(np.abs(np.abs(got) - expect)) <= 1e-12


@pytest.mark.parametrize("zr_mult", [0.5, 2.0, -1.0])
def test_paraxial_limit_within_the_fourth_order_remainder(zr_mult):
    # sqrt(1 - a) - 1 = -a/2 - a^2/8 - ..., so the exact and paraxial phases differ by about
    # 2 pi z lambda^3 f^4 / 8; over a Gaussian beam's spectrum this bounds the field difference
    n, dx, lam, w0px = 256, 1e-5, 550e-9, 10.0
    w0 = w0px * dx
    z = zr_mult * math.pi * w0 * w0 / lam
    u = synth.gaussian_beam(n, w0px)
    ex = oracle.as_propagate_exact(u, dx, lam, z)
    par = oracle.as_propagate(u, dx, lam, z)
    spec = np.abs(oracle.dft2(u))
    k = oracle.signed_index(n)
    f2 = (k[:, None] ** 2 + k[None, :] ** 2) / (n * dx) ** 2
    dphi = 2 * math.pi * abs(z) * lam ** 3 * f2 ** 2 / 8 * 1.01
    bound = np.sqrt(np.sum((spec * dphi) ** 2)) / n          # Parseval: field L2 of the phase error
    err = np.linalg.norm(ex - par)
    assert err <= bound
    assert err >= 0.5 * bound            # the remainder is really there (not a silent paraxial copy)


def test_unitary_and_group_law_on_propagating_fields(rng=np.random.default_rng(4)):
    n, dx, lam = 48, 2e-6, 600e-9      # every grid frequency propagates: f_max = 1/(2 dx) < 1/lambda
    u = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    a = oracle.as_propagate_exact(u, dx, lam, 3e-4)
    assert abs(np.linalg.norm(a) / np.linalg.norm(u) - 1.0) <= 1e-12
    b = oracle.as_propagate_exact(oracle.as_propagate_exact(u, dx, lam, 1e-4), dx, lam, 2e-4)
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(a))
    back = oracle.as_propagate_exact(a, dx, lam, -3e-4)
    assert np.max(np.abs(back - u)) <= 1e-11 * np.max(np.abs(u))
