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


def _grazing_plane_wave(kx, n, wavelength, eps):
    """A grid plane wave of x-frequency (1 + eps) / lambda (just past grazing incidence for
    eps > 0, just before it for eps < 0), with the pitch that puts it there."""
    dx = kx * wavelength / (n * (1.0 + eps))
    x = np.arange(n)[None, :] * np.ones((n, 1))
    return dx, np.exp(2j * np.pi * kx * x / n)


@pytest.mark.parametrize("z_over_lambda", [10.3, -7.7, 3.45])
def test_transfer_is_continuous_across_the_cutoff(z_over_lambda):
    # At grazing incidence the propagation angle reaches 90 degrees: cos(theta) -> 0, so the
    # exact (piston-free) eigenvalue exp(2 pi i z (cos(theta) - 1) / lambda) tends to
    # exp(-2 pi i z / lambda) from the propagating side. The evanescent side must reach the
    # same value (its decay -> 1 and its phase is the piston's), for either sign of z: a dropped
    # or sign-flipped piston factor fails here (z / lambda is not an integer).
    n, kx, lam = 64, 20, 633e-9
    z = z_over_lambda * lam
    limit = np.exp(-2j * np.pi * z_over_lambda)
    eps = 1e-10
    # distance of either side from the limit: 2 pi |z| / lambda * sqrt(2 eps) to first order
    tol = 1.1 * 2.0 * math.pi * abs(z_over_lambda) * math.sqrt(2.0 * eps)
    vals = []
    for e in (-eps, eps):
        dx, u = _grazing_plane_wave(kx, n, lam, e)
        got = oracle.as_propagate_exact(u, dx, lam, z)
        h = got / u
        assert np.max(np.abs(h - h[0, 0])) <= 1e-9        # still an eigenfunction
        assert abs(h[0, 0] - limit) <= tol
        vals.append(h[0, 0])
    assert abs(vals[0] - vals[1]) <= 2 * tol
    # and the two sides really straddle the cutoff: the propagating side keeps |H| = 1
    assert abs(abs(vals[0]) - 1.0) <= 1e-12
    assert abs(vals[1]) < 1.0 - 1e-5


def test_backward_step_is_the_adjoint_on_every_frequency(rng=np.random.default_rng(11)):
    # Reading for z < 0: evanescent components decay in either direction, so that the step over
    # -z is the exact adjoint of the step over z on the whole grid (the inverse on the
    # propagating frequencies, where |H| = 1). The z > 0 decay is physics (pinned above); this
    # fixes the z < 0 branch relative to it: <AS(z) u, v> = <u, AS(-z) v> with a pitch below
    # lambda / 2, where most grid frequencies are evanescent.
    n, dx, lam, z = 32, 0.3e-6, 633e-9, 0.4e-6
    u = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    v = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    lhs = np.vdot(v, oracle.as_propagate_exact(u, dx, lam, z))
    rhs = np.vdot(oracle.as_propagate_exact(v, dx, lam, -z), u)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # evanescent waves lose the same fraction of amplitude over -z as over +z
    y, x = np.mgrid[0:n, 0:n]
    w = np.exp(2j * np.pi * (13 * x - 9 * y) / n)
    f = math.hypot(13, 9) / (n * dx)
    assert f > 1.0 / lam
    decay = math.exp(-2.0 * math.pi * abs(z) * math.sqrt(f * f - 1.0 / lam ** 2))
    for zz in (z, -z):
        assert np.max(np.abs(np.abs(oracle.as_propagate_exact(w, dx, lam, zz)) - decay)) <= 1e-12
