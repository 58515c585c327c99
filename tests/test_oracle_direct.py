"""Pins for the oracle's direct (single-transform) Fresnel step (O9): the complex Gaussian-beam
closed form on the output grid, Parseval with the pitch change, and its exact agreement with the
independently pinned angular-spectrum step (O3) at the distance n dx^2 / lambda, where the
output pitch equals the input pitch and the Fresnel kernel exp(i pi m^2 / n) is n-periodic, so
that the linear and the circular convolution coincide (Gauss sum: the constant dx^2/(i lambda z)
is then exactly the AS step's)."""

import math

import numpy as np
import pytest

import oracle
from paper_1806_06467_amd import synth


def _gaussian_closed_form(n, pitch, lam, w0, z):
    """exp(-r^2/(w0^2 (1 + i zeta))) / (1 + i zeta), zeta = z / z_R, on the grid c(k) pitch."""
    zeta = z / (math.pi * w0 * w0 / lam)
    r2 = (synth.radius_grid(n) * pitch) ** 2
    q = 1.0 + 1j * zeta
    return np.exp(-r2 / (w0 * w0 * q)) / q


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("n,dx", [(64, 1e-5), (96, 3e-6), (128, 2.5e-5)])
def test_direct_equals_angular_spectrum_at_periodic_distance(n, dx, sign):
    lam = 550e-9
    z = sign * n * dx * dx / lam
    rng = np.random.default_rng(n)
    u = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    got, dx2 = oracle.direct_fresnel(u, dx, lam, z)
    assert abs(dx2 - dx) <= 1e-15 * dx
    ref = oracle.as_propagate(u, dx, lam, z)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("zr_mult", [0.5, 2.0, 4.0, -3.0])
def test_direct_gaussian_beam_closed_form(zr_mult):
    n, dx, lam, w0px = 512, 1e-5, 550e-9, 12.0
    w0 = w0px * dx
    z = zr_mult * math.pi * w0 * w0 / lam
    got, dx2 = oracle.direct_fresnel(synth.gaussian_beam(n, w0px), dx, lam, z)
    assert abs(dx2 - lam * abs(z) / (n * dx)) <= 1e-15 * dx2
    ref = _gaussian_closed_form(n, dx2, lam, w0, z)
    assert np.max(np.abs(got - ref)) <= 1e-12


def test_direct_parseval_with_pitch_change():
    n, dx, lam = 80, 7e-6, 633e-9
    rng = np.random.default_rng(5)
    u = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    for z in (0.013, 0.5, 3.7):
        got, dx2 = oracle.direct_fresnel(u, dx, lam, z)
        e1 = np.sum(np.abs(u) ** 2) * dx * dx
        e2 = np.sum(np.abs(got) ** 2) * dx2 * dx2
        assert abs(e2 / e1 - 1.0) <= 1e-12


def test_direct_rows_and_argument_checks():
    n, dx, lam, z = 48, 1e-5, 550e-9, 0.3
    rng = np.random.default_rng(7)
    u = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    full, _ = oracle.direct_fresnel(u, dx, lam, z)
    rows = [0, 1, 23, 24, 47]
    assert np.max(np.abs(oracle.direct_fresnel_rows(u, dx, lam, z, rows) - full[rows])) <= 1e-13
    assert np.max(np.abs(oracle.direct_fresnel_rows(u, dx, lam, -z, rows) - oracle.direct_fresnel(u, dx, lam, -z)[0][rows])) <= 1e-13
    with pytest.raises(ValueError):
        oracle.direct_fresnel(u, dx, lam, 0.0)


@pytest.mark.parametrize("n,z", [(32, 0.02), (48, 0.7), (40, -0.3)])
def test_direct_adjoint_identity_and_inverse(n, z):
    # the adjoint by the dot-product identity against the (pinned) forward step, and the inverse
    # (adjoint times (dx2/dx)^2) undoing the forward step
    dx, lam = 9e-6, 700e-9
    rng = np.random.default_rng(n)
    u = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    v = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    du, dx2 = oracle.direct_fresnel(u, dx, lam, z)
    lhs = np.vdot(v, du)
    rhs = np.vdot(oracle.direct_fresnel_adjoint(v, dx, lam, z), u)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    back = oracle.direct_fresnel_adjoint(du, dx, lam, z) * (dx2 / dx) ** 2
    assert np.max(np.abs(back - u)) <= 1e-12 * np.max(np.abs(u))


def test_direct_negative_distance_is_the_conjugate_step():
    # the Fresnel integral over -z is the complex conjugate of the one over z applied to the
    # conjugate field (its kernel exp(i pi r^2 / (lambda z)) / (i lambda z) is conjugated by z -> -z)
    n, dx, lam = 40, 1.1e-5, 633e-9
    rng = np.random.default_rng(9)
    u = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    for z in (0.05, 1.3):
        neg, dxn = oracle.direct_fresnel(u, dx, lam, -z)
        pos, dxp = oracle.direct_fresnel(np.conj(u), dx, lam, z)
        assert dxn == dxp
        assert np.max(np.abs(neg - np.conj(pos))) <= 1e-13 * np.max(np.abs(pos))
