"""Pins for the oracle's optic multiply (O2) and angular-spectrum step (O3): the complex
Gaussian-beam closed form, the Talbot self-imaging closed form of the paper's Appendix A
example (without its aperture), the thin-lens q-parameter law, and exact invariants."""

import cmath
import json
import math
import os

import numpy as np
import pytest
from scipy.special import jv

import oracle
from paper_1806_06467_amd import synth


def _gaussian_closed_form(n, dx, lam, w0, z):
    """exp(-r^2/(w0^2 (1 + i zeta))) / (1 + i zeta), zeta = z / z_R, z_R = pi w0^2 / lambda."""
    zeta = z / (math.pi * w0 * w0 / lam)
    r2 = (synth.radius_grid(n) * dx) ** 2
    q = 1.0 + 1j * zeta
    return np.exp(-r2 / (w0 * w0 * q)) / q


@pytest.mark.parametrize("zr_mult", [0.5, 1.0, 2.0, -1.0])
def test_gaussian_beam_closed_form(zr_mult):
    n, dx, lam, w0px = 512, 1e-5, 550e-9, 12.0
    w0 = w0px * dx
    z = zr_mult * math.pi * w0 * w0 / lam
    u0 = synth.gaussian_beam(n, w0px)
    got = oracle.as_propagate(u0, dx, lam, z)
    ref = _gaussian_closed_form(n, dx, lam, w0, z)
    assert np.max(np.abs(got - ref)) <= 1e-12
    # the beam radius law w(z) = w0 sqrt(1 + (z/zR)^2), read off the second moment of |E|^2
    inten = np.abs(got) ** 2
    r2 = (synth.radius_grid(n) * dx) ** 2
    w_meas = math.sqrt(2.0 * np.sum(r2 * inten) / np.sum(inten))
    assert abs(w_meas - w0 * math.sqrt(1.0 + zr_mult ** 2)) <= 1e-10 * w0


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _talbot_setup(n):
    # Appendix A: beam radius 2 cm sampled by 256 px (dx = 156.25 um), lambda = 0.5 um,
    # 5 nm sine WFE at 500 cycles/m (period 2 mm), Talbot length 2 p^2 / lambda = 16 m
    with open(os.path.join(GOLDEN, "talbot_appendix_a.json")) as f:
        g = json.load(f)
    dx = 2 * g["beam_radius_m"] / g["npix"]
    lam, period, amp = g["wavelength_m"], 1.0 / g["sine_spatial_freq_per_m"], g["sine_amplitude_m"]
    assert n % g["npix"] == 0
    opd = synth.sine_opd(n, dx, period, amp)
    return dx, lam, period, amp, opd


def test_talbot_length_eq1():
    with open(os.path.join(GOLDEN, "talbot_appendix_a.json")) as f:
        g = json.load(f)
    p = 1.0 / g["sine_spatial_freq_per_m"]
    assert abs(2 * p * p / g["wavelength_m"] - g["talbot_length_m"]) < 1e-12
    assert g["npix"] * g["oversample"] == 2048


@pytest.mark.parametrize("n", [256, pytest.param(2048, marks=pytest.mark.slow)])
def test_talbot_quarter_length_converts_phase_to_amplitude(n):
    dx, lam, period, amp, opd = _talbot_setup(n)
    z_t = 2.0 * period ** 2 / lam
    assert abs(z_t - 16.0) < 1e-12
    got = oracle.fresnel_step(np.ones((n, n)), dx, lam, z_t / 4.0, opd=opd)
    a = 2.0 * math.pi * amp / lam
    theta = 2.0 * math.pi * ((np.arange(n) - n // 2) * dx) / period
    ref_row = np.cos(a * np.sin(theta)) + np.sin(a * np.sin(theta))
    assert np.max(np.abs(got - ref_row[None, :])) <= 1e-12
    # the field is real: the sine phase error has become a pure amplitude error
    assert np.max(np.abs(got.imag)) <= 1e-12
    inten = np.abs(got[0]) ** 2
    assert abs(inten.max() - 1.0 - math.sin(2 * a)) < 1e-3   # +/- 0.1253 modulation


@pytest.mark.parametrize("frac", [0.05, 0.13])
def test_talbot_partial_distance_bessel_series(frac):
    n = 256
    dx, lam, period, amp, opd = _talbot_setup(n)
    z = frac * 2.0 * period ** 2 / lam
    got = oracle.fresnel_step(np.ones((n, n)), dx, lam, z, opd=opd)
    a = 2.0 * math.pi * amp / lam
    theta = 2.0 * math.pi * ((np.arange(n) - n // 2) * dx) / period
    ref = np.zeros(n, complex)
    for m in range(-9, 10):
        ref += jv(m, a) * np.exp(1j * m * theta) * np.exp(-1j * math.pi * m * m * lam * z / period ** 2)
    assert np.max(np.abs(got - ref[None, :])) <= 1e-12


def test_thin_lens_q_law():
    # Gaussian waist at a thin lens f, then a step z: 1/q' = 1/q0 - 1/f, q(z) = q' + z and
    # E = (q'/q) exp(i pi r^2 / (lambda q)) with q0 = -i z_R in this sign convention
    n, dx, lam, w0px, f = 512, 1e-5, 550e-9, 12.0, 0.5
    w0 = w0px * dx
    zr = math.pi * w0 * w0 / lam
    q0 = -1j * zr
    qp = 1.0 / (1.0 / q0 - 1.0 / f)
    r2 = (synth.radius_grid(n) * dx) ** 2
    for z in (0.0, 0.03, 0.12):
        got = oracle.fresnel_step(synth.gaussian_beam(n, w0px), dx, lam, z, lens_focal=f)
        q = qp + z
        ref = (qp / q) * np.exp(1j * math.pi * r2 / (lam * q))
        assert np.max(np.abs(got - ref)) <= 1e-12


def test_optic_phasor_eq3_and_lens_pointwise(rng):
    n, dx, lam, f = 16, 3e-5, 633e-9, 0.7
    amp = rng.uniform(0.2, 1.0, (n, n))
    opd = rng.normal(0, 200e-9, (n, n))
    ph = oracle.optic_phasor(n, dx, lam, amp=amp, opd=opd, lens_focal=f)
    for (y, x) in [(0, 0), (3, 11), (8, 8), (15, 2)]:
        r2 = ((y - n // 2) ** 2 + (x - n // 2) ** 2) * dx * dx
        ref = amp[y, x] * cmath.exp(2j * math.pi * opd[y, x] / lam) * cmath.exp(-1j * math.pi * r2 / (lam * f))
        assert abs(ph[y, x] - ref) <= 1e-13
    surf = rng.normal(0, 5e-9, (n, n))
    ph2 = oracle.optic_phasor(n, dx, lam, surface=surf)
    assert np.allclose(ph2, np.exp(4j * math.pi * surf / lam), atol=1e-14)


def test_as_invariants(rng):
    n, dx, lam = 64, 2e-5, 600e-9
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    z1, z2 = 0.37, -0.11
    a = oracle.as_propagate(oracle.as_propagate(u, dx, lam, z1), dx, lam, z2)
    b = oracle.as_propagate(u, dx, lam, z1 + z2)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(u))
    back = oracle.as_propagate(oracle.as_propagate(u, dx, lam, z1), dx, lam, -z1)
    assert np.max(np.abs(back - u)) <= 1e-13 * np.max(np.abs(u))
    ident = oracle.as_propagate(u, dx, lam, 0.0)
    assert np.max(np.abs(ident - u)) <= 1e-13 * np.max(np.abs(u))
    e0 = np.sum(np.abs(u) ** 2)
    e1 = np.sum(np.abs(oracle.as_propagate(u, dx, lam, z1)) ** 2)
    assert abs(e1 - e0) <= 1e-13 * e0


def test_transfer_function_factorises_and_is_even():
    n, dx, lam, z = 48, 1e-5, 500e-9, 0.8
    h = oracle.transfer_function(n, dx, lam, z)
    hx = h[0, :]
    # the phase runs to ~1000 turns here, so float64 rounding of the argument is ~1e-13 rad
    assert np.max(np.abs(h - np.outer(hx, hx))) <= 2e-12
    k = oracle.signed_index(n)
    assert np.max(np.abs(hx - np.exp(-1j * math.pi * lam * z * (k / (n * dx)) ** 2))) <= 1e-12


def test_fresnel_step_adjoint_identity(rng):
    n, dx, lam, z, f = 32, 4e-5, 550e-9, 0.9, 1.3
    amp = rng.uniform(0.0, 1.0, (n, n))
    opd = rng.normal(0, 100e-9, (n, n))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    fx = oracle.fresnel_step(x, dx, lam, z, amp=amp, opd=opd, lens_focal=f)
    fhy = oracle.fresnel_step(y, dx, lam, z, amp=amp, opd=opd, lens_focal=f, adjoint=True)
    lhs = np.vdot(fx, y)
    rhs = np.vdot(x, fhy)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_as_propagate_rows_equals_full_step():
    # the separable (circulant) form of the paraxial step gives the same rows as the 2-D
    # definition, on even and odd edges and at distances whose phases wrap many turns
    rng = np.random.default_rng(5)
    for n, z in ((64, 0.3), (100, 2.0), (45, 7.5)):
        u = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        rows = [0, 1, n // 2, n - 1]
        full = oracle.as_propagate(u, 2e-5, 600e-9, z)[rows]
        part = oracle.as_propagate_rows(u, 2e-5, 600e-9, z, rows)
        assert np.max(np.abs(part - full)) <= 1e-12 * np.max(np.abs(full))


def test_as_propagate_rows_gaussian_closed_form():
    # rows of a propagated Gaussian beam against the closed form (independent of the 2-D path)
    n, dx, lam, w0px = 256, 1e-5, 550e-9, 12.0
    w0 = w0px * dx
    zr = np.pi * w0 * w0 / lam
    u = synth.gaussian_beam(n, w0px)
    rows = [n // 2, n // 2 + 7, n // 2 - 20, 3]
    got = oracle.as_propagate_rows(u, dx, lam, 1.5 * zr, rows)
    r2 = (synth.radius_grid(n) * dx) ** 2
    ref = (np.exp(-r2 / (w0 * w0 * (1 + 1.5j))) / (1 + 1.5j))[rows]
    assert np.linalg.norm(got - ref) <= 1e-6 * np.linalg.norm(ref)
