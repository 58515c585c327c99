"""GPU parity of fresnel_step_f64 (the Fresnel plane of fresnel_step in float64, the paper's
precision) against the FP64 oracle, closed forms and invariants. Bar: field relative L2 <= 1e-12
(float64 transforms of length n accumulate about log2(n) 1e-16; the tables are built from exact
integer phases in float64, as the oracle builds its transfer function per pixel)."""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_1806_06467_amd import fresnel as fb
from paper_1806_06467_amd import synth
from tests.gpu_common import banner, grid_plane_wave_sum, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _gpu(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda:0")


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _case(n, seed):
    rng = np.random.default_rng(seed)
    field = synth.random_field(n, seed)
    amp = rng.uniform(0.3, 1.0, (n, n))
    opd = rng.normal(0.0, 60e-9, (n, n))
    dx, lam = 2e-5, 550e-9
    z = 0.4 * n * dx * dx / lam
    return field, amp, opd, dx, lam, z, 5.0 * n * dx * dx / lam


@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024, 2048, 4096])
def test_fresnel_step_f64_matches_oracle(n, adjoint):
    banner(f"fresnel_step_f64 n={n} adjoint={adjoint}")
    field, amp, opd, dx, lam, z, f = _case(n, 640 + n + adjoint)
    t = _gpu(field)
    st = fb.fresnel_step_f64(t, dx, lam, z, amp=_gpu(amp, torch.float64), opd=_gpu(opd, torch.float64),
                             lens_focal=f, adjoint=adjoint)
    assert st == 0
    ref = oracle.fresnel_step(field, dx, lam, z, amp=amp, opd=opd, lens_focal=f, adjoint=adjoint)
    assert rel_l2(_np(t), ref) <= TOL


def test_fresnel_step_f64_adjoint_identity_and_round_trip():
    """<A x, y> = <x, A^H y> for the step with its optic; without an optic the adjoint (the step
    over -z) undoes the step."""
    n = 1024
    banner("fresnel_step_f64 adjoint identity, round trip")
    field, amp, opd, dx, lam, z, f = _case(n, 17)
    y = synth.random_field(n, 18)
    a_g, o_g = _gpu(amp, torch.float64), _gpu(opd, torch.float64)
    ax = _gpu(field)
    fb.fresnel_step_f64(ax, dx, lam, z, amp=a_g, opd=o_g, lens_focal=f)
    ahy = _gpu(y)
    fb.fresnel_step_f64(ahy, dx, lam, z, amp=a_g, opd=o_g, lens_focal=f, adjoint=True)
    lhs = np.vdot(y, _np(ax))
    rhs = np.vdot(_np(ahy), field)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(field) * np.linalg.norm(y)
    t = _gpu(field)
    fb.fresnel_step_f64(t, dx, lam, z)
    fb.fresnel_step_f64(t, dx, lam, z, adjoint=True)
    assert rel_l2(_np(t), field) <= TOL


def test_fresnel_step_f64_gaussian_beam_closed_form():
    """A Gaussian beam of waist w0 at 1.5 z_R: exp(-r^2 / (w0^2 (1 + i zeta))) / (1 + i zeta)."""
    n, w0px, dx, lam = 512, 12.0, 1e-4, 550e-9
    w0 = w0px * dx
    zr = math.pi * w0 * w0 / lam
    banner("fresnel_step_f64 Gaussian beam n=512")
    t = _gpu(synth.gaussian_beam(n, w0px))
    fb.fresnel_step_f64(t, dx, lam, 1.5 * zr)
    r2 = (synth.radius_grid(n) * dx) ** 2
    ref = np.exp(-r2 / (w0 * w0 * (1 + 1.5j))) / (1 + 1.5j)
    assert rel_l2(_np(t), ref) <= TOL


@pytest.mark.parametrize("adjoint", [False, True])
def test_fresnel_step_f64_8192_plane_waves_closed_form(adjoint):
    """The largest edge on the whole plane: each grid plane wave of a sum is multiplied by the
    paraxial transfer function of its frequency, exp(-i pi lambda z f^2) in float64 (conjugated
    for the adjoint), frequencies up to the Nyquist corner. The corner's phase is about 900 turns,
    whose float64 rounding (about 1e-13 turns, on either side) sets the bar here at 5e-12."""
    n, dx, lam, z = 8192, 1.25e-5, 550e-9, 1.0
    banner(f"fresnel_step_f64 n=8192 plane waves adjoint={adjoint}")
    waves = [(1, 0, 1.0), (-37, 1500, 0.6j), (4000, -2500, 0.5), (-4096, -4096, 0.25), (2048, 7, -0.4)]
    t = _gpu(grid_plane_wave_sum(n, waves))
    fb.fresnel_step_f64(t, dx, lam, z, adjoint=adjoint)
    expected = []
    for kx, ky, a in waves:
        hk = np.exp(-1j * np.pi * lam * z * (kx * kx + ky * ky) / (n * dx) ** 2)
        expected.append((kx, ky, a * (np.conj(hk) if adjoint else hk)))
    got = _np(t)
    del t
    assert rel_l2(got, grid_plane_wave_sum(n, expected)) <= 5e-12
