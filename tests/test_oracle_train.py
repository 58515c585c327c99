"""Pins for the oracle's DM synthesis (O6), Lyot train (O5) and gradient (O7/O8) on a small
geometry: single-actuator closed form, total rejection of a full-band occulter (Babinet
normalisation), the dot-product identity of the whole linear map, finite differences and a
Taylor test of the gradient, for one and for two mirrors."""

import math

import numpy as np
import pytest

import oracle
from paper_1806_06467_amd import synth


def _geom(n_d=32, occ_m=32, occ_du=8.0 / 32, det_m=32, det_du=0.5, opd_seed=0):
    amp = synth.pupil_amplitude(n_d, 0.1, 0.04)
    return oracle.TrainGeometry(
        n_d=n_d, d_m=n_d * 25e-6, z_m=0.05, occ_m=occ_m, occ_du_c=occ_du, det_m=det_m,
        det_du_c=det_du, lambda_c=550e-9, pupil_amp=amp,
        occ_mask=synth.occulter_spot(occ_m, occ_du, 3.0), lyot=synth.lyot_stop(n_d, 0.9),
        pupil_opd=synth.power_law_opd(n_d, amp, 10e-9, -3.0, opd_seed))


def test_dm_single_actuator_closed_form():
    n, n_d, n_act = 40, 24, 6
    h = np.zeros((n_act, n_act))
    h[2, 4] = 3e-9
    s = oracle.dm_surface(h, n, n_d)
    p = n_d / n_act
    ya, xa = (2 - (n_act - 1) / 2) * p, (4 - (n_act - 1) / 2) * p
    c = np.arange(n) - n // 2
    ref = 3e-9 * np.exp(-((c[:, None] - ya) ** 2 + (c[None, :] - xa) ** 2) / (2 * p * p))
    assert np.max(np.abs(s - ref)) <= 1e-24
    # here the actuator centre (-2, +6) px falls on a pixel, which then holds the full height
    assert abs(s[n // 2 - 2, n // 2 + 6] - 3e-9) <= 1e-24
    # one pitch away along x the surface has dropped to exp(-1/2) (sigma = one pitch)
    assert abs(s[n // 2 - 2, n // 2 + 10] - 3e-9 * math.exp(-0.5)) <= 1e-24


def test_full_band_occulter_rejects_everything():
    # occulter grid = the padded plane's own DFT lattice and a spot covering all of it: the
    # Babinet subtraction must then remove the whole field (normalisation of MFT and MFT^H)
    n_d, n = 32, 64
    g = _geom(n_d, occ_m=n, occ_du=n_d / n)
    g.occ_mask = np.ones((n, n))
    e = oracle.train_forward(g, 550e-9, n, [synth.dm_heights(8, 1)], occulter=True).e_det
    ref = oracle.train_forward(g, 550e-9, n, [synth.dm_heights(8, 1)], occulter=False).e_det
    assert np.max(np.abs(e) ** 2) <= 1e-26 * np.max(np.abs(ref) ** 2)


def test_no_occulter_is_lyot_stopped_pupil_mft():
    n_d, n = 32, 64
    g = _geom(n_d)
    g.z_m = 0.0
    e = oracle.train_forward(g, 550e-9, n, [], occulter=False).e_det
    pupil = g.pupil_amp * np.exp(2j * np.pi * g.pupil_opd / 550e-9)
    ref = oracle.mft(g.lyot * pupil, n_d, g.det_m, g.det_du_c)
    assert np.max(np.abs(e - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("lam", [550e-9, 500e-9])
def test_linear_map_adjoint_identity(lam, rng):
    n_d, n = 32, 64
    g = _geom(n_d)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal((g.det_m, g.det_m)) + 1j * rng.standard_normal((g.det_m, g.det_m))
    lhs = np.vdot(oracle.dm_to_detector(g, lam, x), y)
    rhs = np.vdot(x, oracle.dm_to_detector_adjoint(g, lam, n, y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _setup(n_dm, n_lambda):
    n_d, n, n_act = 32, 64, 8
    g = _geom(n_d)
    heights = [synth.dm_heights(n_act, 1 + i) for i in range(n_dm)]
    lams = synth.wavelengths(n_lambda)
    ns = [n] * n_lambda
    w = [1.0 / n_lambda] * n_lambda
    ref = oracle.train_psf(g, lams, ns, w, heights, occulter=False)
    dh = synth.dark_hole(g.det_m, g.det_du_c, 3.0, 7.0)
    return g, heights, lams, ns, w, dh, float(ref.max())


@pytest.mark.parametrize("n_dm,n_lambda", [(1, 1), (1, 2), (2, 2)])
def test_gradient_matches_finite_differences(n_dm, n_lambda):
    g, heights, lams, ns, w, dh, mref = _setup(n_dm, n_lambda)
    grad = oracle.train_grad(g, lams, ns, w, heights, dh, mref)
    acts = [(d, r, c) for d in range(n_dm) for (r, c) in [(3, 4), (2, 6), (5, 1)]]
    fd = oracle.fd_grad(g, lams, ns, w, heights, dh, mref, acts, h=1e-12)
    an = np.array([grad[d][r, c] for d, r, c in acts])
    scale = np.max(np.abs(np.concatenate([x.ravel() for x in grad])))
    assert np.max(np.abs(an - fd)) <= 1e-6 * scale
    for a, f in zip(an, fd):
        if abs(a) > 0.05 * scale:
            assert abs(a - f) <= 1e-6 * abs(a)


def test_gradient_taylor_remainder_is_second_order(rng):
    g, heights, lams, ns, w, dh, mref = _setup(2, 1)
    grad = oracle.train_grad(g, lams, ns, w, heights, dh, mref)
    d = [rng.standard_normal(h.shape) * 1e-9 for h in heights]
    l0 = oracle.train_loss(g, lams, ns, w, heights, dh, mref)
    slope = sum(float(np.sum(gg * dd)) for gg, dd in zip(grad, d))
    rem = []
    for eps in (1e-1, 5e-2, 2.5e-2):
        hs = [h + eps * dd for h, dd in zip(heights, d)]
        rem.append(abs(oracle.train_loss(g, lams, ns, w, hs, dh, mref) - l0 - eps * slope))
    # halving eps divides an O(eps^2) remainder by about 4
    assert 3.0 < rem[0] / rem[1] < 5.0 and 3.0 < rem[1] / rem[2] < 5.0


@pytest.mark.parametrize("lam", [500e-9, 550e-9, 600e-9])
def test_focal_grid_fixed_in_reference_units(lam):
    # a pupil tilt of alpha rad puts the PSF centre at alpha D / lambda_c in lambda_c/D units for
    # every wavelength; with a symmetric pupil the PSF is mirror-symmetric about that sample
    n_d, n = 32, 64
    g = _geom(n_d)
    g.z_m = 0.0
    shift = 2                                       # detector samples off axis
    alpha = shift * g.det_du_c * g.lambda_c / g.d_m
    x = (np.arange(n_d) - n_d // 2) * g.dx
    g.pupil_opd = np.broadcast_to(alpha * x, (n_d, n_d)).copy()
    e = oracle.train_forward(g, lam, n, [], occulter=False).e_det
    inten = np.abs(e) ** 2
    k0 = g.det_m // 2
    row = inten[k0]
    assert int(np.argmax(row)) == k0 + shift
    for d in (1, 2, 3):
        assert abs(row[k0 + shift + d] - row[k0 + shift - d]) <= 1e-11 * row.max()


def test_step_cache_is_pure_memoisation():
    g, heights, lams, ns, w, dh, mref = _setup(1, 2)
    cache = {}
    a = oracle.train_loss(g, lams, ns, w, heights, dh, mref)
    b = oracle.train_loss(g, lams, ns, w, heights, dh, mref, step_cache=cache)
    c = oracle.train_loss(g, lams, ns, w, heights, dh, mref, step_cache=cache)
    assert a == b == c and len(cache) == 2


def test_one_pixel_axial_spot_removes_the_mean_term():
    # A spot of one focal pixel on the optical axis (u = 0) blocks only the zero-frequency MFT
    # sample, (du/n_d) sum(E) over the whole padded plane (the DC term, pinned in the MFT
    # tests); its adjoint spreads that value evenly over the pupil window with the same factor.
    # So the Babinet step must leave lyot * (window(E) - (du/n_d)^2 sum(E)) at the Lyot plane:
    # a sign, mask, window-offset or normalisation mistake in the train fails this.
    n_d, n, lam = 32, 64, 550e-9
    g = _geom(n_d)
    g.occ_mask = np.zeros((g.occ_m, g.occ_m))
    g.occ_mask[g.occ_m // 2, g.occ_m // 2] = 1.0
    fwd = oracle.train_forward(g, lam, n, [synth.dm_heights(8, 1)], occulter=True)
    e_dm = fwd.e_dm[-1]
    du = g.occ_du_c * g.lambda_c / lam
    off = (n - n_d) // 2
    e_lyot = g.lyot * (e_dm[off:off + n_d, off:off + n_d] - (du / n_d) ** 2 * e_dm.sum())
    ref = oracle.mft(e_lyot, n_d, g.det_m, g.det_du_c * g.lambda_c / lam)
    assert np.max(np.abs(fwd.e_det - ref)) <= 1e-12 * np.max(np.abs(ref))
