"""The Gaussian pilot-beam planner fr_plan_route (host arithmetic only, no GPU): which step
carries a field between two planes, and the pitch on each side, for every near / far pairing."""

import ctypes
import math

import pytest

from paper_1806_06467_amd import fresnel as fb

LAM, W0, N, DX = 600e-9, 2e-3, 1024, 2e-5
ZR = math.pi * W0 * W0 / LAM          # 20.9 m


def route(z_from, z_to, dx=DX, z_waist=0.0):
    return fb.plan_route(W0, z_waist, LAM, N, dx, z_from, z_to)


def far_pitch(d, dx_w=DX):
    return LAM * abs(d) / (N * dx_w)


def test_near_to_near_is_one_angular_spectrum_step():
    assert route(-0.3 * ZR, 0.8 * ZR) == [(fb.FR_ROUTE_AS, 1.1 * ZR, DX, DX)]
    assert route(0.5 * ZR, 0.5 * ZR) == []


def test_near_to_far_goes_through_the_waist():
    (k1, z1, a1, b1), (k2, z2, a2, b2) = route(0.4 * ZR, 3.0 * ZR, z_waist=0.0)
    assert (k1, a1, b1) == (fb.FR_ROUTE_AS, DX, DX) and z1 == pytest.approx(-0.4 * ZR, rel=1e-15)
    assert (k2, z2, a2) == (fb.FR_ROUTE_DIRECT, 3.0 * ZR, DX) and b2 == pytest.approx(far_pitch(3 * ZR))
    # starting on the waist plane: only the direct step
    assert route(0.0, -2.0 * ZR) == [(fb.FR_ROUTE_DIRECT, -2.0 * ZR, DX, far_pitch(2 * ZR))]


def test_far_to_near_returns_by_the_inverse_step():
    dx_far = far_pitch(4.0 * ZR)
    (k1, z1, a1, b1), (k2, z2, a2, b2) = route(4.0 * ZR, 0.25 * ZR, dx=dx_far)
    assert (k1, z1, a1) == (fb.FR_ROUTE_DIRECT_INVERSE, 4.0 * ZR, dx_far) and b1 == pytest.approx(DX, rel=1e-14)
    assert (k2, a2) == (fb.FR_ROUTE_AS, b1) and z2 == pytest.approx(0.25 * ZR) and b2 == b1


def test_far_to_far_on_either_side():
    dx_far = far_pitch(-5.0 * ZR)
    for z_to in (-2.0 * ZR, 7.0 * ZR):
        (k1, z1, a1, b1), (k2, z2, a2, b2) = route(-5.0 * ZR, z_to, dx=dx_far)
        assert (k1, z1) == (fb.FR_ROUTE_DIRECT_INVERSE, -5.0 * ZR) and b1 == pytest.approx(DX, rel=1e-14)
        assert (k2, z2) == (fb.FR_ROUTE_DIRECT, z_to) and b2 == pytest.approx(far_pitch(z_to), rel=1e-14)


def test_waist_offset_and_rayleigh_boundary():
    zw = 3.0
    assert route(zw + ZR, zw - ZR, z_waist=zw)[0][0] == fb.FR_ROUTE_AS       # both exactly at z_R: near
    ks = [s[0] for s in route(zw + 1.01 * ZR, zw, z_waist=zw)]
    assert ks == [fb.FR_ROUTE_DIRECT_INVERSE]                                 # far plane back to the waist


def test_argument_errors():
    L = fb.lib()
    steps = (fb.FrRouteStep * 2)()
    assert L.fr_plan_route(0.0, 0.0, LAM, N, DX, 0.0, 1.0, steps, 2) == fb.FR_EINVAL
    assert L.fr_plan_route(W0, 0.0, LAM, 0, DX, 0.0, 1.0, steps, 2) == fb.FR_EINVAL
    assert L.fr_plan_route(W0, 0.0, LAM, N, DX, float("nan"), 1.0, steps, 2) == fb.FR_EINVAL
    assert L.fr_plan_route(W0, 0.0, LAM, N, DX, 0.0, 1.0, steps, 1) == fb.FR_EINVAL
    assert L.fr_plan_route(W0, 0.0, LAM, N, DX, 0.0, 1.0, None, 2) == fb.FR_EINVAL
