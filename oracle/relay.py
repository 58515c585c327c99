"""O11. A multi-optic system propagated plane by plane (App. B: the paper's benchmark relay of an
aperture, thin-lens mirrors, a shaped pupil, a focal-plane mask and a final focus, with Fresnel
propagation between them; Sec. 1.1: the direct and the angular-spectrum methods carry the
wavefront, a Gaussian pilot beam choosing between them after Lawrence).

TEST INFRASTRUCTURE (see the package docstring): plain float64, one definition after another.

Reading of the paper (it names the pilot beam but not its rule): a plane within one Rayleigh
distance z_R = pi w0^2 / lambda of the pilot beam's waist is near and holds the field on the
waist plane's pitch; a farther plane is far and holds the field on the pitch lambda |d| / (n dx_w)
of the direct step from the waist over its distance d. Between two near planes the field moves
by one angular-spectrum step; otherwise it goes through the waist plane: from a far plane by the
inverse of the direct step, from a near one by the angular spectrum, and on to a far plane by
the direct step, to a near one by the angular spectrum. A thin lens of focal f changes the
pilot beam by the law of the complex beam parameter, 1/q' = 1/q - 1/f, with q = (z - z_waist) -
i z_R in the sign convention of the transfer function exp(-i pi lambda z f^2) (under which a
Gaussian beam is (q0 / q) exp(i pi r^2 / (lambda q))). The pilot beam starts collimated with its
waist on the first plane.
"""

import numpy as np

from .core import as_propagate, direct_fresnel, direct_fresnel_adjoint, direct_pitch, optic_phasor


def pilot_through_lens(w0, z_waist, wavelength, z_lens, focal):
    """The pilot beam (waist radius, waist position) after a thin lens of focal `focal` at
    z_lens."""
    z_r = np.pi * w0 * w0 / wavelength
    q = complex(z_lens - z_waist, -z_r)
    q2 = 1.0 / (1.0 / q - 1.0 / focal)
    z_r2 = -q2.imag
    return float(np.sqrt(wavelength * z_r2 / np.pi)), float(z_lens - q2.real)


def route(w0, z_waist, wavelength, n, pitch, z_from, z_to):
    """The steps from z_from to z_to: a list of ("as", z), ("direct", d) and ("inverse", d)
    with the pitch each step leaves the field on, as (kind, distance, pitch_before, pitch_after)."""
    z_r = np.pi * w0 * w0 / wavelength
    d_from, d_to = z_from - z_waist, z_to - z_waist
    near_from, near_to = abs(d_from) <= z_r, abs(d_to) <= z_r
    # the waist plane's pitch, from the pitch the field has on z_from
    dx_w = pitch if near_from else wavelength * abs(d_from) / (n * pitch)
    steps = []
    if z_to == z_from:
        return steps
    if near_from and near_to:
        return [("as", z_to - z_from, dx_w, dx_w)]
    if not near_from:
        steps.append(("inverse", d_from, pitch, dx_w))
    elif d_from != 0.0:
        steps.append(("as", -d_from, dx_w, dx_w))
    if near_to:
        if d_to != 0.0:
            steps.append(("as", d_to, dx_w, dx_w))
    else:
        steps.append(("direct", d_to, dx_w, direct_pitch(n, dx_w, wavelength, d_to)))
    return steps


def system_plan(n, dx, wavelength, beam_radius, optics):
    """Per plane its pitch (on which its masks are sampled), the steps to the next plane, and
    the number of 2-D transforms (two per angular-spectrum step, one per direct step).
    optics: (z from the previous plane, lens focal length or 0, amp or None, opd or None)."""
    w0, z_w = float(beam_radius), 0.0
    z, pitch = 0.0, float(dx)
    pitches, routes, transforms = [], [], 0
    for i, (dz, focal, _amp, _opd) in enumerate(optics):
        if i > 0:
            z += dz
        pitches.append(pitch)
        if focal:
            w0, z_w = pilot_through_lens(w0, z_w, wavelength, z, focal)
        if i + 1 == len(optics):
            routes.append([])
            break
        steps = route(w0, z_w, wavelength, n, pitch, z, z + optics[i + 1][0])
        routes.append(steps)
        for kind, _d, _p0, p1 in steps:
            transforms += 2 if kind == "as" else 1
            pitch = p1
    return pitches, routes, transforms


def propagate_system(u, dx, wavelength, beam_radius, optics):
    """The field at the last plane (after its optic) and that plane's pitch: at every plane the
    optic multiplies the field (transmission, OPD phasor of Eq. 3, thin lens, on the plane's
    pitch), then the planned steps carry it to the next plane."""
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[0]
    pitches, routes, _ = system_plan(n, dx, wavelength, beam_radius, optics)
    for i, (_dz, focal, amp, opd) in enumerate(optics):
        u = u * optic_phasor(n, pitches[i], wavelength, amp=amp, opd=opd, lens_focal=focal)
        for kind, d, p0, p1 in routes[i]:
            if kind == "as":
                u = as_propagate(u, p0, wavelength, d)
            elif kind == "direct":
                u, _ = direct_fresnel(u, p0, wavelength, d)
            else:
                # the inverse of the direct step from the waist plane (pitch p1) over d
                u = direct_fresnel_adjoint(u, p1, wavelength, d) * (p0 / p1) ** 2
    return u, pitches[-1]


def gaussian_through_system(n, pitch, wavelength, w0, optics):
    """Closed form: a Gaussian beam exp(-r^2 / w0^2) with its waist on the first plane, carried
    through the thin lenses and distances of `optics` (masks ignored), sampled on the last
    plane's grid of pitch `pitch`: (q0 / q) exp(i pi r^2 / (lambda q)) with q = d - i z_R at the
    waist, q -> q + dz over a distance, 1/q -> 1/q - 1/f at a lens, and the amplitude factor
    carried as the running product of q_before / q_after over the distances."""
    z_r = np.pi * w0 * w0 / wavelength
    q = complex(0.0, -z_r)
    amp = 1.0 + 0.0j
    for i, (dz, focal, _a, _o) in enumerate(optics):
        if i > 0 and dz != 0.0:
            amp *= q / (q + dz)
            q = q + dz
        if focal:
            q = 1.0 / (1.0 / q - 1.0 / focal)
    c = np.arange(n) - n // 2
    r2 = (c[:, None] ** 2 + c[None, :] ** 2) * float(pitch) ** 2
    return amp * np.exp(1j * np.pi * r2 / (wavelength * q))
