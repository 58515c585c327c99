"""Seeded synthetic inputs for the Fresnel + MFT path (pupils, phase maps, masks, DM heights,
wavelength grids, random fields).

This module holds input generation only and none of the propagation arithmetic: the
tests, the benchmark and the smoke check build one set of float64 master inputs here and
hand the same arrays to both the GPU library and the CPU reference.

The paper's own optics (the shaped-pupil system of its Appendix B) come from data files that
are not available, so these generators stand in for them with the regime the paper describes
(Sec. 1.2: 32x32 to 64x64-actuator mirrors, pupils sampled by hundreds to thousands of pixels,
N = 2048 ... 8192 padded grids). Masks are arrays shared by both sides, so no parity result
depends on how a boundary pixel is decided.
"""

import numpy as np

LAMBDA_C = 550e-9


def _coords(n):
    return np.arange(n, dtype=np.float64) - (n // 2)


def radius_grid(n):
    """Distance of every pixel centre from pixel (n//2, n//2), in pixels."""
    c = _coords(n)
    return np.hypot(c[:, None], c[None, :])


def circular_aperture(n, radius_px):
    """1 inside r < radius (strict), 0 outside."""
    return (radius_grid(n) < radius_px).astype(np.float64)


def pupil_amplitude(n_d, obscuration=0.1, spider_width=0.01, n_spiders=4):
    """Clear circle of diameter n_d px with a central obscuration of diameter obscuration*D and
    n_spiders=4 radial arms (a '+') each spider_width*D wide; 1 = clear."""
    c = _coords(n_d)
    r = np.hypot(c[:, None], c[None, :])
    a = (r < n_d / 2.0) & ~(r < obscuration * n_d / 2.0)
    if n_spiders:
        if n_spiders != 4:
            raise ValueError("only the 4-arm '+' spider is provided")
        half = spider_width * n_d / 2.0
        a &= ~(np.abs(c)[:, None] < half)
        a &= ~(np.abs(c)[None, :] < half)
    return a.astype(np.float64)


def power_law_opd(n_d, clear, rms_m=10e-9, psd_exponent=-3.0, seed=0):
    """Phase map with PSD ~ f^psd_exponent: complex white noise times f^(psd_exponent/2)
    (f in cycles per D, f = 0 removed), inverse transformed, real part, mean removed and scaled
    to rms_m over the clear pixels, zero outside. PCG64 default_rng(seed)."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n_d, n_d)) + 1j * rng.standard_normal((n_d, n_d))
    k = np.fft.fftfreq(n_d) * n_d
    f = np.hypot(k[:, None], k[None, :])
    filt = np.zeros_like(f)
    filt[f > 0] = f[f > 0] ** (psd_exponent / 2.0)
    opd = np.fft.ifft2(white * filt).real
    m = clear > 0
    opd = opd - opd[m].mean()
    opd = opd * (rms_m / np.sqrt(np.mean(opd[m] ** 2)))
    opd[~m] = 0.0
    return opd


def dm_heights(n_act, seed, sigma_m=2e-9):
    """Actuator surface heights N(0, sigma_m), PCG64 default_rng(seed)."""
    return np.random.default_rng(seed).normal(0.0, sigma_m, (n_act, n_act))


def focal_coords(m, du):
    """Focal-plane coordinate of pixel k, (k - m//2) du, in lambda/D."""
    return (np.arange(m, dtype=np.float64) - (m // 2)) * du


def occulter_spot(m=256, du=8.0 / 256, radius=3.0):
    """Opaque spot of the given radius [lambda_c/D] on an m x m grid: 1 where blocked (r < radius)."""
    u = focal_coords(m, du)
    return (np.hypot(u[:, None], u[None, :]) < radius).astype(np.float64)


def lyot_stop(n_d, diameter_frac=0.9):
    """Clear circle of diameter diameter_frac * D on the n_d grid."""
    return circular_aperture(n_d, diameter_frac * n_d / 2.0)


def dark_hole(m=512, du=0.25, r_in=3.0, r_out=10.0):
    """Half annulus r_in <= rho <= r_out [lambda_c/D] with u > 0 (right half) on the detector."""
    u = focal_coords(m, du)
    rho = np.hypot(u[:, None], u[None, :])
    return ((rho >= r_in) & (rho <= r_out) & (u[None, :] > 0)).astype(np.float64)


def wavelengths(n, lo=500e-9, hi=600e-9):
    """n wavelengths uniform over [lo, hi] inclusive (a single one is LAMBDA_C)."""
    if n == 1:
        return np.array([LAMBDA_C])
    return np.linspace(lo, hi, n)


def _smooth7(v):
    for p in (2, 3, 5, 7):
        while v % p == 0:
            v //= p
    return v == 1


def padded_sizes(n_lambda=21, lo=3584, hi=4096):
    """Per-wavelength padded grid edges: for wavelength k the 7-smooth multiple of 16 nearest
    lo + (hi - lo) k / (n_lambda - 1), ties going up."""
    out = []
    for k in range(n_lambda):
        target = lo + (hi - lo) * k / max(n_lambda - 1, 1)
        cands = [v for v in range(16, 2 * hi + 16, 16) if _smooth7(v)]
        best = min(cands, key=lambda v: (abs(v - target), -v))
        out.append(best)
    return out


def random_field(n, seed, dtype=np.complex128):
    """Complex field with N(0,1) real and imaginary parts (seeded)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(dtype)


def gaussian_beam(n, w0_px):
    """exp(-r^2 / w0^2) on pixel units, axis at pixel n//2."""
    r = radius_grid(n)
    return np.exp(-(r / float(w0_px)) ** 2)


def sine_opd(n, dx, period_m, amplitude_m):
    """1-D sinusoidal OPD along x: amplitude sin(2 pi x / period), x = (i - n//2) dx."""
    x = _coords(n) * dx
    return np.broadcast_to(amplitude_m * np.sin(2 * np.pi * x / period_m), (n, n)).copy()


def embed_centred(a, n):
    """An n_d x n_d map placed in an n x n zero map with its centre pixel on (n//2, n//2)."""
    a = np.asarray(a)
    m = a.shape[0]
    out = np.zeros((n, n), dtype=a.dtype)
    o = n // 2 - m // 2
    out[o:o + m, o:o + m] = a
    return out


def shaped_pupil(n_d, bars=3, bar_width=0.06):
    """A binary pupil standing in for a shaped-pupil mask: a clear circle of diameter n_d px
    crossed by `bars` opaque horizontal bars of width bar_width D, evenly spaced."""
    c = _coords(n_d) / n_d  # in units of D
    r = np.hypot(c[:, None], c[None, :])
    clear = r < 0.5
    for k in range(bars):
        y0 = -0.5 + (k + 1) / (bars + 1)
        clear &= ~(np.abs(c[:, None] - y0) < bar_width / 2)
    return clear.astype(np.float64)


def bowtie_mask(n, px_per_lamd, r_in=2.5, r_out=9.0, opening_deg=65.0):
    """A focal-plane mask: clear between r_in and r_out lambda/D inside two opposite wedges of
    full angle opening_deg about the x axis, opaque elsewhere; px_per_lamd pixels per lambda/D."""
    c = _coords(n) / float(px_per_lamd)
    x, y = c[None, :], c[:, None]
    r = np.hypot(x, y)
    ang = np.degrees(np.arctan2(np.abs(y), np.abs(x)))
    return ((r >= r_in) & (r < r_out) & (ang <= opening_deg / 2)).astype(np.float64)

