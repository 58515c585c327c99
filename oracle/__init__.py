"""FP64 CPU oracle for the Fresnel + matrix-Fourier-transform hot path of
Douglas & Perrin, "Accelerated Modeling of Near and Far-Field Diffraction for
Coronagraphic Optical Systems" (SPIE 2018, arXiv:1806.06467).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library
and its Python binding) never does, and this package imports nothing from it.

Every routine here is the plain definition of what the paper's method computes,
written out in float64 with explicit DFT / MFT matrices and no FFT: slow on
purpose, so that it can be checked against the paper and the mathematics by eye.

Pins (see tests/test_oracle_*.py): brute-force DFT on tiny grids, Parseval,
the complex Gaussian-beam closed form, the Talbot self-imaging closed form,
the thin-lens q-parameter law, the Airy pattern, the direct Fresnel step's agreement with
the angular-spectrum step where its kernel is periodic, the exact DFT special case of
the MFT, dot-product (adjoint) identities, the AS/MFT lattice invariance,
finite differences and a Taylor test of the gradient; the multi-optic system (O11) by the
complex Gaussian beam carried through lenses and a focus by the q-law, exact energy
conservation across near and far planes, and the relay's pitch ratios.

The composed Lyot-train intensity (O5) is pinned through its parts and by three
whole-train cases: a full-band occulter rejects everything, no occulter leaves the
Lyot-stopped pupil MFT, and a one-pixel spot on the axis removes exactly the field's
mean term (plus the dot-product identity of the whole linear map). The exact transfer
function's evanescent branch (O10) is pinned by continuity at grazing incidence (its
piston phase) and by the adjoint identity between the steps over z and -z (its decay
for z < 0). No oracle function is parity unpinned.
"""

from .core import (  # noqa: F401
    centred, signed_index, dft_matrix, dft2, idft2, transfer_function,
    as_propagate, as_propagate_rows, optic_phasor, fresnel_step, mft_matrix, mft, mft_adjoint,
    direct_pitch, quadratic_phase, direct_kernel_matrix, direct_fresnel, direct_fresnel_rows,
    direct_fresnel_adjoint, transfer_function_exact, as_propagate_exact,
)
from .relay import (  # noqa: F401
    pilot_through_lens, route, system_plan, propagate_system, gaussian_through_system,
)
from .train import (  # noqa: F401
    embed, extract, dm_influence, dm_surface, TrainGeometry, train_forward,
    dm_to_detector, dm_to_detector_adjoint,
    train_psf, train_backward, train_loss, train_grad, fd_grad,
)
