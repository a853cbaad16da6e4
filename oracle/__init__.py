"""FP64 CPU oracle for the idealized binned power spectrum and bispectrum.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
It shares no code with the HIP path.

Parity status of each function (what pins it is in ``tests/test_oracle.py``
and ``tests/test_oracle_pins.py``):

* ``power_spectrum``       pinned: Parseval, plane-wave closed form,
                           invariances, statistical recovery of the input P.
* ``triangle_triplets``    pinned: the 196 (= 2 x 98) configurations printed
                           for 8 bins in the bispectrum validation set-up.
* ``triangle_counts``      pinned: brute-force mode counting, integrality,
                           and the continuum Bessel-integral N_0 (end of
                           Sec. IV.D.1) within the shells' discreteness.
* ``bispectrum``           pinned: brute-force k-triplet sums, plane-wave
                           closed form, invariances, Gaussian null and the
                           tree-level bispectrum of a quadratic field.
* ``triplet_sums_sample``, ``count_sample`` (a triplet subset, for large
                           grids) pinned: equal to the full ``bispectrum``
                           entries (sums, absolute sums, exact counts) on
                           32^3 and 64^3 fields, a = b = c included; a
                           shuffled bin remap fails the check.
* ``windowed_polyspectra`` pinned: unbiased means for a field with local
                           2- and 3-point functions under random windows.
* ``masked`` (Monte Carlo Fisher of the masked power spectrum) pinned: the
                           exact expectation equals (1/2) diag(N_b) without a
                           window and a brute-force double sum with one; the
                           Monte Carlo average converges to it; the
                           unwindowed estimate is unbiased for a flat
                           spectrum under a window.
* ``multipoles`` (global line of sight) pinned: the separable bispectrum
                           multipole sum equals explicit mode-triangle loops
                           with the Legendre weight on k_3; the power
                           multipoles with the discrete Fisher matrix are
                           unbiased for an anisotropic Gaussian field;
                           invariance under x-y exchange and z reflection.
* ``weighted`` (P_fid weights, pixel window, shot noise) pinned: weighted
                           sums equal explicit mode-triangle loops; constant
                           P_fid reduces to the unweighted estimators; window
                           deconvolution undoes a window applied in Fourier
                           space; the window sinc(pi n / N)^p equals the
                           average over a particle's position in its cell of
                           the DFT of explicit NGP / CIC / TSC assignment
                           (Gauss-Legendre quadrature, every n incl. Nyquist;
                           a wrong argument or exponent fails); Poisson noise
                           of a uniform field is removed on average from P
                           and B.
* ``injection`` (expectation under an injected bispectrum) pinned: the
                           separable bin average equals explicit loops over
                           closed triangles; the oracle estimator's linear
                           response to the injection averages to it over
                           seeds.
* ``noncubic`` (Nx x Ny x Nz grids, Lx x Ly x Lz boxes) pinned: a cubic
                           geometry reproduces ``polyspec``; separable sums and
                           counts equal explicit mode-triangle loops on small
                           grids (cubic and anisotropic boxes); P of Gaussian
                           fields and the tree-level B of quadratic fields on
                           an anisotropic box average to their expectations.
* ``bk_fisher`` (bispectrum multipoles with the discrete ideal Fisher matrix
                           and the degeneracy factors) pinned: the separable
                           Fisher blocks, N_l and numerators equal explicit
                           loops over closed triangles in every degeneracy
                           case; l_max = 0 gives the monopole estimator; on
                           an alias-free grid the blocks approach the
                           continuum diagonal form.
"""

from .polyspec import (  # noqa: F401
    Result,
    bin_of_modes,
    bispectrum,
    count_sample,
    dft,
    filtered_fields,
    freqs,
    idft,
    kmag2,
    max_component,
    mode_counts,
    window_moments,
    windowed_polyspectra,
    power_spectrum,
    triangle_counts,
    triangle_triplets,
    triple_sums,
    triplet_sums_sample,
    unit_fields,
)
from .brute import brute_sums  # noqa: F401
from . import masked  # noqa: F401,E402
from . import multipoles  # noqa: F401,E402
from . import weighted  # noqa: F401,E402
from . import injection  # noqa: F401,E402
from . import noncubic  # noqa: F401,E402
from . import bk_fisher  # noqa: F401,E402
