"""Tolerances of the multipole and masked-power parity tests, derived from
the conditioning of the matrices the estimators invert.

Power multipoles P_l = F^-1 p per bin (the discrete Fisher matrix of
eq. pk-limit, F[l][l'] = sum over the bin's modes of L_l L_l' (w)).  The
numerators p_l carry the FP32-FFT error of |D|^2 times |L_l| <= 1, at most
eps p_0 each, so |dP_l| <= eps * a_l * P_0 with the gain
a_l = F_00 sum_l' |F^-1_{l l'}| (5 for l = 2 and 9 for l = 4 in the
continuum, 1 for the monopole; larger on shells the cubic grid truncates).
With eps = 1e-6 (ten times the measured FP32-FFT error of P) the gate is
1e-6 * max(10, a_l) * |P_0|: 1e-5 |P_0| on ordinary shells.

Masked power P = F^-1 p (Monte Carlo Fisher matrix): with errors of at most
eps relative in F and p, |dP| <= 2 eps * s |P| for s the Skeel condition
number || |F^-1| |F| ||_inf (about 2 for the tested windows), eps = 1e-5.
"""

import numpy as np

from oracle.multipoles import legendre


def multipole_gain(bin_idx, mu2, nb, lmax, weight=None):
    """a[l, b] = F_00 sum_l' |F^-1_{l l'}| of bin b's discrete Fisher matrix."""
    ells = list(range(0, lmax + 1, 2))
    mu = np.sqrt(np.clip(mu2, 0.0, 1.0))  # even multipoles depend on mu^2 only
    L = np.stack([legendre(l, mu) for l in ells])
    out = np.zeros((len(ells), nb))
    for b in range(nb):
        m = bin_idx == b
        Lb = L[:, m]
        w = np.ones(Lb.shape[1]) if weight is None else weight[m]
        F = (Lb * w[None, :]) @ Lb.T
        out[:, b] = F[0, 0] * np.abs(np.linalg.inv(F)).sum(axis=1)
    return out


def multipole_power_gate(gain, p0):
    """Allowed |dP_l| per (l, bin) for reference monopole p0 (per bin)."""
    return 1e-6 * np.maximum(10.0, gain) * np.abs(p0)[None, :]


def masked_power_rtol(F):
    """Allowed |dP| / |P| of the masked power spectrum for Fisher matrix F."""
    F = np.asarray(F, dtype=np.float64)
    s = np.linalg.norm(np.abs(np.linalg.inv(F)) @ np.abs(F), np.inf)
    return 2e-5 * s
