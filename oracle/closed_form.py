"""Closed-form solution of the Neumann box problem.

Test infrastructure only (see the package docstring).

On an unjittered mesh whose active cells form an axis-aligned box, every
open face along axis d has the same coefficient c_d, and the operator is
    L = sum_d c_d * (I (x) T_{m_d} (x) I),
with T_m the 1-D second difference matrix with reflecting (Neumann) ends.
The DCT-II vectors cos(pi k (j + 1/2) / m) diagonalise T_m with eigenvalues
4 sin^2(pi k / (2 m)), so for a right-hand side with zero sum the solution
with zero mean is IDCT(DCT(b) / lambda) (mode k = 0 dropped).  The pinned
solution is that function shifted so that it vanishes at the pin.
"""
from __future__ import annotations

import numpy as np
from scipy.fft import dctn, idctn


def neumann_box_solve(b_box, coeffs, pin_index=(0, 0, 0)):
    """b_box: [mx, my, mz] right-hand side with zero sum; coeffs: (c_x, c_y,
    c_z) face coefficients per axis.  Returns p with p[pin_index] = 0."""
    b_box = np.asarray(b_box, dtype=np.float64)
    lam = np.zeros(b_box.shape)
    for d, m in enumerate(b_box.shape):
        k = np.arange(m)
        ev = 4.0 * np.sin(np.pi * k / (2.0 * m)) ** 2
        shape = [1, 1, 1]
        shape[d] = m
        lam = lam + coeffs[d] * ev.reshape(shape)
    bh = dctn(b_box, type=2, norm="ortho")
    ph = np.zeros_like(bh)
    nz = lam > 0
    ph[nz] = bh[nz] / lam[nz]
    p = idctn(ph, type=2, norm="ortho")
    return p - p[pin_index]
