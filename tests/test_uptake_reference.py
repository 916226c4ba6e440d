"""The sharp-interface reference of uptake onto a circular drop (bench.radial_uptake,
the 2-D analogue of eq 30 that the adsorption workload is checked against),
pinned to facts other than itself: it conserves the surfactant, starts at the
adsorption rate of a clean interface, and ends at the Langmuir equilibrium
that the global balance of the closed domain fixes."""
import numpy as np
import pytest
from scipy.optimize import brentq

import bench

R, D, ra, rd, pinf, phi0 = 25.0, 0.02, 0.1, 0.05, 1.0, 0.05
R_OUT = 128.0 / np.sqrt(np.pi)   # the disk of the periodic 128 x 128 box's area


def total(psi, r, phi, nr):
    dr = (R_OUT - R) / nr
    return R * psi + float((r * dr * phi).sum())


def test_conserves_surfactant():
    nr = 200
    for mode in (0, 1):
        ps, r, ph = bench.radial_uptake(R, R_OUT, D, ra, rd, pinf, phi0, [0.0], source_mode=mode, nr=nr)
        m0 = total(ps[0], r, ph, nr)
        ps, r, ph = bench.radial_uptake(R, R_OUT, D, ra, rd, pinf, phi0, [300.0], source_mode=mode, nr=nr)
        assert ps[0] > 0.0
        assert total(ps[0], r, ph, nr) == pytest.approx(m0, rel=1e-12)


def test_initial_rate_is_that_of_a_clean_interface():
    t = 0.002
    ps, _, _ = bench.radial_uptake(R, R_OUT, D, ra, rd, pinf, phi0, [t], nr=400, dt=0.0001)
    assert ps[0] / t == pytest.approx(ra * pinf * phi0, rel=2e-3)


def test_ends_at_the_global_langmuir_equilibrium():
    """psi = psi_inf ra phi / (ra phi + rd) with phi from the balance
    phi0 A = phi A + psi 2 pi R over the bulk area A (uniform phi at the end)."""
    A = np.pi * (R_OUT ** 2 - R ** 2)
    f = lambda ph: phi0 * A - ph * A - 2 * np.pi * R * pinf * ra * ph / (ra * ph + rd)
    ph_f = brentq(f, 0.0, phi0)
    psi_eq = pinf * ra * ph_f / (ra * ph_f + rd)
    ps, r, ph = bench.radial_uptake(R, R_OUT, D, ra, rd, pinf, phi0, [3.0e6], nr=100, dt=100.0)
    assert ps[0] == pytest.approx(psi_eq, rel=1e-6)
    assert np.abs(ph - ph_f).max() <= 1e-6 * ph_f
    # the values of this balance for the adsorption workload
    assert ph_f == pytest.approx(0.049027, abs=1e-6) and psi_eq == pytest.approx(0.089298, abs=1e-6)
