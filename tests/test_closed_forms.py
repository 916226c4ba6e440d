"""The closed forms the validations compare against, pinned to facts other than
their own transcription: eq 30 is the time integral of the surface value of
eq 29 (with the dimensionally consistent denominator), the surface value tends
to the steady uptake of a sphere with a linear flux condition, 1/(1 + mR),
and eq 29 tends to 1 far from the drop."""
import numpy as np
import pytest
from scipy.integrate import quad

import bench


P = dict(R=30.0, D=0.1, ra=0.2, psi_inf=1.0, phi0=0.0005)


def test_eq30_is_the_integral_of_eq29_at_the_surface():
    R, D, ra, pinf, phi0 = P["R"], P["D"], P["ra"], P["psi_inf"], P["phi0"]
    surf = lambda t: bench.adsorption_theory(t, [R], R, D, ra, pinf, phi0)[1][0]
    for T in (50.0, 500.0, 27000.0):
        integral, _ = quad(lambda t: ra * phi0 * surf(t), 0.0, T, limit=200)
        psi, _ = bench.adsorption_theory(T, [R], R, D, ra, pinf, phi0)
        assert psi == pytest.approx(integral, rel=1e-8)


def test_eq29_limits():
    R, D, ra, pinf, phi0 = P["R"], P["D"], P["ra"], P["psi_inf"], P["phi0"]
    m = ra * pinf / D
    # long times: the steady sphere solution phi = phi0 (1 - (mR/(1+mR)) R/r) at r = R
    _, s = bench.adsorption_theory(1e14, [R], R, D, ra, pinf, phi0)
    assert s[0] == pytest.approx(1.0 / (1.0 + m * R), rel=1e-5)
    # far from the drop nothing has changed yet; the profile rises with r
    r = np.linspace(R, 6 * R, 50)
    _, prof = bench.adsorption_theory(2000.0, r, R, D, ra, pinf, phi0)
    assert prof[-1] == pytest.approx(1.0, abs=1e-12)
    assert (np.diff(prof) > 0).all()
    # start: the surface value starts at 1 and falls like 1 - m sqrt(pi D t)
    t = 1e-10
    _, s0 = bench.adsorption_theory(t, [R], R, D, ra, pinf, phi0)
    assert 1.0 - s0[0] == pytest.approx(m * np.sqrt(np.pi * D * t), rel=1e-3)


def test_eq30_initial_slope():
    """d(psi/psi_inf)/dt = ra phi0 at t = 0 (the bulk next to a clean interface is at phi0)."""
    R, D, ra, pinf, phi0 = P["R"], P["D"], P["ra"], P["psi_inf"], P["phi0"]
    t = 1e-8
    psi, _ = bench.adsorption_theory(t, [R], R, D, ra, pinf, phi0)
    assert psi / t == pytest.approx(ra * phi0, rel=1e-4)
