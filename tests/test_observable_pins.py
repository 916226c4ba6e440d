"""Pins of the oracle's observables and initial state against closed forms.

The observables (the drop velocity of eqs 33-34, the deformation from the
second moments, the interface band of psi statistics) and the initial shear
profile feed every GPU observable comparison; these tests fix them against
results that follow from their definitions on constructed fields, not against
the oracle's own code:

* deformation: a colour field whose level sets are similar ellipses (or
  ellipsoids) with semi-axes a, b (, c) has second moments proportional to
  a^2, b^2 (, c^2), so D = (L - B)/(L + B) = (a - b)/(a + b) (3-D: largest
  and smallest axes) whatever the profile across the interface, up to the
  lattice sampling of a smooth profile; a rotation of the axes and an
  off-centre position must not change it;
* eq 33 velocity: equilibrium populations at a velocity that is U_in on nodes
  with rhoN >= 0 and something else elsewhere give exactly U_in, with the tie
  rhoN = 0 counted inside (eq 34);
* psi_min / psi_max: taken over |rhoN| <= 0.5, ties at exactly 0.5 included;
* initial shear: the profile u_x = shear (y - (ny - 1)/2) meets walls at
  y = -1/2 and ny - 1/2 moving at -/+ u_w when shear = 2 u_w / ny, and is the
  steady Couette state there (it stays put under the whole step).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import bruteforce as bf


def _pops_at_rest(rhoR, rhoB, three):
    """Colour populations at rest: all mass on the rest direction, so that
    rho^k is exactly the given value (no rounding in the direction sum)."""
    Q = 19 if three else 9
    fR = np.zeros((Q,) + rhoR.shape)
    fB = np.zeros((Q,) + rhoB.shape)
    fR[0] = rhoR
    fB[0] = rhoB
    return fR, fB


def _oracle_with_colour(shape, rhoN, lattice, **over):
    nz, ny, nx = shape
    p = W.finalize(dict(lattice=lattice, nx=nx, ny=ny, nz=nz, sigma0=0.0, E0=0.0, fd_enable=0, **over))
    o = oracle.Oracle(p)
    fR, fB = _pops_at_rest(0.5 * (1 + rhoN), 0.5 * (1 - rhoN), lattice == W.D3Q19)
    o.set_field("fR", fR)
    o.set_field("fB", fB)
    return o


def _ellipse_field(shape, centre, axes, rot, width):
    """rhoN = tanh(2 s (1 - r_e)/W), r_e the elliptic radius in the frame
    rotated by `rot` (columns: the principal directions), s the geometric mean
    of the semi-axes: level sets are similar ellipses (ellipsoids)."""
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    # coordinates in (x, y, z) order
    D = len(axes)
    X = np.stack([grids[len(shape) - 1 - a] - centre[a] for a in range(D)])
    Y = np.tensordot(rot.T, X, axes=1)          # components along the principal directions
    re = np.sqrt(sum((Y[a] / axes[a]) ** 2 for a in range(D)))
    s = float(np.prod(axes)) ** (1.0 / D)
    return np.tanh(2.0 * s * (1.0 - re) / width)


def _rot2(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s], [s, c]])


@pytest.mark.parametrize("a,b,theta,width", [(24.0, 16.0, 0.0, 3.0), (24.0, 16.0, np.pi / 6, 3.0),
                                             (30.0, 12.0, 1.1, 5.0), (20.0, 19.0, 0.4, 3.0)])
def test_deformation_of_an_ellipse(a, b, theta, width):
    """2-D: D = (a - b)/(a + b) for every interface width and orientation."""
    shape = (1, 96, 104)
    rN = _ellipse_field(shape[1:], (51.3, 47.6), (a, b), _rot2(theta), width)[None]
    o = _oracle_with_colour(shape, rN, W.D2Q9)
    ob = o.observables()
    D = oracle.deformation(ob["second"], 2)
    assert abs(D - (a - b) / (a + b)) < 2e-5 * (a - b) / (a + b) + 1e-7, (D, (a - b) / (a + b))
    # the centroid is the centre of the construction
    assert abs(ob["centroid"][0] - 51.3) < 1e-4 and abs(ob["centroid"][1] - 47.6) < 1e-4


def test_deformation_of_an_ellipsoid():
    """3-D: D = (a - c)/(a + c) from the largest and smallest semi-axes, for an
    ellipsoid turned about two axes."""
    t1, t2 = 0.5, -0.3
    Rz = np.array([[np.cos(t1), -np.sin(t1), 0], [np.sin(t1), np.cos(t1), 0], [0, 0, 1]])
    Ry = np.array([[np.cos(t2), 0, np.sin(t2)], [0, 1, 0], [-np.sin(t2), 0, np.cos(t2)]])
    a, b, c = 14.0, 10.0, 7.0
    shape = (40, 44, 48)
    rN = _ellipse_field(shape, (23.7, 21.2, 19.9), (a, b, c), Rz @ Ry, 3.0)
    o = _oracle_with_colour(shape, rN, W.D3Q19)
    D = oracle.deformation(o.observables()["second"], 3)
    assert abs(D - (a - c) / (a + c)) < 2e-5 * (a - c) / (a + c), (D, (a - c) / (a + c))


def test_deformation_of_a_circle_is_zero_and_scale_free():
    shape = (1, 64, 64)
    rN = _ellipse_field(shape[1:], (31.5, 31.5), (15.0, 15.0), np.eye(2), 3.0)[None]
    o = _oracle_with_colour(shape, rN, W.D2Q9)
    assert oracle.deformation(o.observables()["second"], 2) < 1e-9


def _equilibrium(e, w, rho, u):
    """Second-order Maxwellian equilibrium (the textbook form), per node."""
    D = u.shape[0]
    eu = np.tensordot(e[:, :D].astype(np.float64), u, axes=1)
    uu = (u * u).sum(0)
    return w[:, None, None, None] * rho[None] * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * uu[None])


@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_eq33_velocity_is_the_mean_over_the_indicator(lattice):
    """Eqs 33-34: U = sum u N / sum N with N = [rhoN >= 0]. Populations at
    equilibrium with velocity U_in where rhoN > 0, U_tie where rhoN = 0
    exactly, U_out where rhoN < 0, and no force (clean, no gravity): the
    result is (n_in U_in + n_tie U_tie)/(n_in + n_tie)."""
    three = lattice == W.D3Q19
    shape = (6, 9, 10) if three else (1, 12, 14)
    D = 3 if three else 2
    e, w, _ = bf.lattice(three)
    rng = np.random.default_rng(5)
    cls = rng.integers(0, 3, shape)                 # 0 outside, 1 inside, 2 tie
    rhoR = np.where(cls == 1, 0.9, np.where(cls == 2, 0.5, 0.1))
    rhoB = np.where(cls == 1, 0.1, np.where(cls == 2, 0.5, 0.9))
    U = {1: np.array([0.012, -0.007, 0.004]), 2: np.array([-0.02, 0.011, 0.009]),
         0: np.array([0.003, 0.015, -0.013])}
    u = np.zeros((D,) + shape)
    for c, v in U.items():
        for a in range(D):
            u[a][cls == c] = v[a]
    fR = _equilibrium(e, w, rhoR, u)
    fB = _equilibrium(e, w, rhoB, u)
    p = W.finalize(dict(lattice=lattice, nx=shape[2], ny=shape[1], nz=shape[0], sigma0=0.0, E0=0.0,
                        fd_enable=0))
    o = oracle.Oracle(p)
    o.set_field("fR", fR)
    o.set_field("fB", fB)
    ob = o.observables()
    n_in, n_tie = int((cls == 1).sum()), int((cls == 2).sum())
    expect = (n_in * U[1] + n_tie * U[2]) / (n_in + n_tie)
    for a in range(D):
        assert abs(ob["velocity"][a] - expect[a]) < 1e-15, (a, ob["velocity"][a], expect[a])
    assert ob["nsum"] == n_in + n_tie
    # the tie rhoN = 0 is exact here: moving the tie class outside changes U
    assert np.abs(expect[:D] - U[1][:D]).max() > 1e-3


def test_psi_band_statistics():
    """psi_min / psi_max over |rhoN| <= 0.5 (ties included); larger and
    smaller psi on nodes just outside the band are ignored; psi_av = sum G psi /
    sum G equals a uniform psi."""
    shape = (1, 10, 12)
    rng = np.random.default_rng(7)
    cls = rng.integers(0, 5, shape[1:])[None]
    # rho^R, rho^B exactly representable: rhoN = 0.5, -0.5, 0.25, 0.75, -0.75
    rR = np.choose(cls, [0.75, 0.25, 0.625, 0.875, 0.125])
    rhoN = 2 * rR - 1
    o = _oracle_with_colour(shape, rhoN, W.D2Q9)
    psi = rng.uniform(0.2, 0.4, shape)
    band = np.abs(rhoN) <= 0.5
    assert band.sum() > 10 and (~band).sum() > 10
    # the band's own extremes on the tie nodes |rhoN| = 0.5 exactly
    ties = np.argwhere(np.abs(rhoN) == 0.5)
    psi[tuple(ties[0])] = 0.05
    psi[tuple(ties[1])] = 0.61
    # bigger extremes just outside the band
    out = np.argwhere(~band)
    psi[tuple(out[0])] = 0.01
    psi[tuple(out[1])] = 0.9
    o.set_field("psi", psi)
    o.set_field("phi", np.zeros(shape))
    ob = o.observables()
    assert ob["psi_min"] == 0.05 and ob["psi_max"] == 0.61
    o.set_field("psi", np.full(shape, 0.3))
    assert abs(o.observables()["psi_av"] - 0.3) < 1e-15


@pytest.mark.parametrize("ny,u_w", [(24, 0.01), (31, 0.02)])
def test_initial_shear_profile_is_the_couette_state(ny, u_w):
    """u_x = shear (y - (ny - 1)/2) with shear = 2 u_w / ny: linear, zero on
    the centre line, extrapolating to -/+ u_w at the walls (y = -1/2 and
    ny - 1/2), and steady under the whole step with half-way bounce-back at
    walls moving at -/+ u_w (a profile shifted by half a node would drift)."""
    shear = 2 * u_w / ny
    p = W.finalize(dict(lattice=W.D2Q9, nx=8, ny=ny, bc=[W.PERIODIC, W.WALL, W.PERIODIC],
                        wall_u=[[0, 0, 0], [0, 0, 0], [-u_w, 0, 0], [u_w, 0, 0], [0, 0, 0], [0, 0, 0]],
                        sigma0=0.0, E0=0.0, fd_enable=0, muR0=0.1, muB0=0.1))
    o = oracle.Oracle(p).init(dict(W.BASE_INIT, drops=[], shear_rate=shear))
    ux = o.field("u")[0, 0]
    y = np.arange(ny)
    assert np.abs(ux - ux[:, :1]).max() == 0.0
    col = ux[:, 0]
    slope, icpt = np.polyfit(y, col, 1)
    assert abs(slope - shear) < 1e-14 and np.abs(col - (slope * y + icpt)).max() < 1e-16
    assert abs((slope * -0.5 + icpt) + u_w) < 1e-15 and abs((slope * (ny - 0.5) + icpt) - u_w) < 1e-15
    assert np.abs(o.field("u")[1]).max() < 1e-18
    # steady under the step to rounding (a slope 2 % off drifts by ~1e-2 u_w)
    o.step(400)
    col2 = o.field("u")[0, 0, :, 0]
    assert np.abs(col2 - col).max() < 1e-14, np.abs(col2 - col).max()
