"""Pins of the oracle's field gather and of its analytic initial fields.

The gather (Sec. 3.3, on the staggered lattices of eq. (offseteq)) is pinned
by what bilinear interpolation of a cell-shaped particle must do: reproduce
exactly any bilinear function sampled at each component's own staggered
nodes, continue the half-integer-j components across the axis with their
parity (r components even, theta and phi components odd), and see no plasma
field inside the conductors.  The analytic fields (Sec. 5.2 for the monopole,
Sec. 4.3 for the dipole with its corotation field) are pinned by the
equations they must satisfy -- a divergence-free and curl-free vacuum B, the
ideal-conductor field E = -(Omega x r) x B / c inside the star, and a static
vacuum E outside it -- evaluated here by finite differences and Cartesian
cross products, never by restating the oracle's expressions.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1407_1810_amd import workloads as W

# staggered position (sx, sy) of each component's node (i, j), eq. (offseteq)
OFFSETS = {"Er": (0.5, 0.0), "Eth": (0.0, 0.5), "Eph": (0.0, 0.0),
           "Br": (0.0, 0.5), "Bth": (0.5, 0.0), "Bph": (0.5, 0.5)}
# parity across the axis: r components even, theta and phi components odd
PARITY = {"Er": 1.0, "Eth": -1.0, "Eph": -1.0, "Br": 1.0, "Bth": -1.0, "Bph": -1.0}
SLOT = {"Er": (0, 0), "Eth": (0, 1), "Eph": (0, 2), "Br": (1, 0), "Bth": (1, 1), "Bph": (1, 2)}

NR, NTH = 14, 12


def _oracle(**kw):
    p = W.grid_params(NR, NTH, 5.0)
    p.update(dict(n_filt=1, absorb_cells=0, sigma_max=0.0, mover="vay", bg_kind="none", B0=0.0, q_over_m=1.0))
    p.update(kw)
    return O.Oracle(p), p


def _coef(comp):
    """Coefficients (a, b, c, d) of f = a + b X + c Y + d X Y, different for
    every component so that a gather that read one component's lattice for
    another, or swapped X and Y, would fail."""
    k = list(OFFSETS).index(comp)
    return 0.3 + 0.1 * k, 0.011 * (k + 1), -0.017 + 0.005 * k, 0.0013 * (2 - k)


def _f(comp, X, Y):
    a, b, c, d = _coef(comp)
    return a + b * X + c * Y + d * X * Y


def _load_bilinear(o):
    for comp, (sx, sy) in OFFSETS.items():
        rows, cols, _ = o.shape(comp)
        X = (np.arange(rows) + sx)[:, None]
        Y = (np.arange(cols) + sy)[None, :]
        o.set_field(comp, _f(comp, X, Y) + 0.0 * X * Y)


def _gather(o, x, y, comp):
    E, B = o.gather(x, y)
    a, c = SLOT[comp]
    return (E, B)[a][c]


def test_gather_reproduces_bilinear_fields_on_every_lattice():
    """Inside each lattice's own node range the gather returns the bilinear
    function the nodes sample, to rounding: a wrong staggering offset, a
    swapped weight or a component read from another lattice would shift or
    mix the result by O(0.01)."""
    o, _ = _oracle()
    _load_bilinear(o)
    rng = np.random.default_rng(11)
    for comp, (sx, sy) in OFFSETS.items():
        rows, cols, _ = o.shape(comp)
        xs = rng.uniform(sx, rows - 1 + sx, 200)
        ys = rng.uniform(sy, cols - 1 + sy, 200)
        # also the nodes themselves and the corners of the range
        xs = np.concatenate([xs, [sx, rows - 1 + sx, sx + 3.0]])
        ys = np.concatenate([ys, [sy, cols - 1 + sy, sy + 2.0]])
        got = np.array([_gather(o, x, y, comp) for x, y in zip(xs, ys)])
        assert np.abs(got - _f(comp, xs, ys)).max() < 1e-13, comp


@pytest.mark.parametrize("comp", ["Eth", "Br", "Bph"])
def test_gather_axis_parity_of_half_integer_components(comp):
    """Between a pole and the first half-node the lattice is continued across
    the axis with the component's parity: an even component (B_r) keeps the
    half-node's value, an odd one (E_theta, B_phi) falls linearly to zero on
    the axis -- 2 y times the half-node's value in the north, 2 (nth - y)
    times it in the south."""
    o, _ = _oracle()
    _load_bilinear(o)
    sx, sy = OFFSETS[comp]
    rows, _, _ = o.shape(comp)
    rng = np.random.default_rng(12)
    for x in rng.uniform(sx, rows - 1 + sx, 10):
        for y in np.concatenate([rng.uniform(0.0, 0.5, 6), [0.0]]):
            v = _f(comp, x, 0.5)
            want = v if PARITY[comp] > 0 else 2.0 * y * v
            assert _gather(o, x, y, comp) == pytest.approx(want, abs=1e-13)
        for y in np.concatenate([rng.uniform(NTH - 0.5, NTH, 6), [float(NTH)]]):
            v = _f(comp, x, NTH - 0.5)
            want = v if PARITY[comp] > 0 else 2.0 * (NTH - y) * v
            assert _gather(o, x, y, comp) == pytest.approx(want, abs=1e-13)


@pytest.mark.parametrize("comp", ["Er", "Bth", "Bph"])
def test_gather_sees_no_plasma_field_inside_the_conductors(comp):
    """The half-integer-i lattices end half a cell inside the domain; between
    a conductor and the first half-node the field falls linearly to the zero
    that the conductor holds half a cell beyond."""
    o, _ = _oracle()
    _load_bilinear(o)
    rng = np.random.default_rng(13)
    y = 5.7 if OFFSETS[comp][1] == 0.5 else 6.0
    for x in np.concatenate([rng.uniform(0.0, 0.5, 6), [0.0]]):
        want = (x + 0.5) * _f(comp, 0.5, y)
        assert _gather(o, x, y, comp) == pytest.approx(want, abs=1e-13)
    for x in np.concatenate([rng.uniform(NR - 0.5, NR, 6), [float(NR)]]):
        want = (NR + 0.5 - x) * _f(comp, NR - 0.5, y)
        assert _gather(o, x, y, comp) == pytest.approx(want, abs=1e-13)


# --------------------------------------------------------------------------
# Analytic initial fields: the dipole of Sec. 4.3 and the monopole of Sec. 5.2
# --------------------------------------------------------------------------

def _bg_oracle(bg, **kw):
    p = W.grid_params(64, 48, 8.0)
    p.update(dict(n_filt=0, absorb_cells=0, sigma_max=0.0, mover="vay", bg_kind=bg, B0=1.7, omega=0.013,
                  q_over_m=1.0))
    p.update(kw)
    o = O.Oracle(p)
    dxi = math.log(p["r_out"] / p["r_in"]) / p["nr"]

    def at(r, th, t=50.0):
        """Local (r, theta, phi) E and B at radius r, colatitude th."""
        x = math.log(r / p["r_in"]) / dxi
        y = p["nth"] * (1.0 - math.cos(th)) / 2.0
        return o.background(x, y, t)

    return o, p, at


def _to_cart(v, th):
    """Local (r, theta, phi) components at phi = 0 to Cartesian."""
    s, k = math.sin(th), math.cos(th)
    return np.array([s * v[0] + k * v[1], v[2], k * v[0] - s * v[1]])


def _div_curl(F, r, th, h=1e-3):
    """Divergence and the azimuthal curl of an axisymmetric field with no
    phi dependence, by fourth-order central differences of F(r, th) (local
    components): truncation O(h^4), far below the bounds used here."""
    def d(g, a, step):
        return (-g(a + 2 * step) + 8 * g(a + step) - 8 * g(a - step) + g(a - 2 * step)) / (12 * step)

    dr, dt = h * r, h
    s = math.sin(th)
    div = d(lambda q: q * q * F(q, th)[0], r, dr) / (r * r) + d(lambda a: math.sin(a) * F(r, a)[1], th, dt) / (r * s)
    curl = d(lambda q: q * F(q, th)[1], r, dr) / r - d(lambda a: F(r, a)[0], th, dt) / r
    return div, curl


@pytest.mark.parametrize("bg", ["dipole", "monopole"])
def test_background_b_is_a_vacuum_field(bg):
    """B is divergence-free and curl-free outside the star, and B0 is its
    strength on the conductor surface: the dipole's field is 2 B0 radial at
    the pole and B0 meridional at the equator, the monopole's B0 radial."""
    o, p, at = _bg_oracle(bg)
    r0 = p["r_in"]
    B = lambda r, th: at(r, th)[1]
    for r in (1.3 * r0, 2.7 * r0, 5.5 * r0):
        for th in (0.3, 1.1, 2.0, 2.9):
            div, curl = _div_curl(B, r, th)
            scale = np.abs(B(r, th)).max() / r
            assert abs(div) < 1e-9 * scale and abs(curl) < 1e-9 * scale, (r, th, div, curl)
    if bg == "dipole":
        assert B(r0, 0.0)[0] == pytest.approx(2 * p["B0"], rel=1e-12)
        assert B(r0, 0.5 * math.pi)[1] == pytest.approx(p["B0"], rel=1e-12)
        assert abs(B(r0, 0.5 * math.pi)[0]) < 1e-12 * p["B0"]
        # a dipole falls off as r^-3 along every direction
        assert B(4 * r0, 1.0)[0] == pytest.approx(B(2 * r0, 1.0)[0] / 8, rel=1e-12)
    else:
        assert B(r0, 1.2)[0] == pytest.approx(p["B0"], rel=1e-12)
        assert B(3 * r0, 0.4)[0] == pytest.approx(p["B0"] / 9, rel=1e-12)
    assert all(abs(B(2 * r0, th)[2]) == 0.0 for th in (0.2, 1.5))


@pytest.mark.parametrize("bg", ["dipole", "monopole"])
def test_corotation_field_inside_the_star(bg):
    """Inside the conductor the plasma corotates: E = -(Omega z x r) x B / c
    (the ideal-conductor condition of Sec. 4.3 and Sec. 5.2), formed here in
    Cartesian components, so that E . B = 0 (force-free)."""
    o, p, at = _bg_oracle(bg)
    r0, c, om = p["r_in"], p["c"], p["omega"]
    for r in (0.55 * r0, 0.8 * r0, 0.99 * r0):
        for th in (0.0, 0.4, 1.3, 1.9, 3.0):
            E, B = at(r, th)
            Rc = r * _to_cart([1.0, 0.0, 0.0], th)
            v = np.cross([0.0, 0.0, om], Rc)
            want = -np.cross(v, _to_cart(B, th)) / c
            got = _to_cart(E, th)
            assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max() + 1e-16, (r, th, got, want)
            assert abs(np.dot(E, B)) <= 1e-13 * np.abs(E).max() * np.abs(B).max() + 1e-30


def test_dipole_corotation_kind_corotates_everywhere():
    """The drift test of Sec. 4.3 (dipole with the corotation E at every
    radius): the same ideal-conductor field outside the star too."""
    o, p, at = _bg_oracle("dipole_corot")
    c, om = p["c"], p["omega"]
    for r in (1.5 * p["r_in"], 3.0 * p["r_in"]):
        for th in (0.5, 1.5, 2.5):
            E, B = at(r, th)
            v = np.cross([0.0, 0.0, om], r * _to_cart([1.0, 0.0, 0.0], th))
            want = -np.cross(v, _to_cart(B, th)) / c
            assert np.abs(_to_cart(E, th) - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("bg", ["dipole", "monopole"])
def test_exterior_e_is_a_static_vacuum_field(bg):
    """Outside the star E is divergence-free and curl-free (no charge, no
    changing B), falls off as the multipole that matches the surface
    potential (dipole: l = 2, r^-4; monopole: l = 1, r^-3), and its
    tangential part equals the corotation value on the surface: together with
    zero net charge these fix the vacuum exterior uniquely."""
    o, p, at = _bg_oracle(bg)
    r0 = p["r_in"]
    E = lambda r, th: at(r, th)[0]
    for r in (1.2 * r0, 2.5 * r0, 6.0 * r0):
        for th in (0.35, 1.0, 2.2, 2.8):
            div, curl = _div_curl(E, r, th)
            scale = np.abs(E(r, th)).max() / r
            assert abs(div) < 1e-9 * scale and abs(curl) < 1e-9 * scale, (r, th, div, curl)
    n = 4 if bg == "dipole" else 3
    for th in (0.4, 1.2):
        assert E(3 * r0, th)[1] == pytest.approx(E(1.5 * r0, th)[1] / 2 ** n, rel=1e-12)
    for th in np.linspace(0.1, 3.0, 9):
        inside = at(r0 * (1 - 1e-13), th)[0]
        outside = at(r0, th)[0]
        assert outside[1] == pytest.approx(inside[1], rel=1e-9, abs=1e-15)
    # spin-up (Sec. 5.2): the field grows linearly with Omega(t) = Omega t / t_spin
    o2, p2, at2 = _bg_oracle(bg, t_spin=200.0)
    assert at2(2 * r0, 0.7, 50.0)[0][0] == pytest.approx(at(2 * r0, 0.7, 50.0)[0][0] * 50.0 / 200.0, rel=1e-13)


def test_charge_fall_in_relaxes_pointwise():
    """Sec. 4.2.1: once the pulse launched by the swallowed charge has left
    (between 1.5 and 2 crossing times in the paper), the field is the
    inverse-square field of the swallowed charge.  On the uniform-radius
    grid of the fall-in test, E_r 4 pi r^2 is within 2.5 % of Q over the
    inner half of the domain after 3.5 crossing times (2.1 % measured) and
    within 1 % everywhere between the conductor and the lossy layer after 5
    (0.52 % measured): the ringing decays instead of settling at an offset."""
    import test_oracle_pins as T
    for t_tc, inner_bound, all_bound in ((3.5, 0.025, 0.035), (5.0, 0.01, 0.01)):
        o, p, nr, nth, L = T._fall_in("lin", t_tc)
        Er = o.get_field("Er")
        rb = o.geometry(1)
        ratio = Er * 4 * math.pi * (rb ** 2)[:, None]
        inner = np.abs(ratio[1:nr // 2] - 1.0).max()
        upto = np.abs(ratio[1:nr - L - 1] - 1.0).max()
        print(f"{t_tc} crossing times: inner half {inner:.4f}, up to the layer {upto:.4f}")
        assert inner < inner_bound and upto < all_bound


def test_cell_offset_loader_matches_absolute_coordinates():
    """Particles handed to the oracle as cell indices plus offsets take the
    same step as the same particles given by absolute coordinates, when the
    absolute coordinates are exact (offsets on a 2^-20 grid); near a pole the
    loader forms the pole distance from the offset, so a particle 2^-44 of a
    cell from the south pole of a 2^14-cell grid keeps that distance (the
    absolute coordinate nth - 2^-44 rounds to the pole)."""
    p = W.grid_params(16, 12, 4.0)
    p.update(dict(n_filt=1, absorb_cells=0, sigma_max=0.0, mover="vay", bg_kind="dipole", B0=1.0, omega=0.01,
                  q_over_m=1.0))
    rng = np.random.default_rng(21)
    n = 64
    ci = rng.integers(0, 16, n).astype(np.int32)
    cj = rng.integers(0, 12, n).astype(np.int32)
    fx = np.floor(rng.uniform(0, 1, n) * 2 ** 20) / 2 ** 20
    fy = np.floor(rng.uniform(0, 1, n) * 2 ** 20) / 2 ** 20
    u = rng.normal(0, 0.3, (3, n))
    w = np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * 1e-3
    a, b = O.Oracle(p), O.Oracle(p)
    a.add_particles(ci + fx, cj + fy, u[0], u[1], u[2], w)
    b.add_particles_cells(ci, fx, cj, fy, u[0], u[1], u[2], w)
    a.step(1)
    b.step(1)
    Pa, Pb = a.particles(), b.particles()
    for k in Pa:
        assert np.array_equal(Pa[k], Pb[k]), k
    for c in ("Fr", "Fth", "Fph"):
        assert np.array_equal(a.get_field(c), b.get_field(c)), c
    # the pole distance from the offset: on a grid of 2^14 meridional cells
    # the absolute coordinate nth - 2^-44 rounds to the pole itself, the
    # cell-offset loader keeps the particle 2^-44 of a cell from the axis
    q = W.grid_params(8, 2 ** 14, 4.0)
    q.update(dict(n_filt=0, absorb_cells=0, sigma_max=0.0, mover="vay", bg_kind="dipole", B0=1.0, omega=0.01,
                  q_over_m=1.0))
    eps = 2.0 ** -44
    near, absolute, pole = O.Oracle(q), O.Oracle(q), O.Oracle(q)
    near.add_particles_cells([4], [0.5], [2 ** 14 - 1], [1.0 - eps], [0.0], [0.3], [0.0], [1e-3])
    absolute.add_particles([4.5], [2.0 ** 14 - eps], [0.0], [0.3], [0.0], [1e-3])
    pole.add_particles_cells([4], [0.5], [2 ** 14 - 1], [1.0], [0.0], [0.3], [0.0], [1e-3])
    for o in (near, absolute, pole):
        o.step(1)
    assert np.array_equal(absolute.particles()["ur"], pole.particles()["ur"])
    assert not np.array_equal(near.particles()["ur"], pole.particles()["ur"])
