"""Host checks of the parity helpers' momentum scale: the update's field
terms against their definition in fields the oracle holds exactly."""
import math

import numpy as np

from oracle.oracle import Oracle
from paper_1407_1810_amd import workloads as W
from parity_util import update_term_scale, widen_by_update_terms


def _oracle(bg):
    p = W.small_config(bg=bg, nr=16, nth=12)["params"]
    return Oracle(p), p


def test_magnetic_term_in_a_uniform_field():
    """Uniform B_z = B0, no plasma field: the rotation term alone,
    |eps| B0 |u| / gamma."""
    o, p = _oracle("uniform_bz")
    o.step(1)  # the scale reads the time of the step just taken
    u = np.array([0.3, -0.4, 1.2])
    before = dict(id=np.array([5, 9], np.uint64), x=np.array([3.25, 7.5]), y=np.array([4.5, 6.0]),
                  ur=np.array([u[0], 0.0]), ut=np.array([u[1], 0.0]), up=np.array([u[2], 0.0]))
    got = update_term_scale(o, before, np.array([9, 5], np.uint64))
    eps = abs(p["q_over_m"]) / (2 * p["c"])
    um = float(np.linalg.norm(u))
    assert got[0] == 0.0
    assert math.isclose(got[1], eps * p["B0"] * um / math.sqrt(1 + um * um), rel_tol=1e-12)


def test_electric_term_from_a_constant_plasma_field():
    """A constant plasma E_r (every node of its lattice) and no background:
    the kick term 2 |eps| |E| at rest, whatever the position; beyond the
    outer conductor no force and no term."""
    o, p = _oracle("none")
    o.step(1)
    o.set_field("Er", np.full(o.get_field("Er").shape, 0.7))
    before = dict(id=np.array([1, 2, 3], np.uint64), x=np.array([2.3, 11.9, p["nr"] + 0.5]),
                  y=np.array([5.5, 1.2, 3.0]), ur=np.zeros(3), ut=np.zeros(3), up=np.zeros(3))
    got = update_term_scale(o, before, np.array([1, 2, 3], np.uint64))
    eps = abs(p["q_over_m"]) / (2 * p["c"])
    assert np.allclose(got[:2], 2 * eps * 0.7, rtol=1e-12, atol=0)
    assert got[2] == 0.0


def test_widening_touches_only_failing_particles():
    o, p = _oracle("uniform_bz")
    o.step(1)
    ids = np.array([1, 2], np.uint64)
    before = dict(id=ids, x=np.array([4.0, 5.0]), y=np.array([3.0, 3.0]), ur=np.array([1.0, 1.0]),
                  ut=np.zeros(2), up=np.zeros(2))
    umag = np.array([1e-6, 1e-6])
    du = np.array([1e-12, 1e-6])  # the first passes against umag alone
    new, raised = widen_by_update_terms(o, before, ids, umag, du, 1e-5)
    assert new[0] == umag[0] and new[1] > umag[1] and raised == 1
