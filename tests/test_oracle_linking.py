"""Pins of the oracle's secant ray linking (oracle.linking; Sections 4 and 6.3 of the paper).

Closed forms: in a homogeneous medium the linked ray is the chord from emitter to receiver,
with T = |x_r - x_e| / c0 and the 2D free-space amplitude [8 pi k0 |x_r - x_e|]^-1/2
(Appendix B); in a medium with a linear sound-speed gradient the linked ray is a circular
arc with the textbook travel time between its two end points. Invariants: every linked ray
ends on its receiver within the stopping tolerance, retracing its launch angle reproduces
it, and the pairs with a fan bracket are the linked pairs.
"""
import math

import numpy as np

from oracle import binning
from oracle.linking import ACCEPT, MAX_ITER, TOL, link_receivers
from oracle.medium import Grid, Ring, refractive_index
from oracle.trace import trace
from tests.test_oracle_trace import _arccosh_time, _linear_medium, _setup

C0 = 1500.0


def test_water_linked_rays_are_chords():
    g = _setup()
    ring = Ring(12, 0.02)
    ns = np.ones((g.ny, g.nx))
    lk = link_receivers(ns, g, ring, 40, 0.2e-3, 400, emitters=[0, 5])
    pos = ring.positions()
    for a, e in enumerate([0, 5]):
        for r in range(ring.n):
            if r == e:
                assert not lk.valid[a, r]
                continue
            assert lk.valid[a, r], (e, r)
            chord = math.hypot(*(pos[r] - pos[e]))
            assert abs(lk.T[a, r] - chord / C0) <= 1e-9 * chord / C0
            assert abs(lk.A[a, r] * math.sqrt(8 * math.pi * chord) - 1.0) <= 1e-8
            assert lk.K[a, r] == 0 and lk.miss[a, r] <= TOL
            # the chord's direction from e
            want = math.atan2(pos[r, 1] - pos[e, 1], pos[r, 0] - pos[e, 0])
            d = (lk.gamma[a, r] - want + math.pi) % (2 * math.pi) - math.pi
            assert abs(d) <= 1e-8


def test_linear_gradient_linked_time_closed_form():
    gvec = (500.0, -200.0)
    g, c = _linear_medium(*gvec)
    ns = refractive_index(c, C0)
    ring = Ring(10, 0.02)
    lk = link_receivers(ns, g, ring, 48, 0.2e-3, 400, emitters=[0, 3, 7])
    pos = ring.positions()
    worst = 0.0
    n_valid = 0
    for a, e in enumerate([0, 3, 7]):
        for r in range(ring.n):
            if not lk.valid[a, r]:
                continue
            n_valid += 1
            Tc = _arccosh_time(C0, gvec, pos[e], pos[r][None, :])[0]
            worst = max(worst, abs(lk.T[a, r] - Tc) / Tc)
    assert n_valid >= 3 * (ring.n - 3)
    assert worst < 2e-6, worst


def test_heterogeneous_invariants():
    import phantoms as ph

    g = _setup(R=0.02, dx=0.4e-3)
    c = ph.gaussian_inclusion(g.nx, g.ny, g.dx, g.x0, g.y0, seed=11, amp=45.0, sigma=4e-3,
                              centre_radius=6e-3, mask_radius=g.mask_radius)
    ns = refractive_index(c, C0)
    ring = Ring(16, 0.02)
    emitters = [0, 9]
    fan = trace(ns, g, ring, 90, 0.2e-3, 260, emitters=emitters)
    lk = link_receivers(ns, g, ring, 90, 0.2e-3, 260, emitters=emitters)
    for a, e in enumerate(emitters):
        rv = binning.receivers_emitter(fan, e, ring)[0]
        # linked exactly where the fan brackets the receiver (no fold in this medium)
        assert np.array_equal(lk.valid[a], rv)
        v = lk.valid[a]
        assert np.all(lk.miss[a, v] <= TOL)
        assert np.all(lk.rays[a] <= MAX_ITER)
        # retracing the linked launch angles lands on the receivers again
        rs = np.flatnonzero(v)
        s = trace(ns, g, ring, 90, 0.2e-3, 260, emitters=[e], angles=lk.gamma[a, rs][None, :])
        m = s.M
        beta = np.mod(np.arctan2(s.y[np.arange(rs.size), m], s.x[np.arange(rs.size), m])
                      - ring.angles()[e], 2 * math.pi)
        br = 2 * math.pi * ((rs - e) % ring.n) / ring.n
        assert np.all(np.abs(beta - br) <= TOL)
        assert np.allclose(s.T[np.arange(rs.size), m], lk.T[a, rs], rtol=0, atol=1e-18)
        # the fan's interpolation is close to the linked values (first-order accurate)
        Tf = binning.receivers_emitter(fan, e, ring)[1]
        assert np.max(np.abs(Tf[v] - lk.T[a, v]) / lk.T[a, v]) < 1e-4
    assert ACCEPT >= TOL
