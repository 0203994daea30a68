"""Pins of the oracle's pairwise separation (eq. avoidance): brute force over
tracks on tiny inputs, and exact-boundary cases (distance equal to the
required separation is safe)."""
import math

import numpy as np

from oracle import rollout as ro
from oracle import wind
from tests.oracle_helpers import mini


def _no_unary(s):
    """Make every unary constraint inactive so feasibility is separation only."""
    s["aircraft"][:, 5] = 1e12        # thrust limit
    s["aircraft"][:, 6] = 0.0         # empty mass
    s["aircraft"][:, 7] = math.pi / 2  # bank limit
    s["aircraft"][:, 8] = math.pi / 2  # climb-angle limit
    s["env"] = np.array([-1e9, 1e9, 0.0, 1e9])
    return s


def _brute_force(track, present, sep_h, sep_v):
    H, L, M, N = present.shape
    feas = np.ones((L, M, N), dtype=bool)
    for l in range(L):
        for m in range(M):
            for k in range(H):
                for i in range(N):
                    for j in range(N):
                        if i == j or not (present[k, l, m, i] and present[k, l, m, j]):
                            continue
                        a, b = track[k + 1, l, m, i], track[k + 1, l, m, j]
                        dh2 = (a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2
                        if dh2 < sep_h ** 2 and abs(a[2] - b[2]) < sep_v:
                            feas[l, m, i] = False
    return feas


def test_brute_force_agreement_on_tiny_inputs():
    rng = np.random.default_rng(11)
    hits = 0
    for trial in range(6):
        N = int(rng.integers(2, 5))
        H = int(rng.integers(2, 6))
        st = np.zeros((N, 6))
        st[:, 0] = rng.uniform(-6e3, 6e3, N)
        st[:, 1] = rng.uniform(-6e3, 6e3, N)
        st[:, 2] = rng.uniform(2000, 2600, N)
        st[:, 3] = rng.uniform(120, 200, N)
        st[:, 4] = rng.uniform(-math.pi, math.pi, N)
        st[:, 5] = 60e3
        kact = rng.integers(0, H, N)
        s = _no_unary(mini(N=N, H=H, S=1, M=2, L=3, sigma=5.0, states=st,
                           k_active=kact))
        u = rng.uniform(0, 1, (3, N, 1, 3))
        W = wind.sample_field(s, 0)
        r = ro.rollout(s, u, W, record=True)
        bf = _brute_force(r["track"], r["present"], s["sep_h"], s["sep_v"])
        assert np.array_equal(r["feas"], bf)
        hits += int((~bf).sum())
    assert hits > 0


def _pair(dx, dz):
    st = [[0.0, 0.0, 0.0, 150.0, math.pi / 2, 60e3],
          [dx, 0.0, dz, 150.0, math.pi / 2, 60e3]]
    s = _no_unary(mini(N=2, H=3, S=1, states=st))
    s["ctrl_lo"] = np.array([-0.05, 100.0, -15.0])
    s["ctrl_hi"] = np.array([0.05, 200.0, 15.0])
    u = np.full((1, 2, 1, 3), 0.5)
    G = int(np.prod(s["grid"]))
    return ro.rollout(s, u, np.zeros((1, G, 2)))["feas"][0, 0]


def test_exact_boundary_is_safe():
    sh, sv = 5556.0, 304.8
    assert _pair(sh, 0.0).all()                 # horizontal distance == 2 P_r
    assert not _pair(sh - 1.0, 0.0).any()       # inside in both senses
    assert _pair(0.0, sv).all()                 # vertical distance == 2 P_h
    assert not _pair(0.0, sv - 0.01).any()
    assert _pair(sh - 1.0, sv + 0.01).all()     # either condition suffices


def test_inactive_and_landed_aircraft_are_not_tested():
    st = [[0.0, 0.0, 1000.0, 150.0, 0.0, 60e3], [100.0, 0.0, 1000.0, 150.0, 0.0, 60e3]]
    s = _no_unary(mini(N=2, H=4, S=1, states=st, k_active=[0, -1]))
    u = np.full((1, 2, 1, 3), 0.5)
    G = int(np.prod(s["grid"]))
    r = ro.rollout(s, u, np.zeros((1, G, 2)))
    assert r["feas"].all() and r["cost"][0, 0, 1] == 0.0
