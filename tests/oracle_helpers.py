"""Small hand-built scenarios for the oracle pins (CPU only)."""
import math

import numpy as np

import synth


def mini(N=1, kinds=None, H=10, S=1, dt=5.0, M=1, L=1, box=(60e3, 60e3, 6e3),
         grid=(4, 4, 3), sigma=0.0, wind_mean=(0.0, 0.0), states=None,
         k_active=None, **over):
    """A scenario dict with explicit small sizes; unspecified fields come from
    the C1 generator."""
    s = synth.c1()
    kinds = [1] * N if kinds is None else kinds
    s.update(N=N, H=H, S=S, dt=dt, M=M, L=L, box=np.array(box, float),
             grid=np.array(grid, dtype=np.int32), wind_sigma=sigma,
             wind_mean=np.array(wind_mean, float),
             kind=np.array(kinds, dtype=np.int8))
    ac = np.tile(s["aircraft"][:1], (N, 1))
    ac[:, 0] = 122.6
    ac[:, 1] = 0.025
    s["aircraft"] = ac
    s["targets"] = np.tile(np.array([[0.5, 5000.0, 200.0, 27e3]]), (N, 1))
    if states is None:
        states = np.tile(np.array([[0.0, 0.0, 3000.0, 200.0, 0.3, 60e3]]), (N, 1))
    s["states"] = np.array(states, float)
    s["k_active"] = (np.zeros(N, np.int32) if k_active is None
                     else np.array(k_active, np.int32))
    s["env"] = np.array([0.0, box[2], 110.0, 250.0])
    s.update(over)
    return s


def const_controls(L, N, S, value=0.5):
    return np.full((L, N, S, 3), value)


def zero_field(scen, M=1):
    G = int(np.prod(scen["grid"]))
    W = np.zeros((M, G, 2))
    W += np.asarray(scen["wind_mean"])[None, None, :]
    return W


def isa_table():
    """Standard-atmosphere densities [kg/m^3] from published ISA tables."""
    return {0.0: 1.2250, 1000.0: 1.1117, 2000.0: 1.0066, 5000.0: 0.73643,
            11000.0: 0.36391}


DEG = math.pi / 180
