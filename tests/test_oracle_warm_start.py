"""Pins of the warm start of the receding-horizon loop (Sec. "Model
Predictive Control", "Rolling Window": the window moves by the applied
part, the first control segment): the next update's initial particle l is
the previous final particle l moved one segment earlier, its last segment
drawn as a fresh initialisation draws it."""
import numpy as np

import synth
from oracle import mpc as ompc
from oracle import smc as osmc


def _scen(**kw):
    return synth.shrink(synth.c1(), L=16, K=3, **kw)


def test_shift_by_one_segment_and_fresh_tail():
    s = dict(_scen(), warm_start=1)
    L, N, S = s["L"], s["N"], s["S"]
    # every element distinct, so a shift along another axis cannot pass
    u_prev = np.arange(L * N * S * 3, dtype=np.float64).reshape(L, N, S, 3) / (L * N * S * 3)
    u = osmc.warm_start_particles(s, u_prev, mpc_step=5)
    for s_ in range(S - 1):
        assert np.array_equal(u[:, :, s_], u_prev[:, :, s_ + 1])
    fresh = osmc.init_particles(s, 5)
    assert np.array_equal(u[:, :, S - 1], fresh[:, :, S - 1])
    assert not np.array_equal(u[:, :, S - 1], u_prev[:, :, S - 1])
    assert np.all((u >= 0) & (u < 1))


def test_update_starts_from_the_shifted_population():
    """The first weighting pass of a warm-started update sees the shifted
    population; without warm start (or without a previous population) it
    sees the fresh draw."""
    s = dict(_scen(), warm_start=1)
    first = osmc.smc_mpc_step(s, mpc_step=0)
    u_prev = first["result"]["u"]
    tr = []
    osmc.smc_mpc_step(s, mpc_step=1, trace=tr, u_prev=u_prev)
    assert np.array_equal(tr[0]["u"], osmc.warm_start_particles(s, u_prev, 1))
    tr_cold = []
    osmc.smc_mpc_step(dict(s, warm_start=0), mpc_step=1, trace=tr_cold, u_prev=u_prev)
    assert np.array_equal(tr_cold[0]["u"], osmc.init_particles(s, 1))


def test_rolling_window_passes_the_final_population():
    """The loop hands each update's final population to the next: with warm
    start the second update's controls differ from a cold loop's, the first
    update's are the same."""
    s = _scen()
    cold = ompc.rolling_window(s, 2)
    warm = ompc.rolling_window(dict(s, warm_start=1), 2)
    assert np.array_equal(cold[0]["controls"], warm[0]["controls"])
    assert not np.array_equal(cold[1]["controls"], warm[1]["controls"])
