"""Error paths of smc_mpc_init that are decided on the host before any
device work, so they run without a GPU: SMC_ENOMEM for a context whose
buffers no device can hold (the library sums its largest buffers first),
and SMC_ENOTSPD for a wind covariance whose per-axis factorisation fails
(Sec. "Wind Model": the covariance must be positive definite to be
factorised).  A refused initialisation leaves no context behind and sets
smc_last_error(NULL)."""
import ctypes as C

import numpy as np
import pytest

import paper_1506_02869_amd as smc
import synth


def _init(scen):
    sc, keep = smc.make_scenario_struct(scen)
    h = C.c_void_p()
    st = smc.lib().smc_mpc_init(C.byref(sc), C.byref(h))
    return st, h.value, (smc.lib().smc_last_error(None) or b"").decode()


def test_huge_particle_count_is_refused_with_enomem():
    # 40 aircraft, 2^24 particles (one control segment, so that the
    # particle array stays within the Philox element range), 4096 samples:
    # the per-world costs alone take 4096 * 2^24 * 40 * 9 bytes = 25 TB
    s = synth.shrink(synth.c5(), L=1 << 24, M=4096, S=1, grid=(4, 4, 3))
    st, h, msg = _init(s)
    assert st == smc.SMC_ENOMEM, (st, msg)
    assert h is None
    assert "device memory" in msg


def test_enomem_is_raised_by_the_binding():
    s = synth.shrink(synth.c5(), L=1 << 24, M=4096, S=1, grid=(4, 4, 3))
    with pytest.raises(smc.SmcError) as e:
        smc.smc_mpc_init(s)
    assert e.value.status == smc.SMC_ENOMEM


def test_singular_wind_covariance_is_refused_with_enotspd():
    # no nugget and a length scale far beyond the box: the per-axis Gram
    # matrix is all ones to rounding, so its Cholesky factorisation fails
    s = synth.shrink(synth.c1(), grid=(16, 16, 4))
    s = dict(s, wind_nugget=0.0, wind_ell=1e9)
    st, h, msg = _init(s)
    assert st == smc.SMC_ENOTSPD, (st, msg)
    assert h is None
    assert "positive definite" in msg


def test_the_same_grid_with_its_nugget_factorises():
    """Control case: the scenario of the previous test with the default
    nugget is not refused for its covariance (without a device it fails
    later, at the first device call)."""
    s = synth.shrink(synth.c1(), grid=(16, 16, 4))
    st, h, msg = _init(s)
    assert st != smc.SMC_ENOTSPD
    if st != smc.SMC_OK:
        assert st in (smc.SMC_EDEVICE, smc.SMC_ENOMEM)
    else:
        smc.lib().smc_destroy(C.c_void_p(h))


@pytest.mark.parametrize("case", ["value", "paper_controls"])
def test_warm_start_refusals(case):
    """warm_start must be 0 or 1 and takes the kinematic segment controls
    (the shift is by one control segment)."""
    if case == "value":
        s = dict(synth.shrink(synth.c1(), L=16, K=2), warm_start=2)
    else:
        s = dict(synth.shrink(synth.make_scenario("W", n_arr=1, n_dep=1, box=(60e3, 60e3, 6e3),
                                                  grid=(4, 4, 2), H=6, dt=10.0, S=6, M=2,
                                                  L=16, K=2, controls="paper")), warm_start=1)
    st, h, msg = _init(s)
    assert st == smc.SMC_EINVAL and h is None
    assert "warm_start" in msg
