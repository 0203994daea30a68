"""The binding refuses wrongly typed or sized arguments before any library
call (host only: the context carries the scenario's sizes, no device
handle is needed for the checks)."""
import numpy as np
import pytest
import torch

import paper_1506_02869_amd as smc
import synth


@pytest.fixture(scope="module")
def ctx():
    s = synth.c1()                      # FP64, N = 2, S = 6, M = 16, G = 1024
    return smc.Context(None, s)


def _cpu(shape, dtype):
    return torch.zeros(shape, dtype=dtype)


def test_dtype_and_size_refused_before_the_device_check(ctx):
    N, S, M, P = ctx.N, ctx.S, ctx.M, 7
    u = _cpu((P, N, S, 3), torch.float32)          # FP64 context
    with pytest.raises(ValueError, match="dtype"):
        smc.smc_k_init_particles(ctx, 0, P, u)
    with pytest.raises(ValueError, match="elements"):
        smc.smc_k_init_particles(ctx, 0, P + 1, _cpu((P, N, S, 3), torch.float64))
    with pytest.raises(ValueError, match="device"):
        smc.smc_k_init_particles(ctx, 0, P, _cpu((P, N, S, 3), torch.float64))
    # an int64 activation vector would be misread as int32 by the kernels
    args = [_cpu((P, N, S, 3), torch.float64), P, _cpu((M, ctx.G, 2), torch.float64),
            _cpu((N, 6), torch.float64), _cpu((N,), torch.int64), ctx.H,
            _cpu((M, P, N), torch.float64), _cpu((M, P, N), torch.uint8)]
    with pytest.raises(ValueError, match="k_active"):
        smc.smc_k_rollout(ctx, *args)
    args[4] = _cpu((N,), torch.int32)
    args[6] = _cpu((M, P - 1, N), torch.float64)   # short cost buffer
    with pytest.raises(ValueError, match="cost"):
        smc.smc_k_rollout(ctx, *args)


def test_mpc_step_dev_checks_every_buffer(ctx):
    N, S = ctx.N, ctx.S
    good = dict(states=_cpu((N, 6), torch.float64), k_active=_cpu((N,), torch.int32),
                controls_out=_cpu((N, S, 3), torch.float64), cost_out=_cpu((1 + N,), torch.float64))
    for name, bad in [("states", _cpu((N, 5), torch.float64)),
                      ("k_active", _cpu((N,), torch.float64)),
                      ("controls_out", _cpu((N, S, 2), torch.float64)),
                      ("cost_out", _cpu((N,), torch.float64))]:
        kw = dict(good, **{name: bad})
        with pytest.raises(ValueError, match=name):
            smc.smc_mpc_step_dev(ctx, 0, kw["states"], kw["k_active"], np.zeros(2), ctx.H,
                                 kw["controls_out"], kw["cost_out"])
    with pytest.raises(ValueError, match="status_out"):
        smc.smc_mpc_step_dev(ctx, 0, good["states"], good["k_active"], np.zeros(2), ctx.H,
                             good["controls_out"], good["cost_out"],
                             status_out=_cpu((2,), torch.int32))
    with pytest.raises(ValueError, match="wind_mean"):
        smc.smc_mpc_step_dev(ctx, 0, good["states"], good["k_active"], np.zeros(3), ctx.H,
                             good["controls_out"], good["cost_out"])


def test_host_forms_check_shapes(ctx):
    N, S = ctx.N, ctx.S
    with pytest.raises(ValueError, match="particles"):
        smc.smc_eval_cost(ctx, np.zeros((4, N, S + 1, 3)), 0)
    with pytest.raises(ValueError, match="particles"):
        smc.smc_eval_cost(ctx, np.zeros((N, S, 3)), 0)
    with pytest.raises(ValueError, match="states"):
        smc.smc_mpc_step(ctx, states=np.zeros((N + 1, 6)))
    with pytest.raises(ValueError, match="k_active"):
        smc.smc_mpc_step(ctx, k_active=np.zeros(N + 1))
    with pytest.raises(ValueError, match="controls"):
        smc.smc_plant_step(ctx, np.zeros((N, S, 2)), plant_iter=1)


def test_kernel_entries_check_pn_buffers(ctx):
    N, P = ctx.N, 5
    f64, u8, i32 = torch.float64, torch.uint8, torch.int32
    pn = lambda dt: _cpu((P, N), dt)
    with pytest.raises(ValueError, match="feas_prop"):
        smc.smc_k_accept(ctx, P, _cpu((P, N, ctx.S, 3), f64), _cpu((P, N, ctx.S, 3), f64),
                         pn(f64), pn(f64), pn(u8), _cpu((P, N + 1), u8), pn(f64), pn(f64), 0, 0)
    with pytest.raises(ValueError, match="best"):
        smc.smc_k_select(ctx, P, pn(f64), pn(f64), 1.0, _cpu((1,), i32))
    with pytest.raises(ValueError, match="anc"):
        smc.smc_k_resample(ctx, P, pn(f64), _cpu((N,), i32), _cpu((N, P), torch.int64))
    with pytest.raises(ValueError, match="out"):
        smc.smc_k_philox(0, 0, 0, 1, 0, 0, 10, _cpu((10, 3), i32))
