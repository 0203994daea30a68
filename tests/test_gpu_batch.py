"""GPU parity of the batched form: every scenario of a batch gets exactly
(bit for bit) the controls and costs of its own single-scenario update, in
both precisions and every move (jitter, random-walk, Langevin); graph replays
equal eager launches; launch shapes do not change results; a batch scenario
matches the oracle; and C3 at full size matches single-scenario runs."""
import numpy as np
import pytest

import synth
from oracle import smc as osmc
from tests.gpu_helpers import dev, empty, host, rel_err

pytestmark = pytest.mark.gpu


def _mixed(precision="fp64", move="jitter", L=128, M=6, K=4, seed=0):
    """Scenarios of uneven size in one box / grid: N = 2, 5, 9, 13, 20 with
    different horizons and segment counts."""
    shapes = [(1, 1, 60, 6), (3, 2, 75, 5), (5, 4, 90, 6), (8, 5, 70, 7), (12, 8, 64, 4)]
    out = []
    for k, (na, nd, H, S) in enumerate(shapes):
        s = synth.make_scenario(f"b{k}", n_arr=na, n_dep=nd, box=(100e3, 100e3, 8e3),
                                grid=(8, 8, 4), H=H, dt=5.0, S=S, M=M, L=L, K=K,
                                precision=precision, move=move, seed=seed * 100 + k)
        s["scenario_id"] = k
        s["wind_mean"] = np.array([3.0 - k, 0.5 * k])
        out.append(s)
    return out


def _singles(lib, scens, mpc_step=0, horizons=None):
    res = []
    for k, s in enumerate(scens):
        ctx = lib.smc_mpc_init(s)
        h = s["H"] if horizons is None else int(horizons[k])
        ctrl, cost, status, info = lib.smc_mpc_step(ctx, mpc_step=mpc_step, horizon=h)
        res.append((ctrl, cost, status))
        ctx.close()
    return res


def _assert_same(b, out, singles):
    ctrl, cost, status = out[0], out[1], out[2]
    for s, ((c, e), (c1, e1, st1)) in enumerate(zip(b.split(ctrl, cost), singles)):
        assert np.array_equal(c, c1), f"scenario {s}: controls differ"
        assert np.array_equal(e, e1), f"scenario {s}: costs differ"
        assert status[s] == st1


@pytest.mark.parametrize("precision,move", [("fp64", "jitter"), ("fp32", "jitter"),
                                            ("fp32", "rwmh"), ("fp64", "rwmh"),
                                            ("fp32", "mala"), ("fp64", "mala")])
def test_batch_equals_single_scenario_runs(lib, precision, move):
    scens = _mixed(precision, move)
    print(f"batch vs single: {precision} {move} N={[s['N'] for s in scens]}", flush=True)
    b = lib.smc_batch_init(scens)
    out = lib.smc_batch_step(b, mpc_step=2)
    _assert_same(b, out, _singles(lib, scens, mpc_step=2))
    info = out[4]
    assert info["n_scenarios"] == len(scens) and info["aircraft_steps"] > 0
    assert info["rollout_launches"] == len({min(i for i, n in enumerate(lib.BATCH_BUCKET_NMAX)
                                                if s["N"] <= n) for s in scens}) * \
        scens[0]["K"] * (1 if move == "jitter" else 2)
    if move == "rwmh":
        assert 0.0 < info["accept_rate"] < 1.0
    if move == "mala":
        assert 0.0 <= info["accept_rate"] < 1.0


def test_batch_mala_many_samples(lib):
    """Langevin moves with more wind samples than a wavefront (the adjoint
    sums its samples in chunks through the batch's partial buffer)."""
    scens = _mixed("fp32", "mala", L=32, M=80, K=2)
    b = lib.smc_batch_init(scens)
    out = lib.smc_batch_step(b, mpc_step=1)
    _assert_same(b, out, _singles(lib, scens, mpc_step=1))


def test_batch_horizons_and_inputs_per_update(lib):
    """Horizons below horizon_max (the work plan is re-ordered), changed
    states and wind means: still the single-scenario result."""
    scens = _mixed("fp32", "jitter", K=3)
    b = lib.smc_batch_init(scens)
    hz = np.array([s["S"] + 7 * (k + 1) for k, s in enumerate(scens)], dtype=np.int32)
    hz = np.minimum(hz, [s["H"] for s in scens]).astype(np.int32)
    for s in scens:
        s["states"] = s["states"].copy()
        s["states"][:, 3] += 3.0
        s["wind_mean"] = s["wind_mean"] * -1.0
    out = lib.smc_batch_step(b, mpc_step=5, states=np.concatenate([s["states"] for s in scens]),
                             wind_mean=np.stack([s["wind_mean"] for s in scens]), horizons=hz)
    _assert_same(b, out, _singles(lib, scens, mpc_step=5, horizons=hz))


@pytest.mark.parametrize("move", ["rwmh", "mala"])
def test_batch_graph_replays_equal_eager(lib, move):
    """The captured update replayed for several MPC steps (with eager work
    and synchronisations between replays, horizons changing) equals the eager
    launches every time (Langevin batches re-capture when the horizons
    change: the adjoint's launches carry them)."""
    import torch
    scens = _mixed("fp32", move, K=3)
    eager = lib.smc_batch_init(scens)
    graph = lib.smc_batch_init(scens)
    lib.smc_batch_set_graph(graph, True)
    H = np.array([s["H"] for s in scens], dtype=np.int32)
    for rep, mpc in enumerate([0, 1, 7, 1]):
        hz = H - (rep % 2) * np.array([s["S"] // 2 for s in scens], dtype=np.int32)
        print(f"graph replay {rep}: mpc_step {mpc}", flush=True)
        a = lib.smc_batch_step(eager, mpc_step=mpc, horizons=hz)
        x = torch.ones(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        g = lib.smc_batch_step(graph, mpc_step=mpc, horizons=hz)
        assert g[4]["graph"] == 1 and a[4]["graph"] == 0
        assert float(x) == float(1 << 20)
        for k in range(3):
            assert np.array_equal(a[k], g[k]), f"replay {rep}: output {k} differs"


def test_batch_device_form_and_streams(lib):
    """Device-pointer form on a caller stream, with and without info; the
    graph path through the device form."""
    import torch
    scens = _mixed("fp32", "jitter", K=3)
    b = lib.smc_batch_init(scens)
    ref = lib.smc_batch_step(b, mpc_step=4)
    states = dev(np.concatenate([s["states"] for s in scens]))
    kact = dev(np.concatenate([s["k_active"] for s in scens]).astype(np.int32))
    wm = np.stack([s["wind_mean"] for s in scens])
    hz = np.array([s["H"] for s in scens], dtype=np.int32)
    ctrl = empty(int(b.ctrl_off[-1]), torch.float64)
    cost = empty(int(b.cost_off[-1]), torch.float64)
    status = empty(b.ns, torch.int32)
    st = torch.cuda.Stream()
    for use_graph in (False, True):
        lib.smc_batch_set_graph(b, use_graph)
        for want_info in (False, True):
            ctrl.fill_(-1.0)
            # the fill and the inputs were queued on the default stream
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                lib.smc_batch_step_dev(b, 4, states, kact, wm, hz, ctrl, cost, status,
                                       want_info=want_info, stream=st)
            st.synchronize()
            assert np.array_equal(host(ctrl), ref[0])
            assert np.array_equal(host(cost), ref[1])
            assert np.array_equal(host(status), ref[2])


def test_batch_tuning_does_not_change_results(lib):
    scens = _mixed("fp32", "jitter", K=3)
    b = lib.smc_batch_init(scens)
    ref = lib.smc_batch_step(b, mpc_step=3)
    shapes = [
        {"block": [64] * 8, "grid_mult": [2] * 8, "order": 1},
        {"block": [128] * 8, "grid_mult": [1] * 8, "order": 0},
        {"block": [256, 64, 128, 256, 64, 128, 256, 64], "grid_mult": [1, 2] * 4, "order": 0},
    ]
    for t in shapes:
        lib.smc_batch_set_tuning(b, t)
        got = lib.smc_batch_get_tuning(b)
        assert got == t
        out = lib.smc_batch_step(b, mpc_step=3)
        for k in range(3):
            assert np.array_equal(out[k], ref[k])
    t = lib.smc_batch_autotune(b, mpc_step=3, reps=1)
    assert all(v in (64, 128, 256) for v in t["block"]) and all(v in (1, 2) for v in t["grid_mult"])
    out = lib.smc_batch_step(b, mpc_step=3)
    for k in range(3):
        assert np.array_equal(out[k], ref[k])


def test_batch_scenario_matches_oracle(lib):
    """A two-scenario FP64 batch against the oracle's whole SMC run of each
    scenario (returned controls 1e-4, expected cost 1e-5 relative)."""
    scens = _mixed("fp64", "jitter", L=128, M=6, K=5)[:2]
    b = lib.smc_batch_init(scens)
    ctrl, cost, status, r, info = lib.smc_batch_step(b, mpc_step=1)
    for s, (c, e) in zip(scens, b.split(ctrl, cost)):
        ref = osmc.smc_mpc_step(dict(s, mpc_step=1))
        u = (c - s["ctrl_lo"]) / (s["ctrl_hi"] - s["ctrl_lo"])
        assert np.abs(u - ref["u_best"]).max() < 1e-4
        assert abs(e[0] - ref["cost"]) <= 1e-5 * max(abs(ref["cost"]), 1e-3)
        assert np.all(rel_err(e[1:], ref["cost_per"]) < 1e-5)


def test_c3_full_size_matches_single_runs(lib):
    """The 64-scenario batch at full size (4096 particles, 32 wind samples,
    N from 2 to 20, horizons 60..180; 2 iterations to bound the run time):
    the smallest, the largest and a middle scenario equal their own
    single-scenario updates bit for bit."""
    scens = [synth.shrink(s, K=2) for s in synth.c3()]
    print("C3 batch init", flush=True)
    b = lib.smc_batch_init(scens)
    out = lib.smc_batch_step(b, mpc_step=0)
    info = out[4]
    assert info["aircraft_steps"] > 0
    order = np.argsort([s["N"] * 1000 + s["H"] for s in scens], kind="stable")
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    parts = b.split(out[0], out[1])
    for k in pick:
        print(f"C3 single scenario {k} (N={scens[k]['N']}, H={scens[k]['H']})", flush=True)
        ((c1, e1, st1),) = _singles(lib, [scens[k]])
        assert np.array_equal(parts[k][0], c1) and np.array_equal(parts[k][1], e1)
        assert out[2][k] == st1
