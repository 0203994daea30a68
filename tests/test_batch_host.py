"""Host logic of the batched form (CPU only): the work plan of the
persistent rollout, batch validation before any device work, and the
autotune cache."""
import numpy as np
import pytest

import synth
import paper_1506_02869_amd as smc


def test_plan_covers_every_world_once_in_bucket_order():
    N = [3, 20, 2, 11, 20, 7, 16, 13]
    H = [100, 60, 180, 120, 180, 90, 61, 150]
    L, M = 100, 3
    bs, bc, isc, iw = smc.smc_batch_plan(N, H, L, M)
    per = -(-L * M // smc.BATCH_ITEM_WORLDS)
    assert len(isc) == per * len(N) == bc.sum()
    # every (scenario, world block) exactly once
    pairs = set(zip(isc.tolist(), iw.tolist()))
    assert pairs == {(s, t * 64) for s in range(len(N)) for t in range(per)}
    # buckets contiguous, scenario's bucket matches its N
    for b in range(smc.BATCH_BUCKETS):
        seg = isc[bs[b]:bs[b] + bc[b]]
        lo = smc.BATCH_BUCKET_NMAX[b - 1] if b else 0
        assert all(lo < N[s] <= smc.BATCH_BUCKET_NMAX[b] for s in seg)
        # decreasing N^2 H within the bucket, ties by index
        keys = [(-(N[s] ** 2) * H[s], s) for s in seg]
        assert keys == sorted(keys)
    assert np.all(np.diff(bs) >= 0) and bs[0] == 0


def test_plan_scenario_order_and_errors():
    N, H = [5, 5, 3], [60, 180, 120]
    bs, bc, isc, iw = smc.smc_batch_plan(N, H, 64, 2, order=1)
    b4 = smc.BATCH_BUCKET_NMAX.index(4)
    b6 = smc.BATCH_BUCKET_NMAX.index(6)
    assert list(isc[bs[b6]:bs[b6] + bc[b6]]) == [0, 0, 1, 1]
    assert list(isc[bs[b4]:bs[b4] + bc[b4]]) == [2, 2]
    bs, bc, isc, iw = smc.smc_batch_plan(N, H, 64, 2, order=0)
    assert list(isc[bs[b6]:bs[b6] + bc[b6]]) == [1, 1, 0, 0]
    for bad in ([21], [0]):
        with pytest.raises(smc.SmcError):
            smc.smc_batch_plan(bad, [60], 64, 2)


def _tiny(seed, **kw):
    args = dict(n_arr=1, n_dep=1, box=(60e3, 60e3, 6e3), grid=(8, 8, 4), H=60, dt=5.0,
                S=6, M=4, L=64, K=3, precision="fp64", seed=seed)
    args.update(kw)
    return synth.make_scenario(f"t{seed}", **args)


@pytest.mark.parametrize("change,msg", [
    (dict(L=128), "n_particles"), (dict(M=8), "n_wind"), (dict(K=4), "n_iters"),
    (dict(precision="fp32"), "precision"), (dict(grid=(8, 8, 5)), "wind grid"),
    (dict(box=(60e3, 60e3, 7e3)), "wind grid"),
    (dict(n_arr=9, n_dep=12, box=(200e3, 200e3, 6e3)), "at most 20"),
])
def test_batch_init_rejects_mismatch_on_host(change, msg):
    a = _tiny(1)
    b = _tiny(2, **change)
    with pytest.raises(smc.SmcError) as e:
        smc.smc_batch_init([a, b])
    assert e.value.status == smc.SMC_EINVAL and msg in str(e.value)


def test_batch_init_rejects_bad_scenario():
    b = _tiny(1)
    b["dt"] = 0.0
    with pytest.raises(smc.SmcError) as e:
        smc.smc_batch_init([_tiny(1), b])
    assert "scenario 1" in str(e.value)
    with pytest.raises(smc.SmcError):
        smc.smc_batch_init([])


def test_tuning_cache_roundtrip(tmp_path):
    scens = [_tiny(1), _tiny(2, n_arr=2, H=90)]
    k1 = smc.tuning_key(scens, "dev-a")
    assert k1 == smc.tuning_key(list(reversed(scens)), "dev-a")   # order-free
    assert k1 != smc.tuning_key(scens, "dev-b")
    assert k1 != smc.tuning_key(scens[:1], "dev-a")
    path = str(tmp_path / "tune.json")
    assert smc.load_tuning(path, k1) is None
    t = {"block": [64, 128, 256, 0, 0, 0, 0, 256], "grid_mult": [1, 2, 1, 0, 0, 0, 0, 1],
         "order": 0}
    smc.save_tuning(path, k1, t)
    smc.save_tuning(path, "other", dict(t, order=1))
    assert smc.load_tuning(path, k1) == t
    assert smc.load_tuning(path, "other")["order"] == 1
    # corrupt entries are ignored
    smc.save_tuning(path, "bad", dict(t, block=[7] * 8))
    assert smc.load_tuning(path, "bad") is None
    tt = smc.BatchTuning.from_dict(t)
    assert tt.as_dict() == t


@pytest.mark.parametrize("change,msg", [
    (dict(move="mala"), "gradient move"),
    (dict(n_arr=12, n_dep=9), "at most 20 aircraft"),
    (dict(wind_tcorr=0.0), "wind_tcorr"),
    (dict(grid=(65, 64, 2)), "4096 horizontal nodes"),
])
def test_time_correlated_wind_limits_are_checked_on_the_host(change, msg):
    """Scenario checks of the paper's wind model run before any device work."""
    s = _tiny(3, wind_model="ar1", **change)
    with pytest.raises(smc.SmcError) as e:
        smc.smc_mpc_init(s)
    assert msg in str(e.value)
    bad = dict(_tiny(4, wind_model="ar1"))
    bad["wind_beta"] = -1.0
    with pytest.raises(smc.SmcError):
        smc.smc_mpc_init(bad)
    with pytest.raises(smc.SmcError) as e:
        smc.smc_batch_init([_tiny(1), _tiny(2, wind_model="ar1")])
    assert "static wind model" in str(e.value)
