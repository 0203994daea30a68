"""smc_k_resample_noalloc (the resampling entry point with a static scan
workspace, for callers that cannot allocate) against the context entry point
smc_k_resample: two calls in a row on one device, the second with a smaller
input, give the same ancestors (bit for bit) and effective sample sizes, and
the oracle's ancestors."""
import numpy as np
import pytest

import synth
from oracle import smc as osmc
from tests.gpu_helpers import dev, empty, host

pytestmark = pytest.mark.gpu


def _case(N, P, seed):
    rng = np.random.default_rng(seed)
    logw = rng.normal(0, 4, (P, N)) - 30.0
    logw[rng.uniform(size=(P, N)) < 0.3] = -np.inf
    logw[:, N - 1] = -np.inf                       # an all-violating row
    logw[0, 0] = -30.0
    U = rng.integers(0, 2**32, N, dtype=np.uint64).astype(np.uint32)
    return logw, U


def _ctx(lib, N, P):
    n_arr = N // 2
    s = synth.make_scenario("R", n_arr=n_arr, n_dep=N - n_arr, box=(100e3, 100e3, 8e3),
                            grid=(4, 4, 3), H=12, dt=5.0, S=2, M=2, L=P, K=2,
                            precision="fp32", seed=N)
    return lib.smc_mpc_init(s)


def test_noalloc_resample_equals_context_entry(lib):
    import torch
    # the C5 rows (40 x 65536, 2.6 M doubles of scan), then a smaller call
    # that reuses the same static workspace
    for N, P, seed in [(40, 65536, 1), (7, 1000, 2)]:
        logw, U = _case(N, P, seed)
        ctx = _ctx(lib, N, P)
        d_logw, d_U = dev(logw), dev(U.view(np.int32))
        a_ref, e_ref = empty((N, P), torch.int32), empty((N,), torch.float64)
        lib.smc_k_resample(ctx, P, d_logw, d_U, a_ref, e_ref)
        a_got, e_got = empty((N, P), torch.int32), empty((N,), torch.float64)
        lib.smc_k_resample_noalloc(N, P, d_logw, d_U, a_got, e_got)
        torch.cuda.synchronize()
        assert np.array_equal(host(a_got), host(a_ref)), (N, P)
        assert np.array_equal(host(e_got), host(e_ref)), (N, P)
        for i in (0, N // 2, N - 1):
            assert np.array_equal(host(a_got)[i], osmc.resample_row(logw[:, i], int(U[i]))), i
        ctx.close()


def test_noalloc_resample_refuses_beyond_workspace(lib):
    import torch
    N, P = 2, (1 << 21) + 1                        # N P = 2^22 + 2 doubles of scan
    logw = torch.zeros((P, N), dtype=torch.float64, device="cuda")
    U = torch.zeros((N,), dtype=torch.int32, device="cuda")
    anc = torch.empty((N, P), dtype=torch.int32, device="cuda")
    with pytest.raises(lib.SmcError):
        lib.smc_k_resample_noalloc(N, P, logw, U, anc)
