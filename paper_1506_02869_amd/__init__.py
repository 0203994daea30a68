"""Python binding of the MI355X SMC-MPC engine (libsmc_mpc.so).

Argument marshalling only: every step of the optimiser runs in the HIP
kernels behind the C ABI declared in include/smc_mpc.h and
include/smc_kernels.h.  Function names follow the C ABI.  Device arrays are
torch tensors on a HIP device (PyTorch provides device memory and streams);
host arrays are NumPy arrays.

The library must be built first (``python -m paper_1506_02869_amd.build``);
importing this package without it raises at the first call.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmc_mpc.so")

SMC_OK, SMC_INFEASIBLE = 0, 1
SMC_EINVAL, SMC_ENOMEM, SMC_EDEVICE, SMC_ENOTSPD = -1, -2, -3, -4
STATUS_NAMES = {0: "SMC_OK", 1: "SMC_INFEASIBLE", -1: "SMC_EINVAL", -2: "SMC_ENOMEM",
                -3: "SMC_EDEVICE", -4: "SMC_ENOTSPD"}
FP64, FP32 = 0, 1
MOVE_JITTER, MOVE_RWMH, MOVE_MALA = 0, 1, 2
AC_NPAR, COST_NW = 9, 9

# Philox purposes (third counter word)
P_INIT, P_WIND, P_RESAMPLE, P_MOVE, P_ACCEPT, P_MALA = 1, 2, 3, 4, 5, 6


class SmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Scenario(C.Structure):
    _fields_ = [
        ("n_aircraft", C.c_int32), ("n_segments", C.c_int32), ("horizon_max", C.c_int32),
        ("n_particles", C.c_int32), ("n_wind", C.c_int32), ("n_iters", C.c_int32),
        ("dt", C.c_double), ("box", C.c_double * 3), ("grid_n", C.c_int32 * 3),
        ("wind_sigma", C.c_double), ("wind_ell", C.c_double), ("wind_nugget", C.c_double),
        ("sep_h", C.c_double), ("sep_v", C.c_double),
        ("kind", C.POINTER(C.c_int8)), ("aircraft", C.POINTER(C.c_double)),
        ("ctrl_lo", C.c_double * 3), ("ctrl_hi", C.c_double * 3),
        ("env", C.c_double * 4), ("landing", C.c_double * 5),
        ("targets", C.POINTER(C.c_double)), ("cost_w", C.c_double * COST_NW),
        ("time_norm", C.c_double), ("noise_alt", C.c_double),
        ("popdense", C.POINTER(C.c_float)), ("pop_n", C.c_int32 * 2),
        ("precision", C.c_int32), ("move", C.c_int32),
        ("kappa", C.c_double), ("sigma_move", C.c_double), ("mala_step", C.c_double),
        ("seed", C.c_uint64), ("scenario_id", C.c_int32),
    ]


class StepInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("best_particle", C.c_int32),
                ("feasible_frac", C.c_double), ("accept_rate", C.c_double),
                ("ess_min", C.c_double), ("aircraft_steps", C.c_int64),
                ("pair_tests", C.c_int64),
                ("ms_total", C.c_double), ("ms_rollout", C.c_double),
                ("ms_wind", C.c_double), ("rollout_launches", C.c_int32),
                ("wind_launches", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_VP = C.c_void_p
_SIGS = {
    "smc_version": (C.c_char_p, []),
    "smc_last_error": (C.c_char_p, [_VP]),
    "smc_destroy": (None, [_VP]),
    "smc_mpc_init": (C.c_int, [C.POINTER(Scenario), C.POINTER(_VP)]),
    "smc_mpc_step": (C.c_int, [_VP, C.c_int64, _VP, _VP, _VP, C.c_int32, _VP, _VP,
                               C.POINTER(StepInfo)]),
    "smc_mpc_step_dev": (C.c_int, [_VP, C.c_int64, _VP, _VP, _VP, C.c_int32, _VP, _VP, _VP,
                                   C.POINTER(StepInfo), _VP]),
    "smc_eval_cost": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP, _VP, C.c_int32, _VP,
                                C.c_int32, _VP, _VP]),
    "smc_k_philox": (C.c_int, [C.c_uint64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                               C.c_int64, C.c_int64, _VP, _VP]),
    "smc_k_init_particles": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP]),
    "smc_k_wind_normals": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP]),
    "smc_k_wind_gemm": (C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "smc_k_wind_factor": (C.c_int, [_VP, _VP, _VP]),
    "smc_k_rollout": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, C.c_int32, _VP, _VP, _VP,
                                _VP]),
    "smc_k_reduce": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_double, _VP, _VP, _VP, _VP]),
    "smc_k_resample_offsets": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP]),
    "smc_k_resample": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP, _VP]),
    "smc_k_gather_move": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, C.c_int64, C.c_int32,
                                    C.c_int32, _VP]),
    "smc_k_propose": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_int64, C.c_int32, _VP]),
    "smc_k_accept": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                               C.c_int64, C.c_int32, _VP, _VP]),
    "smc_k_select": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_double, _VP, _VP]),
    "smc_set_rollout_layout": (C.c_int, [_VP, C.c_int32]),
    "smc_k_rollout_grad": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, C.c_int32, _VP, _VP]),
    "smc_k_mala_propose": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_double, _VP, C.c_int64,
                                     C.c_int32, _VP]),
    "smc_k_mala_accept": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP, C.c_double, _VP, _VP,
                                    _VP, _VP, _VP, _VP, C.c_int64, C.c_int32, _VP, _VP]),
}

_lib = None


def lib():
    """The loaded C library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1506_02869_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def device_available() -> bool:
    import torch
    return torch.cuda.is_available()


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _hp(a, dtype):
    """Host pointer of a C-contiguous NumPy array of the given dtype."""
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _check(status, ctx=None):
    if status < 0:
        msg = lib().smc_last_error(ctx.handle if ctx is not None else None)
        raise SmcError(status, (msg or b"").decode())
    return status


class Context:
    """Owns an smc_ctx*; created by smc_mpc_init."""

    def __init__(self, handle, scen):
        self.handle = handle
        self.N, self.S, self.H = int(scen["N"]), int(scen["S"]), int(scen["H"])
        self.L, self.M, self.K = int(scen["L"]), int(scen["M"]), int(scen["K"])
        self.G = int(np.prod(scen["grid"]))
        self.precision = int(scen["precision"])
        self.scen = scen

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.precision == FP64 else torch.float32

    def close(self):
        if self.handle:
            lib().smc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_scenario_struct(s: dict):
    """ctypes Scenario from a scenario dict (see synth.scenarios); returns the
    struct and the NumPy arrays it points into (keep them alive)."""
    N = int(s["N"])
    keep = {}
    keep["kind"], p_kind = _hp(s["kind"], np.int8)
    keep["aircraft"], p_ac = _hp(s["aircraft"], np.float64)
    keep["targets"], p_tg = _hp(s["targets"], np.float64)
    if keep["kind"].shape != (N,) or keep["aircraft"].shape != (N, AC_NPAR) or \
            keep["targets"].shape != (N, 4):
        raise ValueError("kind / aircraft / targets shapes do not match N")
    sc = Scenario()
    sc.n_aircraft, sc.n_segments, sc.horizon_max = N, int(s["S"]), int(s["H"])
    sc.n_particles, sc.n_wind, sc.n_iters = int(s["L"]), int(s["M"]), int(s["K"])
    sc.dt = float(s["dt"])
    sc.box[:] = [float(b) for b in s["box"]]
    sc.grid_n[:] = [int(g) for g in s["grid"]]
    sc.wind_sigma, sc.wind_ell, sc.wind_nugget = (float(s["wind_sigma"]), float(s["wind_ell"]),
                                                  float(s["wind_nugget"]))
    sc.sep_h, sc.sep_v = float(s["sep_h"]), float(s["sep_v"])
    sc.kind = C.cast(p_kind, C.POINTER(C.c_int8))
    sc.aircraft = C.cast(p_ac, C.POINTER(C.c_double))
    sc.targets = C.cast(p_tg, C.POINTER(C.c_double))
    sc.ctrl_lo[:] = [float(v) for v in s["ctrl_lo"]]
    sc.ctrl_hi[:] = [float(v) for v in s["ctrl_hi"]]
    sc.env[:] = [float(v) for v in s["env"]]
    sc.landing[:] = [float(v) for v in s["landing"]]
    sc.cost_w[:] = [float(v) for v in s["cost_w"]]
    sc.time_norm, sc.noise_alt = float(s["time_norm"]), float(s["noise_alt"])
    if s.get("popdense") is not None:
        keep["pop"], p_pop = _hp(s["popdense"], np.float32)
        sc.popdense = C.cast(p_pop, C.POINTER(C.c_float))
        sc.pop_n[:] = [keep["pop"].shape[1], keep["pop"].shape[0]]
    else:
        sc.popdense = None
        sc.pop_n[:] = [0, 0]
    sc.precision, sc.move = int(s["precision"]), int(s["move"])
    sc.kappa, sc.sigma_move, sc.mala_step = (float(s["kappa"]), float(s["sigma_move"]),
                                             float(s["mala_step"]))
    sc.seed = int(s["seed"]) & 0xFFFFFFFFFFFFFFFF
    sc.scenario_id = int(s.get("scenario_id", 0))
    return sc, keep


def smc_version() -> str:
    return lib().smc_version().decode()


def smc_mpc_init(scen: dict) -> Context:
    sc, keep = make_scenario_struct(scen)
    h = C.c_void_p()
    st = lib().smc_mpc_init(C.byref(sc), C.byref(h))
    if st < 0:
        raise SmcError(st, (lib().smc_last_error(None) or b"").decode())
    return Context(h, scen)


def smc_mpc_step(ctx: Context, mpc_step=None, states=None, k_active=None, wind_mean=None,
                 horizon=None):
    """Host form: returns (controls [N,S,3], exp_cost [1+N], status, info dict)."""
    s = ctx.scen
    mpc_step = s["mpc_step"] if mpc_step is None else mpc_step
    states = s["states"] if states is None else states
    k_active = s["k_active"] if k_active is None else k_active
    wind_mean = s["wind_mean"] if wind_mean is None else wind_mean
    horizon = ctx.H if horizon is None else horizon
    st_a, p_st = _hp(states, np.float64)
    ka_a, p_ka = _hp(k_active, np.int32)
    wm_a, p_wm = _hp(wind_mean, np.float64)
    ctrl = np.zeros((ctx.N, ctx.S, 3))
    cost = np.zeros(1 + ctx.N)
    info = StepInfo()
    r = lib().smc_mpc_step(ctx.handle, int(mpc_step), p_st, p_ka, p_wm, int(horizon),
                           ctrl.ctypes.data_as(C.c_void_p), cost.ctypes.data_as(C.c_void_p),
                           C.byref(info))
    _check(r, ctx)
    return ctrl, cost, r, info.as_dict()


def smc_mpc_step_dev(ctx: Context, mpc_step, states, k_active, wind_mean, horizon,
                     controls_out, cost_out, status_out=None, want_info=False, stream=None):
    """Device form: states [N,6] f64, k_active [N] i32, outputs device tensors."""
    wm_a, p_wm = _hp(wind_mean, np.float64)
    info = StepInfo() if want_info else None
    r = lib().smc_mpc_step_dev(ctx.handle, int(mpc_step), _ptr(states), _ptr(k_active), p_wm,
                               int(horizon), _ptr(controls_out), _ptr(cost_out),
                               _ptr(status_out), C.byref(info) if info is not None else None,
                               _stream(stream))
    _check(r, ctx)
    return r, (info.as_dict() if info is not None else None)


def smc_eval_cost(ctx: Context, particles, iter_, mpc_step=None, states=None, k_active=None,
                  wind_mean=None, horizon=None):
    s = ctx.scen
    mpc_step = s["mpc_step"] if mpc_step is None else mpc_step
    states = s["states"] if states is None else states
    k_active = s["k_active"] if k_active is None else k_active
    wind_mean = s["wind_mean"] if wind_mean is None else wind_mean
    horizon = ctx.H if horizon is None else horizon
    pa, p_pa = _hp(particles, np.float64)
    P = pa.shape[0]
    st_a, p_st = _hp(states, np.float64)
    ka_a, p_ka = _hp(k_active, np.int32)
    wm_a, p_wm = _hp(wind_mean, np.float64)
    cost = np.zeros((P, ctx.N))
    feas = np.zeros((P, ctx.N), dtype=np.uint8)
    r = lib().smc_eval_cost(ctx.handle, int(mpc_step), int(iter_), p_st, p_ka, p_wm,
                            int(horizon), p_pa, int(P), cost.ctypes.data_as(C.c_void_p),
                            feas.ctypes.data_as(C.c_void_p))
    _check(r, ctx)
    return cost, feas.astype(bool)


# ---- kernel-level entry points (device tensors) -----------------------------

def smc_k_philox(seed, mpc_step, iter_, purpose, scenario, e0, n, out, stream=None):
    _check(lib().smc_k_philox(int(seed) & 0xFFFFFFFFFFFFFFFF, int(mpc_step), int(iter_),
                              int(purpose), int(scenario), int(e0), int(n), _ptr(out),
                              _stream(stream)))


def smc_k_init_particles(ctx, mpc_step, P, u, stream=None):
    _check(lib().smc_k_init_particles(ctx.handle, int(mpc_step), int(P), _ptr(u),
                                      _stream(stream)), ctx)


def smc_k_wind_normals(ctx, mpc_step, iter_, Z, stream=None):
    _check(lib().smc_k_wind_normals(ctx.handle, int(mpc_step), int(iter_), _ptr(Z),
                                    _stream(stream)), ctx)


def smc_k_wind_gemm(ctx, Z, wind_mean, W, stream=None):
    wm_a, p_wm = _hp(wind_mean, np.float64)
    _check(lib().smc_k_wind_gemm(ctx.handle, _ptr(Z), p_wm, _ptr(W), _stream(stream)), ctx)


def smc_k_wind_factor(ctx, out, stream=None):
    _check(lib().smc_k_wind_factor(ctx.handle, _ptr(out), _stream(stream)), ctx)


def smc_k_rollout(ctx, u, P, W, states, k_active, horizon, cost, feas, steps=None, stream=None):
    _check(lib().smc_k_rollout(ctx.handle, _ptr(u), int(P), _ptr(W), _ptr(states),
                               _ptr(k_active), int(horizon), _ptr(cost), _ptr(feas),
                               _ptr(steps), _stream(stream)), ctx)


def smc_k_reduce(ctx, P, cost, feas, beta, chat, feas_pn, logw, stream=None):
    _check(lib().smc_k_reduce(ctx.handle, int(P), _ptr(cost), _ptr(feas), float(beta),
                              _ptr(chat), _ptr(feas_pn), _ptr(logw), _stream(stream)), ctx)


def smc_k_resample_offsets(ctx, mpc_step, iter_, U, stream=None):
    _check(lib().smc_k_resample_offsets(ctx.handle, int(mpc_step), int(iter_), _ptr(U),
                                        _stream(stream)), ctx)


def smc_k_resample(ctx, P, logw, U, anc, ess=None, stream=None):
    _check(lib().smc_k_resample(ctx.handle, int(P), _ptr(logw), _ptr(U), _ptr(anc), _ptr(ess),
                                _stream(stream)), ctx)


def smc_k_gather_move(ctx, P, u_in, anc, u_out, mpc_step, iter_, jitter, stream=None):
    _check(lib().smc_k_gather_move(ctx.handle, int(P), _ptr(u_in), _ptr(anc), _ptr(u_out),
                                   int(mpc_step), int(iter_), int(jitter), _stream(stream)), ctx)


def smc_k_propose(ctx, P, u, u_prop, mpc_step, iter_, stream=None):
    _check(lib().smc_k_propose(ctx.handle, int(P), _ptr(u), _ptr(u_prop), int(mpc_step),
                               int(iter_), _stream(stream)), ctx)


def smc_k_accept(ctx, P, u, u_prop, chat, chat_prop, feas_pn, feas_prop, logw, logw_prop,
                 mpc_step, iter_, accepted=None, stream=None):
    _check(lib().smc_k_accept(ctx.handle, int(P), _ptr(u), _ptr(u_prop), _ptr(chat),
                              _ptr(chat_prop), _ptr(feas_pn), _ptr(feas_prop), _ptr(logw),
                              _ptr(logw_prop), int(mpc_step), int(iter_), _ptr(accepted),
                              _stream(stream)), ctx)


def smc_k_select(ctx, P, logw, chat, beta, best, stream=None):
    _check(lib().smc_k_select(ctx.handle, int(P), _ptr(logw), _ptr(chat), float(beta),
                              _ptr(best), _stream(stream)), ctx)


def smc_set_rollout_layout(ctx, layout):
    """0 automatic, 1 aircraft-per-lane, 2 world-per-lane."""
    _check(lib().smc_set_rollout_layout(ctx.handle, int(layout)), ctx)


def smc_k_rollout_grad(ctx, u, P, W, states, k_active, horizon, grad, stream=None):
    _check(lib().smc_k_rollout_grad(ctx.handle, _ptr(u), int(P), _ptr(W), _ptr(states),
                                    _ptr(k_active), int(horizon), _ptr(grad), _stream(stream)), ctx)


def smc_k_mala_propose(ctx, P, u, grad, beta, u_prop, mpc_step, iter_, stream=None):
    _check(lib().smc_k_mala_propose(ctx.handle, int(P), _ptr(u), _ptr(grad), float(beta),
                                    _ptr(u_prop), int(mpc_step), int(iter_), _stream(stream)), ctx)


def smc_k_mala_accept(ctx, P, u, u_prop, grad, grad_prop, beta, chat, chat_prop, feas_pn,
                      feas_prop, logw, logw_prop, mpc_step, iter_, accepted, stream=None):
    _check(lib().smc_k_mala_accept(ctx.handle, int(P), _ptr(u), _ptr(u_prop), _ptr(grad),
                                   _ptr(grad_prop), float(beta), _ptr(chat), _ptr(chat_prop),
                                   _ptr(feas_pn), _ptr(feas_prop), _ptr(logw), _ptr(logw_prop),
                                   int(mpc_step), int(iter_), _ptr(accepted), _stream(stream)),
           ctx)
