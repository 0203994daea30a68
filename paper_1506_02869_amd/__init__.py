"""Python binding of the MI355X SMC-MPC engine (libsmc_mpc.so).

Argument marshalling only: every step of the optimiser runs in the HIP
kernels behind the C ABI declared in include/smc_mpc.h,
include/smc_kernels.h and include/smc_batch.h.  Function names follow the C ABI.  Device arrays are
torch tensors on a HIP device (PyTorch provides device memory and streams);
host arrays are NumPy arrays.

Streams: device-form calls take ``stream`` (a torch stream; default: torch's
current stream) and queue the library's work on it, so torch work queued
before the call on that stream (filling inputs) completes first and torch
work queued after it sees the outputs.  Torch's default stream has the
handle 0, the null stream, which the library uses as such.

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
        ("wind_model", C.c_int32), ("wind_beta", C.c_double), ("wind_gamma", C.c_double),
        ("wind_tcorr", C.c_double), ("weighting", C.c_int32), ("control_model", C.c_int32),
        ("warm_start", C.c_int32),
    ]


class StepInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("best_particle", C.c_int32),
                ("feasible_frac", C.c_double), ("accept_rate", C.c_double),
                ("ess_min", C.c_double), ("aircraft_steps", C.c_int64),
                ("pair_tests", C.c_int64),
                ("ms_total", C.c_double), ("ms_rollout", C.c_double),
                ("ms_wind", C.c_double), ("rollout_launches", C.c_int32),
                ("wind_launches", C.c_int32), ("ms_grad", C.c_double),
                ("grad_launches", C.c_int32), ("pair_tests_h", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


BATCH_BUCKETS = 8
BATCH_BUCKET_NMAX = (2, 4, 6, 8, 10, 12, 16, 20)
BATCH_ITEM_WORLDS = 64


class BatchTuning(C.Structure):
    _fields_ = [("block", C.c_int32 * BATCH_BUCKETS), ("grid_mult", C.c_int32 * BATCH_BUCKETS),
                ("order", C.c_int32)]

    def as_dict(self):
        return {"block": list(self.block), "grid_mult": list(self.grid_mult),
                "order": int(self.order)}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        t.block[:] = [int(v) for v in d.get("block", [0] * BATCH_BUCKETS)]
        t.grid_mult[:] = [int(v) for v in d.get("grid_mult", [0] * BATCH_BUCKETS)]
        t.order = int(d.get("order", 0))
        return t


class BatchInfo(C.Structure):
    _fields_ = [("n_scenarios", C.c_int32), ("iterations", C.c_int32),
                ("aircraft_steps", C.c_int64), ("pair_tests", C.c_int64),
                ("ms_total", C.c_double), ("accept_rate", C.c_double),
                ("feasible_frac", C.c_double), ("graph", C.c_int32),
                ("rollout_launches", C.c_int32), ("rollout_passes", C.c_int32),
                ("ms_rollout", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_VP = C.c_void_p
_I32P = C.POINTER(C.c_int32)
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
    "smc_plant_step": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP, _VP, _VP, C.c_int32,
                                 C.c_int32, _VP, _VP, _VP]),
    "smc_k_philox": (C.c_int, [C.c_uint64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                               C.c_int64, C.c_int64, _VP, _VP]),
    "smc_k_init_particles": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP]),
    "smc_k_wind_normals": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP]),
    "smc_k_wind_gemm": (C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "smc_k_wind_factor": (C.c_int, [_VP, _VP, _VP]),
    "smc_k_wind_fields": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP, _VP]),
    "smc_k_rollout": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, C.c_int32, _VP, _VP, _VP,
                                _VP]),
    "smc_k_reduce": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_double, _VP, _VP, _VP, _VP]),
    "smc_k_reduce_product": (C.c_int, [_VP, C.c_int32, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP]),
    "smc_k_resample_offsets": (C.c_int, [_VP, C.c_int64, C.c_int32, _VP, _VP]),
    "smc_k_resample": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP, _VP]),
    "smc_k_resample_noalloc": (C.c_int, [C.c_int32, C.c_int32, _VP, _VP, _VP, _VP, _VP]),
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
    "smc_batch_init": (C.c_int, [C.POINTER(Scenario), C.c_int32, C.POINTER(_VP)]),
    "smc_batch_step": (C.c_int, [_VP, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                 C.POINTER(BatchInfo)]),
    "smc_batch_step_dev": (C.c_int, [_VP, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                     C.POINTER(BatchInfo), _VP]),
    "smc_batch_set_graph": (C.c_int, [_VP, C.c_int32]),
    "smc_batch_get_tuning": (C.c_int, [_VP, C.POINTER(BatchTuning)]),
    "smc_batch_set_tuning": (C.c_int, [_VP, C.POINTER(BatchTuning)]),
    "smc_batch_autotune": (C.c_int, [_VP, C.c_int64, _VP, _VP, _VP, _VP, C.c_int32,
                                     C.POINTER(BatchTuning)]),
    "smc_batch_plan": (C.c_int, [C.c_int32, _VP, _VP, C.c_int32, C.c_int32, C.c_int32, _VP, _VP,
                                 _VP, _VP, C.c_int64, C.POINTER(C.c_int64)]),
    "smc_batch_last_error": (C.c_char_p, [_VP]),
    "smc_batch_destroy": (None, [_VP]),
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


def _dtypes(kind):
    """Accepted torch dtypes of an argument kind: 'f64', 'i32', 'u32' (int32
    bit patterns accepted), 'u8', 'u64' (int64 accepted), or a Context's
    'real'."""
    import torch
    table = {"f64": (torch.float64,), "f32": (torch.float32,), "i32": (torch.int32,),
             "u32": tuple(t for t in (torch.int32, getattr(torch, "uint32", None)) if t),
             "u8": (torch.uint8, torch.bool),
             "u64": tuple(t for t in (torch.int64, getattr(torch, "uint64", None)) if t)}
    return table[kind]


def _dev(t, name, kind, numel, optional=False):
    """Checked argument: a tensor of the given kind with exactly `numel`
    elements (None passes if optional).  Raises ValueError before any
    library call, so a wrong dtype or a short buffer never reaches a
    kernel; `_ptrs` then converts the checked tensors to device pointers."""
    import torch
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name}: a device tensor is required")
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    ok = _dtypes(kind) if isinstance(kind, str) else (kind,)
    if t.dtype not in ok:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {' or '.join(map(str, ok))}")
    if t.numel() != int(numel):
        raise ValueError(f"{name}: {t.numel()} elements, expected {int(numel)}")
    return t


def _ptrs(*ts):
    """Device pointers of already checked tensors (the device and contiguity
    checks come after every argument's type and size check)."""
    return tuple(_ptr(t) for t in ts)


def _host(a, name, shape, dtype):
    """Host array converted to dtype with exactly the given shape."""
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.shape != tuple(int(v) for v in shape):
        raise ValueError(f"{name}: shape {a.shape}, expected {tuple(shape)}")
    return a, a.ctypes.data_as(C.c_void_p)


def _count(P, name="P"):
    P = int(P)
    if P < 0:
        raise ValueError(f"{name} must be >= 0")
    return P


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
        # fields per iteration: one per sample, or one per sample and step
        # under the time-correlated wind model
        self.Mf = self.M * (self.H if int(scen.get("wind_model", 0)) == 1 else 1)
        self.scen = scen

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.precision == FP64 else torch.float32

    @property
    def D(self):
        return self.N * self.S * 3

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
    sc.wind_model = int(s.get("wind_model", 0))
    sc.wind_beta = float(s.get("wind_beta", 0.0))
    sc.wind_gamma = float(s.get("wind_gamma", 0.0))
    sc.wind_tcorr = float(s.get("wind_tcorr", 0.0))
    sc.weighting = int(s.get("weighting", 0))
    sc.control_model = int(s.get("control_model", 0))
    sc.warm_start = int(s.get("warm_start", 0))
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
    st_a, p_st = _host(states, "states", (ctx.N, 6), np.float64)
    ka_a, p_ka = _host(k_active, "k_active", (ctx.N,), np.int32)
    wm_a, p_wm = _host(wind_mean, "wind_mean", (2,), np.float64)
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
    """Device form: states [N,6] f64, k_active [N] i32, controls_out [N,S,3]
    f64, cost_out [1+N] f64, status_out [1] i32 (optional): device tensors."""
    wm_a, p_wm = _host(wind_mean, "wind_mean", (2,), np.float64)
    args = _ptrs(_dev(states, "states", "f64", ctx.N * 6), _dev(k_active, "k_active", "i32", ctx.N),
            _dev(controls_out, "controls_out", "f64", ctx.D),
            _dev(cost_out, "cost_out", "f64", 1 + ctx.N),
            _dev(status_out, "status_out", "i32", 1, optional=True))
    info = StepInfo() if want_info else None
    r = lib().smc_mpc_step_dev(ctx.handle, int(mpc_step), args[0], args[1], p_wm,
                               int(horizon), args[2], args[3], args[4],
                               C.byref(info) if info is not None else None, _stream(stream))
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
    pa = np.asarray(particles)
    P = pa.shape[0] if pa.ndim == 4 else -1
    pa, p_pa = _host(pa, "particles", (P, ctx.N, ctx.S, 3), np.float64)
    st_a, p_st = _host(states, "states", (ctx.N, 6), np.float64)
    ka_a, p_ka = _host(k_active, "k_active", (ctx.N,), np.int32)
    wm_a, p_wm = _host(wind_mean, "wind_mean", (2,), np.float64)
    cost = np.zeros((P, ctx.N))
    feas = np.zeros((P, ctx.N), dtype=np.uint8)
    r = lib().smc_eval_cost(ctx.handle, int(mpc_step), int(iter_), p_st, p_ka, p_wm,
                            int(horizon), p_pa, int(P), cost.ctypes.data_as(C.c_void_p),
                            feas.ctypes.data_as(C.c_void_p))
    _check(r, ctx)
    return cost, feas.astype(bool)


def smc_plant_step(ctx: Context, controls, plant_iter, n_steps=None, mpc_step=None, states=None,
                   k_active=None, wind_mean=None, horizon=None):
    """Host form: returns (states [N,6], k_active [N], event [N]) after the
    plant flew n_steps (default: the first control segment) of the plan."""
    s = ctx.scen
    mpc_step = s["mpc_step"] if mpc_step is None else mpc_step
    states = s["states"] if states is None else states
    k_active = s["k_active"] if k_active is None else k_active
    wind_mean = s["wind_mean"] if wind_mean is None else wind_mean
    horizon = ctx.H if horizon is None else horizon
    n_steps = -(-int(horizon) // ctx.S) if n_steps is None else n_steps
    st_a, p_st = _host(states, "states", (ctx.N, 6), np.float64)
    ka_a, p_ka = _host(k_active, "k_active", (ctx.N,), np.int32)
    wm_a, p_wm = _host(wind_mean, "wind_mean", (2,), np.float64)
    c_a, p_c = _host(controls, "controls", (ctx.N, ctx.S, 3), np.float64)
    st_out = np.zeros((ctx.N, 6))
    ka_out = np.zeros(ctx.N, dtype=np.int32)
    ev = np.zeros(ctx.N, dtype=np.int32)
    r = lib().smc_plant_step(ctx.handle, int(mpc_step), int(plant_iter), p_st, p_ka, p_wm, p_c,
                             int(horizon), int(n_steps), st_out.ctypes.data_as(C.c_void_p),
                             ka_out.ctypes.data_as(C.c_void_p), ev.ctypes.data_as(C.c_void_p))
    _check(r, ctx)
    return st_out, ka_out, ev


def rolling_window(ctx: Context, n_updates, plant_iter=None, states=None, k_active=None,
                   mpc_step0=None, wind_mean=None):
    """Receding-horizon loop (Sec. "Model Predictive Control", "Rolling
    Window"): n_updates times solve one MPC update from the current states,
    let the plant fly the first control segment (smc_plant_step, disturbance
    from iteration word plant_iter, default n_iters + 1), move the window.
    Returns one dict per update (controls, cost, states and k_active after the
    plant step, events, info)."""
    s = ctx.scen
    plant_iter = int(s["K"]) + 1 if plant_iter is None else plant_iter
    states = np.array(s["states"] if states is None else states, dtype=np.float64)
    k_active = np.array(s["k_active"] if k_active is None else k_active, dtype=np.int32)
    step0 = int(s["mpc_step"]) if mpc_step0 is None else int(mpc_step0)
    out = []
    for t in range(n_updates):
        step = step0 + t
        ctrl, cost, status, info = smc_mpc_step(ctx, mpc_step=step, states=states,
                                                k_active=k_active, wind_mean=wind_mean)
        states, k_active, ev = smc_plant_step(ctx, ctrl, plant_iter, mpc_step=step,
                                              states=states, k_active=k_active,
                                              wind_mean=wind_mean)
        out.append(dict(controls=ctrl, cost=cost, status=status, states=states.copy(),
                        k_active=k_active.copy(), event=ev, info=info))
    return out


# ---- kernel-level entry points (device tensors) -----------------------------

def smc_k_philox(seed, mpc_step, iter_, purpose, scenario, e0, n, out, stream=None):
    p_out = _ptr(_dev(out, "out", "u32", 4 * _count(n, "n")))
    _check(lib().smc_k_philox(int(seed) & 0xFFFFFFFFFFFFFFFF, int(mpc_step), int(iter_),
                              int(purpose), int(scenario), int(e0), int(n), p_out,
                              _stream(stream)))


def smc_k_init_particles(ctx, mpc_step, P, u, stream=None):
    p_u = _ptr(_dev(u, "u", ctx.real_dtype, _count(P) * ctx.D))
    _check(lib().smc_k_init_particles(ctx.handle, int(mpc_step), int(P), p_u,
                                      _stream(stream)), ctx)


def smc_k_wind_normals(ctx, mpc_step, iter_, Z, stream=None):
    p_z = _ptr(_dev(Z, "Z", ctx.real_dtype, ctx.G * 2 * ctx.M))
    _check(lib().smc_k_wind_normals(ctx.handle, int(mpc_step), int(iter_), p_z,
                                    _stream(stream)), ctx)


def smc_k_wind_gemm(ctx, Z, wind_mean, W, stream=None):
    wm_a, p_wm = _host(wind_mean, "wind_mean", (2,), np.float64)
    p_z, p_w = _ptrs(_dev(Z, "Z", ctx.real_dtype, ctx.G * 2 * ctx.M),
                     _dev(W, "W", ctx.real_dtype, ctx.M * ctx.G * 2))
    _check(lib().smc_k_wind_gemm(ctx.handle, p_z, p_wm, p_w, _stream(stream)), ctx)


def smc_k_wind_factor(ctx, out, stream=None):
    p_o = _ptr(_dev(out, "out", ctx.real_dtype, ctx.G * ctx.G))
    _check(lib().smc_k_wind_factor(ctx.handle, p_o, _stream(stream)), ctx)


def smc_k_wind_fields(ctx, mpc_step, it, wind_mean, W, stream=None):
    wm_a, p_wm = _host(wind_mean, "wind_mean", (2,), np.float64)
    p_w = _ptr(_dev(W, "W", ctx.real_dtype, ctx.Mf * ctx.G * 2))
    _check(lib().smc_k_wind_fields(ctx.handle, int(mpc_step), int(it), p_wm, p_w,
                                   _stream(stream)), ctx)


def smc_k_rollout(ctx, u, P, W, states, k_active, horizon, cost, feas, steps=None, stream=None):
    P = _count(P)
    a = _ptrs(_dev(u, "u", ctx.real_dtype, P * ctx.D), _dev(W, "W", ctx.real_dtype, ctx.Mf * ctx.G * 2),
         _dev(states, "states", "f64", ctx.N * 6), _dev(k_active, "k_active", "i32", ctx.N),
         _dev(cost, "cost", "f64", ctx.M * P * ctx.N), _dev(feas, "feas", "u8", ctx.M * P * ctx.N),
         _dev(steps, "steps", "u64", 128, optional=True))
    _check(lib().smc_k_rollout(ctx.handle, a[0], P, a[1], a[2], a[3], int(horizon), a[4], a[5],
                               a[6], _stream(stream)), ctx)


def smc_k_reduce(ctx, P, cost, feas, beta, chat, feas_pn, logw, stream=None):
    P = _count(P)
    a = _ptrs(_dev(cost, "cost", "f64", ctx.M * P * ctx.N), _dev(feas, "feas", "u8", ctx.M * P * ctx.N),
         _dev(chat, "chat", "f64", P * ctx.N), _dev(feas_pn, "feas_pn", "u8", P * ctx.N),
         _dev(logw, "logw", "f64", P * ctx.N))
    _check(lib().smc_k_reduce(ctx.handle, P, a[0], a[1], float(beta), a[2], a[3], a[4],
                              _stream(stream)), ctx)


def smc_k_reduce_product(ctx, P, M, cost, feas, chat, feas_pn, logw, stream=None):
    P, M = _count(P), _count(M, "M")
    a = _ptrs(_dev(cost, "cost", "f64", M * P * ctx.N), _dev(feas, "feas", "u8", M * P * ctx.N),
         _dev(chat, "chat", "f64", P * ctx.N), _dev(feas_pn, "feas_pn", "u8", P * ctx.N),
         _dev(logw, "logw", "f64", P * ctx.N))
    _check(lib().smc_k_reduce_product(ctx.handle, P, M, a[0], a[1], a[2], a[3], a[4],
                                      _stream(stream)), ctx)


def smc_k_resample_offsets(ctx, mpc_step, iter_, U, stream=None):
    p_u = _ptr(_dev(U, "U", "u32", ctx.N))
    _check(lib().smc_k_resample_offsets(ctx.handle, int(mpc_step), int(iter_), p_u,
                                        _stream(stream)), ctx)


def smc_k_resample(ctx, P, logw, U, anc, ess=None, stream=None):
    P = _count(P)
    a = _ptrs(_dev(logw, "logw", "f64", P * ctx.N), _dev(U, "U", "u32", ctx.N),
         _dev(anc, "anc", "i32", ctx.N * P), _dev(ess, "ess", "f64", ctx.N, optional=True))
    _check(lib().smc_k_resample(ctx.handle, P, a[0], a[1], a[2], a[3], _stream(stream)), ctx)


def smc_k_resample_noalloc(N, P, logw, U, anc, ess=None, stream=None):
    """Context-free resampling with the library's static scan workspace
    (no device allocation; include/smc_kernels.h)."""
    N, P = _count(N, "N"), _count(P)
    a = _ptrs(_dev(logw, "logw", "f64", P * N), _dev(U, "U", "u32", N),
              _dev(anc, "anc", "i32", N * P), _dev(ess, "ess", "f64", N, optional=True))
    _check(lib().smc_k_resample_noalloc(N, P, a[0], a[1], a[2], a[3], _stream(stream)))


def smc_k_gather_move(ctx, P, u_in, anc, u_out, mpc_step, iter_, jitter, stream=None):
    P = _count(P)
    a = _ptrs(_dev(u_in, "u_in", ctx.real_dtype, P * ctx.D), _dev(anc, "anc", "i32", ctx.N * P),
         _dev(u_out, "u_out", ctx.real_dtype, P * ctx.D))
    _check(lib().smc_k_gather_move(ctx.handle, P, a[0], a[1], a[2], int(mpc_step), int(iter_),
                                   int(jitter), _stream(stream)), ctx)


def smc_k_propose(ctx, P, u, u_prop, mpc_step, iter_, stream=None):
    P = _count(P)
    a = _ptrs(_dev(u, "u", ctx.real_dtype, P * ctx.D), _dev(u_prop, "u_prop", ctx.real_dtype, P * ctx.D))
    _check(lib().smc_k_propose(ctx.handle, P, a[0], a[1], int(mpc_step), int(iter_),
                               _stream(stream)), ctx)


def _pn_args(ctx, P, chat, chat_prop, feas_pn, feas_prop, logw, logw_prop):
    n = P * ctx.N
    return (_dev(chat, "chat", "f64", n), _dev(chat_prop, "chat_prop", "f64", n),
            _dev(feas_pn, "feas_pn", "u8", n), _dev(feas_prop, "feas_prop", "u8", n),
            _dev(logw, "logw", "f64", n), _dev(logw_prop, "logw_prop", "f64", n))


def smc_k_accept(ctx, P, u, u_prop, chat, chat_prop, feas_pn, feas_prop, logw, logw_prop,
                 mpc_step, iter_, accepted=None, stream=None):
    P = _count(P)
    a = _ptrs(_dev(u, "u", ctx.real_dtype, P * ctx.D), _dev(u_prop, "u_prop", ctx.real_dtype, P * ctx.D),
              *_pn_args(ctx, P, chat, chat_prop, feas_pn, feas_prop, logw, logw_prop),
              _dev(accepted, "accepted", "i32", P, optional=True))
    _check(lib().smc_k_accept(ctx.handle, P, *a[:8], int(mpc_step), int(iter_), a[8],
                              _stream(stream)), ctx)


def smc_k_select(ctx, P, logw, chat, beta, best, stream=None):
    P = _count(P)
    a = _ptrs(_dev(logw, "logw", "f64", P * ctx.N), _dev(chat, "chat", "f64", P * ctx.N),
         _dev(best, "best", "i32", 2))
    _check(lib().smc_k_select(ctx.handle, P, a[0], a[1], float(beta), a[2], _stream(stream)), ctx)


def smc_set_rollout_layout(ctx, layout):
    """0 automatic, 1 aircraft-per-lane, 2 world-per-lane."""
    _check(lib().smc_set_rollout_layout(ctx.handle, int(layout)), ctx)


def smc_k_rollout_grad(ctx, u, P, W, states, k_active, horizon, grad, stream=None):
    P = _count(P)
    a = _ptrs(_dev(u, "u", ctx.real_dtype, P * ctx.D), _dev(W, "W", ctx.real_dtype, ctx.Mf * ctx.G * 2),
         _dev(states, "states", "f64", ctx.N * 6), _dev(k_active, "k_active", "i32", ctx.N),
         _dev(grad, "grad", "f64", P * ctx.D))
    _check(lib().smc_k_rollout_grad(ctx.handle, a[0], P, a[1], a[2], a[3], int(horizon), a[4],
                                    _stream(stream)), ctx)


def smc_k_mala_propose(ctx, P, u, grad, beta, u_prop, mpc_step, iter_, stream=None):
    P = _count(P)
    a = _ptrs(_dev(u, "u", ctx.real_dtype, P * ctx.D), _dev(grad, "grad", "f64", P * ctx.D),
         _dev(u_prop, "u_prop", ctx.real_dtype, P * ctx.D))
    _check(lib().smc_k_mala_propose(ctx.handle, P, a[0], a[1], float(beta), a[2], int(mpc_step),
                                    int(iter_), _stream(stream)), ctx)


def smc_k_mala_accept(ctx, P, u, u_prop, grad, grad_prop, beta, chat, chat_prop, feas_pn,
                      feas_prop, logw, logw_prop, mpc_step, iter_, accepted, stream=None):
    P = _count(P)
    a = _ptrs(_dev(u, "u", ctx.real_dtype, P * ctx.D), _dev(u_prop, "u_prop", ctx.real_dtype, P * ctx.D),
              _dev(grad, "grad", "f64", P * ctx.D), _dev(grad_prop, "grad_prop", "f64", P * ctx.D),
              *_pn_args(ctx, P, chat, chat_prop, feas_pn, feas_prop, logw, logw_prop),
              _dev(accepted, "accepted", "i32", P))
    _check(lib().smc_k_mala_accept(ctx.handle, P, a[0], a[1], a[2], a[3], float(beta), *a[4:10],
                                   int(mpc_step), int(iter_), a[10], _stream(stream)), ctx)


# ---- batched form (include/smc_batch.h) --------------------------------------

def _bcheck(status, batch=None):
    if status < 0:
        msg = lib().smc_batch_last_error(batch.handle if batch is not None else None)
        raise SmcError(status, (msg or b"").decode())
    return status


class Batch:
    """Owns an smc_batch*; created by smc_batch_init.  Per-scenario arrays
    are concatenated in scenario order (see include/smc_batch.h)."""

    def __init__(self, handle, scens):
        self.handle = handle
        self.scens = scens
        self.ns = len(scens)
        self.N = [int(s["N"]) for s in scens]
        self.S = [int(s["S"]) for s in scens]
        self.H = [int(s["H"]) for s in scens]
        self.ctrl_off = np.concatenate([[0], np.cumsum([n * k * 3 for n, k in
                                                        zip(self.N, self.S)])]).astype(np.int64)
        self.cost_off = np.concatenate([[0], np.cumsum([1 + n for n in self.N])]).astype(np.int64)
        self.row_off = np.concatenate([[0], np.cumsum(self.N)]).astype(np.int64)

    def split(self, controls, costs):
        """Per-scenario ([N, S, 3] controls, [1 + N] costs) from the
        concatenated outputs."""
        out = []
        for s in range(self.ns):
            c = controls[self.ctrl_off[s]:self.ctrl_off[s + 1]].reshape(self.N[s], self.S[s], 3)
            out.append((c, costs[self.cost_off[s]:self.cost_off[s + 1]]))
        return out

    def close(self):
        if self.handle:
            lib().smc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def smc_batch_init(scens) -> Batch:
    arr = (Scenario * len(scens))()
    keep = []
    for k, s in enumerate(scens):
        sc, kp = make_scenario_struct(s)
        arr[k] = sc
        keep.append(kp)
    h = C.c_void_p()
    st = lib().smc_batch_init(arr, len(scens), C.byref(h))
    if st < 0:
        raise SmcError(st, (lib().smc_batch_last_error(None) or b"").decode())
    b = Batch(h, scens)
    b._keep = keep
    return b


def _batch_inputs(b: Batch, states, k_active, wind_mean, horizons):
    sc = b.scens
    states = np.concatenate([s["states"] for s in sc]) if states is None else states
    k_active = np.concatenate([s["k_active"] for s in sc]) if k_active is None else k_active
    wind_mean = np.stack([s["wind_mean"] for s in sc]) if wind_mean is None else wind_mean
    horizons = np.array(b.H) if horizons is None else horizons
    rows = int(b.row_off[-1])
    return (_host(states, "states", (rows, 6), np.float64),
            _host(k_active, "k_active", (rows,), np.int32),
            _host(wind_mean, "wind_mean", (b.ns, 2), np.float64),
            _host(horizons, "horizons", (b.ns,), np.int32))


def smc_batch_step(b: Batch, mpc_step=0, states=None, k_active=None, wind_mean=None,
                   horizons=None):
    """Host form: returns (controls [sum N S 3], costs [sum (1 + N)],
    status [n_scen], return code, info dict)."""
    (st_a, p_st), (ka_a, p_ka), (wm_a, p_wm), (h_a, p_h) = _batch_inputs(
        b, states, k_active, wind_mean, horizons)
    ctrl = np.zeros(int(b.ctrl_off[-1]))
    cost = np.zeros(int(b.cost_off[-1]))
    status = np.zeros(b.ns, dtype=np.int32)
    info = BatchInfo()
    r = lib().smc_batch_step(b.handle, int(mpc_step), p_st, p_ka, p_wm, p_h,
                             ctrl.ctypes.data_as(C.c_void_p), cost.ctypes.data_as(C.c_void_p),
                             status.ctypes.data_as(C.c_void_p), C.byref(info))
    _bcheck(r, b)
    return ctrl, cost, status, r, info.as_dict()


def smc_batch_step_dev(b: Batch, mpc_step, states, k_active, wind_mean, horizons, controls_out,
                       cost_out, status_out=None, want_info=False, stream=None):
    """Device form: states [sum N, 6] f64, k_active [sum N] i32 and the
    outputs are device tensors; wind_mean [n_scen, 2] and horizons are host."""
    wm_a, p_wm = _host(wind_mean, "wind_mean", (b.ns, 2), np.float64)
    h_a, p_h = _host(horizons, "horizons", (b.ns,), np.int32)
    rows = int(b.row_off[-1])
    a = _ptrs(_dev(states, "states", "f64", rows * 6), _dev(k_active, "k_active", "i32", rows),
         _dev(controls_out, "controls_out", "f64", int(b.ctrl_off[-1])),
         _dev(cost_out, "cost_out", "f64", int(b.cost_off[-1])),
         _dev(status_out, "status_out", "i32", b.ns, optional=True))
    info = BatchInfo() if want_info else None
    r = lib().smc_batch_step_dev(b.handle, int(mpc_step), a[0], a[1], p_wm, p_h, a[2], a[3], a[4],
                                 C.byref(info) if info is not None else None, _stream(stream))
    _bcheck(r, b)
    return r, (info.as_dict() if info is not None else None)


def smc_batch_set_graph(b: Batch, enable: bool):
    _bcheck(lib().smc_batch_set_graph(b.handle, 1 if enable else 0), b)


def smc_batch_get_tuning(b: Batch) -> dict:
    t = BatchTuning()
    _bcheck(lib().smc_batch_get_tuning(b.handle, C.byref(t)), b)
    return t.as_dict()


def smc_batch_set_tuning(b: Batch, tuning: dict):
    t = BatchTuning.from_dict(tuning)
    _bcheck(lib().smc_batch_set_tuning(b.handle, C.byref(t)), b)


def smc_batch_autotune(b: Batch, mpc_step=0, states=None, k_active=None, wind_mean=None,
                       horizons=None, reps=3) -> dict:
    (st_a, p_st), (ka_a, p_ka), (wm_a, p_wm), (h_a, p_h) = _batch_inputs(
        b, states, k_active, wind_mean, horizons)
    t = BatchTuning()
    _bcheck(lib().smc_batch_autotune(b.handle, int(mpc_step), p_st, p_ka, p_wm, p_h, int(reps),
                                     C.byref(t)), b)
    return t.as_dict()


def smc_batch_plan(n_aircraft, horizons, n_particles, n_wind, order=0):
    """Host-only work plan: (bucket_start [8], bucket_count [8], item_scen,
    item_world0)."""
    na, p_na = _hp(n_aircraft, np.int32)
    hz, p_hz = _hp(horizons, np.int32)
    bs = np.zeros(BATCH_BUCKETS, dtype=np.int32)
    bc = np.zeros(BATCH_BUCKETS, dtype=np.int32)
    n = C.c_int64()
    per = -(-int(n_particles) * int(n_wind) // BATCH_ITEM_WORLDS)
    cap = per * len(na)
    isc = np.zeros(cap, dtype=np.int32)
    iw = np.zeros(cap, dtype=np.int32)
    _bcheck(lib().smc_batch_plan(len(na), p_na, p_hz, int(n_particles), int(n_wind), int(order),
                                 bs.ctypes.data_as(C.c_void_p), bc.ctypes.data_as(C.c_void_p),
                                 isc.ctypes.data_as(C.c_void_p), iw.ctypes.data_as(C.c_void_p),
                                 cap, C.byref(n)))
    return bs, bc, isc[:n.value], iw[:n.value]


# ---- autotune cache (host logic) -----------------------------------------------

def tuning_key(scens, device_name: str) -> str:
    """Cache key of a batch's launch shapes: device, precision, sizes and
    the bucket histogram with horizons (what the rollout's speed depends on)."""
    import hashlib
    s0 = scens[0]
    parts = [device_name, f"p{int(s0['precision'])}", f"L{int(s0['L'])}", f"M{int(s0['M'])}",
             f"m{int(s0['move'])}"]
    parts += [f"{int(s['N'])}x{int(s['H'])}" for s in sorted(
        scens, key=lambda s: (int(s["N"]), int(s["H"])))]
    return hashlib.sha256("|".join(parts).encode()).hexdigest()[:24]


def load_tuning(path: str, key: str):
    """Tuning dict stored under key in the JSON cache at path, or None."""
    import json
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        try:
            data = json.load(f)
        except json.JSONDecodeError:
            return None
    t = data.get(key)
    if not isinstance(t, dict):
        return None
    ok = (len(t.get("block", [])) == BATCH_BUCKETS and
          len(t.get("grid_mult", [])) == BATCH_BUCKETS and
          all(v in (0, 64, 128, 256) for v in t["block"]) and
          all(0 <= v <= 4 for v in t["grid_mult"]) and t.get("order", 0) in (0, 1))
    return t if ok else None


def save_tuning(path: str, key: str, tuning: dict):
    """Store tuning under key in the JSON cache at path (atomic replace)."""
    import json
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            try:
                data = json.load(f)
            except json.JSONDecodeError:
                data = {}
    data[key] = {"block": [int(v) for v in tuning["block"]],
                 "grid_mult": [int(v) for v in tuning["grid_mult"]],
                 "order": int(tuning.get("order", 0))}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def batch_tune(b: Batch, cache_path=None, device_name=None, reps=3, **inputs) -> dict:
    """Install a cached tuning for this batch shape, or autotune and cache it."""
    if cache_path:
        if device_name is None:
            import torch
            device_name = torch.cuda.get_device_name(0)
        key = tuning_key(b.scens, device_name)
        t = load_tuning(cache_path, key)
        if t is not None:
            smc_batch_set_tuning(b, t)
            return t
    t = smc_batch_autotune(b, reps=reps, **inputs)
    if cache_path:
        save_tuning(cache_path, key, t)
    return t
