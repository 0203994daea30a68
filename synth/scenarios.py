"""Seeded synthetic terminal-area scenarios.

This module only draws inputs: initial aircraft states, targets, aircraft
parameters, activation steps and the optional population grid.  It holds none
of the optimiser's arithmetic (no dynamics, costs, wind factorisation or
resampling), so both the CPU oracle and the GPU path can be fed from it.

Geometry follows the paper's terminal-area setting (Sec. "Simulation Setup"
and Sec. "Trajectory Planning"): a single runway at the origin, x east, y
north, landing and departing east-to-west; departures start at 400 m above
the threshold heading west; arrivals enter on the boundary of the area.

Aircraft parameters are round, narrow-body-like synthetic values.  The paper
takes A320 data from a licensed aircraft database that is not available here,
so none of these numbers claims to be that data.

Every scenario is a plain ``dict`` of Python scalars and NumPy arrays in SI
units (angles in radians).  Field list, in the order the C ABI takes them:

    name, N, S, H, dt, L, M, K, box(3), grid(3), wind_sigma, wind_ell,
    wind_nugget, sep_h, sep_v, kind[N] (0 arrival, 1 departure),
    aircraft[N, 9]  (wing_area, cd0, cd2, cf1, cf2, t_max, m_empty,
                     phi_max, gamma_max),
    ctrl_lo[3], ctrl_hi[3]  (heading rate, true airspeed, climb rate),
    env[4]   (z_min, z_max, v_min, v_max),
    landing[5] (P_runway, P_beta, P_chi, P_vs, beta_f),
    targets[N, 4] (bearing theta_F, altitude Z, speed v_D, exit radius D_TMA),
    cost_w[9] (arr hdg, arr glide, arr fuel, dep brg, dep fuel, dep alt,
               dep spd, alpha_time, alpha_noise),
    time_norm, noise_alt, popdense[ny_p, nx_p] float32 or None,
    precision (0 fp64, 1 fp32), move (0 jitter, 1 rwmh, 2 mala),
    control_model (0 kinematic segment controls, 1 the paper's per-step
    thrust fraction / flight-path angle / bank, S = H), warm_start (1: an
    update after the first starts from the previous update's final
    population shifted by one control segment),
    kappa, sigma_move, mala_step (standard deviation of the Langevin proposal
    in logit coordinates: the time step h = 1e-2 of the differentiable
    workload gives sqrt(h) = 0.1), seed,
    states[N, 6] (x, y, z, v, chi, m), k_active[N], wind_mean[2], mpc_step
"""
from __future__ import annotations

import math

import numpy as np

DEG = math.pi / 180.0

AC_FIELDS = ("wing_area", "cd0", "cd2", "cf1", "cf2", "t_max", "m_empty",
             "phi_max", "gamma_max")
N_AC_PAR = len(AC_FIELDS)

# Objective weights of the paper's coefficient table (Tab. coeff), mapped by
# the "Associated cost" column: arrivals heading 0.25 / nominal altitude 0.65 /
# fuel 0.1, departures bearing 0.4 / fuel 0.1 / altitude 0.25 / speed 0.25.
MIX_WEIGHTS = (0.25, 0.65, 0.10, 0.40, 0.10, 0.25, 0.25)

PRECISION = {"fp64": 0, "fp32": 1}
MOVES = {"jitter": 0, "rwmh": 1, "mala": 2}
WIND_MODELS = {"se": 0, "ar1": 1}   # static squared-exponential; the paper's time recursion
CONTROL_MODELS = {"kinematic": 0, "paper": 1}


def _aircraft_params(rng: np.random.Generator, n: int) -> np.ndarray:
    ac = np.empty((n, N_AC_PAR), dtype=np.float64)
    ac[:, 0] = 122.6          # wing area [m^2]
    ac[:, 1] = 0.025          # zero-lift drag coefficient
    ac[:, 2] = 0.040          # induced drag factor
    ac[:, 3] = 1.5e-5         # fuel-flow coefficient Cf1 [kg/(N s)]
    ac[:, 4] = 1000.0         # fuel-flow speed scale Cf2 [m/s]
    ac[:, 5] = 240_000.0      # maximum thrust [N]
    ac[:, 6] = 42_000.0       # empty mass [kg]
    ac[:, 7] = 35.0 * DEG     # bank limit
    ac[:, 8] = 10.0 * DEG     # climb-angle limit
    # small per-aircraft spread so that aircraft are not identical
    ac[:, 0] *= rng.uniform(0.95, 1.05, n)
    ac[:, 1] *= rng.uniform(0.95, 1.05, n)
    return ac


def _arrival_states(rng, n, box, r_entry, min_sep, z_lo=3048.0, z_hi=4572.0,
                    v0=200.0):
    """Arrivals on a circle of radius ``r_entry`` (the area's boundary),
    flight level 100-150, heading to the origin +-30 deg; pairwise horizontal
    distance at least ``min_sep`` (rejection)."""
    out = np.zeros((n, 6))
    placed = []
    tries = 0
    while len(placed) < n:
        tries += 1
        if tries > 100_000:
            raise RuntimeError("could not place arrivals with the requested separation")
        psi = rng.uniform(0.0, 2.0 * math.pi)
        x, y = r_entry * math.cos(psi), r_entry * math.sin(psi)
        z = rng.uniform(z_lo, z_hi)
        if any(math.hypot(x - p[0], y - p[1]) < min_sep for p in placed):
            continue
        chi = math.atan2(-y, -x) + rng.uniform(-30.0, 30.0) * DEG
        m0 = rng.uniform(55_000.0, 70_000.0)
        placed.append((x, y, z, v0, chi, m0))
    if n:
        out[:] = np.array(placed)
    return out


def _departure_states(rng, n, v0=110.0):
    out = np.zeros((n, 6))
    for j in range(n):
        out[j] = (0.0, 0.0, 400.0, v0, math.pi, rng.uniform(55_000.0, 70_000.0))
    return out


def _departure_targets(rng, n, box, d_tma):
    t = np.zeros((n, 4))
    for j in range(n):
        t[j, 0] = rng.uniform(-math.pi, math.pi)             # bearing theta_F
        t[j, 1] = rng.uniform(0.70, 0.90) * box[2]           # target altitude Z
        t[j, 2] = rng.uniform(180.0, 230.0)                  # target speed v_D
        t[j, 3] = d_tma                                      # exit radius
    return t


def make_scenario(name: str, *, n_arr: int, n_dep: int, box, grid, H: int,
                  dt: float, S: int, M: int, L: int, K: int,
                  precision: str = "fp64", move: str = "jitter",
                  seed: int = 0, dep_spacing: int | None = None,
                  alpha_time: float = 0.2, alpha_noise: float = 0.0,
                  noise_alt: float = 2000.0, pop_n=None, kappa: float = 1.0,
                  sigma_move: float = 0.02, mala_step: float = 0.1,
                  mpc_step: int = 0, wind_model: str = "se",
                  wind_tcorr: float = 1800.0, controls: str = "kinematic",
                  warm_start: bool = False) -> dict:
    rng = np.random.default_rng(seed)
    box = tuple(float(b) for b in box)
    N = n_arr + n_dep
    sep_h, sep_v = 5556.0, 304.8          # 3 NM, 1000 ft
    r_entry = 0.45 * min(box[0], box[1])
    arr = _arrival_states(rng, n_arr, box, r_entry, 1.5 * sep_h)
    dep = _departure_states(rng, n_dep)
    states = np.concatenate([arr, dep], axis=0)
    kind = np.array([0] * n_arr + [1] * n_dep, dtype=np.int8)
    targets = np.zeros((N, 4))
    targets[n_arr:] = _departure_targets(rng, n_dep, box, r_entry)
    # departures released one after the other from the same threshold
    if dep_spacing is None:
        dep_spacing = 12 if 12 * max(n_dep - 1, 0) < H else max(H // max(n_dep, 1), 1)
    k_active = np.zeros(N, dtype=np.int32)
    k_active[n_arr:] = dep_spacing * np.arange(n_dep, dtype=np.int32)
    aircraft = _aircraft_params(rng, N)
    popdense = None
    if pop_n is not None:
        # i.i.d. lognormal(0, 1.5) cells, capped at the 90 % quantile and
        # scaled to [0, 1] (the paper caps its density at 1)
        X = rng.lognormal(mean=0.0, sigma=1.5, size=(pop_n[1], pop_n[0]))
        q90 = math.exp(1.5 * 1.2815515655446004)
        popdense = np.minimum(X / q90, 1.0).astype(np.float32)
    if controls == "paper":
        # the paper's per-step controls: thrust (fraction of T_max, up to
        # about twice the cruise drag), flight-path angle, bank; one control
        # set per step
        S = H
        ctrl_lo = np.array([0.0, -6.0 * DEG, -25.0 * DEG])
        ctrl_hi = np.array([0.5, 6.0 * DEG, 25.0 * DEG])
    else:
        ctrl_lo = np.array([-3.0 * DEG, 110.0, -15.0])
        ctrl_hi = np.array([3.0 * DEG, 250.0, 15.0])
    env = np.array([0.0, box[2], 110.0, 250.0])
    landing = np.array([8000.0, 6.0 * DEG, 15.0 * DEG, 130.0, 3.0 * DEG])
    cost_w = np.array(list(MIX_WEIGHTS) + [alpha_time, alpha_noise])
    time_norm = 2.0 * math.hypot(box[0] / 2, box[1] / 2) / env[2]
    return dict(
        name=name, N=N, S=S, H=H, dt=float(dt), L=L, M=M, K=K,
        box=np.array(box), grid=np.array(grid, dtype=np.int32),
        wind_sigma=5.0, wind_ell=20_000.0, wind_nugget=1e-10,
        sep_h=sep_h, sep_v=sep_v, kind=kind, aircraft=aircraft,
        ctrl_lo=ctrl_lo, ctrl_hi=ctrl_hi, env=env, landing=landing,
        targets=targets, cost_w=cost_w, time_norm=float(time_norm),
        noise_alt=float(noise_alt), popdense=popdense,
        precision=PRECISION[precision], move=MOVES[move], kappa=float(kappa),
        sigma_move=float(sigma_move), mala_step=float(mala_step),
        seed=int(seed), states=states, k_active=k_active,
        wind_mean=np.zeros(2), mpc_step=int(mpc_step),
        # the paper's exponential covariance and time recursion (wind_model
        # 1): beta, gamma [1/m] as quoted there, G_t [s] a stated choice
        wind_model=WIND_MODELS[wind_model], wind_beta=1.6e-6, wind_gamma=1.5e-5,
        wind_tcorr=float(wind_tcorr),
        control_model=CONTROL_MODELS[controls],
        warm_start=int(bool(warm_start)),
    )


# --- the five workload shapes ------------------------------------------------

def c1(seed: int = 0, **kw) -> dict:
    """2 aircraft (1 arrival, 1 departure), 60x60x6 km, H=60, dt=5 s, S=6,
    wind 16x16x4 with M=16, L=256, K=20, FP64."""
    args = dict(n_arr=1, n_dep=1, box=(60e3, 60e3, 6e3), grid=(16, 16, 4),
                H=60, dt=5.0, S=6, M=16, L=256, K=20, precision="fp64",
                seed=seed)
    args.update(kw)
    return make_scenario("C1", **args)


def c2(seed: int = 0, **kw) -> dict:
    """10 aircraft (6 arrivals, 4 departures released at steps 0/12/24/36),
    100x100x8 km, H=120, dt=5 s, S=8, wind 32x32x8 (G=8192) with M=64,
    L=8192, K=40, FP32 rollout."""
    args = dict(n_arr=6, n_dep=4, box=(100e3, 100e3, 8e3), grid=(32, 32, 8),
                H=120, dt=5.0, S=8, M=64, L=8192, K=40, precision="fp32",
                seed=seed)
    args.update(kw)
    return make_scenario("C2", **args)


def c3(seed: int = 0, n_scen: int = 64, **kw) -> list:
    """64 independent scenarios: N ~ U{2..20} (60 % arrivals), H ~ U{60..180},
    S = ceil(H/15), 100x100x8 km, wind 32x32x8 with M=32, L=4096, K=40, FP32."""
    rng = np.random.default_rng(10_000 + seed)
    out = []
    for s in range(n_scen):
        N = int(rng.integers(2, 21))
        n_arr = max(1, int(round(0.6 * N)))
        n_dep = N - n_arr
        H = int(rng.integers(60, 181))
        S = int(math.ceil(H / 15))
        args = dict(n_arr=n_arr, n_dep=n_dep, box=(100e3, 100e3, 8e3),
                    grid=(32, 32, 8), H=H, dt=5.0, S=S, M=32, L=4096, K=40,
                    precision="fp32", seed=seed * 1000 + s)
        args.update(kw)
        sc = make_scenario(f"C3.{s}", **args)
        sc["scenario_id"] = s
        out.append(sc)
    return out


def c4(seed: int = 0, **kw) -> dict:
    """20 aircraft (12 arrivals, 8 departures), 100x100x8 km, H=150, dt=4 s,
    S=10 (600 parameters per particle), wind 32x32x8 with M=64, L=16384,
    MALA moves."""
    args = dict(n_arr=12, n_dep=8, box=(100e3, 100e3, 8e3), grid=(32, 32, 8),
                H=150, dt=4.0, S=10, M=64, L=16384, K=40, precision="fp32",
                move="mala", seed=seed)
    args.update(kw)
    return make_scenario("C4", **args)


def c5(seed: int = 0, **kw) -> dict:
    """40 aircraft (24 arrivals, 16 departures), 150x150x10 km, H=180,
    dt=5 s, S=12, fuel + time + noise objective over a 256x256 lognormal
    population grid, wind 64x64x8 (G=32768) with M=128, L=65536, K=60."""
    args = dict(n_arr=24, n_dep=16, box=(150e3, 150e3, 10e3), grid=(64, 64, 8),
                H=180, dt=5.0, S=12, M=128, L=65536, K=60, precision="fp32",
                alpha_noise=0.1, noise_alt=2000.0, pop_n=(256, 256), seed=seed)
    args.update(kw)
    return make_scenario("C5", **args)


def paper_table(seed: int = 0, **kw) -> dict:
    """The shape of the paper's timing experiment (Sec. "Simulation Setup",
    Table comp_sense): 10 aircraft (8 arrivals, 2 departures released 4
    steps apart), horizon 6 steps of dt = 10 s with the paper's per-step
    (thrust, flight-path angle, bank) controls, a 2 x 2 x 2 wind grid,
    10240 particles, 100 SMC iterations weighted literally over
    SampleSchedule(J) + 1 wind passes (M = SampleSchedule(99) + 1 = 710),
    in a 80 x 80 x 6 km terminal area."""
    K = kw.pop("K", 100)
    M = int(math.floor(3.0 + 5.0 * math.exp(0.05 * (K - 1)))) + 1
    args = dict(n_arr=8, n_dep=2, box=(80e3, 80e3, 6e3), grid=(2, 2, 2), H=6, dt=10.0,
                S=6, M=M, L=10240, K=K, precision="fp32", controls="paper", seed=seed,
                dep_spacing=4)
    args.update(kw)
    s = make_scenario("PAPER", **args)
    s["weighting"] = 1
    return s


def shrink(scen: dict, **kw) -> dict:
    """Copy of ``scen`` with some sizes replaced (L, M, K, H, S, grid ...)."""
    out = dict(scen)
    for k, v in kw.items():
        out[k] = np.array(v, dtype=np.int32) if k == "grid" else v
    return out
