"""Throughput of one SMC-MPC update on one MI355X, with the rollout kernel's
roofline fraction and the CPU oracle timed beside it.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
                [--no-cpu-baseline] [--cpu-particles P] [--no-large]

A step is one MPC update: the whole hot path (particle init, K_smc wind
fields, rollouts with separation, weighting, resampling, moves, final
selection) over one synthetic scenario, inputs resident in device memory.
The default workload is the 10-aircraft plain SMC-MPC step; after its
timed updates the default run also times one update of the 40-aircraft
large form (`large_form` in the record).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "aircraft-step rollouts/sec + ms per MPC step to cost within 1e-3 of oracle"
# the default: the 10-aircraft plain SMC-MPC step (8192 particles, 64 wind
# samples, 40 iterations), which the metric is quoted on
DEFAULT_WORKLOAD = "c2"

# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic work of the rollout: elementary operations of the oracle's
# per-step list (each transcendental, square root or division counted once)
# per simulated aircraft-step, and per separation test between two present
# aircraft; the table is in the design notes.
FLOPS_PER_AIRCRAFT_STEP = 170
FLOPS_PER_PAIR_TEST = 10
# The same list split by what the wind changes: the wind only moves an
# aircraft horizontally, so the speed, climb, bank, drag, thrust, fuel,
# mass, altitude, heading, unary checks and the altitude and speed elements
# (80) are the same in every wind sample of a particle; the horizontal wind
# lookup, horizontal update, geometry and horizontal cost elements (90) are
# per sample.  A pair test is a vertical part (3: difference, abs, compare)
# and a horizontal part (7).
FLOPS_WIND_INDEPENDENT = 80
FLOPS_WIND_DEPENDENT = 90
FLOPS_PAIR_VERTICAL = 3
FLOPS_PAIR_HORIZONTAL = 7
# Adjoint of the fuel + time cost: one primal step plus one reverse step per
# (particle, aircraft, wind sample, step); the recomputation from checkpoints
# is overhead and not counted.
FLOPS_PER_ADJOINT_STEP = 334


WORKLOADS = {
    "c1": ("2 aircraft (1 arrival, 1 departure), 60x60x6 km, H=60 dt=5 s, S=6, wind 16x16x4 "
           "M=16, L=256, K=20, FP64", "c1"),
    "c2": ("10 aircraft (6 arrivals, 4 departures released at steps 0/12/24/36), "
           "100x100x8 km, H=120 dt=5 s, S=8, wind 32x32x8 (G=8192) M=64, L=8192, K=40, "
           "FP32 rollout with FP64 weights and scan, jitter moves", "c2"),
    "c3": ("batched form: 64 scenarios, N ~ U{2..20} (60 % arrivals), H ~ U{60..180}, "
           "S = ceil(H/15), 100x100x8 km, wind 32x32x8 (one shared factor) M=32, L=4096, "
           "K=40, FP32 rollout with FP64 weights and scan, jitter moves; persistent "
           "rollout per aircraft bucket, graph-captured update", "c3"),
    "c4": ("differentiable form: 20 aircraft (12 arrivals, 8 departures), 100x100x8 km, "
           "H=150 dt=4 s, S=10 (600 parameters), wind 32x32x8 M=64, L=16384, K=40, "
           "FP32 rollout and adjoint with FP64 weights, scan and gradient sums, MALA moves "
           "(step 1e-2) driven by the adjoint of the fuel + time cost, checkpoint every "
           "25 steps", "c4"),
    "paper": ("the paper's timing experiment shape: 10 aircraft (8 arrivals, 2 departures "
              "released 4 steps apart), 80x80x6 km, H=6 dt=10 s, per-step (thrust, flight-path "
              "angle, bank) controls, wind 2x2x2 M=709, L=10240, K=100, literal weighting over "
              "SampleSchedule(J)+1 passes at iteration J, FP32 rollout with FP64 weights and scan, "
              "jitter moves", "paper_table"),
    "c5": ("large form: 40 aircraft (24 arrivals, 16 departures, 780 pairs), 150x150x10 km, "
           "H=180 dt=5 s, S=12, fuel + time + noise (256x256 lognormal population below "
           "2 km), wind 64x64x8 (G=32768) M=128, L=65536, K=60, FP32 rollout "
           "(particle tile) with FP64 weights and scan, jitter moves", "c5"),
}


AR1_DESC = ("; the paper's wind model: exponential covariance (beta 1.6e-6, gamma 1.5e-5 1/m, "
            "sigma 5 m/s), time recursion with G_t = 1800 s, one field per step of the "
            "horizon for every sample (H M fields per SMC iteration)")


def _src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1506_02869_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_src: tuple, workload: str, kind: str = "rollout"):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, or
    None when absent, taken on another workload or on a different kernel
    source."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != _src_hash(*kernel_src):
        return None
    return t.get("bytes_per_launch")


# --- the CPU oracle as a baseline ---------------------------------------------
# It runs in a child process started before this process touches the GPU:
# the child forks one worker per host core for the rollouts.

_SHARD = {}


def _rollout_shard(u):
    """One worker's share of an oracle rollout pass (BLAS on one thread)."""
    from threadpoolctl import threadpool_limits

    from oracle import rollout as oro
    with threadpool_limits(limits=1):
        r = oro.rollout(_SHARD["scen"], u, _SHARD["W"])
    return r["cost"], r["feas"], r["steps"]


def host_cpu():
    """Host cores this process may use (the box's share, at most 16 for one
    GPU), nproc, and the CPU model."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return min(avail, 16), os.cpu_count() or 1, model


def cpu_baseline(scen, particles: int, workers: int, iters: int = 2):
    """The oracle, as it stands, on a bounded sample of the same workload:
    `particles` particles, `iters` SMC iterations over all wind samples (or
    the iteration's passes), aircraft and steps, the wind factor and fields
    included; every rollout pass is
    split by particles over `workers` forked processes (one host core each),
    the factor and fields use the BLAS library on the same cores."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import smc as osmc
    from oracle import wind as owind

    s = synth.shrink(scen, L=particles, K=iters)
    note = ""
    if s["move"] == 2:
        # the oracle's Langevin move needs its autograd gradient; the baseline
        # times the oracle's rollout under random-walk moves instead
        s = synth.shrink(s, move=1)
        note = ", random-walk moves in place of MALA"
    steps = 0
    fork = mp.get_context("fork")
    _SHARD["scen"] = s
    t0 = time.perf_counter()
    with threadpool_limits(limits=workers):
        Lfac = owind.factor(s)
    product = osmc.product_weighting(s)

    def evaluate(u, J):
        nonlocal steps
        with threadpool_limits(limits=workers):
            W = owind.sample_field(s, J, s["mpc_step"], Lfac)
        # the literal weighting rolls out the iteration's first passes only
        _SHARD["W"] = W[:osmc.inner_samples(J)] if product else W
        shards = [x for x in np.array_split(u, workers) if len(x)]
        with fork.Pool(len(shards)) as pool:
            parts = pool.map(_rollout_shard, shards)
        steps += sum(p[2] for p in parts)
        cost = np.concatenate([p[0] for p in parts])
        feas = np.concatenate([p[1] for p in parts])
        chat, fe = osmc.expected_cost(cost, feas)
        if product:
            return chat, fe, osmc.product_log_weights(cost, feas)
        return chat, fe

    osmc.run_smc(s, evaluate, s["L"], s["K"], s["N"], s["S"])
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "aircraft-steps/s", "cores": workers, "kind": "oracle",
            "sample": (f"oracle smc loop on {particles} particles x {s['M']} wind samples x "
                       f"{s['N']} aircraft x {s['H']} steps, {iters} SMC iterations "
                       f"({steps} aircraft-steps in {dt:.1f} s; wind factor and fields "
                       f"included; rollouts split by particles over {workers} processes{note})"),
            "seconds": round(dt, 2)}


def cpu_baseline_child(args):
    """--cpu-baseline-only: print the baseline's JSON (no GPU use)."""
    import synth
    key = WORKLOADS[args.workload][1]
    workers, nproc, model = host_cpu()
    iters = 10 if key == "paper_table" else 2
    out = cpu_baseline(getattr(synth, key)(), args.cpu_particles, workers, iters)
    out.update(nproc=nproc, cpu_model=model)
    print(json.dumps(out), flush=True)


def run_cpu_baseline(args):
    """The baseline in a child process (it forks workers, which a process
    holding the GPU should not)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
           "--workload", args.workload, "--cpu-particles", str(args.cpu_particles)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def bench_batch(args, desc):
    """The batched form (C3): one MPC update of all 64 scenarios per step,
    replayed from the captured graph; roofline of the persistent rollout from
    an instrumented (event-timed) update."""
    import numpy as np
    import torch

    import paper_1506_02869_amd as smc
    import synth

    scens = synth.c3(move=args.move) if args.move else synth.c3()
    torch.cuda.set_device(0)
    b = smc.smc_batch_init(scens)
    dev = torch.device("cuda")
    states = torch.as_tensor(np.concatenate([s["states"] for s in scens]), dtype=torch.float64,
                             device=dev)
    kact = torch.as_tensor(np.concatenate([s["k_active"] for s in scens]), dtype=torch.int32,
                           device=dev)
    wm = np.stack([s["wind_mean"] for s in scens])
    hz = np.array([s["H"] for s in scens], dtype=np.int32)
    ctrl = torch.empty(int(b.ctrl_off[-1]), dtype=torch.float64, device=dev)
    cost = torch.empty(int(b.cost_off[-1]), dtype=torch.float64, device=dev)
    status = torch.zeros(b.ns, dtype=torch.int32, device=dev)
    tuning = smc.smc_batch_get_tuning(b)
    if args.autotune:
        tuning = smc.smc_batch_autotune(b, mpc_step=0, reps=2)

    def one(info=False):
        return smc.smc_batch_step_dev(b, 0, states, kact, wm, hz, ctrl, cost, status,
                                      want_info=info)

    _, info0 = one(info=True)          # instrumented, kernel by kernel
    smc.smc_batch_set_graph(b, True)
    for _ in range(max(args.warmup, 1)):   # the first graph update captures
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    aircraft_steps = info0["aircraft_steps"]
    passes = info0["rollout_passes"]
    ms_pass = info0["ms_rollout"] / passes
    flops_pass = (aircraft_steps * FLOPS_PER_AIRCRAFT_STEP
                  + info0["pair_tests"] * FLOPS_PER_PAIR_TEST) / passes
    achieved = flops_pass / (ms_pass * 1e-3) / 1e12
    roof = {"kernel": "k_rollout_wm_batch (all buckets of one pass)", "bound": "alu",
            "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": None,
            "ms_per_pass": round(ms_pass, 4), "launches_per_pass":
                info0["rollout_launches"] // passes,
            "aircraft_steps_per_pass": aircraft_steps // passes,
            "pair_tests_per_pass": info0["pair_tests"] // passes, "flops_per_pass": flops_pass}
    out = {"metric": METRIC, "value": aircraft_steps / (ms_step * 1e-3),
           "unit": "aircraft-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"C3: {desc}" + (f"; {args.move} moves" if args.move else ""),
                      "scenarios": b.ns,
                      "aircraft": [int(n) for n in b.N], "horizons": [int(h) for h in hz],
                      "particles": int(scens[0]["L"]), "wind_samples": int(scens[0]["M"]),
                      "smc_iterations": int(scens[0]["K"]),
                      "aircraft_steps_per_mpc_step": aircraft_steps, "tuning": tuning,
                      "graph": True},
           "roofline": roof, "cpu_baseline": None,
           "step_info": {"ms_total_instrumented": info0["ms_total"],
                         "feasible_frac": info0["feasible_frac"],
                         "accept_rate": info0["accept_rate"]}}
    print(json.dumps(out), flush=True)


def compare_moves(args):
    """Wall time per MPC update for each move (Langevin with the adjoint's
    gradient, random-walk Metropolis, and the paper's jitter) to reach the
    converged expected cost of plain random-walk SMC on the differentiable
    workload (C4).  Every returned control sequence is re-scored by the
    library on one fixed set of wind fields drawn from an iteration word that
    no run uses, so costs are comparable across runs; a run reaches the target
    if its controls are feasible under those fields and score within 1e-3 of
    random-walk SMC at the largest iteration count.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1506_02869_amd as smc
    import synth

    iters = [int(k) for k in args.compare_iters.split(",")]
    j_eval = 1 << 20
    torch.cuda.set_device(0)
    dev = torch.device("cuda")
    runs = {}
    for move in ("rwmh", "mala", "jitter"):
        runs[move] = []
        for K in iters:
            scen = synth.c4(move=move, K=K)
            ctx = smc.smc_mpc_init(scen)
            states = torch.as_tensor(scen["states"], dtype=torch.float64, device=dev)
            kact = torch.as_tensor(scen["k_active"], dtype=torch.int32, device=dev)
            ctrl = torch.empty((scen["N"], scen["S"], 3), dtype=torch.float64, device=dev)
            cost = torch.empty(1 + scen["N"], dtype=torch.float64, device=dev)
            status = torch.zeros(1, dtype=torch.int32, device=dev)

            def one():
                smc.smc_mpc_step_dev(ctx, int(scen["mpc_step"]), states, kact,
                                     scen["wind_mean"], scen["H"], ctrl, cost, status)

            one()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            one()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            _, info = smc.smc_mpc_step_dev(ctx, int(scen["mpc_step"]), states, kact,
                                           scen["wind_mean"], scen["H"], ctrl, cost, status,
                                           want_info=True)
            u = (ctrl.cpu().numpy() - scen["ctrl_lo"]) / (scen["ctrl_hi"] - scen["ctrl_lo"])
            ec, ef = smc.smc_eval_cost(ctx, u[None], j_eval)
            score = float(ec.sum())
            feas = bool(np.all(ef))
            runs[move].append({"K": K, "ms_per_update": round(ms, 1), "score": score,
                               "feasible": feas, "returned_cost": float(cost[0].item()),
                               "accept_rate": round(info["accept_rate"], 6),
                               "feasible_frac": round(info["feasible_frac"], 4)})
            print(f"compare-moves {move} K={K}: {ms:.1f} ms, score {score:.6f} "
                  f"(feasible {feas})", file=sys.stderr, flush=True)
            ctx.close()
    ref = runs["rwmh"][-1]["score"]
    target = ref * (1.0 + 1e-3)

    def reach(move):
        for r in runs[move]:
            if r["feasible"] and r["score"] <= target:
                return r
        return None

    out = {"metric": "wall time per MPC update to reach plain SMC's converged expected cost "
                     "within 1e-3 relative", "workload": WORKLOADS["c4"][0],
           "converged_cost": ref, "converged_from": f"rwmh, K={runs['rwmh'][-1]['K']}",
           "scoring": f"smc_eval_cost on the wind fields of iteration word {j_eval}",
           "runs": runs}
    rr = reach("rwmh")
    for move in ("mala", "jitter"):
        rm = reach(move)
        out[f"{move}_reaches"] = rm
        out[f"{move}_speedup_vs_rwmh"] = (None if rm is None or rr is None
                                          else round(rr["ms_per_update"] / rm["ms_per_update"], 3))
    out["rwmh_reaches"] = rr
    print(json.dumps(out), flush=True)


def compare_moves_batch(args):
    """The same comparison in the batched form (C3: 64 scenarios in one
    batched update): wall time per batched update for each move, the
    acceptance rate of the Metropolis moves, and the summed expected cost
    of the 64 returned control sequences, each re-scored by its own
    scenario's smc_eval_cost on wind fields of an iteration word no run
    draws.  Prints one JSON line."""
    import numpy as np

    import paper_1506_02869_amd as smc
    import synth

    iters = [int(k) for k in args.compare_iters.split(",")]
    j_eval = 1 << 20
    base = synth.c3()
    # one scoring context per scenario (one particle each)
    evals = [smc.smc_mpc_init(synth.shrink(sc, L=8, K=2)) for sc in base]
    runs = {}
    for move in ("rwmh", "mala", "jitter"):
        runs[move] = []
        for K in iters:
            scens = synth.c3(move=move, K=K)
            b = smc.smc_batch_init(scens)
            smc.smc_batch_step(b, 0)                      # warm-up (graph capture off)
            print(f"compare-moves (batched) {move} K={K}: warm-up done", file=sys.stderr,
                  flush=True)
            t0 = time.perf_counter()
            ctrl, cost, status, _, info = smc.smc_batch_step(b, 0)
            ms = (time.perf_counter() - t0) * 1e3
            score, nfeas = 0.0, 0
            for s, sc in enumerate(scens):
                o = int(b.ctrl_off[s])
                c_s = ctrl[o:o + sc["N"] * sc["S"] * 3].reshape(sc["N"], sc["S"], 3)
                u = (c_s - sc["ctrl_lo"]) / (sc["ctrl_hi"] - sc["ctrl_lo"])
                ec, ef = smc.smc_eval_cost(evals[s], u[None], j_eval)
                score += float(ec.sum())
                nfeas += int(np.all(ef))
            runs[move].append({"K": K, "ms_per_update": round(ms, 1), "score": score,
                               "feasible_scenarios": nfeas,
                               "accept_rate": round(float(info.get("accept_rate", 0.0)), 6)})
            print(f"compare-moves (batched) {move} K={K}: {ms:.1f} ms, score {score:.6f} "
                  f"({nfeas} of {len(scens)} scenarios feasible, acceptance "
                  f"{info.get('accept_rate', 0.0):.4f})", file=sys.stderr, flush=True)
            b.close()
    for e in evals:
        e.close()
    ref = runs["rwmh"][-1]["score"]
    ref_feas = runs["rwmh"][-1]["feasible_scenarios"]
    target = ref * (1.0 + 1e-3)

    def reach(move):
        # the summed cost within 1e-3 of the reference with at least as many
        # scenarios feasible on the scoring fields
        for r in runs[move]:
            if r["feasible_scenarios"] >= ref_feas and r["score"] <= target:
                return r
        return None

    out = {"metric": "wall time per batched MPC update to reach plain SMC's converged expected "
                     "cost within 1e-3 relative", "workload": WORKLOADS["c3"][0],
           "converged_cost": ref, "converged_from": f"rwmh, K={runs['rwmh'][-1]['K']}",
           "scoring": f"sum over the 64 scenarios of smc_eval_cost on the wind fields of "
                      f"iteration word {j_eval}",
           "runs": runs}
    rr = reach("rwmh")
    for move in ("mala", "jitter"):
        rm = reach(move)
        out[f"{move}_reaches"] = rm
        out[f"{move}_speedup_vs_rwmh"] = (None if rm is None or rr is None
                                          else round(rr["ms_per_update"] / rm["ms_per_update"], 3))
    out["rwmh_reaches"] = rr
    print(json.dumps(out), flush=True)


def rolling(args):
    """The receding-horizon loop (solve, apply the first control segment to
    the plant, move the window) for --rolling updates of the chosen workload,
    host form: wall time per update including the plant step and the host
    copies.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1506_02869_amd as smc
    import synth

    scen = getattr(synth, WORKLOADS[args.workload][1])()
    torch.cuda.set_device(0)
    ctx = smc.smc_mpc_init(scen)
    smc.rolling_window(ctx, 1)                     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = smc.rolling_window(ctx, args.rolling)
    ms = (time.perf_counter() - t0) * 1e3 / args.rolling
    steps = sum(h["info"]["aircraft_steps"] for h in hist)
    out = {"metric": "wall time per receding-horizon update (MPC update + plant step, host form)",
           "workload": WORKLOADS[args.workload][0], "updates": args.rolling,
           "ms_per_update": round(ms, 2), "aircraft_steps_per_s": steps / (ms * 1e-3 * args.rolling),
           "events": [h["event"].tolist() for h in hist],
           "active": [int((h["k_active"] >= 0).sum()) for h in hist],
           "cost": [float(h["cost"][0]) for h in hist]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-large", action="store_true",
                    help="default workload: skip the one-update measurement of the large form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-particles", type=int, default=None,
                    help="particles of the CPU baseline's sample (default: 32 for c5, "
                         "64 for c4, 2048 for c2 and paper, 256 otherwise)")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="batched workload: autotune the persistent rollout's launch shape first")
    ap.add_argument("--move", choices=["jitter", "rwmh", "mala"], default=None,
                    help="batched workload: move of every scenario (default jitter)")
    ap.add_argument("--compare-moves", action="store_true",
                    help="C4 (or C3 with --workload c3, the batched form): time each move to "
                         "reach plain SMC's converged cost")
    ap.add_argument("--compare-iters", default="5,10,20,40,80,160")
    ap.add_argument("--rolling", type=int, default=0,
                    help="run this many receding-horizon updates (solve + plant) instead")
    ap.add_argument("--wind", choices=["se", "ar1"], default="se",
                    help="wind model: static squared-exponential fields (default) or the "
                         "paper's exponential covariance with its time recursion (c1, c2)")
    ap.add_argument("--weighting", choices=["tempered", "product"], default="tempered",
                    help="SMC weights: tempered mean over all samples (default) or the paper's "
                         "literal product over SampleSchedule(J) + 1 passes")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of the path is described in the design notes)",
              file=sys.stderr)
        sys.exit(2)

    if args.cpu_particles is None:
        args.cpu_particles = {"c5": 32, "c4": 64, "paper": 2048, "c2": 2048}.get(args.workload, 256)
    if args.cpu_baseline_only:
        return cpu_baseline_child(args)
    desc, key = WORKLOADS[args.workload]
    ar1 = args.wind == "ar1"
    # the CPU oracle first, in a child process, before this process uses the GPU
    cpu = None
    single = not (args.compare_moves or args.rolling > 0 or key == "c3")
    if single and not args.no_cpu_baseline and not ar1:
        cpu = run_cpu_baseline(args)
        print(f"bench {args.workload}: cpu baseline {cpu['value']:.4g} aircraft-steps/s on "
              f"{cpu['cores']} cores ({cpu['seconds']} s)", file=sys.stderr, flush=True)

    import numpy as np
    import torch

    import paper_1506_02869_amd as smc
    import synth

    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.compare_moves:
        return compare_moves_batch(args) if key == "c3" else compare_moves(args)
    if args.rolling > 0:
        return rolling(args)
    if ar1 and key not in ("c1", "c2"):
        print("--wind ar1: the time-correlated wind runs in the single-scenario form with up "
              "to 20 aircraft and random-walk or jitter moves (workloads c1, c2)", file=sys.stderr)
        sys.exit(2)
    if args.weighting == "product" and key in ("c3", "c4"):
        print("--weighting product: the literal weighting runs in the single-scenario form with "
              "random-walk or jitter moves (workloads c1, c2, c5)", file=sys.stderr)
        sys.exit(2)
    if key == "c3":
        return bench_batch(args, desc)
    out = bench_single(args, args.workload, args.steps, args.warmup, cpu, not args.no_check)
    if (args.workload == DEFAULT_WORKLOAD and not args.no_large and not ar1
            and args.weighting == "tempered"):
        # the large form, bounded: one instrumented update after the timed
        # ones (its 25-update run does not fit the default run's minutes)
        big = bench_single(args, "c5", 1, 0, None, False)
        out["large_form"] = {k: big[k] for k in ("value", "unit", "ms_per_step", "dtype",
                                                 "config", "roofline", "wind_gemm_roofline",
                                                 "step_info", "status", "smc_ops_roofline")}
    print(json.dumps(out), flush=True)


def smc_ops_bandwidth(smc, torch, ctx, scen, reps=11):
    """HBM rooflines of the SMC steps between rollouts (reduction and
    log-weights, resampling, gather and move, final selection), each timed
    alone at the workload's shape with device events on the stream it runs
    on.  Algorithmic bytes per call:
      k_reduce       M P N (8 + 1) read, P N (8 + 1 + 8) written
      k_resample     P N 8 + 4 N read, 4 N P + 8 N written
      k_gather_move  P D r + 4 N P read, P D r written (D = N S 3 reals of r bytes)
      k_select       16 P N read, 8 written
    (the median of `reps` calls, each between its own events)"""
    import numpy as np
    dev = torch.device("cuda")
    P, N, M, S = scen["L"], scen["N"], scen["M"], scen["S"]
    D = N * S * 3
    rdt = torch.float64 if scen["precision"] == 0 else torch.float32
    r = 8 if scen["precision"] == 0 else 4
    g = torch.Generator(device="cpu").manual_seed(7)
    cost = torch.rand((M, P, N), generator=g, dtype=torch.float64).to(dev)
    feas = (torch.rand((M, P, N), generator=g) < 0.9).to(torch.uint8).to(dev)
    chat = torch.empty((P, N), dtype=torch.float64, device=dev)
    feas_pn = torch.empty((P, N), dtype=torch.uint8, device=dev)
    logw = torch.empty((P, N), dtype=torch.float64, device=dev)
    U = torch.empty(N, dtype=torch.int32, device=dev)
    anc = torch.empty((N, P), dtype=torch.int32, device=dev)
    u_in = torch.rand((P, N, S, 3), generator=g, dtype=torch.float64).to(rdt).to(dev)
    u_out = torch.empty_like(u_in)
    best = torch.empty(2, dtype=torch.int32, device=dev)
    ops = {
        "k_reduce": (lambda: smc.smc_k_reduce(ctx, P, cost, feas, 1.0, chat, feas_pn, logw),
                     M * P * N * 9, P * N * 17),
        "k_resample": (lambda: smc.smc_k_resample(ctx, P, logw, U, anc),
                       P * N * 8 + 4 * N, 4 * N * P + 8 * N),
        "k_gather_move": (lambda: smc.smc_k_gather_move(ctx, P, u_in, anc, u_out, 0, 1, 1),
                          P * D * r + 4 * N * P, P * D * r),
        "k_select": (lambda: smc.smc_k_select(ctx, P, logw, chat, 1.0, best), 16 * P * N, 8),
    }
    ops["k_reduce"][0]()
    smc.smc_k_resample_offsets(ctx, 0, 1, U)
    out = {}
    for name, (fn, rd, wr) in ops.items():
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for e0, e1 in ev:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
        gbs = (rd + wr) / (ms * 1e-3) / 1e9
        out[name] = {"bound": "hbm", "ms_per_launch": round(ms, 4), "bytes": rd + wr,
                     "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs / PEAK_HBM_GBS, 4)}
    return out


def bench_single(args, workload, steps, warmup, cpu=None, check_cost=True):
    """One workload in the single-scenario form: `warmup` untimed MPC
    updates, then `steps` timed ones (each instrumented); returns the JSON
    record.  The context is released before returning."""
    import numpy as np
    import torch

    import paper_1506_02869_amd as smc
    import synth

    desc, key = WORKLOADS[workload]
    ar1 = args.wind == "ar1"
    if ar1:
        desc += (AR1_DESC)
    scen = getattr(synth, key)(**({"wind_model": "ar1"} if ar1 else {}))
    product = args.weighting == "product"
    if product and scen.get("weighting", 0) != 1:
        scen["weighting"] = 1
        desc += ("; the paper's literal weighting: SampleSchedule(J) + 1 passes at iteration J "
                 "(one wind sample each), log W = sum log(1 - cost)")
    product = scen.get("weighting", 0) == 1
    torch.cuda.set_device(0)
    ctx = smc.smc_mpc_init(scen)
    dev = torch.device("cuda")
    states = torch.as_tensor(scen["states"], dtype=torch.float64, device=dev)
    kact = torch.as_tensor(scen["k_active"], dtype=torch.int32, device=dev)
    ctrl = torch.empty((scen["N"], scen["S"], 3), dtype=torch.float64, device=dev)
    cost = torch.empty(1 + scen["N"], dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    wm = scen["wind_mean"]
    step_id = int(scen["mpc_step"])

    def one(info=False):
        return smc.smc_mpc_step_dev(ctx, step_id, states, kact, wm, scen["H"], ctrl, cost,
                                    status, want_info=info)

    def note(msg):
        print(f"bench {workload}: {msg}", file=sys.stderr, flush=True)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    # every timed update is instrumented: per-kernel durations from device
    # events on the stream the kernels run on, and the work counts
    nsteps = max(steps, 1)
    infos = []
    t0 = time.perf_counter()
    for _ in range(nsteps):
        infos.append(one(info=True)[1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / nsteps
    note(f"{nsteps} timed updates, {ms_step:.1f} ms each")
    info0 = infos[0]
    aircraft_steps = info0["aircraft_steps"]
    value = aircraft_steps / (ms_step * 1e-3)

    n_roll = sum(i["rollout_launches"] for i in infos)
    ms_roll = sum(i["ms_rollout"] for i in infos) / n_roll
    n_wind = sum(i["wind_launches"] for i in infos)
    ms_wind = sum(i["ms_wind"] for i in infos) / n_wind
    as_per_launch = aircraft_steps / info0["rollout_launches"]
    pt_per_launch = info0["pair_tests"] / info0["rollout_launches"]
    ph_per_launch = info0["pair_tests_h"] / info0["rollout_launches"]
    N = scen["N"]
    fp64 = scen["precision"] == 0
    # the rollout layout the library picks (world-per-lane up to 20 aircraft,
    # the particle tile above in FP32, aircraft-per-lane otherwise)
    layout = 2 if N <= 20 else (4 if not fp64 else 1)
    # algorithmic work: the per-step operation list for every simulated
    # aircraft-step and every pair of present aircraft, whatever the layout
    # shares between the worlds of a particle
    flops_launch = (as_per_launch * FLOPS_PER_AIRCRAFT_STEP
                    + pt_per_launch * FLOPS_PER_PAIR_TEST)
    split = None
    if layout in (3, 4):
        # what these layouts compute: the wind-independent part of a step once
        # per particle, the wind-dependent part per world; vertical pair tests
        # once per particle, horizontal ones per world for pairs within sep_v
        split = (as_per_launch * FLOPS_WIND_DEPENDENT
                 + as_per_launch / scen["M"] * FLOPS_WIND_INDEPENDENT
                 + pt_per_launch / scen["M"] * FLOPS_PAIR_VERTICAL
                 + ph_per_launch * FLOPS_PAIR_HORIZONTAL)
    achieved = flops_launch / (ms_roll * 1e-3) / 1e12
    peak = PEAK_FP64_VECTOR_TFLOPS if fp64 else PEAK_FP32_VECTOR_TFLOPS
    world_lane = layout == 2
    kname, ksrc = {
        2: ("k_rollout_wm", ("kernels_rollout_wm.hip", "rollout_wm_body.inc", "rollout_math.h")),
        3: ("k_rollout_pw", ("kernels_rollout_pw.hip", "rollout_pw_common.h", "rollout_math.h")),
        4: ("k_rollout_pt", ("kernels_rollout_pt.hip", "rollout_pw_common.h", "rollout_math.h")),
        1: ("k_rollout", ("kernels_rollout.hip", "rollout_math.h"))}[layout]
    if ar1:
        kname = "k_rollout_wm_tv"
    roof = {"kernel": kname, "bound": "alu", "achieved": round(achieved, 3),
            "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": traffic_for(ksrc, workload) if not ar1 else None,
            "ms_per_launch": round(ms_roll, 4),
            "aircraft_steps_per_launch": int(as_per_launch),
            "pair_tests_per_launch": int(pt_per_launch),
            "horizontal_pair_tests_per_launch": int(ph_per_launch),
            "flops_per_launch": flops_launch}
    if split is not None:
        # the operations the layout executes (shared per particle), per second
        roof["executed_split_tflops"] = round(split / (ms_roll * 1e-3) / 1e12, 3)
    G = int(np.prod(scen["grid"]))
    nh, nz = int(scen["grid"][0]) * int(scen["grid"][1]), int(scen["grid"][2])
    # the horizontal factor's triangular GEMM (nx ny rows) over the
    # level-mixed columns: 2 H M nz of them under the time-correlated wind;
    # 2 M nz for the static wind, whose level pass (nz (nz + 1) flops per
    # node and column) runs inside the same timed region
    if ar1:
        gemm_flops = float(nh) * (nh + 1) * 2 * scen["M"] * scen["H"] * nz
        wkern = "k_wind_gemm"
    elif nz <= 16:
        gemm_flops = (float(nh) * (nh + 1) * 2 * scen["M"] * nz
                      + float(nh) * 2 * scen["M"] * nz * (nz + 1))
        wkern = "k_wind_levels + k_wind_gemm"
    else:
        gemm_flops = float(G) * (G + 1) * 2 * scen["M"]
        wkern = "k_wind_gemm"
    gemm_ach = gemm_flops / (ms_wind * 1e-3) / 1e12
    gpeak = PEAK_FP64_MFMA_TFLOPS if fp64 else PEAK_FP32_MFMA_TFLOPS
    wind_roof = {"kernel": wkern, "bound": "mfma", "achieved": round(gemm_ach, 3),
                 "peak": gpeak, "unit": "TFLOP/s", "frac": round(gemm_ach / gpeak, 4),
                 "ms_per_launch": round(ms_wind, 4)}
    grad_roof = None
    n_grad = sum(i["grad_launches"] for i in infos)
    if n_grad:
        # the adjoint runs on the particles of each rollout pass, so its
        # (particle, aircraft, sample) steps equal that pass's aircraft-steps
        ms_grad = sum(i["ms_grad"] for i in infos) / n_grad
        ls_launch = aircraft_steps / info0["grad_launches"]
        gflops = ls_launch * FLOPS_PER_ADJOINT_STEP
        gach = gflops / (ms_grad * 1e-3) / 1e12
        # the sample-independent chain hoisted per (particle, aircraft) for
        # 17 ... 128 samples and horizons up to 160 steps
        gk = ("k_rollout_grad_split" if 16 < scen["M"] <= 128 and scen["H"] <= 160
              else "k_rollout_grad")
        grad_roof = {"kernel": gk, "bound": "alu", "achieved": round(gach, 3),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(gach / peak, 4),
                     "traffic": traffic_for(("kernels_grad.hip", "rollout_math.h"), workload,
                                            "adjoint"),
                     "ms_per_launch": round(ms_grad, 4), "lane_steps_per_launch": int(ls_launch),
                     "flops_per_launch": gflops,
                     "ms_per_mpc_step_in_adjoint": round(ms_grad * info0["grad_launches"], 2)}

    check = None
    if check_cost and not ar1:
        # re-score the returned controls with the FP64 oracle on the last
        # iteration's wind fields
        from oracle import smc as osmc
        c_ctrl = ctrl.cpu().numpy()
        c_cost = cost.cpu().numpy()
        u = (c_ctrl - scen["ctrl_lo"]) / (scen["ctrl_hi"] - scen["ctrl_lo"])
        # the returned cost averages the passes of the last iteration
        sc = dict(scen, M=osmc.inner_samples(scen["K"] - 1)) if product else scen
        rc, rf = osmc.eval_cost(sc, u[None], scen["K"] - 1)
        rel = abs(float(rc.sum()) - float(c_cost[0])) / max(abs(float(rc.sum())), 1e-3)
        check = {"gpu_cost": float(c_cost[0]), "oracle_rescored_cost": float(rc.sum()),
                 "rel_err": rel, "within_1e-3": bool(rel <= 1e-3),
                 "oracle_feasible": bool(rf.all()), "status": int(status.cpu()[0])}


    out = {"metric": METRIC, "value": value, "unit": "aircraft-steps/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if fp64 else "f32", "data": "synthetic",
           "config": {"workload": f"{workload.upper()}: {desc}", "aircraft": N,
                      "particles": scen["L"], "wind_samples": scen["M"],
                      "smc_iterations": scen["K"], "horizon": scen["H"],
                      "segments": scen["S"], "grid": [int(g) for g in scen["grid"]],
                      "aircraft_steps_per_mpc_step": aircraft_steps},
           "roofline": roof, "cpu_baseline": cpu, "wind_gemm_roofline": wind_roof,
           "adjoint_roofline": grad_roof, "cost_check": check,
           "step_info": {k: info0[k] for k in ("feasible_frac", "ess_min", "best_particle",
                                              "ms_total", "accept_rate")},
           "status": int(status.cpu()[0])}
    if key == "paper_table":
        # the paper's own timing (Table comp_sense, best thread layout), on
        # its hardware and traffic: context, not a target
        out["paper_context"] = {
            "seconds_per_update": 56.0, "hardware": "NVIDIA GeForce GTX 580, mostly FP64",
            "workload": "10 aircraft, H=6, dt=10 s, L=10240, 100 iterations of "
                        "SampleSchedule(J) passes, 8-point wind grid (Gatwick traffic)"}
    out["smc_ops_roofline"] = smc_ops_bandwidth(smc, torch, ctx, scen)
    ctx.close()
    return out


if __name__ == "__main__":
    main()
