"""Throughput of the coupled LBRMT step on one MI355X.

Workload (default): the 2048 x 2048 lid-driven cavity with one neo-Hookean disc
(tau 0.6, lid 0.05, disc R = 0.15 L at (0.5 L, 0.6 L), G 0.005, density ratio 1),
FP64, synthetic initial state (fluid at rest), every input resident in HBM.
A step is one full pass of Alg. 1: advection, 11 extrapolation layers,
relabel, stress divergence, SFC + Guo collision with streaming and walls.

Prints ONE JSON line: whole-job MLUPS (interior nodes x steps / s), the roofline
of the dominant kernel (the lattice Boltzmann update of the tiles outside the
solid band, timed with HIP events on its own stream), and the CPU oracle timed
on a bounded sample of the same workload (all OpenMP threads, and one).
The extrapolation launch mode (all layers in one launch, or one launch per
layer) is the library's default for the grid; --autotune chooses it during
the untimed warm-up by timing whole steps (lbrmt_autotune_steps).  The mode
is reported in extra.extrapolation_launch.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
_T0 = time.perf_counter()


def progress(msg):
    """One progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)
METRIC = "coupled LBRMT step MLUPS & % HBM roofline; FP32/batched/adjoint vs FP64 plain"


def _workload(name):
    import workloads
    return getattr(workloads, name)()


def lb_bytes_per_node(precision):
    s = 8 if precision == "f64" else 4
    return 18 * s  # nine populations read, nine written (pull scheme, two lattices)


def traffic_from_profile(kernel, workload, precision):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, or None
    when none exists or the lattice-update sources (k_lb.hip, lb_node.h)
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    csrc = os.path.join(ROOT, "paper_2402_12696_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, n), "rb").read() for n in ("k_lb.hip", "lb_node.h"))
    digest = hashlib.sha256(src).hexdigest()[:16]
    m = re.search(r"source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != digest:
        return None
    return float(t.group(1))


def run_gpu(cfg, precision, steps, warmup, timing_steps, overlap=None, lb_variant=None,
            autotune=False):
    import torch
    from paper_2402_12696_amd import Sim
    from paper_2402_12696_amd.lbrmt import LBRMT_OPT_LB_VARIANT, LBRMT_OPT_OVERLAP
    progress(f"{cfg['name']} {precision}: init")
    sim = Sim(device="cuda:0", precision=precision, **cfg).init()
    if overlap is not None:
        sim.set_option(LBRMT_OPT_OVERLAP, overlap)
    if lb_variant is not None:
        sim.set_option(LBRMT_OPT_LB_VARIANT, lb_variant)
    sim.step(warmup)
    torch.cuda.synchronize()
    progress(f"{precision}: {warmup} warm-up steps done; choosing the extrapolation launch")
    # extrapolation launch mode (one launch for all layers, or one per layer):
    # the library's default (-1: one launch when the bulk update is uncapped,
    # as here), or with autotune chosen by timing whole steps, untimed; the
    # steps it takes are extra warm-up
    if autotune:
        fused, _ = sim.autotune_steps(60)
    else:
        from paper_2402_12696_amd.lbrmt import LBRMT_OPT_FUSED_FIT
        fused = sim.get_option(LBRMT_OPT_FUSED_FIT)
    torch.cuda.synchronize()
    progress(f"{precision}: chose fused_fit={fused}; priming graphs for {steps} steps")
    prime_graphs(sim, steps)
    torch.cuda.synchronize()
    progress(f"{precision}: timing {steps} steps")
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    progress(f"{precision}: {ms_per_step:.4f} ms/step; per-kernel event timing")
    diag = sim.diag(raise_unstable=False)
    band_nodes, window_nodes = sim.band_nodes()
    # per-kernel durations: eager launches bracketed by HIP events on the
    # stream each kernel runs on
    sim.set_timing(True)
    sim.step(timing_steps)
    torch.cuda.synchronize()
    ktimes = {k: sim.kernel_time(k) for k in
              ("advect", "extrap", "relabel", "force", "lb_bulk", "lb_band")}
    sim.set_timing(False)
    # the full-grid lattice update alone (one stream), for reference
    from paper_2402_12696_amd.lbrmt import LBRMT_OPT_OVERLAP as _OV
    keep = sim.get_option(_OV)
    sim.set_option(_OV, 0)
    sim.set_timing(True)
    sim.step(timing_steps // 2)
    torch.cuda.synchronize()
    ktimes["lb_full_alone"] = sim.kernel_time("lb_bulk")
    sim.set_timing(False)
    sim.set_option(_OV, keep)
    sim.close()
    ktimes["fused_fit"] = fused
    return ms_per_step, ktimes, band_nodes, window_nodes, diag


def prime_graphs(sim, steps):
    """Untimed: capture every step graph that a run of `steps` steps from a
    six-step boundary replays, and end on such a boundary.  The library
    replays a captured six-step graph for each whole block of six steps and
    a captured shorter graph for the rest (steps 0 .. r-1 of the period),
    each captured on first use; after this the timed steps only replay
    graphs whatever `steps` is.  At most 17 steps: the 2048^2 workload
    becomes unstable after ~4250 steps, so the timed steps must stay early."""
    sim.step((-sim.step_count) % 6)
    sim.step(6 + steps % 6)
    sim.step((-sim.step_count) % 6)


def step_bytes(precision, nodes, n_band):
    """Algorithmic HBM bytes of one coupled step: 18 s_f per node (nine
    populations read and nine written, pull scheme) plus (9 s_f + 25 s) per
    band node (the band moments, the advection, the extrapolation and
    relabel, the force, the collision's force and level-set reads), s_f the
    population size and s the size of a reference-map, level-set or force
    value (8 in FP64, 4 in FP32)."""
    s = 8 if precision == "f64" else 4
    return 18 * s * nodes + (9 * s + 25 * s) * n_band


def step_traffic_from_profile(workload, precision):
    """HBM bytes per step (FETCH_SIZE + WRITE_SIZE of every kernel of a
    step, scaled by the copy-kernel factors) from a committed rocprofv3
    summary, or None when none exists or a kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"lbrmt_step_{workload}_{precision}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"sources_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_step:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != sources_digest():
        return None
    return float(t.group(1))


def sources_digest():
    """Hash of every HIP source of the library (16 hex digits)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2402_12696_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def copy_ceiling(nbytes, reps=20):
    """HBM rate of a plain streaming copy on this GPU: FP32 negation of nbytes
    into a second buffer and back (ping-pong, as the lattice update reads one
    lattice and writes the other), timed with events on torch's stream."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.neg(b, out=a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        if r % 2:
            torch.neg(b, out=a)
        else:
            torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def run_ensemble(precision, steps, seq_steps=120, seq_warmup=12):
    """The seeded 96-member cavity ensemble: one batch (autotuned tile shape)
    for `steps` steps, against each member stepped alone (same precision and
    FP64) for seq_steps steps after seq_warmup; sequential times are per-step
    averages scaled to `steps`."""
    import torch
    import workloads
    from paper_2402_12696_amd import Batch, Sim
    cfgs = workloads.cavity_ensemble()
    nodes = sum(c["nx"] * c["ny"] for c in cfgs)
    out = {"workload": "cavity_ensemble_96 (seed 4)", "members": len(cfgs), "nodes": nodes,
           "steps": steps, "precision": precision}
    batch = Batch(cfgs, precision=precision).init()
    batch.step(12)
    out["autotuned_variant"], _ = batch.autotune(reps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps - 12)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / (steps - 12)
    out["ms_per_step"] = ms
    out["mlups"] = nodes / (ms * 1e-3) / 1e6
    bad = [k for k in range(len(cfgs))
           if any(v for v in batch.member(k).diag(raise_unstable=False)["health"].values())]
    out["members_with_health_flags"] = bad
    batch.close()
    for prec in (precision, "f64") if precision != "f64" else ("f64",):
        tot = 0.0
        for c in cfgs:
            sim = Sim(device="cuda:0", precision=prec, **c).init()
            sim.step(seq_warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(seq_steps)
            torch.cuda.synchronize()
            tot += (time.perf_counter() - t0) * 1e3 / seq_steps
            sim.close()
        out[f"sequential_{prec}_ms_per_step"] = tot
        out[f"speedup_vs_sequential_{prec}"] = tot / ms
    return out


def run_suspension(precision, steps, warmup=24):
    """The seeded 4096^2 periodic suspension of 400 soft discs and ellipses
    (several-solid path with contact): whole-step time after `warmup` steps."""
    import torch
    import workloads
    from paper_2402_12696_amd import Sim
    cfg = workloads.suspension()
    sim = Sim(device="cuda:0", precision=precision, **cfg).init()
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    nodes = cfg["nx"] * cfg["ny"]
    d = sim.diag(raise_unstable=False)
    sim.close()
    return {"workload": cfg["name"] + " (seed 240212696)", "solids": len(cfg["solids"]),
            "precision": precision, "steps": steps, "ms_per_step": ms,
            "mlups": nodes / (ms * 1e-3) / 1e6,
            "health_flags": {k: v for k, v in d["health"].items() if v}}


def run_adjoint(T=600):
    """The 256^2 inverse-problem scene (disc R 40 at (128, 153.6), tau 0.7, lid
    0.08, G 0.01, u_0 ~ N(0, 1e-3^2) from default_rng(5)); the loss follows
    the centroid and mean displacement of a G* = 0.008 run.  Forward with
    sqrt(T) checkpoints, then the adjoint (replays and reverse steps); T = 600:
    this scene blows up after ~700 steps with that noise (explicit stress
    update at tau 0.7)."""
    import numpy as np
    import torch
    import workloads
    from paper_2402_12696_amd import adjoint as AD
    cfg = workloads.make(nx=256, ny=256, tau=0.7, lid_ux=0.08,
                         solid=dict(cx=128.0, cy=153.6, R=40.0, G=0.01, rho_s=1.0))
    tgt = AD.trajectory(cfg, 0.008, 0.08, T)
    u0 = np.random.default_rng(5).normal(0.0, 1e-3, size=(2, 256, 256))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = AD.Trajectory(cfg, 0.01, 0.08, u0, T, tgt)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    gG, gU, gu0 = tr.backward()
    tb = time.perf_counter() - t0
    out = {"workload": "cavity_disc_256 inverse problem", "steps": T, "checkpoints": tr.K,
           "loss": tr.loss, "forward_s": tf, "adjoint_s": tb, "adjoint_over_forward": tb / tf,
           "dL_dG": gG, "dL_dU": gU, "max_abs_dL_du0": float(gu0.abs().max()),
           "health_flags": tr.health}
    tr.close()
    return out


def cpu_baseline(cfg, seconds=15.0):
    from oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = Oracle(**cfg).init()
    o.step(1)
    n, t = 0, 0.0
    while t < seconds and n < 50:
        t0 = time.perf_counter()
        o.step(1)
        t += time.perf_counter() - t0
        n += 1
    mlups = cfg["nx"] * cfg["ny"] * n / t / 1e6
    return {"value": mlups, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of {cfg['name']} after 1 warm-up step "
                      f"({t:.1f} s, OpenMP threads {threads})",
            "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count(),
            "single_thread": _oracle_one_thread(cfg),
            "parity_vs_gpu": parity_vs_oracle(cfg)}


def parity_vs_oracle(cfg, precision="f64", steps=20, amp=0.01, cells=4, seed=7):
    """The GPU step against the CPU oracle at full size on a deforming
    solid: the workload's grid, disc and parameters with a seeded cellular
    flow (amplitude amp) that shears and carries the disc from the first
    step; errors after `steps` steps of both: rho, each velocity component
    against its own maximum, xi, and the deviations rho - rho_f and xi - x
    (over the nodes with phi < eps); node and solid sets must agree."""
    import numpy as np
    import workloads
    from oracle import Oracle
    from paper_2402_12696_amd import Sim
    c = dict(cfg)
    c.pop("steps", None)
    c.pop("name", None)
    u0 = workloads.cellular_velocity(c["nx"], c["ny"], amp, cells, seed)
    ref = Oracle(**c).init(u0)
    ref.step(steps)
    sim = Sim(device="cuda:0", precision=precision, **c).init(u0)
    sim.step(steps)
    rho, ux, uy = (t.cpu().numpy() for t in sim.macro())
    X, Y, P = (t.cpu().numpy() for t in sim.refmap())
    sim.close()
    rr, ru, rv = ref.macro()
    RX, RY, RP = ref.refmap()

    def rel(a, b):
        m = np.max(np.abs(b))
        return float(np.max(np.abs(a - b)) / m) if m > 0 else float(np.max(np.abs(a)))

    mg, mr = ~np.isnan(X), ~np.isnan(RX)
    same = bool(np.array_equal(mg, mr) and np.array_equal(P[mg] < 0, RP[mr] < 0))
    y, x = np.mgrid[0:c["ny"], 0:c["nx"]] + 0.5
    ms = mr & (RP < c.get("eps", 1.5))
    rf = c.get("rho_f", 1.0)
    return {"workload": f"{cfg['name']} with a cellular flow (amp {amp}, {cells} cells, seed {seed})",
            "precision": precision, "steps": steps, "node_sets_equal": same,
            "rho": rel(rho, rr), "ux": rel(ux, ru), "uy": rel(uy, rv),
            "xi": max(rel(X[mr], RX[mr]), rel(Y[mr], RY[mr])),
            "rho_minus_rho_f": rel(rho - rf, rr - rf),
            "xi_minus_x": max(rel(X[ms] - x[ms], RX[ms] - x[ms]),
                              rel(Y[ms] - y[ms], RY[ms] - y[ms])),
            "max_xi_minus_x": float(max(np.max(np.abs(RX[ms] - x[ms])),
                                        np.max(np.abs(RY[ms] - y[ms]))))}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ONE_THREAD = """
import json, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import Oracle
cfg = json.loads(sys.argv[2])
o = Oracle(**cfg).init()
o.step(1)
n, t = 0, 0.0
while t < float(sys.argv[3]) and n < 20:
    t0 = time.perf_counter()
    o.step(1)
    t += time.perf_counter() - t0
    n += 1
print(json.dumps({"steps": n, "seconds": t}))
"""


def _oracle_one_thread(cfg, seconds=8.0):
    """The same oracle on one OpenMP thread, in a child process (the thread
    count of this process's OpenMP runtime is already fixed)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_THREAD, ROOT, json.dumps(cfg), str(seconds)],
                       env=env, capture_output=True, text=True, timeout=300, check=True)
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": cfg["nx"] * cfg["ny"] * d["steps"] / d["seconds"] / 1e6, "unit": "MLUPS",
            "cores": 1, "sample": f"{d['steps']} steps of {cfg['name']} after 1 warm-up step "
                                  f"({d['seconds']:.1f} s, OpenMP threads 1)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=120)
    ap.add_argument("--autotune", action="store_true",
                    help="choose the extrapolation launch mode by timing whole steps "
                         "(default: the library's choice for the grid)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="the default; kept for older command lines")
    ap.add_argument("--workload", default="cavity_disc_2048")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--timing-steps", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--overlap", type=int, default=None, choices=[0, 1],
                    help="1: reference-map chain on a side stream (library default 1)")
    ap.add_argument("--lb-variant", type=int, default=None,
                    help="lattice tile variant (library default 3 for f64, 5 for f32)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 96-member ensemble (batched vs sequential)")
    ap.add_argument("--batch-steps", type=int, default=600,
                    help="steps of the ensemble (its stiffest members blow up after ~700)")
    ap.add_argument("--no-suspension", action="store_true",
                    help="skip the 4096^2 suspension of 400 solids (several-solid path)")
    ap.add_argument("--suspension-steps", type=int, default=400)
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint of the 256^2 inverse-problem scene")
    ap.add_argument("--suspension-only", action="store_true",
                    help="run only the suspension (in --precision) and print its record "
                         "(for profiling; not the benchmark line)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one plain elementwise copy (FP32 negation) reading and "
                         "writing this many bytes: the reference dispatch that scales HBM "
                         "counters (FETCH_SIZE, WRITE_SIZE) of a profiled run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the "
              "multi-GPU slab decomposition is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.suspension_only:
        print(json.dumps(run_suspension(args.precision, args.suspension_steps)), flush=True)
        return

    if args.copy_bytes > 0:
        import torch
        a = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    cfg = _workload(args.workload)
    nodes = cfg["nx"] * cfg["ny"]
    ms, kt, band, window, diag = run_gpu(cfg, args.precision, args.steps, args.warmup,
                                         args.timing_steps, args.overlap, args.lb_variant,
                                         args.autotune and not args.no_autotune)
    mlups = nodes / (ms * 1e-3) / 1e6

    bulk_ms, bulk_n = kt["lb_bulk"]
    # with overlap (the library default) the bulk launch updates every node
    # outside the window (the force pass updates the window's nodes, which
    # lbrmt_band_nodes reports then); without it, every node
    bulk_nodes = nodes - band if (kt["lb_band"][1] > 0 or args.overlap != 0) else nodes
    bpn = lb_bytes_per_node(args.precision)
    alg_bytes = bpn * bulk_nodes
    achieved = alg_bytes / (bulk_ms * 1e-3) / 1e9 if bulk_ms > 0 else None
    traffic = traffic_from_profile("lb_bulk", args.workload, args.precision)
    ceiling = copy_ceiling(bpn // 2 * nodes)  # one lattice, as the update reads one and writes one
    alone_ms = kt["lb_full_alone"][0]
    alone = bpn * nodes / (alone_ms * 1e-3) / 1e9 if alone_ms > 0 else None
    roof = {"kernel": "lb_bulk", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic, "bytes_per_launch": alg_bytes, "nodes_per_launch": bulk_nodes,
            "avg_launch_ms": bulk_ms, "launches": bulk_n,
            "copy_ceiling_GBs": ceiling,
            "frac_of_copy_ceiling": achieved / ceiling if achieved else None,
            "full_grid_update_alone": {"avg_launch_ms": alone_ms, "achieved": alone,
                                       "frac": alone / HBM_PEAK_GBS if alone else None,
                                       "frac_of_copy_ceiling": alone / ceiling if alone else None}}

    n_band = int(diag["n_band"])
    b_step = step_bytes(args.precision, nodes, n_band)
    a_step = b_step / (ms * 1e-3) / 1e9
    roof["step"] = {"what": "whole coupled step: algorithmic bytes per step / ms_per_step",
                    "bytes_per_step": b_step, "n_band": n_band, "achieved": a_step,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a_step / HBM_PEAK_GBS,
                    "frac_of_copy_ceiling": a_step / ceiling,
                    "traffic_per_step": step_traffic_from_profile(args.workload, args.precision)}
    fused = kt.pop("fused_fit")
    extra = {"kernel_avg_ms": {k: v[0] for k, v in kt.items()},
             "extrapolation_launch": "one launch, all layers" if fused else "one launch per layer",
             "band_region_nodes": band, "window_nodes": window,
             "n_solid": diag["n_solid"], "n_band": diag["n_band"],
             "health": diag["health"]}
    if args.precision == "f64" and not args.no_f32:
        ms32, kt32, _, _, d32 = run_gpu(cfg, "f32", args.steps, args.warmup, args.timing_steps,
                                        args.overlap, args.lb_variant,
                                        args.autotune and not args.no_autotune)
        b32 = step_bytes("f32", nodes, int(d32["n_band"]))
        extra["f32"] = {"ms_per_step": ms32, "mlups": nodes / (ms32 * 1e-3) / 1e6,
                        "speedup_vs_f64": ms / ms32,
                        "step_roofline": {"bytes_per_step": b32,
                                          "achieved": b32 / (ms32 * 1e-3) / 1e9,
                                          "frac": b32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                          "frac_of_copy_ceiling":
                                              b32 / (ms32 * 1e-3) / 1e9 / ceiling,
                                          "traffic_per_step": step_traffic_from_profile(
                                              args.workload, "f32")},
                        "lb_bulk_avg_ms": kt32["lb_bulk"][0],
                        "extrapolation_launch": "one launch, all layers" if kt32["fused_fit"]
                        else "one launch per layer"}
    if not args.no_batch:
        progress("ensemble")
        extra["batched"] = run_ensemble("f32", args.batch_steps)
    if not args.no_suspension:
        progress("suspension")
        extra["suspension"] = {p: run_suspension(p, args.suspension_steps)
                               for p in ("f32", "f64")}
    if not args.no_adjoint:
        progress("adjoint")
        extra["adjoint"] = run_adjoint()
    line = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": cfg["name"], "nx": cfg["nx"], "ny": cfg["ny"], "tau": cfg["tau"],
                   "lid_ux": cfg["lid_ux"], "solid": cfg["solid"], "layers": cfg["layers"],
                   "eps": cfg["eps"]},
        "roofline": roof,
        "cpu_baseline": None if args.no_cpu_baseline else (progress("cpu oracle"),
                                                           cpu_baseline(cfg))[1],
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
