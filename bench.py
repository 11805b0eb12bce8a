"""Benchmark: linear solves per second at 4.49M DOF on one MI355X.

One step = one linear solve of an inexact-Newton iteration on the 60x220x85
channelised dual-porosity model: residual/Jacobian assembly, CPR-FPF setup
(decoupling, block ILU(0), pressure AMG) and GMRES(30) to a relative residual
of 1e-6, re-assembled and set up from scratch in every step.  The Jacobians
are those of the model's run: its first 20 ten-day steps are taken first
(untimed), and the timed solves are spread over the Jacobians at their
converged states (--workload first times the third Newton iterate of the
first step instead).  The headline value uses the FP32 preconditioner under
the FP64 Krylov loop; the plain FP64 form is measured in the same run.

Prints one JSON line.  --gpus N with N > 1 exits: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch from two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE),
# each scaled by what the counter reads for a plain copy of known size, with the
# source file of the kernel and its SHA-256 prefix at the time of measurement;
# the figures were taken on the 60x220x85 model in the FP32-preconditioner form
# and are reported only for it, and only while that source is unchanged.  A
# group whose bytes per launch vary with its arguments (the basis passes grow
# with the iteration index) has its measured ratio of traffic to algorithmic
# bytes instead, applied to the timed launches' algorithmic bytes.
TRAFFIC = {
    "amg_rowwise_products": dict(bytes=378.2e6, source="paper_1808_04338_amd/csrc/segsort.hip",
                                 sha256="05515b972e4df1b2"),
    "block_ilu0_solve": dict(bytes=318.3e6, source="paper_1808_04338_amd/csrc/linalg.hip",
                             sha256="be6d0719d26b6576"),
    "amg_vcycle": dict(bytes=560.1e6, source="paper_1808_04338_amd/csrc/amg.hip",
                       sha256="8a1f304235d7fd5a"),
    "gmres_basis_passes": dict(ratio=1.035, source="paper_1808_04338_amd/csrc/krylov.hip",
                               sha256="32ec252621936214"),
}


def traffic_for(name, bytes_per_launch):
    import hashlib

    t = TRAFFIC.get(name)
    if t is None:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha256"]:
            return None
    return t["bytes"] if "bytes" in t else t["ratio"] * bytes_per_launch


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_model(nz):
    import synth

    return synth.model_channelised(nz=nz, steps=20)


def slab(model, nz):
    """The top nz layers of a model (fields cut, wells cut to the slab)."""
    import copy

    m = copy.deepcopy(model)
    n = m["nx"] * m["ny"] * nz
    for k in ("kx", "ky", "kz", "km", "phi_f", "phi_m"):
        m[k] = m[k][:n].copy()
    m["p0"] = m["p0"][:2 * n].copy()
    m["sw0"] = m["sw0"][:2 * n].copy()
    m["nz"] = nz
    for w in m["wells"]:
        w["k1"] = min(w["k1"], nz - 1)
    return m


def prepare(sim, model, newton_its):
    """Start the first timestep and take newton_its Newton iterations: returns dt."""
    dt = model["schedule"][0]
    sim.mark_old()
    for _ in range(newton_its):
        sim.newton_step(dt, 1e-6)
    return dt


def one_solve(sim, dt, rtol):
    """Assembly + CPR-FPF setup + GMRES; returns (iterations, final relative
    decoupled residual).  A solve that stops above rtol is kept and counted by
    the caller (it is not a solve to rtol)."""
    sim.assemble(dt)
    sim.setup()
    its, rel = sim.solve(rtol, 300, allow_noconv=True)
    return its, rel


RUN_STEPS = 20  # the run whose Jacobians form the benchmark set


def jacobians_of_run(model, nsteps=RUN_STEPS):
    """The Jacobian set: the run is advanced through its first nsteps timesteps
    (FP32 preconditioner, fixed forcing term) and the converged state of every
    step is kept; Jacobian k is taken at state k with old state k-1.  Returns a
    list of (old state, state, dt)."""
    from paper_1808_04338_amd import Sim

    sim = Sim(model, precision="fp32")
    states = [sim.get_state()]
    for k in range(nsteps):
        a = time.perf_counter()
        info = sim.timestep(model["schedule"][k])
        states.append(sim.get_state())
        log("run step %d/%d: %d Newton, %d cuts, %.2f s" % (k + 1, nsteps, info["newton_iters"], info["cuts"],
                                                           time.perf_counter() - a))
    sim.close()
    return [(states[k], states[k + 1], model["schedule"][k]) for k in range(nsteps)]


def jacobian_of_first_step(model):
    """A single Jacobian: the third Newton iterate of the first timestep."""
    from paper_1808_04338_amd import Sim

    sim = Sim(model, precision="fp32")
    old = sim.get_state()
    dt = prepare(sim, model, 3)
    cur = sim.get_state()
    sim.close()
    return [(old, cur, dt)]


def timed_form(model, precision, jset, steps, warmup, rtol, kernels=True, **opts):
    """Time `steps` linear solves (assembly + CPR setup + GMRES) over the Jacobian
    set: solve i takes Jacobian i*len/steps when the set is longer than the run
    of solves (evenly spread), else i mod len.  Loading a Jacobian's states is
    input staging and stays outside the timed region; every solve is bracketed
    by device synchronisations."""
    import torch

    from paper_1808_04338_amd import Sim

    sim = Sim(model, precision=precision, lin_rtol=rtol, **opts)
    loaded = [None]

    def load(j):
        if loaded[0] != j:
            old, cur, _ = jset[j]
            sim.set_state(*old)
            sim.mark_old()
            sim.set_state(*cur)
            loaded[0] = j
        return jset[j][2]

    def pick(i):
        n = len(jset)
        return (i * n) // steps if steps < n else i % n

    dt = load(pick(0))
    for _ in range(warmup):
        one_solve(sim, dt, rtol)
    # live kernel timers over the timed region (HIP events on the handle's stream)
    for k in range(len(sim.TIMED_KERNELS)):
        sim.kernel_timer(k, True)
    lat = []
    its_l = []
    rels = []
    for i in range(steps):
        dt = load(pick(i))
        torch.cuda.synchronize()
        a = time.perf_counter()
        its, rel = one_solve(sim, dt, rtol)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
        its_l.append(its)
        rels.append(rel)
    wall = float(np.sum(lat))
    live = []
    for k, name in enumerate(sim.TIMED_KERNELS):
        ms, n, b = sim.kernel_time(k)
        sim.kernel_timer(k, False)
        if n > 0:
            live.append(dict(name=name, launches=n, total_ms=ms, avg_ms=ms / n, bytes_per_launch=b / n,
                             gbs=b / (ms * 1e-3) / 1e9))
    # per-phase device times of one more solve (the last Jacobian timed)
    sim.enable_timing(True)
    one_solve(sim, dt, rtol)
    phases = {name: sim.phase_time(i)[0] for i, name in enumerate(
        ["assembly_ms", "setup_ms", "solve_ms", "spmv_ms_total", "precond_ms_total"])}
    sim.enable_timing(False)
    kern = sim.bench_kernels(20) if kernels else []
    levels = sim.amg_info()
    global_sorts = sim.amg_global_sort_products()
    out = dict(wall=wall, lat=lat, iters=its_l, rel=rel, rels=rels, picks=[pick(i) for i in range(steps)],
               phases=phases, kern=kern, live=live,
               amg_rows=[int(r) for r in levels[1]], amg_nnz=[int(r) for r in levels[2]],
               amg_global_sorts=global_sorts,
               footprint=sim.footprint, n_dof=sim.n_dof, nnz=sim.nnz)
    sim.close()
    return out


def cpu_info():
    """CPU model and the number of cores this process may run on."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def slab_state(state, n_slab):
    """The top layers of a canonical-order state (p, sw, bhp): the first 2 n_slab
    nodes; the wells keep their p_b."""
    p, sw, bhp = state
    return p[:2 * n_slab].copy(), sw[:2 * n_slab].copy(), np.array(bhp, dtype=np.float64).copy()


def cpu_baseline(model, jset, picks, rtol, nz_sample):
    """The oracle's CPR-FPF (textbook, NumPy/SciPy) timed on the top nz_sample
    layers of the benchmark's own Jacobians: for each picked Jacobian of the
    run, the slab's residual and Jacobian at that state (old state: the one
    before it), setup and GMRES to rtol.  Returns one (seconds, slab DOF,
    iterations) record per pick."""
    from oracle import cpr as ocpr
    from oracle import physics as oph

    m = slab(model, nz_sample)
    geo = oph.Geometry(m)
    ctrl = [w["control"] for w in m["wells"]]
    ns = m["nx"] * m["ny"] * nz_sample
    out = []
    for j in picks:
        old, cur, dt = jset[j]
        x_old = oph.pack_state(*slab_state(old, ns))
        x = oph.pack_state(*slab_state(cur, ns))
        t0 = time.perf_counter()
        acc = oph.accumulation(geo, x_old)
        R = oph.residual(geo, x, acc, dt, ctrl)
        J = oph.jacobian(geo, x, dt, ctrl)
        _, its, rel = ocpr.solve(geo, J, -R, rtol=rtol)
        out.append((time.perf_counter() - t0, geo.N, its, j))
        log("oracle on the %d-layer slab of Jacobian %d: %d iterations, %.1f s" % (nz_sample, j, its, out[-1][0]))
    return out


def layered_run(steps=None):
    """The 144k-DOF configuration end to end: the 60x60x10 layered five-spot
    model over its schedule of 5-day steps (30), FP32 preconditioner, GMRES(30)
    to 1e-6 per Newton iteration, the library's default Newton settings."""
    import torch

    import synth
    from paper_1808_04338_amd import Sim

    model = synth.model_layered()
    sched = model["schedule"] if steps is None else model["schedule"][:steps]
    sim = Sim(model, precision="fp32")
    newton = lin = cuts = 0
    mb = 0.0
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dt in sched:
        a = time.perf_counter()
        info = sim.timestep(dt)
        lat.append(time.perf_counter() - a)
        newton += info["newton_iters"]
        lin += info["lin_iters"]
        cuts += info["cuts"]
        mb = max(mb, info["mb_oil"], info["mb_water"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = dict(grid=[model["nx"], model["ny"], model["nz"]], dof=sim.n_dof, timesteps=len(sched),
               days=sum(sched) / 86400.0, newton_iters=newton, linear_iters=lin, cuts=cuts,
               max_material_balance=mb, wall_s=wall, timesteps_per_s=len(sched) / wall,
               p50_step_ms=float(np.percentile(lat, 50)) * 1e3, p99_step_ms=float(np.percentile(lat, 99)) * 1e3)
    sim.close()
    log("60x60x10 run: %d steps, %d Newton, %d GMRES iterations, %d cuts, %.2f s" % (
        len(sched), newton, lin, cuts, wall))
    return out


def precision_deviation(model, jset, k, rtol):
    """FP32-preconditioner and FP64 forms against a tightly converged FP64
    reference after one timestep from the run's state k (the state after step
    k of the run): the 4.49M-DOF model, the library's default Newton settings
    for the two forms, CNV <= 1e-9 and GMRES to 1e-10 for the reference."""
    from paper_1808_04338_amd import Sim

    start, _, dt = jset[k]
    res = {}
    for name, prec, opts in (("reference_fp64", "fp64", dict(newton_tol=1e-9, lin_rtol=1e-10)),
                             ("fp64", "fp64", dict(lin_rtol=rtol)), ("fp32", "fp32", dict(lin_rtol=rtol))):
        sim = Sim(model, precision=prec, **opts)
        sim.set_state(*start)
        info = sim.timestep(dt)
        res[name] = (sim.get_state(), info)
        sim.close()
        log("one step from state %d, %s: %d Newton, %d GMRES iterations" % (k, name, info["newton_iters"],
                                                                           info["lin_iters"]))
    (pr, sr, br), _ = res["reference_fp64"]
    out = {"start_state": k, "dt_days": dt / 86400.0, "dof": int(4 * model["nx"] * model["ny"] * model["nz"] +
                                                                  2 * len(model["wells"]))}
    for name in ("fp64", "fp32"):
        (p, sw, b), info = res[name]
        out[name] = {"newton_iters": info["newton_iters"], "gmres_iters": info["lin_iters"],
                     "cuts": info["cuts"],
                     "pressure_max_rel_err": float(np.abs(p - pr).max() / np.abs(pr).max()),
                     "saturation_max_abs_err": float(np.abs(sw - sr).max()),
                     "bhp_max_rel_err": float(np.abs(b - br).max() / np.abs(br).max()) if len(br) else None}
    (p32, s32, _), _ = res["fp32"]
    (p64, s64, _), _ = res["fp64"]
    out["fp32_vs_fp64"] = {"pressure_max_rel": float(np.abs(p32 - p64).max() / np.abs(p64).max()),
                           "saturation_max_abs": float(np.abs(s32 - s64).max())}
    return out


SERVED_MAX_LARGE = 4  # resident requests above 4 GiB (the 4.49M-DOF class)


def served_leg(count):
    """Poisson arrivals (4/s), sizes uniform over five classes, 10 five-day steps
    each, FP32 preconditioner, admission against a 200 GB budget with at most
    SERVED_MAX_LARGE requests above 4 GiB resident at once."""
    import synth
    from paper_1808_04338_amd import Request, serve

    stream = synth.served_stream(count=count)
    reqs = [Request(r, synth.served_realisation(r, size), t, tag="%dx%dx%d" % size)
            for t, r, size in stream]
    done = [0]
    lock = threading.Lock()

    def on_done(r):
        with lock:
            done[0] += 1
            k = done[0]
        log("served %d/%d finished: request %d (%s), %d steps, %s" % (k, len(reqs), r.rid, r.tag,
                                                                      len(r.latencies), r.status))

    res, summ = serve(reqs, budget_bytes=200 << 30, precision="fp32", on_done=on_done,
                      max_large=SERVED_MAX_LARGE, large_bytes=4 << 30)
    summ["unit"] = "timesteps/s"
    summ["admission"] = "FIFO by footprint, 200 GiB, at most %d resident requests above 4 GiB" % SERVED_MAX_LARGE
    summ["failures"] = [{"rid": r.rid, "class": r.tag, "steps_done": len(r.latencies),
                         "error": r.error} for r in res.values() if r.status != "ok"]
    return summ


def forcing_study(steps):
    """Fixed eta (lin_rtol 1e-6) against the three adaptive forcing terms of
    Eq. (13): the first `steps` 5-day steps of the 144k-DOF layered model, FP32
    preconditioner.  Returns one record per choice."""
    import torch

    import synth
    from paper_1808_04338_amd import Sim

    model = synth.model_layered()
    out = []
    for choice in (0, 1, 2, 3):
        sim = Sim(model, precision="fp32", forcing=choice)
        newton = lin = cuts = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            info = sim.timestep(model["schedule"][k])
            newton += info["newton_iters"]
            lin += info["lin_iters"]
            cuts += info["cuts"]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        out.append(dict(forcing=choice, timesteps=steps, newton_iters=newton, lin_iters=lin, cuts=cuts,
                        lin_per_newton=lin / max(newton, 1), wall_s=wall))
        log("forcing %d: %d Newton, %d GMRES iterations, %.2f s" % (choice, newton, lin, wall))
    return out


def precond_study(nz, steps, rtol):
    """Each decoupling of Sec. 3.2 (Gauss-Jordan, ABF, true-IMPES) with each
    composition (FPF, FP): the benchmarked solve (the third Newton iterate of the
    first step of the 60x220xnz model, FP32 preconditioner, GMRES to rtol), the
    same state for every combination.  One record per combination."""
    model = make_model(nz)
    out = []
    jset = jacobian_of_first_step(model)
    for dec in ("gj", "abf", "ti"):
        for cpr in ("fpf", "fp"):
            r = timed_form(model, "fp32", jset, steps, 1, rtol, kernels=False, decoupling=dec, cpr_variant=cpr)
            rec = dict(decoupling=dec, cpr=cpr, gmres_iters=r["iters"], rel=r["rel"],
                       solves_per_s=steps / r["wall"], ms_per_solve=1e3 * r["wall"] / steps,
                       setup_ms=r["phases"]["setup_ms"], solve_ms=r["phases"]["solve_ms"],
                       precond_ms_total=r["phases"]["precond_ms_total"])
            out.append(rec)
            log("%s/%s: %s iterations, %.2f solves/s" % (dec, cpr, r["iters"], rec["solves_per_s"]))
    return out


def example_run(number, grid, days, forcing, precision):
    """A whole run of the paper's Example 1 or 2 (Sec. 4) over its printed
    period, optionally on a larger grid with the same cells (the paper's Example 3
    is Example 1 on 500x500x50).  Every timestep prints one progress line."""
    import torch

    import synth
    from paper_1808_04338_amd import Sim

    t0 = time.perf_counter()
    model = synth.paper_example(number, grid=grid, days=days)
    log("example %d on %dx%dx%d: model built in %.1f s" % (number, model["nx"], model["ny"], model["nz"],
                                                           time.perf_counter() - t0))
    sim = Sim(model, precision=precision, forcing=forcing)
    log("handle created: %d DOF, %.1f GB of device memory" % (sim.n_dof, sim.footprint / 1e9))
    torch.cuda.synchronize()
    newton = lin = cuts = substeps = 0
    t_day = 0.0
    t0 = time.perf_counter()
    for k, dt in enumerate(model["schedule"]):
        a = time.perf_counter()
        info = sim.timestep(dt)
        newton += info["newton_iters"]
        lin += info["lin_iters"]
        cuts += info["cuts"]
        substeps += info["substeps"]
        t_day += dt / 86400.0
        log("step %d/%d t=%.0f d: %d Newton, %d linear, %d cuts, %.2f s" % (
            k + 1, len(model["schedule"]), t_day, info["newton_iters"], info["lin_iters"], info["cuts"],
            time.perf_counter() - a))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = dict(example=number, grid=[model["nx"], model["ny"], model["nz"]], dof=sim.n_dof,
               days=t_day, timesteps=len(model["schedule"]), substeps=substeps, cuts=cuts,
               newton_iters=newton, linear_iters=lin, wall_s=wall, footprint_gb=sim.footprint / 1e9,
               precision=precision, forcing=forcing)
    sim.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--nz", type=int, default=85)
    ap.add_argument("--cpu-layers", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-example3", action="store_true",
                    help="skip the paper's Example 3 shape (500x500x50, 50M DOF) run")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32/FP64 state deviation after one step at full size")
    ap.add_argument("--no-layered", action="store_true",
                    help="skip the 30-step run of the 144k-DOF layered five-spot model")
    ap.add_argument("--amg-coarse-max", type=int, default=0,
                    help="largest coarsest AMG level (0: the library default)")
    ap.add_argument("--amg-theta", type=float, default=0.0,
                    help="AMG strength threshold (0: the library default)")
    ap.add_argument("--amg-trunc", type=int, default=0,
                    help="interpolation entries kept per row (0: the library default)")
    ap.add_argument("--no-kernels", action="store_true",
                    help="skip the per-kernel timings (kernels list and roofline)")
    ap.add_argument("--served", type=int, default=32,
                    help="requests of the served-ensemble leg (0 to skip)")
    ap.add_argument("--forcing-study", type=int, default=0,
                    help="instead of the benchmark: that many timesteps of the 144k-DOF model with "
                         "each forcing choice of Eq. (13)")
    ap.add_argument("--precond-study", type=int, default=0,
                    help="instead of the benchmark: that many timed solves with each decoupling and "
                         "CPR composition")
    ap.add_argument("--workload", choices=("run", "first"), default="run",
                    help="run: the Jacobians of the 20-step run (default); first: the third Newton "
                         "iterate of the first step, repeated")
    ap.add_argument("--example", type=int, default=0,
                    help="instead of the benchmark: a whole run of the paper's Example 1 or 2")
    ap.add_argument("--grid", type=int, nargs=3, default=None,
                    help="with --example: grid dimensions (same cells as printed)")
    ap.add_argument("--days", type=float, default=None, help="with --example: simulated period")
    ap.add_argument("--forcing", type=int, default=0, help="with --example: forcing choice of Eq. (13)")
    ap.add_argument("--precision", default="fp32", help="with --example: preconditioner precision")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (a sharded solve "
              "would split the grid into slabs along y, one per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.forcing_study > 0:
        rec = forcing_study(args.forcing_study)
        print(json.dumps({"study": "inexact-Newton forcing terms (Eq. (13)) vs fixed eta = 1e-6",
                          "workload": "dual-porosity oil-water 60x60x10 layered five-spot, 144,010 DOF, "
                                      "5-day steps, FP32 preconditioner",
                          "data": "synthetic", "results": rec}))
        return
    if args.example > 0:
        rec = example_run(args.example, tuple(args.grid) if args.grid else None, args.days, args.forcing,
                          args.precision)
        print(json.dumps({"study": "whole run of the paper's Example %d (Sec. 4)" % args.example,
                          "data": "synthetic (printed inputs, stated readings)", "results": rec}))
        return
    if args.precond_study > 0:
        rec = precond_study(args.nz, args.precond_study, args.rtol)
        print(json.dumps({"study": "decoupling (Gauss-Jordan, ABF, true-IMPES) x CPR composition (FPF, FP)",
                          "workload": "dual-porosity oil-water 60x220x%d channelised, third Newton iterate of "
                                      "the first 10-day step, FP32 preconditioner, GMRES to %g"
                                      % (args.nz, args.rtol),
                          "data": "synthetic", "results": rec}))
        return
    log("generating the 60x220x%d model" % args.nz)
    model = make_model(args.nz)
    opts = {}
    if args.amg_coarse_max:
        opts["amg_coarse_max"] = args.amg_coarse_max
    if args.amg_theta:
        opts["amg_theta"] = args.amg_theta
    if args.amg_trunc:
        opts["amg_trunc"] = args.amg_trunc
    if args.workload == "run":
        log("the Jacobian set: %d steps of the run" % RUN_STEPS)
        jset = jacobians_of_run(model)
        wdesc = ("Jacobians at the converged states of the %d ten-day steps of the run (%d timed solves "
                 "spread over them)" % (RUN_STEPS, args.steps))
    else:
        jset = jacobian_of_first_step(model)
        wdesc = "the third Newton iterate of the first ten-day step, solved %d times" % args.steps
    log("FP32-preconditioner form")
    r32 = timed_form(model, "fp32", jset, args.steps, args.warmup, args.rtol, kernels=not args.no_kernels,
                     **opts)
    r64 = None
    if not args.no_fp64:
        log("FP64 form")
        r64 = timed_form(model, "fp64", jset, args.steps, args.warmup, args.rtol,
                         kernels=not args.no_kernels, **opts)
    ms = 1000.0 * r32["wall"] / args.steps
    value = args.steps / r32["wall"]
    lat = np.array(r32["lat"]) * 1000.0
    # roofline of the timed kernel with the largest device time in the timed region
    roof = None
    if r32["live"]:
        k = max(r32["live"], key=lambda e: e["total_ms"])
        roof = dict(bound="hbm", kernel=k["name"], achieved=k["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=k["gbs"] / HBM_PEAK_GBS,
                    traffic=traffic_for(k["name"], k["bytes_per_launch"]) if args.nz == 85 else None,
                    bytes_per_launch=k["bytes_per_launch"], avg_ms=k["avg_ms"], launches=k["launches"],
                    ms_per_step=k["total_ms"] / args.steps)
    above = [i for i, r in enumerate(r32["rels"]) if not r <= args.rtol]
    prec_dev = None
    if not args.no_precision and args.workload == "run":
        log("FP32 and FP64 forms against a converged FP64 step at full size")
        prec_dev = precision_deviation(model, jset, len(jset) // 2, args.rtol)
    cpu = None
    if not args.no_cpu:
        cpu_model, cores_avail = cpu_info()
        tp = r32["picks"]
        picks = sorted({tp[0], tp[len(tp) // 2], tp[-1]})
        log("oracle CPU baseline on %d-layer slabs of Jacobians %s" % (args.cpu_layers, picks))
        recs = cpu_baseline(model, jset, picks, args.rtol, args.cpu_layers)
        full = r32["n_dof"]
        rates = [(1.0 / t) * (ndof / full) for t, ndof, its, j in recs]
        gpu_its = {r32["picks"][i]: r32["iters"][i] for i in range(len(r32["picks"]))}
        cpu = dict(value=float(np.mean(rates)), unit="solves/s", cores=1, kind="oracle",
                   sample="assembly + CPR-FPF setup + GMRES(30) to %g by the oracle on the top %d layers "
                          "(%d DOF) of the run's Jacobians %s (the states the timed solves use): %s s, "
                          "%s GMRES iterations (the GPU's on the full Jacobians: %s); the rate is "
                          "extrapolated by DOF to the full %d-DOF model"
                          % (args.rtol, args.cpu_layers, recs[0][1], [r[3] for r in recs],
                             [round(r[0], 1) for r in recs], [r[2] for r in recs],
                             [gpu_its.get(r[3]) for r in recs], full),
                   cpu_model=cpu_model, cores_available=cores_avail,
                   threads_note="SciPy sparse products, triangular solves and SuperLU run on one core")
    layered = None
    if not args.no_layered:
        log("the 144k-DOF layered five-spot model over its 30 five-day steps")
        layered = layered_run()
    ex3 = None
    if not args.no_example3:
        log("the paper's Example 3 shape: Example 1 on 500x500x50")
        ex3 = example_run(1, (500, 500, 50), None, 2, "fp32")
        ex3["paper_context"] = {"timesteps": 68, "newton_iters": 273, "linear_iters": 641,
                                "wall_s_64_processes": 2531.91, "wall_s_8_processes": 20009.71,
                                "hardware": "a CPU cluster, not stated further", "source": "Sec. 4, Example 3 table"}
    out = {
        "metric": "linear solves/s at 4.5M DOF, FP32-precond vs FP64 to 1e-6 rtol; p50/p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 Krylov + f32 preconditioner",
        "data": "synthetic",
        "config": {"workload": "dual-porosity oil-water 60x%dx%d channelised, %d DOF, assembly + "
                               "CPR-FPF setup + GMRES(30) to rtol %g, FP32 preconditioner; %s"
                               % (220, args.nz, r32["n_dof"], args.rtol, wdesc),
                   "dof": r32["n_dof"], "nnz": r32["nnz"], "jacobians": len(jset)},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "gmres_iters": r32["iters"],
        "phases_ms": r32["phases"],
        "amg_rows": r32["amg_rows"],
        "amg_nnz": r32["amg_nnz"],
        "amg_global_sort_products": r32["amg_global_sorts"],
        "roofline": roof,
        "timed_kernels": r32["live"],
        "kernels_isolated": r32["kern"],
        "cpu_baseline": cpu,
        "timed_solves_above_rtol": above,
        "max_rel_res": float(max(r32["rels"])),
        "precision_deviation": prec_dev,
        "layered_144k_run": layered,
        "example3": ex3,
    }
    if args.served > 0:
        log("served ensemble: %d requests" % args.served)
        out["served"] = served_leg(args.served)
    if r64 is not None:
        lat64 = np.array(r64["lat"]) * 1000.0
        out["fp64"] = {"value": args.steps / r64["wall"], "unit": "solves/s",
                       "ms_per_step": 1000.0 * r64["wall"] / args.steps,
                       "p50_ms": float(np.percentile(lat64, 50)),
                       "p99_ms": float(np.percentile(lat64, 99)),
                       "gmres_iters": r64["iters"], "phases_ms": r64["phases"],
                       "kernel": r64["kern"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
