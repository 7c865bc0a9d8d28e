"""Benchmark: element updates per second of the ALE ADER-WENO scheme with
local time stepping on one MI355X.

Default workload (the metric's configuration, its largest single mesh): the
cylindrical explosion EP1 on the unit disk, seeded 8:1 radially graded mesh of
~400k triangles, transmissive boundary, mesh moving with the fluid, WENO M=2,
LTS with 4 dyadic levels against GTS on the same mesh, FP64.  One step = one
LTS macro step (every element reaches the common time again).  value =
element updates / wall time of the timed macro steps (state resident in HBM).

Also reported: GTS and free local steps (every element at its own CFL step)
over the same physical interval and the time-to-solution ratios; the
per-kernel breakdown from HIP events recorded on the solver's stream; the
roofline of the dominant kernel and the HBM rate of the flux, update, node
and scheduling kernels; the CPU oracle timed on a bounded sample of the same
recipe; one adjoint step against one forward step of the adjoint workload.

Other workloads (separate lines): --workload vortex (isentropic vortex, 80k
triangles, M=2, 3 levels), sod (RP1 shock tube, 2k triangles, M=1, GTS),
batched (256 independent instances in the same launches), adjoint
(gradient through 100 global steps with checkpoints, against the run) or
adjoint_lts (gradient through 100 LTS macro steps, 3 levels, against the run).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload explosion]
                       [--n-elems N] [--M M] [--levels L]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6     # MI355X, published
PEAK_HBM_GBS = 8000.0              # MI355X HBM3E, published
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1408_3719_amd", "csrc", n) for n in ("kernels.hip", "basis.h")]

# HBM bytes per unit of work of the step kernels for each persistent-grid
# setting (workgroups per CU; 0 = one grid over all items) of the list-driven
# kernels (k_reconstruct, k_predict, k_update, k_sched) and of the node and
# edge sweeps (k_node, k_patch): the rocprofv3 FETCH_SIZE and WRITE_SIZE of the profiled LTS pass's
# launches on the 400k explosion mesh at M=2 (4 levels), scaled by what the
# same counters read for a plain 256 MiB copy, divided by the units those
# launches processed (element updates; patches; moved nodes; for the scheduler
# the elements of the mesh). Valid only for the kernel code they were taken on
# (sha256 of kernels.hip and basis.h with comments and whitespace removed);
# otherwise traffic is reported null.
TRAFFIC_SWEEP = (0, 4, 8, 16, 32)
MEASURED_TRAFFIC = {
    "workload": "explosion",
    "source_sha256": "9a8b6ba5a837561b330d64f70a288df398708a542e0cd68f2993f1ee46cb8014",
    "k_reconstruct": {0: 1552, 4: 1606, 8: 1583, 16: 1564, 32: 1557},
    "k_predict": {0: 1501, 4: 1502, 8: 1502, 16: 1502, 32: 1502},
    "k_patch": {0: 1042, 4: 1072, 8: 1048, 16: 1042, 32: 1042},
    "k_update": {0: 724, 4: 726, 8: 724, 16: 724, 32: 724},
    "k_node": {w: 1775 for w in TRAFFIC_SWEEP},
    "k_sched": {w: 88 for w in TRAFFIC_SWEEP},
}


def kernel_source_sha() -> str:
    """sha256 of the step kernels' sources with comments and whitespace removed."""
    text = ""
    for path in KERNEL_SOURCES:
        with open(path) as f:
            text += f.read() + "\n"
    code = re.sub(r"//[^\n]*", " ", re.sub(r"/\*.*?\*/", " ", text, flags=re.S))
    return hashlib.sha256(" ".join(code.split()).encode()).hexdigest()


# ---------------------------------------------------------------------------
# Algorithmic work per unit (operation counts of the algorithm)
# ---------------------------------------------------------------------------
def recon_flops(M: int) -> int:
    """FP64 operations of one element reconstruction + CFL step, counting
    7 stencils of n_e - 1 least-squares rows each, without the projection
    arithmetic (which same-time neighbours skip)."""
    nb = (M + 1) * (M + 2) // 2
    nu = nb - 1
    ne = 2 * nb
    # quadrature points of the rule exact to degree M and the flops that place
    # each (centroid 6, edge midpoint 4, vertex 0)
    point_cost = {1: [6], 2: [4, 4, 4], 3: [0, 0, 0, 4, 4, 4, 6]}[M]
    ref = 3 * 8                                   # vertices into the element's frame
    means = sum(c + 2 * nb + 2 * nb for c in point_cost)   # point, monomials, weighted sums
    arow = nu + 4                                 # shift by the reference means + right-hand side
    givens = nu * (8 + 24) + 6 * nu * (nu - 1) // 2
    row = ref + means + arow + givens
    stencil = (ne - 1) * row + 4 * nu * (nu + 1) + 4 * (2 * nu * nu + 2 * nu) + 20 + 8 * nu
    out = nb * 4 * 2 * nu                         # nodal values from the weighted coefficients
    cfl = 4 * 40
    return 7 * stencil + out + cfl


def predict_flops(M: int, npic: int | None = None) -> int:
    """FP64 operations of one element predictor (npic Picard sweeps + publish)."""
    nb = (M + 1) * (M + 2) // 2
    T = M + 1
    npic = npic or M + 1
    per_node = 2 + 8 * nb + 4 * T + 18 + 20 + 48 * nb + 48 + 8 * M
    sweep = nb * T * per_node + nb * M * (4 * T + 4) + 4 * nb * M
    publish = 4 * T * 2 * nb + 3 * (M + 1) * T * 4 * 2 * nb + 3 * T * 2
    return npic * sweep + publish


def patch_bytes(M: int) -> int:
    """Compulsory HBM bytes of one space-time patch: two corner states per node
    (x, y, tick), both elements' edge traces at nG points and T time nodes,
    their tick and step, the edge record, and the flux/normal written back."""
    T = nG = M + 1
    return 2 * 2 * (16 + 4) + 2 * nG * T * 4 * 8 + 2 * 8 + 7 * 4 + 7 * 8 + 4


# ---------------------------------------------------------------------------
def bench_adjoint(a):
    """Gradient through a run of global steps: EP1 explosion on a 50k-triangle
    8:1 graded disk, M=2, Rusanov flux, 100 steps of a fixed dt, checkpoints
    every 10 steps. Default: the mesh moving with the fluid (dt = 0.3 x the
    smallest initial CFL step), J = energy carried at the final time by the
    elements that start inside r < 0.3 (their moved areas included), gradient
    with respect to the initial averages and node positions. With
    --mesh-velocity eulerian: the fixed mesh (dt = half the smallest CFL step),
    J = total energy inside r < 0.3, gradient with respect to the initial
    averages. value = backward time (the adjoint steps and the recomputation
    inside the checkpoint segments) / forward time of the run. Also per step:
    the step adjoint against one ader_step_gts from the same state. States
    resident in HBM throughout."""
    import numpy as np
    import torch

    from paper_1408_3719_amd import Config, Solver
    from paper_1408_3719_amd.trajectory import gts_trajectory, lagrangian_trajectory
    from workloads import explosion_case

    n = a.n_elems or 50_000
    M = a.M or 2
    lagr = a.mesh_velocity == "lagrangian"
    n_steps, every = 100, 10
    mesh, Q0 = explosion_case(n, seed=7)
    NE = mesh.n_elems
    s = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=M, levels=1, mesh_velocity=a.mesh_velocity))
    if lagr:
        # 0.8 x the smallest of 100 free-running global CFL steps: the mesh
        # compresses and the CFL step shrinks along the run
        t = [0.0] + [s.step_gts(1e9, 1)["t"] for _ in range(n_steps)]
        dt = 0.8 * float(np.diff(t).min())
    else:
        dt = 0.5 * float(s.dump("DTCFL").min())
    c = mesh.nodes[mesh.tris].mean(axis=1)
    inner_np = np.hypot(c[:, 0], c[:, 1]) < 0.3
    inner = torch.tensor(np.nonzero(inner_np)[0], device="cuda")
    tris = torch.tensor(mesh.tris, dtype=torch.long, device="cuda")[inner]

    def area(x):
        p = x[tris]
        return 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                      - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    A0 = area(torch.tensor(mesh.nodes, device="cuda"))
    sync = torch.cuda.synchronize

    def run(every):
        t_f = t_b = 0.0
        for k in range(a.warmup + a.steps):
            q0 = torch.tensor(Q0.T.copy(), device="cuda", requires_grad=True)
            x0 = torch.tensor(mesh.nodes, device="cuda", requires_grad=True)
            sync()
            t0 = time.perf_counter()
            if lagr:
                qn, xn = lagrangian_trajectory(s, q0, x0, dt, n_steps, every=every)
                Jv = (area(xn) * qn[3][inner]).sum()
            else:
                qn = gts_trajectory(s, q0, dt, n_steps, every=every)
                Jv = (A0 * qn[3][inner]).sum()
            sync()
            t1 = time.perf_counter()
            Jv.backward()
            sync()
            t2 = time.perf_counter()
            if k >= a.warmup:
                t_f += t1 - t0
                t_b += t2 - t1
        assert torch.isfinite(q0.grad).all()
        return t_f, t_b, q0.grad

    t_f, t_b, g10 = run(every)
    t_f1, t_b1, g1 = run(1)
    # the checkpoint spacing changes only rounding (recomputed steps restart
    # from a checkpoint's time)
    assert float((g10 - g1).abs().max()) <= 1e-10 * float(g1.abs().max())
    per_step = (lagrangian_adjoint_step_ratio if lagr else adjoint_step_ratio)(n_elems=n, M=M)
    mesh_desc = ("mesh moving with the fluid, J = energy carried by the elements starting in r < 0.3, "
                 "gradient w.r.t. initial averages and node positions" if lagr else
                 "fixed mesh, J = energy inside r < 0.3, gradient w.r.t. initial averages")
    line = {
        "metric": "adjoint/forward time (gradient of J through 100 global steps)",
        "value": t_b / t_f,
        "unit": "ratio",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": t_b / a.steps * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"EP1 explosion, {NE}-triangle 8:1 radially graded disk, M={M}, {mesh_desc}, "
                               f"{n_steps} global steps of a fixed dt ({'0.8 x the smallest of 100 free-running CFL steps' if lagr else 'half the smallest initial CFL step'}), "
                               f"checkpoints every {every}, Rusanov", "dt": dt,
                   "n_elems": NE, "M": M, "n_steps": n_steps, "checkpoint_every": every,
                   "mesh_velocity": a.mesh_velocity, "parallelism": "single GPU"},
        "forward_s_per_run": t_f / a.steps,
        "gradient_s_per_run": t_b / a.steps,
        "per_step": {"forward_ms": per_step["forward_ms"], "adjoint_ms": per_step["adjoint_ms"],
                     "ratio": per_step["value"]},
        "all_states_kept": {"forward_s_per_run": t_f1 / a.steps, "gradient_s_per_run": t_b1 / a.steps,
                            "ratio": t_b1 / t_f1},
        "note": "steps are timed one host call each; ms_per_step is the gradient time of one run",
        "cpu_baseline": None if a.no_cpu_baseline else cpu_baseline_adjoint(a.mesh_velocity, M=M),
    }
    print(json.dumps(line))


def bench_adjoint_lts(a):
    """Gradient through macro steps of the local time stepping on the mesh
    moving with the fluid: EP1 explosion on a 50k-triangle 8:1 graded disk,
    M=2, 3 dyadic levels, Rusanov flux, 100 macro steps from t = 0; J = energy
    carried at the end by the elements that start inside r < 0.3 (their moved
    areas included), gradient with respect to the initial averages and node
    positions through ader_adjoint_lts (schedule held fixed). value = time of
    the gradient call (its own forward run saving every macro-step start, a
    replay of every macro step saving the state after each cycle, and the
    reverse sweep) / time of the forward run alone (ader_step_lts over the same
    macro steps). States resident in HBM."""
    import numpy as np
    import torch

    from paper_1408_3719_amd import Config, Solver
    from workloads import explosion_case

    n = a.n_elems or 50_000
    M = a.M or 2
    L = a.levels or 3
    n_macro = 100
    mesh, Q0 = explosion_case(n, seed=7)
    NE = mesh.n_elems
    s = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=M, levels=L, mesh_velocity="lagrangian"))
    sync = torch.cuda.synchronize
    c = mesh.nodes[mesh.tris].mean(axis=1)
    inner = torch.tensor(np.nonzero(np.hypot(c[:, 0], c[:, 1]) < 0.3)[0], device="cuda")
    tris = torch.tensor(mesh.tris, dtype=torch.long, device="cuda")[inner]

    def area(x):
        p = x[tris]
        return 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                      - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))

    runs = max(1, min(a.steps, 3))
    t_f, st = 0.0, None
    for k in range(1 + runs):
        s.upload_state(Q0)
        sync()
        t0 = time.perf_counter()
        s.step_lts(1e9, n_macro)
        sync()
        if k:
            t_f += time.perf_counter() - t0
        st = s.stats()
    q = s.download_q().clone().requires_grad_(True)
    x = s.download_x().clone().requires_grad_(True)
    (area(x) * q[3][inner]).sum().backward()
    qb, xb = q.grad.detach(), x.grad.detach()
    t_g, done = 0.0, 0
    for k in range(1 + runs):
        s.upload_state(Q0)
        sync()
        t0 = time.perf_counter()
        gq, gx, done = s.adjoint_lts(n_macro, 1e9, qb, xb)
        sync()
        if k:
            t_g += time.perf_counter() - t0
    assert done == n_macro and bool(torch.isfinite(gq).all()) and bool(torch.isfinite(gx).all())
    line = {
        "metric": "adjoint/forward time (gradient of J through 100 LTS macro steps)",
        "value": t_g / t_f,
        "unit": "ratio",
        "n_gpus": 1, "steps": runs, "warmup": 1,
        "ms_per_step": t_g / runs * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"EP1 explosion, {NE}-triangle 8:1 radially graded disk, M={M}, {L} dyadic levels, "
                               f"mesh moving with the fluid, {n_macro} macro steps from t = 0, J = energy carried by "
                               "the elements starting in r < 0.3, gradient w.r.t. initial averages and node "
                               "positions, schedule held fixed, Rusanov",
                   "n_elems": NE, "M": M, "levels": L, "n_macro": n_macro, "parallelism": "single GPU"},
        "forward_s_per_run": t_f / runs,
        "gradient_s_per_run": t_g / runs,
        "element_updates_per_run": int(st["element_updates"]),
        "cycles_per_run": int(st["cycles"]) if "cycles" in st else None,
        "t_end": float(st["t"]),
        "note": "ms_per_step is the gradient time of one run; the gradient call includes its own forward run",
        "cpu_baseline": None if a.no_cpu_baseline else cpu_baseline_adjoint_lts(M=M, levels=L),
    }
    print(json.dumps(line))


def cpu_baseline_adjoint_lts(n_elems: int = 2000, M: int = 2, levels: int = 3):
    """The reverse-mode oracle of the local time stepping (torch.autograd
    through the oracle's LTS macro step, CPU, one thread) on a bounded sample
    of the workload's recipe: one macro step's vector-Jacobian product against
    the same macro step forward, in a single-threaded subprocess."""
    code = f"""
import json, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np, torch
torch.set_num_threads(1)
from oracle.adjoint import LagrangianLTS, lts_schedule
from oracle.scheme import Config, Solver
from workloads import explosion_case
mesh, Q0 = explosion_case({n_elems}, seed=7)
cfg = Config(M={M}, levels={levels}, mesh_velocity="lagrangian")
o = Solver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
sched = lts_schedule(o, 1e9, 1)
lt = LagrangianLTS(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
rng = np.random.default_rng(0)
qb, xb = rng.standard_normal(Q0.shape), rng.standard_normal(mesh.nodes.shape)
t = time.perf_counter()
lt.vjp(Q0, mesh.nodes, sched, qb, xb)
ta = time.perf_counter() - t
t = time.perf_counter()
lt.run(Q0, mesh.nodes, sched)
tf = time.perf_counter() - t
print(json.dumps(dict(adjoint_s=ta, forward_s=tf, n_elems=mesh.n_elems, updates=int(o.st.updates))))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    r = json.loads(out.stdout.strip().splitlines()[-1])
    cpu = host_cpu()
    return dict(value=r["adjoint_s"] / r["forward_s"], unit="ratio", cores=1, kind="oracle",
                adjoint_element_updates_per_s=r["updates"] / r["adjoint_s"],
                sample=f"explosion recipe at {r['n_elems']} triangles, M={M}, {levels} levels, mesh moving with "
                       f"the fluid, one macro step ({r['updates']} element updates): the oracle's reverse mode "
                       f"{r['adjoint_s']:.2f} s (its forward included) against its forward {r['forward_s']:.2f} s "
                       "(one host thread)",
                host_cpu_model=cpu["model"], host_logical_cpus=cpu["logical_cpus"],
                host_cpus_available=cpu["cpus_available"])


def bench_batched(a):
    """Uneven batch of independent Riemann and explosion instances (log-uniform
    1k-50k triangles, random left/right density and pressure), M=2, LTS 3
    levels, all instances in the same kernel launches, against the same
    instances stepped one after another in their own contexts. Instances
    whose solution breaks down when run alone within the horizon (the
    unlimited scheme on strong random jumps) are left out of both, and listed."""
    import torch

    from paper_1408_3719_amd import AderError, Config, Solver
    from workloads import batched_cases, concat_instances

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    M, L = a.M or 2, a.levels or 3
    cases = batched_cases(n_instances=a.instances, seed=256)
    note(f"{len(cases)} instances generated")
    cfg = Config(M=M, levels=L, flux=a.flux)
    far = 1e9                                    # a fixed number of macro steps, no target time
    sync = torch.cuda.synchronize
    # one after another, each in its own context
    seq_t, seq_upd, kept, dropped = 0.0, 0, [], []
    for k, (mesh, q) in enumerate(cases):
        if k % 32 == 0:
            note(f"sequential: instance {k}")
        one = Solver(mesh.nodes, mesh.tris, mesh.bedges, q, cfg)
        try:
            one.step_lts(far, a.warmup)
            u0 = one.stats()["element_updates"]
            sync()
            t0 = time.perf_counter()
            one.step_lts(far, a.steps)
            sync()
            dt = time.perf_counter() - t0
        except AderError as e:
            dropped.append({"instance": k, "n_elems": int(mesh.n_elems), "error": str(e)})
            del one
            continue
        seq_t += dt
        seq_upd += one.stats()["element_updates"] - u0
        kept.append((mesh, q))
        del one
    nodes, tris, bedges, Q0, first = concat_instances(kept)
    note(f"batch of {len(kept)} instances, {tris.shape[0]} triangles")
    s = Solver(nodes, tris, bedges, Q0, cfg, instance_first=first)
    s.step_lts(far, a.warmup)
    st0 = s.stats()
    sync()
    t0 = time.perf_counter()
    s.step_lts(far, a.steps)
    sync()
    t_batch = time.perf_counter() - t0
    upd = s.stats()["element_updates"] - st0["element_updates"]
    note(f"batched: {upd} updates in {t_batch:.3f} s")
    line = {
        "metric": "element-updates/s at 1e-10 rel err vs FP64 oracle, LTS vs GTS",
        "value": upd / t_batch, "unit": "element-updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": t_batch / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch of {len(kept)} Riemann/explosion instances, "
                               f"{tris.shape[0]} triangles in all (1k-50k each), M={M}, "
                               f"LTS {L} levels, {a.flux} flux, one step = one macro step of "
                               "every instance", "instances": len(kept),
                   "n_elems": int(tris.shape[0]), "M": M, "levels": L, "parallelism": "single GPU"},
        "sequential": {"value": seq_upd / seq_t, "updates": seq_upd, "seconds": seq_t},
        "batched_over_sequential": (upd / t_batch) / (seq_upd / seq_t),
        "dropped": dropped,
        "roofline": None, "cpu_baseline": None,
    }
    assert seq_upd == upd, (seq_upd, upd)
    print(json.dumps(line))


METRIC = "element-updates/s at 1e-10 rel err vs FP64 oracle, LTS vs GTS; adjoint/forward ratio"

# Algorithmic work per unit of the hot path (what the method must compute or
# move, independent of this implementation): reconstruction and predictor
# flops per element update, compulsory HBM bytes per space-time patch, per
# active-element update, per moved node and per scheduling candidate.
UNIT_WORK = {
    "recon_flops": {1: 5_000, 2: 25_000, 3: 120_000},
    "predict_flops": {1: 3_600, 2: 27_000, 3: 120_000},
    "patch_bytes": {1: 464, 2: 784, 3: 1232},
    "update_bytes": {1: 364, 2: 364, 3: 364},
    "node_bytes": {1: 450, 2: 550, 3: 650},
    "sched_bytes": {1: 180, 2: 180, 3: 200},
}


def rate_entry(per_unit: float, units: float, total_ms: float, launches: int, peak: float, scale: float):
    """Algorithmic rate of one kernel: per_unit x (units / launches) per
    launch, divided by the average launch duration (total_ms / launches), in
    units of `scale` per second, and its fraction of `peak`."""
    avg_s = total_ms / max(launches, 1) * 1e-3
    upl = units / max(launches, 1)
    achieved = per_unit * upl / avg_s / scale if avg_s > 0 else 0.0
    return {"achieved": achieved, "peak": peak, "frac": achieved / peak, "units_per_launch": upl,
            "launches": launches, "avg_launch_us": avg_s * 1e6}


def host_cpu():
    """Model name and logical CPU count of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = None
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_available": avail}


def cpu_baseline_case(workload: str, n_elems: int, M: int, levels: int, macro_steps: int, t_end: float):
    """Time the oracle on a bounded sample of the workload's recipe in a
    single-threaded subprocess (one host core)."""
    make = {"explosion": "explosion_case({n}, seed=7)", "vortex": "vortex_case({n}, seed=1)",
            "sod": "sod_case({n}, seed=1408)"}[workload].format(n=n_elems)
    code = f"""
import json, os, sys, time
sys.path.insert(0, {ROOT!r})
from oracle.scheme import Config, Solver
from workloads import explosion_case, sod_case, vortex_case
mesh, Q0 = {make}
s = Solver(mesh.nodes, mesh.tris, Q0, Config(M={M}, levels={levels}), bedges=mesh.bedges)
t = time.perf_counter()
s.run({t_end}, max_macro_steps={macro_steps})
dt = time.perf_counter() - t
print(json.dumps(dict(updates=s.st.updates, seconds=dt, n_elems=mesh.n_elems)))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    r = json.loads(out.stdout.strip().splitlines()[-1])
    cpu = host_cpu()
    return dict(value=r["updates"] / r["seconds"], unit="element-updates/s", cores=1, kind="oracle",
                sample=f"{workload} recipe at {r['n_elems']} triangles, M={M}, {levels} levels, first "
                       f"{macro_steps} macro steps ({r['updates']} element updates in {r['seconds']:.1f} s, "
                       f"one host thread)",
                host_cpu_model=cpu["model"], host_logical_cpus=cpu["logical_cpus"],
                host_cpus_available=cpu["cpus_available"])


def cpu_baseline_adjoint(mesh_velocity: str, n_elems: int = 5000, M: int = 2, reps: int = 3):
    """The reverse-mode oracle (torch.autograd through the oracle's global
    step, CPU, one thread) on a bounded sample of the adjoint workload's
    recipe: one step's vector-Jacobian product against one forward step, in a
    single-threaded subprocess."""
    cls = "LagrangianStep" if mesh_velocity == "lagrangian" else "EulerianStep"
    code = f"""
import json, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np, torch
torch.set_num_threads(1)
from oracle.adjoint import {cls} as Step
from oracle.scheme import Config, GTSSolver
from workloads import explosion_case
mesh, Q0 = explosion_case({n_elems}, seed=7)
cfg = Config(M={M}, levels=1, mesh_velocity={mesh_velocity!r})
o = GTSSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
dt = 0.5 * float(o.dtcfl.min())
st = Step(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
rng = np.random.default_rng(0)
qb, xb = rng.standard_normal(Q0.shape), rng.standard_normal(mesh.nodes.shape)
lag = {mesh_velocity == "lagrangian"}
t = time.perf_counter()
for _ in range({reps}):
    st.vjp(Q0, mesh.nodes, dt, qb, xb) if lag else st.vjp(Q0, dt, qb)
ta = (time.perf_counter() - t) / {reps}
t = time.perf_counter()
for _ in range({reps}):
    st.step(Q0, mesh.nodes, dt) if lag else st.step(Q0, dt)
tf = (time.perf_counter() - t) / {reps}
print(json.dumps(dict(adjoint_s=ta, forward_s=tf, n_elems=mesh.n_elems)))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    r = json.loads(out.stdout.strip().splitlines()[-1])
    cpu = host_cpu()
    return dict(value=r["adjoint_s"] / r["forward_s"], unit="ratio", cores=1, kind="oracle",
                adjoint_element_steps_per_s=r["n_elems"] / r["adjoint_s"],
                forward_element_steps_per_s=r["n_elems"] / r["forward_s"],
                sample=f"explosion recipe at {r['n_elems']} triangles, M={M}, {mesh_velocity} mesh, one global "
                       f"step: the oracle's reverse-mode step {r['adjoint_s']:.2f} s against its forward step "
                       f"{r['forward_s']:.2f} s (mean of {reps}, one host thread)",
                host_cpu_model=cpu["model"], host_logical_cpus=cpu["logical_cpus"],
                host_cpus_available=cpu["cpus_available"])


def adjoint_step_ratio(n_elems: int = 50_000, M: int = 2, reps: int = 20):
    """One adjoint step against one forward step from the same state, on the
    adjoint workload (explosion recipe, fixed mesh, dt = half the smallest CFL
    step): the per-step adjoint/forward time ratio."""
    import numpy as np
    import torch

    from paper_1408_3719_amd import Config, Solver
    from workloads import explosion_case
    mesh, Q0 = explosion_case(n_elems, seed=7)
    s = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=M, levels=1, mesh_velocity="eulerian"))
    dt = 0.5 * float(s.dump("DTCFL").min())
    qb = torch.tensor(np.random.default_rng(0).standard_normal((4, mesh.n_elems)), device="cuda")
    sync = torch.cuda.synchronize
    for _ in range(3):
        s.adjoint_gts_step(dt, qb)
        s.upload_state(Q0, 0.0)
        s.step_gts(dt, 1)
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.adjoint_gts_step(dt, qb)
    sync()
    ms_adj = (time.perf_counter() - t0) / reps * 1e3
    ms_fwd = 0.0
    for _ in range(reps):
        s.upload_state(Q0, 0.0)
        sync()
        t0 = time.perf_counter()
        s.step_gts(dt, 1)
        sync()
        ms_fwd += (time.perf_counter() - t0) / reps * 1e3
    return {"value": ms_adj / ms_fwd, "adjoint_ms": ms_adj, "forward_ms": ms_fwd,
            "workload": f"one global step on the {mesh.n_elems}-triangle explosion, fixed mesh, M={M}"}


def lagrangian_adjoint_step_ratio(n_elems: int = 50_000, M: int = 2, reps: int = 20):
    """One adjoint step of the moving-mesh global step (averages and node
    positions differentiated, ader_adjoint_lagrangian_step) against one forward
    Lagrangian global step from the same state, explosion recipe, dt = half
    the smallest CFL step."""
    import numpy as np
    import torch

    from paper_1408_3719_amd import Config, Solver
    from workloads import explosion_case
    mesh, Q0 = explosion_case(n_elems, seed=7)
    s = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=M, levels=1, mesh_velocity="lagrangian"))
    dt = 0.5 * float(s.dump("DTCFL").min())
    rng = np.random.default_rng(0)
    qb = torch.tensor(rng.standard_normal((4, mesh.n_elems)), device="cuda")
    xb = torch.tensor(rng.standard_normal((mesh.n_nodes, 2)), device="cuda")
    sync = torch.cuda.synchronize
    for _ in range(3):
        s.adjoint_lagrangian_step(dt, qb, xb)
        s.upload_state(Q0, 0.0)
        s.step_gts(dt, 1)
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.adjoint_lagrangian_step(dt, qb, xb)
    sync()
    ms_adj = (time.perf_counter() - t0) / reps * 1e3
    ms_fwd = 0.0
    for _ in range(reps):
        s.upload_state(Q0, 0.0)
        sync()
        t0 = time.perf_counter()
        s.step_gts(dt, 1)
        sync()
        ms_fwd += (time.perf_counter() - t0) / reps * 1e3
    return {"value": ms_adj / ms_fwd, "adjoint_ms": ms_adj, "forward_ms": ms_fwd,
            "workload": f"one global step on the {mesh.n_elems}-triangle explosion, Lagrangian mesh, M={M}"}


def lts_gradient_ratio(n_elems: int = 50_000, M: int = 2, levels: int = 3, n_macro: int = 20, reps: int = 2):
    """The gradient through n_macro LTS macro steps on the mesh moving with
    the fluid (ader_adjoint_lts, its own forward included) against the forward
    run over the same macro steps (ader_step_lts), explosion recipe from t = 0."""
    import numpy as np
    import torch

    from paper_1408_3719_amd import Config, Solver
    from workloads import explosion_case
    mesh, Q0 = explosion_case(n_elems, seed=7)
    s = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=M, levels=levels, mesh_velocity="lagrangian"))
    rng = np.random.default_rng(0)
    qb = torch.tensor(rng.standard_normal((4, mesh.n_elems)), device="cuda")
    xb = torch.tensor(rng.standard_normal((mesh.n_nodes, 2)), device="cuda")
    sync = torch.cuda.synchronize
    t_f = t_g = 0.0
    for k in range(reps + 1):
        s.upload_state(Q0)
        sync()
        t0 = time.perf_counter()
        s.step_lts(1e9, n_macro)
        sync()
        t1 = time.perf_counter()
        s.upload_state(Q0)
        sync()
        t2 = time.perf_counter()
        _, _, done = s.adjoint_lts(n_macro, 1e9, qb, xb)
        sync()
        t3 = time.perf_counter()
        assert done == n_macro
        if k:
            t_f += t1 - t0
            t_g += t3 - t2
    return {"value": t_g / t_f, "gradient_ms": t_g / reps * 1e3, "forward_ms": t_f / reps * 1e3,
            "workload": f"{n_macro} LTS macro steps ({levels} levels) from t = 0 on the {mesh.n_elems}-triangle "
                        f"explosion, Lagrangian mesh, M={M}; the gradient call includes its own forward"}


def mfma_probe(n_elems: int = 400_000, iters: int = 64, reps: int = 5):
    """The predictor's derivative contraction (D_xi, D_eta of the M=2 nodal
    basis on ten fields at six nodes, fed back `iters` times) on the vector
    ALUs and on the matrix cores (ader_probe_contraction), best of `reps`
    launches each; useful work 2 x 12 x 6 x 10 = 1,440 flop per element and
    round (the MFMA variant issues 7 tiles x 2 k-steps x 16x16x4 per ten
    elements, 2,867 flop per element and round, padding included)."""
    import numpy as np
    import torch

    from paper_1408_3719_amd import Config, Solver
    from workloads import vortex_case
    mesh, Q0 = vortex_case(400, seed=5)
    s = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=2, levels=1))
    F = torch.tensor(np.random.default_rng(0).standard_normal((n_elems, 10, 6)), device="cuda")
    out = {}
    res = {}
    for name, mf in (("valu", False), ("mfma", True)):
        best = None
        for _ in range(reps):
            r, ms = s.probe_contraction(F, iters, mf)
            best = ms if best is None else min(best, ms)
        res[name] = r
        useful = 1440.0 * n_elems * iters
        out[name] = {"ms": best, "useful_tflops": useful / (best * 1e-3) / 1e12}
    d = float((res["valu"] - res["mfma"]).abs().max() / res["valu"].abs().max())
    return {"n_elems": n_elems, "rounds": iters, **out, "mfma_over_valu_time": out["mfma"]["ms"] / out["valu"]["ms"],
            "max_rel_difference": d}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["explosion", "vortex", "sod", "batched", "adjoint", "adjoint_lts"],
                    default="explosion")
    ap.add_argument("--instances", type=int, default=256, help="batched workload: instances")
    ap.add_argument("--n-elems", type=int, default=None)
    ap.add_argument("--M", type=int, default=None)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--step-fraction", type=float, default=None,
                    help="nominal finest dyadic step / smallest CFL step (library default if unset)")
    ap.add_argument("--flux", choices=["rusanov", "osher", "hll"], default="rusanov")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: pick launch settings with the library's autotuner before timing")
    ap.add_argument("--free", type=int, default=1,
                    help="1: also run free local steps (levels = 0) over the timed interval")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="1: also time one adjoint step against one forward step (adjoint workload)")
    ap.add_argument("--mesh-velocity", choices=["lagrangian", "eulerian"], default="lagrangian",
                    help="adjoint workload: mesh moving with the fluid, or fixed")
    ap.add_argument("--mfma-probe", type=int, default=1,
                    help="1: time the predictor's derivative contraction on MFMA against VALU")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-elems", type=int, default=None)
    ap.add_argument("--cpu-steps", type=int, default=None)
    ap.add_argument("--traffic-sweep", action="store_true",
                    help="repeat the profiled pass for every workgroups-per-CU setting (counter runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {a.gpus}); "
              "the multi-GPU layout is a design note, not an implementation.", file=sys.stderr)
        sys.exit(2)

    if a.workload == "batched":
        return bench_batched(a)
    if a.workload == "adjoint":
        return bench_adjoint(a)
    if a.workload == "adjoint_lts":
        return bench_adjoint_lts(a)

    import numpy as np  # noqa: F401
    import torch

    from paper_1408_3719_amd import Config, Solver
    from workloads import explosion_case, sod_case, vortex_case

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    # workload defaults: mesh size, order, levels, target time, CPU sample (size, macro steps)
    dflt = {"explosion": (400_000, 2, 4, 0.25, (4000, 6)), "vortex": (80_000, 2, 3, 1.0, (5000, 8)),
            "sod": (2_000, 1, 1, 0.2, (2000, 40))}[a.workload]
    a.n_elems = a.n_elems or dflt[0]
    a.M = a.M or dflt[1]
    a.levels = a.levels or dflt[2]
    t_end = dflt[3]
    if a.workload == "vortex":
        mesh, Q0 = vortex_case(a.n_elems, seed=1)
        desc = "isentropic vortex, {}-triangle 4:1 graded mesh"
    elif a.workload == "explosion":
        mesh, Q0 = explosion_case(a.n_elems, seed=7)
        desc = "EP1 explosion, {}-triangle 8:1 radially graded disk"
    else:
        mesh, Q0 = sod_case(a.n_elems, seed=1408)
        desc = "RP1 shock tube, {}-triangle strip"
    note(f"{a.workload}: {mesh.n_elems} triangles")
    extra = {} if a.step_fraction is None else {"lts_step_fraction": a.step_fraction}
    cfg = Config(M=a.M, levels=a.levels, flux=a.flux, **extra)
    s = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, cfg)
    sync = torch.cuda.synchronize
    tune = s.autotune(2) if a.autotune else None      # state restored: not part of the run
    note(f"autotune {tune}")

    # ---- LTS: warm-up then the timed macro steps --------------------------------
    s.step_lts(t_end, a.warmup)
    st0 = s.stats()
    sync()
    t0 = time.perf_counter()
    s.step_lts(t_end, a.steps)
    sync()
    t_lts = time.perf_counter() - t0
    st1 = s.stats()
    lts_updates = st1["element_updates"] - st0["element_updates"]
    T_a, T_b = st0["t"], st1["t"]
    value = lts_updates / t_lts
    lts = {"updates": lts_updates, "seconds": t_lts, "physical_interval": [T_a, T_b]}
    for k in ("cycles", "extra_cycles", "long_macro_steps", "cfl_overshoots", "macro_steps"):
        lts[k] = st1[k] - st0[k]
    lts["max_gcl_residual"] = st1["max_gcl_residual"]
    note(f"LTS {value / 1e6:.1f} M updates/s over [{T_a:.4g}, {T_b:.4g}]")

    # ---- GTS over the same physical interval [T_a, T_b] ---------------------------
    s.upload_state(Q0, 0.0)
    s.step_gts(T_a)
    s.step_gts(T_a)                    # graph of one level already captured
    g0 = s.stats()
    sync()
    t0 = time.perf_counter()
    s.step_gts(T_b)
    sync()
    t_gts = time.perf_counter() - t0
    g1 = s.stats()
    gts_updates = g1["element_updates"] - g0["element_updates"]
    note(f"GTS {gts_updates / t_gts / 1e6:.1f} M updates/s")

    # ---- free local steps over the same interval (each element at its CFL step) --
    free = None
    if a.free:
        f = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=a.M, levels=0, flux=a.flux))
        if tune:
            f.set_tune(sched_chunk=tune["sched_chunk"], list_wg_per_cu=tune["list_wg_per_cu"],
                       sweep_wg_per_cu=tune["sweep_wg_per_cu"])
        f.step_lts(T_a)
        f0 = f.stats()
        sync()
        t0 = time.perf_counter()
        f.step_lts(T_b)
        sync()
        t_free = time.perf_counter() - t0
        f1 = f.stats()
        fu = f1["element_updates"] - f0["element_updates"]
        free = {"value": fu / t_free, "updates": fu, "seconds": t_free,
                "cycles_launched": f1["cycles"] - f0["cycles"],
                "cfl_overshoots": f1["cfl_overshoots"] - f0["cfl_overshoots"],
                "updates_over_lts": fu / max(lts_updates, 1),
                "time_over_lts": t_free / t_lts}
        del f
        note(f"free steps {fu / t_free / 1e6:.1f} M updates/s")

    # ---- profiled LTS pass: per-kernel times from HIP events ----------------------
    s.upload_state(Q0, 0.0)
    s.step_lts(t_end, a.warmup)
    p0 = s.stats()
    s.set_profiling(True)
    s.step_lts(t_end, a.steps)
    kt = s.kernel_times()
    s.set_profiling(False)
    p1 = s.stats()
    units = {
        "recon": p1["element_updates"] - p0["element_updates"],
        "predict": p1["predictor_evals"] - p0["predictor_evals"],
        "patch": p1["patches"] - p0["patches"],
        "update": p1["element_updates"] - p0["element_updates"],
        "node": p1["node_moves"] - p0["node_moves"],
    }
    units["sched"] = mesh.n_elems * kt["sched"][1]         # every element is a candidate
    source_sha = kernel_source_sha()
    kname = {"recon": "k_reconstruct", "predict": "k_predict", "patch": "k_patch",
             "sched": "k_sched", "node": "k_node", "update": "k_update"}

    def traffic(kernel, units_per_launch):
        axis = "sweep_wg_per_cu" if kernel in ("k_node", "k_patch") else "list_wg_per_cu"
        per = MEASURED_TRAFFIC.get(kernel, {}).get(tune[axis] if tune else 0)
        if (per is None or MEASURED_TRAFFIC["source_sha256"] != source_sha or a.M != 2
                or MEASURED_TRAFFIC.get("workload") != a.workload or a.flux != "rusanov"):
            return None
        return per * units_per_launch

    def alu_roof(k, flops_key):
        per = UNIT_WORK[flops_key][a.M]
        r = rate_entry(per, units[k], kt[k][0], kt[k][1], PEAK_FP64_VECTOR_TFLOPS, 1e12)
        return dict(bound="alu", achieved=r["achieved"], peak=r["peak"], unit="TFLOP/s", frac=r["frac"],
                    traffic=traffic(kname[k], r["units_per_launch"]), kernel=kname[k], flops_per_unit=per,
                    units_per_launch=r["units_per_launch"], launches=r["launches"],
                    avg_launch_us=r["avg_launch_us"],
                    kernel_count_flops_per_unit=(recon_flops(a.M) if k == "recon" else predict_flops(a.M)))

    def hbm_rate(k, bytes_key):
        per = UNIT_WORK[bytes_key][a.M]
        r = rate_entry(per, units[k], kt[k][0], kt[k][1], PEAK_HBM_GBS, 1e9)
        return dict(r, unit="GB/s", bytes_per_unit=per, traffic=traffic(kname[k], r["units_per_launch"]))

    total_ms = sum(v[0] for v in kt.values())
    dom = max(("recon", "predict"), key=lambda k: kt[k][0])
    roof = alu_roof(dom, "recon_flops" if dom == "recon" else "predict_flops")
    fp64_kernels = {kname[k]: alu_roof(k, f) for k, f in (("recon", "recon_flops"), ("predict", "predict_flops"))}
    hbm_kernels = {kname[k]: hbm_rate(k, b) for k, b in (("patch", "patch_bytes"), ("update", "update_bytes"),
                                                         ("node", "node_bytes"), ("sched", "sched_bytes"))}

    if a.traffic_sweep:
        # the profiled pass again for every persistent-grid setting of the
        # list-driven kernels and the sweeps (both at the same setting), in
        # this order, one JSON line each (counter runs)
        chunk = tune["sched_chunk"] if tune else 0
        for w in TRAFFIC_SWEEP:
            s.set_tune(sched_chunk=chunk, list_wg_per_cu=w, sweep_wg_per_cu=w)
            s.upload_state(Q0, 0.0)
            s.step_lts(t_end, a.warmup)
            q0 = s.stats()
            s.set_profiling(True)
            s.step_lts(t_end, a.steps)
            kq = s.kernel_times()
            s.set_profiling(False)
            q1 = s.stats()
            print(json.dumps({"traffic_sweep": w, "launches": {k: kq[k][1] for k in kq},
                              "units": {"recon": q1["element_updates"] - q0["element_updates"],
                                        "predict": q1["predictor_evals"] - q0["predictor_evals"],
                                        "patch": q1["patches"] - q0["patches"],
                                        "node": q1["node_moves"] - q0["node_moves"]}}),
                  flush=True)
        if tune:
            s.set_tune(sched_chunk=tune["sched_chunk"], list_wg_per_cu=tune["list_wg_per_cu"],
                       sweep_wg_per_cu=tune["sweep_wg_per_cu"])

    if a.calib_copy_mib:
        n = a.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        sync()
    del s

    adj = adj_lag = adj_lts = None
    if a.adjoint:
        adj = adjoint_step_ratio()
        note(f"adjoint/forward per step {adj['value']:.3f}")
        adj_lag = lagrangian_adjoint_step_ratio()
        note(f"moving-mesh adjoint/forward per step {adj_lag['value']:.3f}")
        adj_lts = lts_gradient_ratio()
        note(f"LTS gradient/forward over {adj_lts['workload'].split()[0]} macro steps {adj_lts['value']:.3f}")

    probe = mfma_probe() if a.mfma_probe else None
    if probe:
        note(f"contraction probe: VALU {probe['valu']['ms']:.3f} ms, MFMA {probe['mfma']['ms']:.3f} ms")

    cpu = None
    if not a.no_cpu_baseline:
        ce, cs = dflt[4]
        cpu = cpu_baseline_case(a.workload, a.cpu_elems or ce, a.M, a.levels, a.cpu_steps or cs, t_end)
        note(f"cpu oracle {cpu['value']:.0f} updates/s")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "element-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": t_lts / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc.format(mesh.n_elems) + f", M={a.M}, LTS {a.levels} levels vs GTS, "
                        f"{a.flux} flux, Lagrangian mesh motion, t from 0 (first {a.warmup} macro steps untimed)",
            "flux": a.flux,
            "n_elems": mesh.n_elems, "M": a.M, "levels": a.levels,
            "lts_step_fraction": cfg.lts_step_fraction,
            "parallelism": "single GPU",
        },
        "gts": {"value": gts_updates / t_gts, "updates": gts_updates, "seconds": t_gts},
        "lts": lts,
        "lts_time_to_solution_speedup": t_gts / t_lts,
        "gts_over_lts_updates": gts_updates / max(lts_updates, 1),
        "free_steps": free,
        "adjoint_forward": adj,
        "adjoint_lagrangian_forward": adj_lag,
        "adjoint_lts_forward": adj_lts,
        "autotune": tune,
        "kernel_ms": {k: round(v[0], 3) for k, v in kt.items()},
        "kernel_launches": {k: v[1] for k, v in kt.items()},
        "work_units": units,
        "kernel_share": {k: round(v[0] / total_ms, 3) for k, v in kt.items()},
        "roofline": roof,
        "fp64_kernels": fp64_kernels,
        "hbm_kernels": hbm_kernels,
        "mfma": {"used": False, "utilisation": 0.0,
                 "note": "no kernel of the step issues MFMA instructions; the probe times the predictor's "
                         "derivative contraction on the matrix cores against the vector ALUs",
                 "probe": probe},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
