#!/usr/bin/env python3
"""Hubbard steps/s on one MI355X (one step = project + occupations + ACBN0
U/J + apply, for every site, k-point, spin and state).

Default workload: the batched real-time loop (36 bohr cube, 120^3 grid,
64 uneven p/d/f sites on a 4x4x4 lattice, 1024 real Gamma-point states,
f = 1 for 512), synthetic states; between steps the FP64 master states are
rotated (Givens rotations of angle ~1e-3, the synthetic propagator) and
converted to FP32, outside the timed region.  ``value`` is the FP32-storage
path (FP64 orbital table, FP64 sums) run as one captured hipGraph per step;
the plain FP64 path (one launch per site and stage, no graph) and the FP64
graph path are timed beside it.  The FP32 gate: occupations and U/J of the
FP32 path against the FP64 oracle run on the FP64 master states (the CPU
leg), at most 1e-9 absolute; a failed gate withholds ``value``.  The
NiO-like collinear antiferromagnet (48^3, 2 Ni d + 2 O p, 2x2x2 k-points, 64
complex states per k and spin) is measured beside it (``detail.side``).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
Prints one JSON line.
"""

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
# velocity-gauge runs: no current; the current from the step's own
# projection pass (hub_step_current); the current as a call of its own after
# the step (hub_current)
GAUGE_RUNS = (("gauge_steps_per_s", None), ("gauge_current_steps_per_s", "step"),
              ("gauge_current_separate_steps_per_s", "separate"))
# sources of the projection and apply kernels (the counter files record
# their hash: traffic measured on other sources is not reported)
KERNEL_SOURCES = ["kcommon.h", "k_project.h", "k_project_f32.hip", "k_project_f64.hip", "k_apply.h",
                  "k_apply_f32.hip", "k_apply_f64.hip", "k_apply_grouped_f32.hip", "k_apply_grouped_f64.hip"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="rt_batched",
                    choices=["nio_afm", "rt_batched", "gamma_d", "spinor_layers", "forces_fcc"])
    ap.add_argument("--side", default="nio_afm",
                    help="second workload summarized in detail.side (FP32 graph steps/s, stage rates, velocity "
                         "gauge); 'none' skips it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="time only the FP32 graph path")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="whole oracle steps timed (default 3; 1 for the three large workloads)")
    ap.add_argument("--cpu-single-thread", action="store_true",
                    help="also time one oracle step on one host thread")
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel shapes")
    ap.add_argument("--chunk", type=int, default=None, help="sphere entries per work-list chunk")
    ap.add_argument("--classes", default="merged", choices=["merged", "sequential", "concurrent"],
                    help="launch policy of the grouped work list's function-count classes")
    ap.add_argument("--worklist", default="grouped", choices=["grouped", "persite"],
                    help="batched work list: every grid point once with all its covers, or per-site layers")
    ap.add_argument("--shapes", default=None,
                    help="fixed kernel shapes PCPL,PWAVES,PLAYOUT,ACPL,AWAVES,ALAYOUT instead of autotuning "
                         "(profiling runs use the shapes the autotuner picked)")
    ap.add_argument("--no-gauge", action="store_true",
                    help="skip the velocity-gauge timing (complex workloads)")
    ap.add_argument("--rc-sweep", default=None,
                    help="instead of the bench line: steps/s and grid points against the sphere radius of the "
                         "d shells (comma-separated radii in bohr; 'cell' and 'tN' (threshold 1e-N) select a "
                         "radius by the Sec. II methods)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB three times (counter calibration)")
    return ap.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_08935_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def union_points(hub):
    import numpy as np
    gs = [hub.site_points(s)[0] for s in range(hub.nsites)]
    return int(np.unique(np.concatenate(gs)).size)


def time_steps(hub, psi, f, hpsi, mode, steps, warmup, bufs, rotate=None):
    """Wall-clock (and HIP-event) time of ``steps`` Hubbard steps.  With
    ``rotate`` the states change between steps and only the Hubbard steps are
    timed (events around each step on the current stream)."""
    import torch
    for _ in range(warmup):
        hub.step(psi, f, hpsi, mode=mode, bufs=bufs)
    torch.cuda.synchronize()
    if rotate is None:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            hub.step(psi, f, hpsi, mode=mode, bufs=bufs)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, e0.elapsed_time(e1) / 1e3
    evs = []
    t0 = time.perf_counter()
    for i in range(steps):
        rotate(i)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        hub.step(psi, f, hpsi, mode=mode, bufs=bufs)
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, sum(a.elapsed_time(b) for a, b in evs) / 1e3


def apply_block(cfg):
    """State columns per block of the oracle's V_U psi, so that one block's
    complex output stays within about 2 GB of host memory."""
    ncomp = 2 if cfg.spin == "spinor" else 1
    per_col = cfg.nq * cfg.G * 16 * ncomp
    return int(max(1, min(cfg.nstates, 2e9 // per_col)))


def cpu_baseline(cfg, psi_host, f, nsteps):
    """The FP64 oracle (sphere form) timed on the host cores: whole steps
    (every site, set and state), V_U psi evaluated in column blocks.  Returns
    (median seconds per step, BLAS threads, the last step's results)."""
    from threadpoolctl import threadpool_info

    from oracle import projection as OP
    from oracle import step as OS
    from tests.helpers import to_system
    sys_ = to_system(cfg)
    sps = OP.all_spheres(sys_)
    t0 = time.perf_counter()
    tens = OS.site_tensors(sys_, sps)
    log(f"oracle Coulomb tensors (setup, untimed): {time.perf_counter() - t0:.1f} s")
    block = apply_block(cfg)
    times = []
    ref = None
    for i in range(nsteps):
        t0 = time.perf_counter()
        ref = OS.hubbard_step(sys_, psi_host, f, sps, tens, form="sphere", apply_block=block)
        times.append(time.perf_counter() - t0)
        log(f"oracle step {i}: {times[-1]:.2f} s (V_U psi in blocks of {block} columns)")
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return statistics.median(times), threads, ref, block


def gate_errors(hub, b32, ref):
    """max |n - n_oracle| over every site and block, and max |U - U_oracle|,
    |J - J_oracle| (Hartree): the FP32 path's results against the oracle's."""
    import numpy as np
    n = b32["n"].cpu().numpy()
    dn = 0.0
    for I in range(hub.nsites):
        L = hub.site_L[I]
        r = np.asarray(ref["n"][I])
        if hub.spin == "spinor":
            g = np.array([[n[I][2 * s_ + t, :L, :L] for t in range(2)] for s_ in range(2)])
        else:
            g = n[I][:, :L, :L]
        dn = max(dn, float(np.max(np.abs(g - r))))
    du = max(float(np.max(np.abs(b32["U"].cpu().numpy() - ref["U"]))),
             float(np.max(np.abs(b32["J"].cpu().numpy() - ref["J"]))))
    return dn, du


def cpu_single_thread(cfg, psi_host, f):
    """One oracle step with the BLAS pools held to one thread, and the host
    it ran on."""
    from threadpoolctl import threadpool_limits

    from oracle import projection as OP
    from oracle import step as OS
    from tests.helpers import to_system
    sys_ = to_system(cfg)
    sps = OP.all_spheres(sys_)
    tens = OS.site_tensors(sys_, sps)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        OS.hubbard_step(sys_, psi_host, f, sps, tens, form="sphere")
        t = time.perf_counter() - t0
    log(f"oracle step, one thread: {t:.2f} s")
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"oracle_single_thread_steps_per_s": round(1.0 / t, 4), "host_cpu": model,
            "host_cpus_visible": os.cpu_count()}


def rc_sweep(args):
    """Sphere-radius sweep (Sec. II, the radius discussion and its figure of
    grid points against the d-orbital radius): the d shells of the workload
    take each radius in turn, the other shells keep theirs; U_eff is fixed
    (as in the paper's sweep), so no Coulomb tensors are built.  Per radius:
    points per d sphere, union of covered points, passes of the grouped
    apply (points with more than 16 functions are split over passes), graph
    steps/s and the algorithmic bytes of project + apply per second."""
    import numpy as np
    import torch

    import paper_1711_08935_amd as H
    from paper_1711_08935_amd.tune import autotune
    from synth import make_config, make_occupations, make_states

    cfg = make_config(args.workload)
    dsites = [i for i, s in enumerate(cfg.sites) if s["l"] == 2]
    psi64 = make_states(cfg, device="cuda")
    f_d = torch.from_numpy(make_occupations(cfg)).cuda()
    esz = 8 if cfg.is_complex else 4
    ncol = cfg.nstates * (2 if cfg.spin == "spinor" else 1)
    out = []
    for tok in args.rc_sweep.split(","):
        d0 = cfg.sites[dsites[0]]
        if tok == "cell":
            rc, how = H.sphere_radius("cell", cell=cfg.cell), "cell"
        elif tok.startswith("t"):
            rc, how = H.sphere_radius("threshold", l=2, zeta=d0["zeta"], threshold=10.0 ** (-int(tok[1:]))), tok
        else:
            rc, how = float(tok), "given"
        sites = [dict(s, rc=rc) if i in dsites else s for i, s in enumerate(cfg.sites)]
        hub = H.Hubbard(cfg.cell, cfg.ngrid, sites, kpts=cfg.kpts, kweights=cfg.kweights, spin=cfg.spin,
                        is_complex=cfg.is_complex, precision="f32", chunk=args.chunk)
        for i in range(len(sites)):
            hub.set_fixed_ueff(i, 0.15)
        psi = psi64.to(hub.state_dtype)
        bufs = hub.step_buffers(cfg.nstates)
        h = torch.zeros_like(psi)
        hub.step(psi, f_d, h, mode="batched", bufs=bufs)
        if not args.no_tune:
            autotune(hub, psi, bufs["c"], bufs["n"], bufs["Ueff"])
        wall, ev = time_steps(hub, psi, f_d, h, "graph", args.steps, args.warmup, bufs)
        pts = union_points(hub)
        alg = 3 * pts * ncol * esz * hub.nsets
        row = {"rc": round(rc, 4), "method": how, "points_per_d_sphere": int(hub.site_npts[dsites[0]]),
               "union_points": pts, "grouped_passes": hub.query(14), "functions_per_point_max": hub.query(12),
               "steps_per_s": round(args.steps / ev, 2), "step_GBs": round(alg / (ev / args.steps) / 1e9, 1)}
        log(str(row))
        out.append(row)
        del hub, psi, bufs, h
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "Hubbard steps/s against the d-sphere radius", "unit": "Hubbard steps/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "dtype": "f64",
                      "data": "synthetic", "config": {"workload": cfg.name, "grid": list(cfg.ngrid),
                                                      "storage": "f32 states", "ueff": "fixed 0.15 Ha"},
                      "sweep": out}))


def side_summary(name, args):
    """FP32 graph steps/s of a second workload with the kernel shapes the
    autotuner picks for it, the projection's and apply's fractions of peak
    HBM bandwidth (library HIP events around each stage, algorithmic bytes
    over the union of sphere points), and for complex workloads the velocity
    gauge without and with the DFT+U current every step."""
    import numpy as np
    import torch

    import paper_1711_08935_amd as H
    from paper_1711_08935_amd.tune import autotune
    from synth import make_config, make_occupations, make_states

    cfg = make_config(name)
    log(f"side workload {name}")
    psi = make_states(cfg, device="cuda")
    f_d = torch.from_numpy(make_occupations(cfg)).cuda()
    hub = H.Hubbard(cfg.cell, cfg.ngrid, cfg.sites, kpts=cfg.kpts, kweights=cfg.kweights, spin=cfg.spin,
                    is_complex=cfg.is_complex, precision="f32", chunk=args.chunk)
    psi = psi.to(hub.state_dtype)
    hub.coulomb(-1)
    S = cfg.nstates
    bufs = hub.step_buffers(S)
    h = torch.zeros_like(psi)
    hub.step(psi, f_d, h, mode="batched", bufs=bufs)
    if not args.no_tune:
        autotune(hub, psi, bufs["c"], bufs["n"], bufs["Ueff"])
    _, ev = time_steps(hub, psi, f_d, h, "graph", args.steps, args.warmup, bufs)
    out = {"workload": name, "steps_per_s": round(args.steps / ev, 2)}
    hub.profile(True)
    for _ in range(max(5, min(args.steps, 30))):
        hub.step(psi, f_d, h, mode="batched", bufs=bufs)
    pr = hub.profile_read()
    hub.profile(False)
    proj_bytes = union_points(hub) * hub.ncol(S) * psi.element_size() * hub.nsets
    for k, b in (("project", proj_bytes), ("apply", 2 * proj_bytes)):
        ms = pr[k][0] / max(1, pr[k][1])
        out[f"{k}_ms"] = round(ms, 4)
        out[f"{k}_frac"] = round(b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    out["small_kernels_us"] = round(1e3 * sum(pr[k][0] / max(1, pr[k][1])
                                              for k in ("reduce", "nbar", "occupations", "acbn0")), 1)
    if cfg.is_complex and not args.no_gauge:
        A0 = np.array([0.05, 0.02, 0.0])
        jcur = torch.empty((hub.nsites, 3), dtype=torch.float64, device="cuda")
        for key, with_current in GAUGE_RUNS:
            def run(nsteps, i0):
                for i in range(nsteps):
                    hub.set_vector_potential(A0 * np.sin(0.1 * (i0 + i)))
                    hub.step(psi, f_d, h, mode="graph", bufs=bufs, current=jcur if with_current == "step" else None)
                    if with_current == "separate":
                        hub.current(psi, bufs["c"], f_d, bufs["Ueff"], bufs["n"])
            run(3, 0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run(args.steps, 3)
            e1.record()
            torch.cuda.synchronize()
            out[key] = round(args.steps / (e0.elapsed_time(e1) * 1e-3), 2)
        hub.set_vector_potential(None)
    log(f"side workload: {out}")
    del hub, psi, bufs, h
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this library runs on one GPU; sharding over GPUs is a design only, "
                          "so --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.rc_sweep:
        rc_sweep(args)
        return
    import numpy as np
    import torch

    import paper_1711_08935_amd as H
    from paper_1711_08935_amd.tune import autotune, autotune_steps
    from synth import make_config, make_occupations, make_states

    cfg = make_config(args.workload)
    log(f"workload {cfg.name}: grid {cfg.ngrid}, {len(cfg.sites)} sites, {cfg.nk} k, spin {cfg.spin}, "
        f"{cfg.nstates} states")
    t0 = time.perf_counter()
    psi64 = make_states(cfg, device="cuda")
    f = make_occupations(cfg)
    f_d = torch.from_numpy(f).cuda()
    torch.cuda.synchronize()
    log(f"states generated in {time.perf_counter() - t0:.1f} s")

    def ctx(prec):
        hub = H.Hubbard(cfg.cell, cfg.ngrid, cfg.sites, kpts=cfg.kpts, kweights=cfg.kweights, spin=cfg.spin,
                        is_complex=cfg.is_complex, precision=prec, chunk=args.chunk)
        hub.set_worklist(args.worklist == "grouped")
        hub.set_class_launch(args.classes)
        return hub

    hub32 = ctx("f32")
    psi32 = psi64.to(hub32.state_dtype)
    S = cfg.nstates
    t0 = time.perf_counter()
    hub32.coulomb(-1)
    torch.cuda.synchronize()
    coulomb_s = time.perf_counter() - t0
    log(f"Coulomb tensors (setup) {coulomb_s * 1e3:.1f} ms")

    rotate = None
    if cfg.name == "rt_batched":
        half = S // 2
        rng = np.random.default_rng(cfg.seed + 100)
        theta = torch.from_numpy(1e-3 * rng.uniform(0.5, 1.0, size=half) * rng.choice([-1.0, 1.0], size=half)).cuda()
        cth, sth = torch.cos(theta), torch.sin(theta)

        def rotate(i):
            # synthetic propagator: Givens rotation of state pairs (i, i + S/2)
            a = psi64[:, :, :half].clone()
            b = psi64[:, :, half:2 * half]
            psi64[:, :, :half] = cth * a - sth * b
            psi64[:, :, half:2 * half] = sth * a + cth * b
            psi32.copy_(psi64)

    bufs32 = hub32.step_buffers(S)
    hpsi32 = torch.zeros_like(psi32)
    tuned = None
    if args.shapes:
        v = [int(x) for x in args.shapes.split(",")]
        pc, pw, ps, ac, aw, asp = v if len(v) == 6 else (v[0], v[1], -1, v[2], v[3], -1)
        hub32.set_tuning(0, pc, pw, ps)
        hub32.set_tuning(1, ac, aw, asp)
        log(f"fixed shapes: project {pc}x{pw} layout {ps}, apply {ac}x{aw} layout {asp}")
    elif not args.no_tune:
        # setup: fill the step buffers once, then pick kernel shapes on them
        hub32.step(psi32, f_d, hpsi32, mode="batched", bufs=bufs32)
        tuned = autotune(hub32, psi32, bufs32["c"], bufs32["n"], bufs32["Ueff"])
        log(f"autotune: project {tuned['project']}, apply {tuned['apply']}")
    wall, ev = time_steps(hub32, psi32, f_d, hpsi32, "graph", args.steps, args.warmup, bufs32, rotate)
    hub_time = ev if rotate is not None else wall
    value = args.steps / hub_time
    log(f"f32 graph: {value:.1f} steps/s ({hub_time / args.steps * 1e3:.3f} ms/step, wall {wall:.3f} s)")

    forces_on = {}
    if cfg.name == "forces_fcc":
        # Hubbard forces (Sec. IV) after every step, eager launches: the
        # orbital-gradient form (<grad phi|psi>) and the state-gradient form
        # (<phi|D psi> over the dilated spheres), each with the force contraction
        for form in ("orbital", "state"):
            for _ in range(2):
                hub32.step(psi32, f_d, hpsi32, mode="graph", bufs=bufs32)
                hub32.forces(psi32, bufs32["c"], f_d, bufs32["Ueff"], bufs32["n"], form=form)
            torch.cuda.synchronize()
            fe0, fe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            fe0.record()
            for _ in range(args.steps):
                hub32.step(psi32, f_d, hpsi32, mode="graph", bufs=bufs32)
                hub32.forces(psi32, bufs32["c"], f_d, bufs32["Ueff"], bufs32["n"], form=form)
            fe1.record()
            torch.cuda.synchronize()
            forces_on[form] = args.steps / (fe0.elapsed_time(fe1) * 1e-3)
            log(f"f32 graph step + forces ({form} gradient): {forces_on[form]:.1f} steps/s")
        # per-stage times of the force calls alone: gradient projection (state
        # rows of every sphere / dilated-sphere entry plus the 3L table values),
        # its reduction and the contraction
        row = cfg.nstates * (8 if cfg.is_complex else 4)
        forces_stages = {}
        for form, q in (("orbital", 4), ("state", 13)):
            hub32.profile(True)
            for _ in range(20):
                hub32.forces(psi32, bufs32["c"], f_d, bufs32["Ueff"], bufs32["n"], form=form)
            pr = hub32.profile_read()
            hub32.profile(False)
            entries = hub32.query(q)
            L = hub32.site_L[0]
            alg = entries * hub32.nsets * (row + 3 * L * 8)
            ms = pr["gradproject"][0] / max(1, pr["gradproject"][1])
            forces_stages[form] = {"gradproject_ms": round(ms, 4), "reduce_ms": round(pr["reduce"][0] / 20, 4),
                                   "forces_ms": round(pr["forces"][0] / 20, 4), "entries": int(entries),
                                   "gradproject_GBs": round(alg / (ms * 1e-3) / 1e9, 1)}
        log(f"force stages: {forces_stages}")

    gauge = None
    if cfg.is_complex and not args.no_gauge:
        # real-time velocity gauge (Sec. V): a new uniform A(t) before every
        # step (device tables updated on the stream, then the graph replay),
        # without and with the DFT+U current correction per step
        A0 = np.array([0.05, 0.02, 0.0])

        def field(i):
            return A0 * np.sin(0.1 * i)

        jcur = torch.empty((hub32.nsites, 3), dtype=torch.float64, device="cuda")

        def run(nsteps, with_current, i0):
            for i in range(nsteps):
                hub32.set_vector_potential(field(i0 + i))
                hub32.step(psi32, f_d, hpsi32, mode="graph", bufs=bufs32,
                           current=jcur if with_current == "step" else None)
                if with_current == "separate":
                    hub32.current(psi32, bufs32["c"], f_d, bufs32["Ueff"], bufs32["n"])

        gauge = {}
        for key, with_current in GAUGE_RUNS:
            run(3, with_current, 0)
            torch.cuda.synchronize()
            ge0, ge1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ge0.record()
            run(args.steps, with_current, 3)
            ge1.record()
            torch.cuda.synchronize()
            gauge[key] = round(args.steps / (ge0.elapsed_time(ge1) * 1e-3), 2)
        # per-stage times under a field (batched steps, library HIP events)
        hub32.set_vector_potential(A0)
        hub32.profile(True)
        for _ in range(max(5, min(args.steps, 30))):
            hub32.step(psi32, f_d, hpsi32, mode="batched", bufs=bufs32)
        gprof = hub32.profile_read()
        # and with the current taken in the step's projection pass: every
        # stage's average time per step (ms)
        for _ in range(max(5, min(args.steps, 30))):
            hub32.step(psi32, f_d, hpsi32, mode="batched", bufs=bufs32, current=jcur)
        cprof = hub32.profile_read()
        gauge["current_step_stage_ms"] = {k: round(v[0] / max(5, min(args.steps, 30)), 4)
                                          for k, v in cprof.items() if v[1]}
        hub32.profile(False)
        hub32.set_vector_potential(None)
        log(f"velocity gauge: {gauge}")

    spindep = None
    if cfg.spin == "spinor":
        # spin-dependent spinor orbitals (App. A): spin-down exponents
        # (d 2.0 -> 2.6, p 1.4 -> 1.1), fixed U_eff, per-site work list; beside
        # it the spin-independent context on the same per-site list
        sd_sites = [dict(s, zeta_dn=(s["zeta"] + 0.6 if s["l"] == 2 else s["zeta"] - 0.3)) for s in cfg.sites]
        hsd = H.Hubbard(cfg.cell, cfg.ngrid, sd_sites, kpts=cfg.kpts, kweights=cfg.kweights, spin=cfg.spin,
                        is_complex=cfg.is_complex, precision="f32", chunk=args.chunk)
        for i in range(hsd.nsites):
            hsd.set_fixed_ueff(i, 0.15)
        bsd = hsd.step_buffers(S)
        hsd_out = torch.zeros_like(psi32)
        hsd.step(psi32, f_d, hsd_out, mode="batched", bufs=bsd)
        if not args.no_tune:
            autotune(hsd, psi32, bsd["c"], bsd["n"], bsd["Ueff"])
        _, sd_ev = time_steps(hsd, psi32, f_d, hsd_out, "graph", args.steps, args.warmup, bsd)
        hsd.profile(True)
        for _ in range(max(5, min(args.steps, 30))):
            hsd.step(psi32, f_d, hsd_out, mode="batched", bufs=bsd)
        sd_prof = hsd.profile_read()
        hsd.profile(False)
        hub32.set_worklist(False)
        _, ps_ev = time_steps(hub32, psi32, f_d, hpsi32, "graph", args.steps, args.warmup, bufs32)
        hub32.set_worklist(args.worklist == "grouped")
        spindep = {"steps_per_s": round(args.steps / sd_ev, 2),
                   "spin_independent_persite_steps_per_s": round(args.steps / ps_ev, 2)}
        log(f"spin-dependent orbitals: {spindep}")
        del hsd, bsd, hsd_out

    if args.calibrate_copy_mb > 0:
        n = args.calibrate_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 3 x {args.calibrate_copy_mb} MiB")
        del src, dst

    # reference: a plain device-to-device copy of 2 GiB (read + write)
    src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_GBs = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    detail = {"coulomb_setup_ms": round(coulomb_s * 1e3, 2), "device_copy_GBs": round(copy_GBs, 1)}
    if gauge is not None:
        detail.update(gauge)
    if forces_on:
        detail["forces_off_steps_per_s"] = round(value, 2)
        detail["forces_on_steps_per_s"] = round(forces_on["orbital"], 2)
        detail["forces_state_gradient_on_steps_per_s"] = round(forces_on["state"], 2)
        detail["force_stages"] = forces_stages
    if tuned is not None:
        detail["tuned_shapes"] = {"project": list(tuned["project"][0]), "apply": list(tuned["apply"][0]),
                                  "candidates_ms": tuned["table"]}
    # ---------------------------------------------------------- profile pass
    hub32.profile(True)
    for _ in range(max(5, min(args.steps, 30))):
        hub32.step(psi32, f_d, hpsi32, mode="batched", bufs=bufs32)
    prof = hub32.profile_read()
    hub32.profile(False)
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}
    detail["stage_avg_ms_f32"] = {k: round(v, 4) for k, v in stage_ms.items() if v > 0}
    U_pts = union_points(hub32)
    ncol = hub32.ncol(S)
    esz = psi32.element_size()
    proj_bytes = U_pts * ncol * esz * hub32.nsets               # psi read at every sphere point once
    apply_bytes = 2 * proj_bytes                                # hpsi read + write
    detail["algorithmic_bytes_per_step"] = int(proj_bytes + apply_bytes)
    for tag, pr in (("gauge", gprof if gauge is not None else None),
                    ("spin_dependent", sd_prof if spindep is not None else None)):
        if pr is None:
            continue
        rates = {}
        for k, b in (("project", proj_bytes), ("apply", apply_bytes)):
            ms = pr[k][0] / max(1, pr[k][1])
            rates[f"{k}_ms"] = round(ms, 4)
            rates[f"{k}_GBs"] = round(b / (ms * 1e-3) / 1e9, 1)
        if tag == "gauge":
            detail["gauge_stages"] = rates
        else:
            spindep.update(rates)
    if spindep is not None:
        detail["spin_dependent_orbitals"] = spindep
    detail["step_GBs"] = round((proj_bytes + apply_bytes) * value / 1e9, 1)
    grouped = args.worklist == "grouped"
    kernels = {
        "project": (proj_bytes, stage_ms["project"], "k_project (row gather + FP64 contraction)"),
        "apply": (apply_bytes, stage_ms["apply"],
                  ("k_apply_grouped" if grouped else "k_apply") + " (row read-modify-write, FP64 sums)"),
    }
    for k, (b, ms, _) in kernels.items():
        detail[f"{k}_GBs"] = round(b / (ms * 1e-3) / 1e9, 1)
        detail[f"{k}_frac"] = round(b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    # the roofline entry describes the kernel with the longest stage time
    dom = max(kernels, key=lambda k: kernels[k][1])
    b, ms, name = kernels[dom]
    achieved = b / (ms * 1e-3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"traffic_{dom}_{cfg.name}.json")
    if os.path.exists(tf):
        with open(tf) as fh:
            tr = json.load(fh)
        if tr.get("kernel_hash") == kernel_hash() and tr.get("worklist", "grouped") == args.worklist:
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": name,
                "bytes_per_launch": int(b), "avg_launch_ms": round(ms, 4)}

    # ------------------------------------------------ FP64 comparison paths
    if not args.no_compare:
        hub64 = ctx("f64")
        hub64.coulomb(-1)
        bufs64 = hub64.step_buffers(S)
        hpsi64 = torch.zeros_like(psi64)
        if not args.no_tune:
            hub64.step(psi64, f_d, hpsi64, mode="batched", bufs=bufs64)
        k64 = max(5, args.steps // 2)
        # where the speedup comes from: the FP64 paths' projection and apply
        # time per step against the same union-point bytes at FP64 storage
        esz64 = psi64.element_size()
        bytes64 = {"project": U_pts * ncol * esz64 * hub64.nsets, "apply": 2 * U_pts * ncol * esz64 * hub64.nsets}

        def fp64_path(mode):
            """Steps/s of one FP64 path with shapes tuned for it (whole
            per-site steps for the plain path), and its stage rates."""
            if not args.no_tune:
                if mode == "persite":
                    autotune_steps(hub64, psi64, f_d, hpsi64, bufs64, mode="persite")
                else:
                    autotune(hub64, psi64, bufs64["c"], bufs64["n"], bufs64["Ueff"])
            w, e = time_steps(hub64, psi64, f_d, hpsi64, mode, k64, 2, bufs64, rotate)
            rate = k64 / (e if rotate is not None else w)
            hub64.profile(True)
            for _ in range(k64):
                hub64.step(psi64, f_d, hpsi64, mode="persite" if mode == "persite" else "batched", bufs=bufs64)
            pr = hub64.profile_read()
            hub64.profile(False)
            rates = {}
            for k, b in bytes64.items():
                ms = pr[k][0] / k64
                rates[f"{k}_ms_per_step"] = round(ms, 4)
                rates[f"{k}_launches_per_step"] = pr[k][1] // k64
                rates[f"{k}_frac"] = round(b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
            return rate, rates

        plain, detail["fp64_plain_stages"] = fp64_path("persite")
        g64, detail["fp64_batched_stages"] = fp64_path("graph")
        log(f"f64 plain per-site: {plain:.1f} steps/s, f64 graph: {g64:.1f} steps/s")
        detail.update(fp64_plain_steps_per_s=round(plain, 2), fp64_graph_steps_per_s=round(g64, 2),
                      speedup_vs_fp64_plain=round(value / plain, 3))
        # accuracy: one step of each path on the current master states
        b32 = hub32.step(psi32, f_d, torch.zeros_like(psi32), mode="batched", bufs=hub32.step_buffers(S))
        b64 = hub64.step(psi64, f_d, torch.zeros_like(psi64), mode="batched", bufs=hub64.step_buffers(S))
        up = psi32.to(psi64.dtype)
        b64r = hub64.step(up, f_d, torch.zeros_like(up), mode="batched", bufs=hub64.step_buffers(S))
        torch.cuda.synchronize()
        d_end = (b32["n"] - b64["n"]).abs().max().item()
        d_ar = (b32["n"] - b64r["n"]).abs().max().item()
        du = max((b32["U"] - b64["U"]).abs().max().item(), (b32["J"] - b64["J"]).abs().max().item())
        du_ar = max((b32["U"] - b64r["U"]).abs().max().item(), (b32["J"] - b64r["J"]).abs().max().item())
        detail.update(f32_occ_err_vs_gpu_f64_master=d_end, f32_occ_err_arithmetic=d_ar,
                      f32_uj_err_vs_gpu_f64_master=du, f32_uj_err_arithmetic=du_ar)
        log(f"f32 occupation error: vs GPU FP64 path on the master {d_end:.2e}, arithmetic {d_ar:.2e}; "
            f"U/J {du:.2e} / {du_ar:.2e}")
        del hub64, b64, b64r, up
    else:
        b32 = hub32.step(psi32, f_d, torch.zeros_like(psi32), mode="batched", bufs=hub32.step_buffers(S))
        torch.cuda.synchronize()

    # ---------------------------------------------------------- CPU oracle
    # The oracle timed on the host cores, on the FP64 master states that the
    # FP32 path's last accuracy step was rounded from; its n, U and J are the
    # reference of the FP32 gate.
    cpu = None
    gate = {"bar": 1e-9, "reference": None}
    if not args.no_cpu_baseline:
        psi_host = psi64.cpu().numpy()
        nsteps = args.cpu_steps or (1 if cfg.name in ("rt_batched", "spinor_layers", "forces_fcc") else 3)
        t_step, threads, ref, block = cpu_baseline(cfg, psi_host, f, nsteps)
        cpu = {"value": round(1.0 / t_step, 4), "unit": "Hubbard steps/s", "cores": threads, "kind": "oracle",
               "sample": f"median of {nsteps} whole FP64 oracle step(s) (sphere form: all {hub32.nsets} state "
                         f"sets, {S} states, {len(cfg.sites)} sites; V_U psi in blocks of {block} columns to bound "
                         f"host memory) on the FP64 master states of the last GPU step; Coulomb setup excluded"}
        dn, duj = gate_errors(hub32, b32, ref)
        gate.update(reference="FP64 oracle on the FP64 master states", occ_err=dn, uj_err=duj,
                    passed=bool(dn <= 1e-9 and duj <= 1e-9))
        log(f"FP32 gate vs oracle: max|dn| {dn:.2e}, max|dU|,|dJ| {duj:.2e} (bar 1e-9)")
        if args.cpu_single_thread:
            detail.update(cpu_single_thread(cfg, psi_host, f))
        del psi_host, ref
    elif "f32_occ_err_vs_gpu_f64_master" in detail:
        gate.update(reference="GPU FP64 path (pinned to the oracle by the GPU tests) on the FP64 master states",
                    occ_err=detail["f32_occ_err_vs_gpu_f64_master"], uj_err=detail["f32_uj_err_vs_gpu_f64_master"])
        gate["passed"] = bool(gate["occ_err"] <= 1e-9 and gate["uj_err"] <= 1e-9)
    detail["fp32_gate"] = gate
    del b32

    if args.side != "none" and args.side != cfg.name:
        del hub32, bufs32, hpsi32, psi32, psi64
        torch.cuda.empty_cache()
        detail["side"] = side_summary(args.side, args)

    out = {
        "metric": "Hubbard steps/s (project+occ+U/J+apply), FP32-split vs FP64 at 1e-9 occ err",
        "value": round(value, 2) if gate.get("passed", True) else None, "unit": "Hubbard steps/s", "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(hub_time / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": {"workload": cfg.name, "grid": list(cfg.ngrid), "sites": len(cfg.sites),
                                        "kpoints": cfg.nk, "spin": cfg.spin, "states": S,
                                        "mode": "hipGraph per step", "storage": "f32 states, f64 orbital table",
                                        "worklist": args.worklist, "chunk": args.chunk or 512,
                                        "classes": args.classes,
                                        "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "detail": detail,
    }
    if not gate.get("passed", True):
        out["error"] = "FP32 gate failed: occupations or U/J of the FP32 path differ from the reference by more " \
                       "than 1e-9; value withheld"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
