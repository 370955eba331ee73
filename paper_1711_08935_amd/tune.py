"""Autotuner for the kernel shapes of the projection and apply kernels.

For a given context and state layout it times every candidate shape
(columns per lane x waves per work-group x lane layout: one state set
per wave, or narrow sets packed across the lanes) with the library's per-stage HIP
event profiler on the caller's own buffers, and keeps the fastest for each
kernel (``hub_set_tuning``).  Results depend only on timing, never on values:
every shape computes the same sums (the GPU tests check this).
"""

import torch

CANDIDATES = tuple((cpl, waves, layout) for layout in (0, 1) for cpl in (1, 2, 4) for waves in (1, 2, 4))


def autotune(hub, psi, c, n, ueff, reps=5, candidates=CANDIDATES):
    """Pick the fastest shape for hub_project (which=0) and hub_apply (1).

    psi: the states the step will read; c, n, ueff: device buffers of the
    right shape (their values do not matter).  Returns
    {"project": ((cpl, waves, layout), ms), "apply": (...), "table": {...}}.
    """
    scratch = torch.zeros_like(psi)
    table = {}
    best = {}
    for which, name in ((0, "project"), (1, "apply")):
        timings = {}
        for cpl, waves, layout in candidates:
            hub.set_tuning(which, cpl, waves, layout)
            # one untimed call compiles nothing but warms caches and sizes buffers
            if which == 0:
                hub.project(psi, out=c)
            else:
                hub.apply(ueff, n, c, scratch)
            hub.profile(True)
            for _ in range(reps):
                if which == 0:
                    hub.project(psi, out=c)
                else:
                    hub.apply(ueff, n, c, scratch)
            prof = hub.profile_read()
            hub.profile(False)
            ms, cnt = prof[name]
            timings[(cpl, waves, layout)] = ms / max(cnt, 1)
        shape = min(timings, key=timings.get)
        hub.set_tuning(which, *shape)
        best[name] = (shape, timings[shape])
        table[name] = {f"{k[0]}x{k[1]}{'w' if k[2] else 'p'}": round(v, 4) for k, v in timings.items()}
    torch.cuda.synchronize()
    best["table"] = table
    return best


def autotune_steps(hub, psi, f, hpsi, bufs, mode="persite", reps=3, candidates=CANDIDATES):
    """Pick the projection and apply shapes for whole steps of one step mode
    (``persite``: one launch per site and stage, whose small grids favour
    other shapes than one launch over every chunk).  Every candidate runs
    reps steps with the library's per-stage events; the fastest shape is
    kept per kernel.  hpsi accumulates the steps' updates.  Returns the same
    structure as autotune."""
    times = {"project": {}, "apply": {}}
    for shape in candidates:
        hub.set_tuning(0, *shape)
        hub.set_tuning(1, *shape)
        hub.step(psi, f, hpsi, mode=mode, bufs=bufs)
        hub.profile(True)
        for _ in range(reps):
            hub.step(psi, f, hpsi, mode=mode, bufs=bufs)
        prof = hub.profile_read()
        hub.profile(False)
        for name in times:
            times[name][shape] = prof[name][0] / reps
    best = {}
    table = {}
    for which, name in ((0, "project"), (1, "apply")):
        shape = min(times[name], key=times[name].get)
        hub.set_tuning(which, *shape)
        best[name] = (shape, times[name][shape])
        table[name] = {f"{k[0]}x{k[1]}{'w' if k[2] else 'p'}": round(v, 4) for k, v in times[name].items()}
    torch.cuda.synchronize()
    best["table"] = table
    return best
