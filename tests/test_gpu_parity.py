"""GPU parity of every entry point against the FP64 oracle on the same inputs.

Reduced workloads (all five shapes, both storage precisions) that still span
several chunks, column tiles and a ragged tail of columns.  Bars:
* FP64 states: normwise relative error <= 1e-12 for c, n, P-bar, N-bar, the
  Coulomb tensors, U-bar, J-bar, E_U, V_U psi, forces and the App. A
  energy terms (N, m, E_DC, E_ee).
* FP32 states: the oracle runs on the FP32-rounded states upcast to FP64, so
  what is compared is the kernels' arithmetic; occupations and U/J must agree
  to 1e-9 absolute (they agree far better), V_U psi to the FP32 rounding of
  the output (normwise 2e-7).
The end-to-end effect of FP32 storage (FP32 results against the oracle on
the FP64 master states) is asserted at full size in test_gpu_fullsize.py.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1711_08935_amd as H  # noqa: E402
from oracle import fll as OFL  # noqa: E402
from oracle import forces as OF  # noqa: E402
from oracle import potential as OPOT  # noqa: E402
from synth import make_config  # noqa: E402
from tests.gpu_common import (c_to_oracle, device_states, make_hub, n_site, oracle_case,  # noqa: E402
                              states_and_occupations)
from tests.helpers import normwise  # noqa: E402

CASES = [("gamma_d", "f64"), ("nio_afm", "f64"), ("nio_afm", "f32"), ("rt_batched", "f64"),
         ("rt_batched", "f32"), ("spinor_layers", "f64"), ("spinor_layers", "f32"), ("forces_fcc", "f32")]


@pytest.fixture(scope="module", params=CASES, ids=[f"{a}-{b}" for a, b in CASES])
def case(request):
    name, prec = request.param
    print(f"\n[case] {name} {prec}", flush=True)
    cfg = make_config(name, small=True)
    psi, f = states_and_occupations(cfg)
    hub = make_hub(cfg, prec, chunk=256)
    psi_d, psi_used = device_states(hub, psi)
    sys_, sps, tens, ref = oracle_case(cfg, psi_used, f)
    f_d = torch.from_numpy(f).cuda()
    hub.coulomb(-1)
    c = hub.project(psi_d)
    n, pbar, nbar = hub.occupations(c, f_d)
    U, J, Ueff, st = hub.acbn0(n, pbar)
    hpsi = torch.zeros_like(psi_d)
    hub.apply(Ueff, n, c, hpsi)
    EU = hub.energy(Ueff, n)
    torch.cuda.synchronize()
    return dict(name=name, prec=prec, cfg=cfg, hub=hub, psi=psi, psi_d=psi_d, psi_used=psi_used, f=f, f_d=f_d,
                sys=sys_, sps=sps, tens=tens, ref=ref, c=c, n=n, pbar=pbar, nbar=nbar, U=U, J=J, Ueff=Ueff,
                st=st, hpsi=hpsi, EU=EU)


def test_projection(case):
    hub, ref = case["hub"], case["ref"]
    c = c_to_oracle(hub, case["c"])
    rc = ref["c"] if hub.is_complex else ref["c"].real
    for I in range(hub.nsites):
        sl = slice(hub.site_orb0[I], hub.site_orb0[I] + hub.site_L[I])
        assert normwise(c[:, sl], rc[:, sl]) < 1e-12, I


def test_occupations_nbar_pbar(case):
    hub, ref = case["hub"], case["ref"]
    bar = 1e-12
    for I in range(hub.nsites):
        L = hub.site_L[I]
        assert normwise(n_site(hub, case["n"], I, L), ref["n"][I]) < bar
        assert normwise(n_site(hub, case["pbar"], I, L), ref["pbar"][I]) < bar
        assert np.max(np.abs(n_site(hub, case["n"], I, L) - ref["n"][I])) < 1e-9
    assert normwise(case["nbar"].cpu().numpy(), ref["nbar"]) < bar
    # unused corners of the 7x7 blocks are written as zeros
    nn = case["n"].cpu().numpy()
    for I in range(hub.nsites):
        L = hub.site_L[I]
        assert np.all(nn[I][:, L:, :] == 0) and np.all(nn[I][:, :, L:] == 0)


def test_coulomb_tensors(case):
    hub = case["hub"]
    for I in range(hub.nsites):
        T = hub.coulomb(I).cpu().numpy()
        assert normwise(T, case["tens"][I]) < 1e-12, I


def test_acbn0_u_j(case):
    ref = case["ref"]
    U = case["U"].cpu().numpy()
    J = case["J"].cpu().numpy()
    assert np.max(np.abs(U - ref["U"])) <= 1e-12 * max(1e-3, np.max(np.abs(ref["U"])))
    assert np.max(np.abs(J - ref["J"])) <= 1e-12 * max(1e-3, np.max(np.abs(ref["J"])))
    np.testing.assert_array_equal(case["st"].cpu().numpy(), ref["status"])


def test_apply_and_energy(case):
    hub, ref = case["hub"], case["ref"]
    h = case["hpsi"].cpu().numpy()
    rh = ref["hpsi"] if hub.is_complex else ref["hpsi"].real
    bar = 1e-12 if case["prec"] == "f64" else 2e-7
    assert normwise(h, rh) < bar
    assert normwise(case["EU"].cpu().numpy(), ref["EU"]) < 1e-12
    # points off every sphere are untouched
    covered = np.zeros(hub.G, bool)
    for sp in case["sps"]:
        covered[sp.g] = True
    assert np.all(h[:, ~covered] == 0)


def test_energy_fll(case):
    """N, m, E_DC and E_ee (App. A) from each side's own n, U-bar, J-bar."""
    hub, ref = case["hub"], case["ref"]
    out = hub.energy_fll(case["U"], case["J"], case["n"]).cpu().numpy()
    sys_ = case["sys"]
    rows = []
    for I in range(hub.nsites):
        N, m = OFL.moments(sys_, ref["n"][I])
        U, J = ref["U"][I], ref["J"][I]
        rows.append([N, *m, OFL.double_counting(N, m, U, J), OFL.hf_energy(sys_, ref["n"][I], U, J)])
    rows = np.array(rows)
    assert normwise(out[:, :4], rows[:, :4]) < 1e-12
    scale = max(1e-3, np.abs(rows[:, 4:]).max())
    assert np.max(np.abs(out[:, 4:] - rows[:, 4:])) <= 1e-12 * scale


def test_state_set_ranges(case):
    """hub_project_sets / hub_apply_sets on one set at a time and on a range
    reproduce the slices of the all-set calls (each set keeps its k-point)."""
    hub = case["hub"]
    psi_d, c_all, hpsi_all = case["psi_d"], case["c"], case["hpsi"]
    nq = psi_d.shape[0]
    ranges = [(q, 1) for q in range(nq)] + ([(1, nq - 1)] if nq > 1 else [])
    for q0, m in ranges:
        cs = hub.project(psi_d[q0:q0 + m], sets=(q0, m))
        h = torch.zeros_like(psi_d[q0:q0 + m])
        hub.apply(case["Ueff"], case["n"], cs, h, sets=(q0, m))
        torch.cuda.synchronize()
        assert normwise(cs.cpu().numpy(), c_all[q0:q0 + m].cpu().numpy()) < 1e-14, (q0, m)
        bar = 1e-14 if case["prec"] == "f64" else 1e-7
        assert normwise(h.cpu().numpy(), hpsi_all[q0:q0 + m].cpu().numpy()) < bar, (q0, m)
    with pytest.raises(H.HubError):
        hub.project(psi_d[:1], sets=(nq, 1))


def test_step_modes_agree_and_graph_replays(case):
    hub = case["hub"]
    psi_d, f_d = case["psi_d"], case["f_d"]
    outs = {}
    for mode in ("batched", "persite", "graph"):
        hpsi = torch.zeros_like(psi_d)
        b = hub.step(psi_d, f_d, hpsi, alpha=1.0, mode=mode)
        torch.cuda.synchronize()
        outs[mode] = (hpsi.clone(), {k: v.clone() for k, v in b.items()})
    # graph replays the batched launches: bitwise equal
    assert torch.equal(outs["graph"][0], outs["batched"][0])
    for k in ("c", "n", "pbar", "nbar", "U", "J", "Ueff"):
        assert torch.equal(outs["graph"][1][k], outs["batched"][1][k]), k
    # one launch per site uses the per-site work list: same sums, other order.
    # In FP32 storage the per-site path rounds the output after each covering
    # site's add (up to 3 sites cover one point here), the grouped path once
    # after summing every cover in FP64: they differ by up to (3 + 1) * 2^-24
    # relative to the partial sums.
    bar = 1e-13 if case["prec"] == "f64" else 4 * 2.0 ** -24 * 1.5
    assert normwise(outs["persite"][0].cpu().numpy(), outs["batched"][0].cpu().numpy()) < bar
    for k in ("c", "n", "pbar", "nbar", "U", "J", "Ueff"):
        assert normwise(outs["persite"][1][k].cpu().numpy(), outs["batched"][1][k].cpu().numpy()) < 1e-12, k
    assert torch.equal(outs["batched"][1]["c"], case["c"])
    assert torch.equal(outs["batched"][1]["Ueff"], case["Ueff"])
    # graph replays on fixed buffers with eager work in between
    hpsi = torch.zeros_like(psi_d)
    bufs = hub.step_buffers(outs["batched"][1]["nbar"].shape[2])
    for r in range(4):
        hpsi.zero_()
        hub.step(psi_d, f_d, hpsi, mode="graph", bufs=bufs)
        torch.cuda.synchronize()
        assert torch.equal(hpsi, outs["batched"][0]), r
        assert torch.equal(bufs["n"], outs["batched"][1]["n"]), r
        _ = (psi_d.abs() * 2).sum().item()          # unrelated eager work between replays


def test_forces(case):
    hub, ref = case["hub"], case["ref"]
    F = hub.forces(case["psi_d"], case["c"], case["f_d"], case["Ueff"], case["n"]).cpu().numpy()
    sys_, sps = case["sys"], case["sps"]
    d = OF.gradient_projections(sys_, case["psi_used"], sps)
    Fo = OF.forces_analytic(sys_, ref["c"], d, ref["V"], case["f"])
    assert normwise(F, Fo) < 1e-11


def test_autograd_energy_gradients(case):
    """dE_U/dpsi* (PyTorch's convention, spinors included) and dE_U/dR from
    hub_energy_gradient through the autograd wrapper, at the oracle's U_eff
    held fixed, against the oracle's adjoint and forces; the wrapper refuses
    a U_eff that is not given."""
    hub = case["hub"]
    with pytest.raises(ValueError):
        H.HubbardEnergy.apply(case["psi_d"], None, hub, case["f_d"], None)
    psi = case["psi_d"].clone().requires_grad_(True)
    R = torch.zeros((hub.nsites, 3), dtype=torch.float64, device="cuda", requires_grad=True)
    E = H.HubbardEnergy.apply(psi, R, hub, case["f_d"], case["Ueff"])
    E.backward()
    ref = case["ref"]
    sys_, sps = case["sys"], case["sps"]
    g_or = OF.psi_gradient(sys_, case["psi_used"], case["f"], ref["Ueff"], sps, OPOT.apply_fullgrid)
    g_or = 2.0 * (g_or if hub.is_complex else g_or.real)
    bar = 1e-12 if case["prec"] == "f64" else 2e-7
    assert normwise(psi.grad.cpu().numpy(), g_or) < bar
    assert abs(E.item() - ref["EU"].sum()) < 1e-12 * max(1.0, abs(ref["EU"].sum()))
    d = OF.gradient_projections(sys_, case["psi_used"], sps)
    Fo = OF.forces_analytic(sys_, ref["c"], d, ref["V"], case["f"])
    assert normwise(-R.grad.cpu().numpy(), Fo) < 1e-11


def test_tuning_variants_agree(case):
    """Every kernel shape (columns per lane x waves per work-group x lane
    layout) gives the
    same projections and V_U psi up to summation order."""
    hub = case["hub"]
    psi_d = case["psi_d"]
    try:
        for cpl, waves, layout in [(c, w, s) for s in (0, 1) for c in (1, 2, 4) for w in (1, 2, 4)]:
            hub.set_tuning(0, cpl, waves, layout)
            hub.set_tuning(1, cpl, waves, layout)
            c = hub.project(psi_d)
            h = torch.zeros_like(psi_d)
            hub.apply(case["Ueff"], case["n"], case["c"], h)
            torch.cuda.synchronize()
            assert normwise(c.cpu().numpy(), case["c"].cpu().numpy()) < 1e-13, (cpl, waves, layout)
            bar = 1e-13 if case["prec"] == "f64" else 1e-7
            assert normwise(h.cpu().numpy(), case["hpsi"].cpu().numpy()) < bar, (cpl, waves, layout)
    finally:
        hub.set_tuning(0, 0, 4, -1)
        hub.set_tuning(1, 0, 4, -1)


def test_step_tuner_keeps_results(case):
    """tune.autotune_steps picks the shapes from whole per-site steps; the
    per-site step with the picked shapes gives the outputs of the default
    shapes up to summation order."""
    from paper_1711_08935_amd.tune import CANDIDATES, autotune_steps
    hub = case["hub"]
    psi_d, f_d = case["psi_d"], case["f_d"]
    try:
        h0 = torch.zeros_like(psi_d)
        b0 = {k: v.clone() for k, v in hub.step(psi_d, f_d, h0, mode="persite").items()}
        bufs = hub.step_buffers(b0["nbar"].shape[2])
        best = autotune_steps(hub, psi_d, f_d, torch.zeros_like(psi_d), bufs, mode="persite", reps=1)
        assert best["project"][0] in CANDIDATES and best["apply"][0] in CANDIDATES
        assert len(best["table"]["project"]) == len(CANDIDATES)
        h1 = torch.zeros_like(psi_d)
        hub.step(psi_d, f_d, h1, mode="persite", bufs=bufs)
        torch.cuda.synchronize()
    finally:
        hub.set_tuning(0, 0, 4, -1)
        hub.set_tuning(1, 0, 4, -1)
    for k in ("c", "n", "pbar", "U", "J", "Ueff"):
        assert normwise(bufs[k].cpu().numpy(), b0[k].cpu().numpy()) < 1e-12, k
    bar = 1e-13 if case["prec"] == "f64" else 1e-7
    assert normwise(h1.cpu().numpy(), h0.cpu().numpy()) < bar


def test_worklists_agree(case):
    """The grouped work list (each grid point once, all its covers) and the
    per-site list applied in layers give the same projections and V_U psi."""
    hub = case["hub"]
    assert hub.ngrouped > 0
    psi_d = case["psi_d"]
    try:
        hub.set_worklist(False)
        c = hub.project(psi_d)
        h = torch.zeros_like(psi_d)
        hub.apply(case["Ueff"], case["n"], case["c"], h)
        torch.cuda.synchronize()
    finally:
        hub.set_worklist(True)
    assert normwise(c.cpu().numpy(), case["c"].cpu().numpy()) < 1e-13
    # the layered apply rounds FP32 output once per layer (up to 3 here)
    bar = 1e-13 if case["prec"] == "f64" else 4 * 2.0 ** -24 * 1.5
    assert normwise(h.cpu().numpy(), case["hpsi"].cpu().numpy()) < bar


def test_class_launch_policies_agree(case):
    """Merged, sequential and concurrent launches of the grouped work list's
    function-count classes perform the same arithmetic per column (entry
    order, wave split and reduction order do not depend on the policy)."""
    hub = case["hub"]
    psi_d = case["psi_d"]
    outs = {}
    try:
        for pol in ("sequential", "concurrent", "merged"):
            hub.set_class_launch(pol)
            c = hub.project(psi_d)
            h = torch.zeros_like(psi_d)
            hub.apply(case["Ueff"], case["n"], case["c"], h)
            torch.cuda.synchronize()
            outs[pol] = (c, h)
    finally:
        hub.set_class_launch("merged")
    for pol in ("sequential", "concurrent"):
        assert torch.equal(outs[pol][0], outs["merged"][0]), pol
        assert torch.equal(outs[pol][1], outs["merged"][1]), pol
    assert torch.equal(outs["merged"][0], case["c"])
