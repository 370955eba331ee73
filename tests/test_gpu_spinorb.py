"""GPU parity of spin-dependent (spinor) orbitals (App. A) against the FP64
oracle.

The noncollinear layered workload with a spin-down Slater exponent on every
site (d: 2.0 -> 2.6, p: 1.4 -> 1.1) and a fixed U_eff per site, both storage
precisions, both work lists: projections c^sigma = <phi^sigma|psi^sigma>,
occupations, E_U, V_U psi, the batched, graph and per-site steps, both
force forms and the current, and the gauge forms under a vector potential.  The oracle
projects and applies per spin component on the whole cell (its full-grid
definitions).  Bars as in test_gpu_parity.py.  With zeta_dn = zeta the
spin-dependent per-site kernels give results bitwise equal to the
spin-independent per-site path, and the grouped ones agree with the
spin-independent grouped path to rounding.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1711_08935_amd as H  # noqa: E402
from oracle import occupations as OCC  # noqa: E402
from oracle import potential as POT  # noqa: E402
from oracle import spinorb as SO  # noqa: E402
from synth import make_config  # noqa: E402
from tests.gpu_common import c_to_oracle, device_states, n_site, states_and_occupations  # noqa: E402
from tests.helpers import normwise, to_system  # noqa: E402

UEFF = 0.15


def _config(zeta_dn):
    cfg = make_config("spinor_layers", small=True)
    cfg.sites = [dict(s, zeta_dn=zeta_dn(s)) for s in cfg.sites]
    return cfg


def _hub(cfg, prec, worklist_grouped=True):
    hub = H.Hubbard(cfg.cell, cfg.ngrid, cfg.sites, kpts=cfg.kpts, kweights=cfg.kweights, spin=cfg.spin,
                    is_complex=cfg.is_complex, precision=prec, chunk=256)
    hub.set_worklist(worklist_grouped)
    for i in range(hub.nsites):
        hub.set_fixed_ueff(i, UEFF)
    return hub


@pytest.fixture(scope="module", params=["f64", "f32"])
def case(request):
    prec = request.param
    print(f"\n[spinorb case] spinor_layers {prec}", flush=True)
    cfg = _config(lambda s: 2.6 if s["l"] == 2 else 1.1)
    psi, f = states_and_occupations(cfg)
    hub = _hub(cfg, prec)
    psi_d, used = device_states(hub, psi)
    sys_ = to_system(cfg)
    cref = SO.project_spin(sys_, used)
    n, _, _ = OCC.occupations(sys_, cref, f, with_pbar=False)
    V = [POT.potential_matrix(sys_, UEFF, nn) for nn in n]
    ref = dict(c=cref, n=n, V=V, EU=np.array([POT.energy(sys_, UEFF, nn) for nn in n]),
               hpsi=SO.apply_spin(sys_, cref, V))
    return dict(prec=prec, cfg=cfg, hub=hub, psi_d=psi_d, used=used, f=f, f_d=torch.from_numpy(f).cuda(), sys=sys_,
                ref=ref)


@pytest.mark.parametrize("grouped", [True, False], ids=["grouped", "persite"])
def test_projection_occupations_energy_apply(case, grouped):
    hub, ref = case["hub"], case["ref"]
    assert hub.query(11) > 0
    hub.set_worklist(grouped)
    try:
        _check_calls(case, hub, ref)
    finally:
        hub.set_worklist(True)


def _check_calls(case, hub, ref):
    c = hub.project(case["psi_d"])
    n, _, _ = hub.occupations(c, case["f_d"], with_pbar=False)
    ueff = torch.full((hub.nsites,), UEFF, dtype=torch.float64, device="cuda")
    EU = hub.energy(ueff, n)
    h = torch.zeros_like(case["psi_d"])
    hub.apply(ueff, n, c, h)
    torch.cuda.synchronize()
    assert normwise(c_to_oracle(hub, c), ref["c"]) < 1e-12
    for I in range(hub.nsites):
        assert normwise(n_site(hub, n, I, hub.site_L[I]), ref["n"][I]) < 1e-12, I
    assert normwise(EU.cpu().numpy(), ref["EU"]) < 1e-12
    bar = 1e-12 if case["prec"] == "f64" else 2e-7
    assert normwise(h.cpu().numpy(), ref["hpsi"]) < bar


@pytest.mark.parametrize("grouped", [True, False], ids=["grouped", "persite"])
def test_set_ranges(case, grouped):
    """hub_project_sets / hub_apply_sets (one k-point at a time, and a
    range) reproduce the slices of the all-set calls."""
    hub, psi_d = case["hub"], case["psi_d"]
    nq = psi_d.shape[0]
    assert nq > 1
    hub.set_worklist(grouped)
    try:
        c_all = hub.project(psi_d)
        n, _, _ = hub.occupations(c_all, case["f_d"], with_pbar=False)
        ueff = torch.full((hub.nsites,), UEFF, dtype=torch.float64, device="cuda")
        h_all = torch.zeros_like(psi_d)
        hub.apply(ueff, n, c_all, h_all)
        bar = 1e-14 if case["prec"] == "f64" else 1e-7
        for q0, m in [(q, 1) for q in range(nq)] + [(1, nq - 1)]:
            cs = hub.project(psi_d[q0:q0 + m], sets=(q0, m))
            h = torch.zeros_like(psi_d[q0:q0 + m])
            hub.apply(ueff, n, cs, h, sets=(q0, m))
            torch.cuda.synchronize()
            assert normwise(cs.cpu().numpy(), c_all[q0:q0 + m].cpu().numpy()) < 1e-14, (q0, m)
            assert normwise(h.cpu().numpy(), h_all[q0:q0 + m].cpu().numpy()) < bar, (q0, m)
    finally:
        hub.set_worklist(True)


def test_steps(case):
    hub, ref = case["hub"], case["ref"]
    S = case["cfg"].nstates
    outs = {}
    for mode in ("batched", "graph", "persite"):
        bufs = hub.step_buffers(S)
        h = torch.zeros_like(case["psi_d"])
        hub.step(case["psi_d"], case["f_d"], h, mode=mode, bufs=bufs)
        torch.cuda.synchronize()
        outs[mode] = (h, bufs)
    h, bufs = outs["batched"]
    assert torch.equal(outs["graph"][0], h)
    # per-site launches use the per-site list: the same sums in another order
    assert normwise(outs["persite"][0].cpu().numpy(), h.cpu().numpy()) < (1e-13 if case["prec"] == "f64" else 2e-7)
    assert normwise(c_to_oracle(hub, bufs["c"]), ref["c"]) < 1e-12
    assert torch.all(bufs["Ueff"] == UEFF)
    bar = 1e-12 if case["prec"] == "f64" else 2e-7
    assert normwise(h.cpu().numpy(), ref["hpsi"]) < bar


def test_forces_and_current(case):
    """Forces through each component's orbital gradients and the current
    through its position moments, against the oracle."""
    from oracle import forces as OF
    from oracle import gauge as GA
    hub, ref, sys_ = case["hub"], case["ref"], case["sys"]
    c = hub.project(case["psi_d"])
    n, _, _ = hub.occupations(c, case["f_d"], with_pbar=False)
    ueff = torch.full((hub.nsites,), UEFF, dtype=torch.float64, device="cuda")
    F = hub.forces(case["psi_d"], c, case["f_d"], ueff, n).cpu().numpy()
    J = hub.current(case["psi_d"], c, case["f_d"], ueff, n).cpu().numpy()
    torch.cuda.synchronize()
    used = case["used"]
    Fo = OF.forces_analytic(sys_, ref["c"], SO.gradient_projections_spin(sys_, used), ref["V"], case["f"])
    Jo = GA.current(sys_, ref["c"], SO.moment_projections_spin(sys_, used), ref["V"], case["f"])
    assert np.abs(Fo).max() > 1e-6 and np.abs(Jo).max() > 1e-8
    assert normwise(F, Fo) < 1e-11
    assert normwise(J, Jo) < 1e-11


def test_velocity_gauge(case):
    """Under a field: c^A, V^A psi and the current against the oracle, and
    the graph step follows the field; the per-site list has no gauge form."""
    from oracle import gauge as GA
    hub, sys_ = case["hub"], case["sys"]
    A = np.array([0.137, -0.291, 0.083])
    hub.set_vector_potential(A)
    try:
        c = hub.project(case["psi_d"])
        n, _, _ = hub.occupations(c, case["f_d"], with_pbar=False)
        ueff = torch.full((hub.nsites,), UEFF, dtype=torch.float64, device="cuda")
        h = torch.zeros_like(case["psi_d"])
        hub.apply(ueff, n, c, h)
        J = hub.current(case["psi_d"], c, case["f_d"], ueff, n).cpu().numpy()
        bufs = hub.step_buffers(case["cfg"].nstates)
        hg = torch.zeros_like(case["psi_d"])
        hub.step(case["psi_d"], case["f_d"], hg, mode="graph", bufs=bufs)
        # the step with the current from its own pass: each component's
        # moments about its site from the spin-dependent orbitals, summed in
        # the moment launch's order (to rounding hub_current's)
        bufs2 = hub.step_buffers(case["cfg"].nstates)
        hs = torch.zeros_like(case["psi_d"])
        Js = torch.empty((hub.nsites, 3), dtype=torch.float64, device="cuda")
        hub.step(case["psi_d"], case["f_d"], hs, mode="graph", bufs=bufs2, current=Js)
        torch.cuda.synchronize()
        Js = Js.cpu().numpy()
        assert normwise(hs.cpu().numpy(), hg.cpu().numpy()) < (1e-12 if case["prec"] == "f64" else 2e-7)
        assert normwise(Js, J) < 1e-12
        hub.set_worklist(False)
        with pytest.raises(H.HubError):
            hub.project(case["psi_d"])
    finally:
        hub.set_worklist(True)
        hub.set_vector_potential(None)
    used, f = case["used"], case["f"]
    cA = SO.project_gauge_spin(sys_, used, A)
    assert normwise(c_to_oracle(hub, c), cA) < 1e-12
    nA, _, _ = OCC.occupations(sys_, cA, f, with_pbar=False)
    V = [POT.potential_matrix(sys_, UEFF, nn) for nn in nA]
    href = SO.apply_gauge_spin(sys_, cA, V, A)
    bar = 1e-12 if case["prec"] == "f64" else 2e-7
    assert normwise(h.cpu().numpy(), href) < bar
    assert normwise(hg.cpu().numpy(), href) < bar
    Jo = GA.current(sys_, cA, SO.moment_projections_spin(sys_, used, A), V, f)
    assert normwise(J, Jo) < 1e-11
    assert normwise(Js, Jo) < 1e-11


def test_state_gradient_forces(case):
    """Forces through <phi^sigma|D psi^sigma> against the oracle."""
    from oracle import stencil as SG
    hub, ref, sys_ = case["hub"], case["ref"], case["sys"]
    c = hub.project(case["psi_d"])
    n, _, _ = hub.occupations(c, case["f_d"], with_pbar=False)
    ueff = torch.full((hub.nsites,), UEFF, dtype=torch.float64, device="cuda")
    F = hub.forces(case["psi_d"], c, case["f_d"], ueff, n, form="state").cpu().numpy()
    e = SO.state_gradient_projections_spin(sys_, case["used"])
    Fo = SG.forces_state_gradient(sys_, ref["c"], e, ref["V"], case["f"])
    assert np.abs(Fo).max() > 1e-6
    assert normwise(F, Fo) < 1e-11


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_equal_exponents_match_spin_independent_path(prec):
    cfg_same = _config(lambda s: s["zeta"])
    cfg_plain = make_config("spinor_layers", small=True)
    psi, f = states_and_occupations(cfg_plain)
    # grouped lists: the same sums, split over different passes
    a = _hub(cfg_same, prec)
    b = _hub(cfg_plain, prec)
    psi_d, _ = device_states(a, psi)
    f_d = torch.from_numpy(f).cuda()
    ca, cb = a.project(psi_d), b.project(psi_d)
    na, _, _ = a.occupations(ca, f_d, with_pbar=False)
    ueff = torch.full((a.nsites,), UEFF, dtype=torch.float64, device="cuda")
    ha, hb = torch.zeros_like(psi_d), torch.zeros_like(psi_d)
    a.apply(ueff, na, ca, ha)
    b.apply(ueff, na, ca, hb)
    torch.cuda.synchronize()
    assert normwise(ca.cpu().numpy(), cb.cpu().numpy()) < 1e-14
    assert normwise(ha.cpu().numpy(), hb.cpu().numpy()) < (1e-14 if prec == "f64" else 1e-7)
    # per-site lists: bitwise
    a = _hub(cfg_same, prec, worklist_grouped=False)
    b = _hub(cfg_plain, prec, worklist_grouped=False)
    psi_d, _ = device_states(a, psi)
    f_d = torch.from_numpy(f).cuda()
    ca, cb = a.project(psi_d), b.project(psi_d)
    na, _, _ = a.occupations(ca, f_d, with_pbar=False)
    nb, _, _ = b.occupations(cb, f_d, with_pbar=False)
    ueff = torch.full((a.nsites,), UEFF, dtype=torch.float64, device="cuda")
    ha, hb = torch.zeros_like(psi_d), torch.zeros_like(psi_d)
    a.apply(ueff, na, ca, ha)
    b.apply(ueff, nb, cb, hb)
    torch.cuda.synchronize()
    assert torch.equal(ca, cb)
    assert torch.equal(na, nb)
    assert torch.equal(ha, hb)
