"""GPU edge cases against the oracle: a single state, a padded odd leading
dimension (forces one column per lane), an s shell next to p/d/f shells, a
site on the cell corner whose sphere overlaps its own periodic images
(duplicate grid points inside one site, several apply layers), a non-cubic
cell with complex k-points, and argument errors raised before any launch."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1711_08935_amd as H  # noqa: E402
from synth import Config  # noqa: E402
from tests.gpu_common import c_to_oracle, device_states, make_hub, n_site, oracle_case  # noqa: E402
from tests.helpers import normwise  # noqa: E402


def _cfg(spin="collinear", nstates=5, cplx=True):
    sites = [dict(R=np.array([0.0, 0.0, 0.0]), l=2, zeta=1.8, rc=3.3, species=0),
             dict(R=np.array([3.1, 2.2, 4.05]), l=0, zeta=1.2, rc=2.0, species=1),
             dict(R=np.array([1.3, 4.4, 1.9]), l=3, zeta=2.1, rc=2.6, species=2),
             dict(R=np.array([4.7, 0.6, 2.8]), l=1, zeta=1.5, rc=2.2, species=1)]
    kp = np.array([[0.25, -0.5, 0.125], [0.0, 0.25, 0.0]]) if cplx else np.zeros((1, 3))
    return Config(name="edge", cell=(6.0, 5.5, 6.5), ngrid=(15, 14, 16), sites=sites, kpts=kp,
                  kweights=np.full(len(kp), 1.0 / len(kp)), spin=spin, is_complex=cplx, nstates=nstates, seed=9)


def _rand_psi(cfg, S, rng):
    shape = (cfg.nk, cfg.G, S, 2) if cfg.spin == "spinor" else (cfg.nq, cfg.G, S)
    a = rng.normal(size=shape)
    if cfg.is_complex:
        a = a + 1j * rng.normal(size=shape)
    return a


def _check(cfg, prec, psi, f, ld_pad=0):
    hub = make_hub(cfg, prec, chunk=64)
    S = cfg.nstates
    if ld_pad:
        ncol = hub.ncol(S)
        full = np.zeros(psi.shape[:2] + (ncol + ld_pad,), dtype=psi.dtype)
        full[..., :ncol] = psi.reshape(psi.shape[0], psi.shape[1], -1)
        big, _ = device_states(hub, full)
        psi_d = big[..., :ncol]
        _, used = device_states(hub, psi)
    else:
        psi_d, used = device_states(hub, psi)
    sys_, sps, tens, ref = oracle_case(cfg, used, f)
    f_d = torch.from_numpy(f).cuda()
    hub.coulomb(-1)
    c = hub.project(psi_d, nstates=S)
    n, pbar, nb = hub.occupations(c, f_d)
    U, J, Ueff, st = hub.acbn0(n, pbar)
    h = torch.zeros_like(psi_d)
    hub.apply(Ueff, n, c, h, nstates=S)
    torch.cuda.synchronize()
    rc = ref["c"] if cfg.is_complex else ref["c"].real
    assert normwise(c_to_oracle(hub, c), rc) < 1e-12
    for I in range(hub.nsites):
        assert normwise(n_site(hub, n, I, hub.site_L[I]), ref["n"][I]) < 1e-12
    assert np.max(np.abs(U.cpu().numpy() - ref["U"])) < 1e-12 * max(1e-3, np.abs(ref["U"]).max())
    hh = h.cpu().numpy()
    if hh.ndim == 3 and cfg.spin == "spinor":
        hh = hh.reshape(hh.shape[0], hh.shape[1], -1, 2)
    rh = ref["hpsi"] if cfg.is_complex else ref["hpsi"].real
    assert normwise(hh, rh) < (1e-12 if prec == "f64" else 2e-7)
    return hub


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_state_and_mixed_shells(prec):
    cfg = _cfg(nstates=1)
    rng = np.random.default_rng(1)
    hub = _check(cfg, prec, _rand_psi(cfg, 1, rng) * 0.1, rng.uniform(0, 1, size=(cfg.nq, 1)))
    assert hub.nlayers >= 2                  # the corner d site overlaps its own images


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_padded_odd_leading_dimension(prec):
    cfg = _cfg(nstates=7)
    rng = np.random.default_rng(2)
    _check(cfg, prec, _rand_psi(cfg, 7, rng) * 0.1, rng.uniform(0, 1, size=(cfg.nq, 7)), ld_pad=2)   # ld = 9


def test_spinor_ragged_and_real_unpolarized():
    rng = np.random.default_rng(3)
    cfg = _cfg(spin="spinor", nstates=3)
    _check(cfg, "f64", _rand_psi(cfg, 3, rng) * 0.1, rng.uniform(0, 1, size=(cfg.nk, 3)))
    cfg2 = _cfg(spin="unpolarized", nstates=67, cplx=False)
    _check(cfg2, "f32", _rand_psi(cfg2, 67, rng) * 0.1, rng.uniform(0, 1, size=(cfg2.nq, 67)))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_step_current_mixed_shells_padded_states(prec):
    """The step with the current (one pass for c and the moments) on s, p, d
    and f shells, a site overlapping its own images, 7 states in rows of 9
    (ragged lanes, caller padding), under a field: the current against
    hub_current after the step and against the oracle."""
    from oracle import gauge as GA
    from oracle import occupations as OCC
    from oracle import potential as POT
    from oracle import projection as OP
    from tests.helpers import to_system
    cfg = _cfg(nstates=7)
    rng = np.random.default_rng(5)
    psi = _rand_psi(cfg, 7, rng) * 0.1
    f = rng.uniform(0, 1, size=(cfg.nq, 7))
    hub = make_hub(cfg, prec, chunk=64)
    ncol = hub.ncol(7)
    full = np.zeros(psi.shape[:2] + (ncol + 2,), dtype=psi.dtype)
    full[..., :ncol] = psi
    big, _ = device_states(hub, full)
    psi_d = big[..., :ncol]
    _, used = device_states(hub, psi)
    f_d = torch.from_numpy(f).cuda()
    hub.coulomb(-1)
    A = np.array([0.11, -0.07, 0.05])
    hub.set_vector_potential(A)
    try:
        h0 = torch.zeros_like(psi_d)
        ref = hub.step(psi_d, f_d, h0, mode="batched", nstates=7)
        Jsep = hub.current(psi_d, ref["c"], f_d, ref["Ueff"], ref["n"], nstates=7).cpu().numpy()
        J = torch.empty((hub.nsites, 3), dtype=torch.float64, device="cuda")
        h = torch.zeros_like(psi_d)
        b = hub.step(psi_d, f_d, h, mode="graph", nstates=7, current=J)
        torch.cuda.synchronize()
    finally:
        hub.set_vector_potential(None)
    J = J.cpu().numpy()
    assert normwise(J, Jsep) < 1e-12
    assert normwise(b["c"].cpu().numpy(), ref["c"].cpu().numpy()) < 1e-13
    sys_ = to_system(cfg)
    sps = OP.all_spheres(sys_)
    cA = GA.project_gauge(sys_, used, sps, A)
    n, _, _ = OCC.occupations(sys_, cA, f, with_pbar=False)
    V = [POT.potential_matrix(sys_, u, nn) for u, nn in zip(ref["Ueff"].cpu().numpy(), n)]
    Jo = GA.current(sys_, cA, GA.moment_projections(sys_, used, sps, A), V, f)
    assert np.abs(Jo).max() > 1e-8
    assert normwise(J, Jo) < 1e-11


def test_argument_errors_raise_before_launch():
    cfg = _cfg(nstates=4)
    hub = make_hub(cfg, "f64")
    psi = torch.zeros((cfg.nq, cfg.G, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(TypeError):
        hub.project(psi.to(torch.complex64))                  # wrong storage type
    with pytest.raises(ValueError):
        hub.project(psi[:1])                                  # wrong number of sets
    with pytest.raises(H.HubError) as e:
        hub.acbn0(hub.empty_n(), hub.empty_n())              # Coulomb tensors not computed yet
    assert e.value.code == H.HUB_ESTATE
    rc = H.lib().hub_project(hub._ctx, psi.data_ptr(), 2, 4, psi.data_ptr())   # ld < nstates
    assert rc == H.HUB_EINVAL
    lib = H.lib()
    p = psi.data_ptr()
    assert lib.hub_project(hub._ctx, p, 4, 0, p) == H.HUB_EINVAL                   # no states
    assert lib.hub_project(hub._ctx, None, 4, 4, p) == H.HUB_EINVAL
    assert lib.hub_project_sets(hub._ctx, p, 4, 4, -1, 1, p) == H.HUB_EINVAL      # set range
    assert lib.hub_project_sets(hub._ctx, p, 4, 4, 0, 0, p) == H.HUB_EINVAL
    assert lib.hub_project_sets(hub._ctx, p, 4, 4, 1, cfg.nq, p) == H.HUB_EINVAL
    assert lib.hub_apply(hub._ctx, p, p, p, 4, None, float("nan"), p, 4) == H.HUB_EINVAL   # alpha
    assert lib.hub_apply_sets(hub._ctx, p, p, p, 4, None, 1.0, p, 4, cfg.nq, 1) == H.HUB_EINVAL
    assert lib.hub_forces(hub._ctx, p, 4, 0, p, p, p, p, p) == H.HUB_EINVAL
    assert lib.hub_current(hub._ctx, None, 4, 4, p, p, p, p, p) == H.HUB_EINVAL
    assert lib.hub_forces_state_gradient(hub._ctx, p, 2, 4, p, p, p, p, p) == H.HUB_EINVAL
    assert lib.hub_energy_fll(hub._ctx, None, p, p, p) == H.HUB_EINVAL
    for A in ([float("nan"), 0.0, 0.0], [0.0, float("inf"), 0.0]):
        with pytest.raises(H.HubError):
            hub.set_vector_potential(A)


@pytest.mark.parametrize("fixed", [False, True])
def test_nonfinite_states_are_flagged(fixed):
    """A NaN in one state at a grid point that only site 0 covers: site 0's
    status is HUB_ENONFINITE (ACBN0: U and J NaN; fixed U_eff kept), and the
    sites of the other species, whose projections and N-bar never see it,
    stay finite with status 0."""
    from synth import make_config, make_occupations, make_states
    cfg = make_config("nio_afm", small=True)
    hub = make_hub(cfg, "f64")
    if fixed:
        for i in range(hub.nsites):
            hub.set_fixed_ueff(i, 0.2)
    else:
        hub.coulomb(-1)
    cover = np.zeros((hub.nsites, hub.G), bool)
    for s in range(hub.nsites):
        cover[s, hub.site_points(s)[0]] = True
    only0 = np.flatnonzero(cover[0] & ~cover[1:].any(axis=0))
    assert only0.size > 0
    psi = make_states(cfg, device="cuda")
    psi[0, int(only0[0]), 3] = float("nan")
    f_d = torch.from_numpy(make_occupations(cfg)).cuda()
    c = hub.project(psi)
    n, pbar, _ = hub.occupations(c, f_d)
    U, J, Ueff, st = hub.acbn0(n, pbar)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st[0] == H.HUB_ENONFINITE
    other = [s for s in range(hub.nsites) if cfg.sites[s]["species"] != cfg.sites[0]["species"]]
    assert other and all(st[s] == 0 for s in other)
    assert np.all(np.isfinite(U.cpu().numpy()[other]))
    if fixed:
        assert np.all(Ueff.cpu().numpy() == 0.2)
    else:
        assert np.isnan(U.cpu().numpy()[0])
    assert H.lib().hub_strerror(H.HUB_ENONFINITE) == b"occupations, U or J not finite"


@pytest.mark.parametrize("cplx,nstates,pad", [(False, 6, 2), (True, 5, 1)])
def test_apply_leaves_padding_columns_untouched(cplx, nstates, pad):
    """hpsi as a padded view whose leading dimension is even while the used
    columns are ragged (FP32 real: 6 of 8; FP32 complex: 5 of 6).  The apply
    writes whole vectors per lane, so the library picks a lane width that
    ends at the last used column: the padding, filled with -0.0, keeps its
    sign bit, and the used columns equal the apply into a contiguous
    buffer."""
    cfg = _cfg(spin="unpolarized" if not cplx else "collinear", nstates=nstates, cplx=cplx)
    rng = np.random.default_rng(4)
    hub = make_hub(cfg, "f32", chunk=64)
    psi_d, _ = device_states(hub, _rand_psi(cfg, nstates, rng) * 0.1)
    f_d = torch.from_numpy(rng.uniform(0, 1, size=(cfg.nq, nstates))).cuda()
    for i in range(hub.nsites):
        hub.set_fixed_ueff(i, 0.3)
    c = hub.project(psi_d)
    n, _, _ = hub.occupations(c, f_d, with_pbar=False, nbar=False)
    ueff = torch.full((hub.nsites,), 0.3, dtype=torch.float64, device="cuda")
    ref = torch.zeros_like(psi_d)
    hub.apply(ueff, n, c, ref)
    big = torch.empty(psi_d.shape[:2] + (nstates + pad,), dtype=psi_d.dtype, device="cuda")
    (torch.view_as_real(big) if cplx else big).fill_(-0.0)          # both parts of a complex value
    view = big[..., :nstates]
    view.zero_()
    for cpl in (0, 4, 2):
        hub.set_tuning(1, cpl, 4, -1)
        view.zero_()
        hub.apply(ueff, n, c, view, nstates=nstates)
        torch.cuda.synchronize()
        padcols = big[..., nstates:]
        parts = torch.view_as_real(padcols) if cplx else padcols
        assert torch.all(parts == 0) and torch.all(torch.signbit(parts)), cpl
        assert torch.equal(view, ref), cpl
    hub.set_tuning(1, 0, 4, -1)


def test_one_electron_in_one_orbital_is_degenerate():
    """psi = phi_m of a d shell on a grid point of a cubic grid (exactly
    orthonormal orbitals), occupied in the spin-up channel only: one
    electron in one orbital.  Both ACBN0 denominators vanish (Eqs. ACBN0_U,
    ACBN0_J), so the site is flagged HUB_WDEGENERATE with U = J = 0, as the
    oracle; n is e_m e_m^T in the up channel and zero in the other, and
    V_U psi = 0 (U_eff = 0)."""
    from synth import make_config
    from tests.gpu_common import oracle_case
    base = make_config("gamma_d")
    cfg = Config(name="one_electron", cell=base.cell, ngrid=base.ngrid, sites=base.sites, kpts=np.zeros((1, 3)),
                 kweights=np.ones(1), spin="collinear", is_complex=False, nstates=1, seed=0)
    hub = make_hub(cfg, "f64")
    g, _, phi, _ = hub.site_points(0)
    m = 2
    psi = np.zeros((2, cfg.G, 1))
    np.add.at(psi[0, :, 0], g, phi[:, m])
    psi[1] = psi[0]
    f = np.array([[1.0], [0.0]])
    psi_d, used = device_states(hub, psi)
    _, _, _, ref = oracle_case(cfg, used, f)
    assert int(ref["status"][0]) == 1 and ref["U"][0] == 0.0 and ref["J"][0] == 0.0
    hub.coulomb(-1)
    hpsi = torch.zeros_like(psi_d)
    b = hub.step(psi_d, torch.from_numpy(f).cuda(), hpsi, mode="graph")
    torch.cuda.synchronize()
    assert int(b["status"][0]) == H.HUB_WDEGENERATE
    assert b["U"][0].item() == 0.0 and b["J"][0].item() == 0.0 and b["Ueff"][0].item() == 0.0
    n = n_site(hub, b["n"], 0, 5)
    e = np.zeros((5, 5))
    e[m, m] = 1.0
    assert np.max(np.abs(n[0] - e)) < 1e-12 and np.max(np.abs(n[1])) == 0.0
    assert normwise(n, ref["n"][0]) < 1e-12
    assert torch.count_nonzero(hpsi).item() == 0


@pytest.mark.parametrize("spin", ["collinear", "spinor"])
def test_empty_shells(spin):
    """Every occupation zero: n = P-bar = 0, both denominators vanish on
    every site (HUB_WDEGENERATE, U = J = 0), E_U = 0 and V_U psi = 0, as the
    oracle."""
    from synth import make_config
    from tests.gpu_common import oracle_case, states_and_occupations
    cfg = make_config("nio_afm" if spin == "collinear" else "spinor_layers", small=True)
    psi, f = states_and_occupations(cfg)
    f = np.zeros_like(f)
    hub = make_hub(cfg, "f64", chunk=256)
    psi_d, used = device_states(hub, psi)
    _, _, _, ref = oracle_case(cfg, used, f)
    assert np.all(ref["status"] == 1)
    hub.coulomb(-1)
    hpsi = torch.zeros_like(psi_d)
    b = hub.step(psi_d, torch.from_numpy(f).cuda(), hpsi, mode="batched")
    EU = hub.energy(b["Ueff"], b["n"])
    torch.cuda.synchronize()
    assert np.all(b["status"].cpu().numpy() == H.HUB_WDEGENERATE)
    assert torch.count_nonzero(b["U"]).item() == 0 and torch.count_nonzero(b["J"]).item() == 0
    assert torch.count_nonzero(b["n"]).item() == 0 and torch.count_nonzero(b["pbar"]).item() == 0
    assert torch.count_nonzero(EU).item() == 0 and torch.count_nonzero(hpsi).item() == 0
    c = c_to_oracle(hub, b["c"])
    assert normwise(c, ref["c"]) < 1e-12
