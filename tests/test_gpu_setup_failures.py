"""Allocation failures and the setup cache, on the GPU.

* HUB_FAIL_ALLOC=N makes a context's N-th device allocation attempt fail
  once.  Whichever call meets it (table upload in hub_finalize, the Coulomb
  temporaries, a step's workspaces, the velocity-gauge tables, the moment
  tables of the step with the current) returns HUB_ENOMEM and can be
  repeated; the context then gives the results of a context that never
  failed, bit for bit, and is destroyed cleanly.
* hub_get_coulomb / hub_set_coulomb (and the .npz cache on them): tensors
  taken from one context and installed in another with the same spheres
  give the same step.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1711_08935_amd as H  # noqa: E402
from synth import make_config, make_occupations, make_states  # noqa: E402

A = np.array([0.05, -0.02, 0.03])


def _context(cfg, finalize=True):
    return H.Hubbard(cfg.cell, cfg.ngrid, cfg.sites, kpts=cfg.kpts, kweights=cfg.kweights, spin=cfg.spin,
                     is_complex=cfg.is_complex, precision="f32", finalize=finalize)


def _retry(fn):
    """Call fn; on an injected HUB_ENOMEM call it once more.  Returns whether
    the failure was met."""
    try:
        fn()
        return False
    except H.HubError as e:
        assert e.code == H.HUB_ENOMEM, e
    fn()
    return True


def _run(hub, cfg, psi, f_d):
    """Setup, a plain step, a step under a field with the current."""
    _retry(hub.finalize) if not hub.finalized else None
    _retry(lambda: hub.coulomb(-1))
    bufs = hub.step_buffers(cfg.nstates)
    h = torch.zeros_like(psi)
    _retry(lambda: hub.step(psi, f_d, h, mode="batched", bufs=bufs))
    _retry(lambda: hub.set_vector_potential(A))
    J = torch.empty((hub.nsites, 3), dtype=torch.float64, device="cuda")
    hg = torch.zeros_like(psi)
    bufs2 = hub.step_buffers(cfg.nstates)
    _retry(lambda: hub.step(psi, f_d, hg, mode="graph", bufs=bufs2, current=J))
    torch.cuda.synchronize()
    return h, bufs["c"].clone(), hg, J.clone()


@pytest.fixture(scope="module")
def clean():
    cfg = make_config("nio_afm", small=True)
    psi64 = make_states(cfg, device="cuda")
    f_d = torch.from_numpy(make_occupations(cfg)).cuda()
    hub = _context(cfg)
    psi = psi64.to(hub.state_dtype)
    counts = [hub.query(15)]                       # allocations after hub_finalize
    out = _run(hub, cfg, psi, f_d)
    counts.append(hub.query(15))                   # after everything
    hub.close()
    return cfg, psi, f_d, out, counts


def test_injected_allocation_failures(clean, monkeypatch):
    cfg, psi, f_d, ref, (n_fin, n_all) = clean
    assert n_all > n_fin > 10
    # the first, a middle and the last upload of hub_finalize, the first
    # allocations after it (Coulomb temporaries, step workspaces), and the
    # last ones (field tables, moment tables, current buffers)
    picks = sorted({1, n_fin // 2, n_fin, n_fin + 1, n_fin + 3, (n_fin + n_all) // 2, n_all - 1, n_all})
    for n in picks:
        print(f"[fail-alloc] attempt {n} of {n_all}", flush=True)
        monkeypatch.setenv("HUB_FAIL_ALLOC", str(n))
        hub = _context(cfg, finalize=False)
        monkeypatch.delenv("HUB_FAIL_ALLOC")
        got = _run(hub, cfg, psi, f_d)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), n
        hub.close()


def test_coulomb_tensors_carry_over(clean):
    cfg, psi, f_d, ref, _ = clean
    a = _context(cfg)
    with pytest.raises(H.HubError) as e:
        a.get_coulomb(0)
    assert e.value.code == H.HUB_ESTATE
    a.coulomb(-1)
    tensors = [a.get_coulomb(s).clone() for s in range(a.nsites)]
    b = _context(cfg)
    with pytest.raises(ValueError):
        b.set_coulomb(0, torch.zeros((2, 2, 2, 2), dtype=torch.float64, device="cuda"))
    for s, t in enumerate(tensors):
        b.set_coulomb(s, t)
        assert torch.equal(b.get_coulomb(s), t)
    outs = []
    for hub in (a, b):
        bufs = hub.step_buffers(cfg.nstates)
        h = torch.zeros_like(psi)
        hub.step(psi, f_d, h, mode="batched", bufs=bufs)
        torch.cuda.synchronize()
        outs.append((h, bufs["U"].clone(), bufs["J"].clone()))
    for x, y in zip(*outs):
        assert torch.equal(x, y)
    assert torch.equal(outs[0][0], ref[0])
    a.close()
    b.close()


def test_coulomb_cache_file(clean, tmp_path):
    """save_coulomb / load_coulomb: an .npz file of the tensors keyed by
    sphere; a context with the same spheres takes them all, one with a
    changed radius on one site takes the others."""
    cfg, psi, f_d, ref, _ = clean
    a = _context(cfg)
    a.coulomb(-1)
    path = str(tmp_path / "coulomb.npz")
    assert a.save_coulomb(path) == a.nsites
    b = _context(cfg)
    assert b.load_coulomb(path) == b.nsites
    for s in range(a.nsites):
        assert torch.equal(a.get_coulomb(s), b.get_coulomb(s))
    bufs = b.step_buffers(cfg.nstates)
    h = torch.zeros_like(psi)
    b.step(psi, f_d, h, mode="batched", bufs=bufs)
    torch.cuda.synchronize()
    assert torch.equal(h, ref[0])
    sites = [dict(s) for s in cfg.sites]
    sites[0]["rc"] = sites[0]["rc"] + 0.1
    d = H.Hubbard(cfg.cell, cfg.ngrid, sites, kpts=cfg.kpts, kweights=cfg.kweights, spin=cfg.spin,
                  is_complex=cfg.is_complex, precision="f32")
    assert d.load_coulomb(path) == d.nsites - 1
    with pytest.raises(H.HubError):
        d.get_coulomb(0)
    for x in (a, b, d):
        x.close()
