"""hub_step_noalloc, called through the C ABI, against hub_step in its
batched mode on the same inputs (the same kernels in the same order: the
outputs must be bitwise equal), on two calls in a row whose second has fewer
states, for a complex collinear (also under a vector potential), a real and
a spinor context.  The context's
device-allocation count (hub_query 15) does not move across the calls, while
a plain hub_step on a fresh context allocates its workspaces; a step whose
workspace exceeds HUB_SCRATCH_BYTES is refused before any launch."""

import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1711_08935_amd as H  # noqa: E402
from synth import make_config  # noqa: E402
from tests.gpu_common import device_states, make_hub, states_and_occupations  # noqa: E402


def _io(psi, ld, nst, f, hpsi, ldh, b):
    return H.StepIO(psi.data_ptr(), ld, nst, f.data_ptr(), hpsi.data_ptr(), ldh, 1.0, b["c"].data_ptr(),
                    b["n"].data_ptr(), b["pbar"].data_ptr(), b["nbar"].data_ptr(), b["U"].data_ptr(),
                    b["J"].data_ptr(), b["Ueff"].data_ptr(), b["status"].data_ptr())


@pytest.mark.parametrize("name,prec,field", [("nio_afm", "f64", False), ("rt_batched", "f32", False),
                                             ("spinor_layers", "f32", False), ("nio_afm", "f32", True)])
def test_noalloc_step_matches_batched_step(name, prec, field):
    print(f"\n[noalloc] {name} {prec} field={field}", flush=True)
    cfg = make_config(name, small=True)
    psi, f = states_and_occupations(cfg)
    hub = make_hub(cfg, prec, chunk=256)
    psi_d, _ = device_states(hub, psi)
    f_d = torch.from_numpy(f).cuda()
    hub.coulomb(-1)
    if field:
        # the velocity gauge's tables are made when the field is set, so the
        # step under a field allocates nothing either
        hub.set_vector_potential([0.05, -0.03, 0.02])
    S = cfg.nstates
    ld = hub.ncol(S)
    lib = H.lib()
    for nst in (S, S // 2 + 1):
        fs = f_d[..., :nst].contiguous()
        bufs = hub.step_buffers(nst)
        h = torch.zeros_like(psi_d)
        before = hub.query(15)
        hub._stream()
        assert lib.hub_step_noalloc(hub._ctx, ctypes.byref(_io(psi_d, ld, nst, fs, h, ld, bufs))) == H.HUB_OK
        torch.cuda.synchronize()
        assert hub.query(15) == before, nst
        ref = hub.step_buffers(nst)
        h_ref = torch.zeros_like(psi_d)
        hub.step(psi_d, fs, h_ref, mode="batched", bufs=ref, nstates=nst)
        torch.cuda.synchronize()
        assert torch.equal(h, h_ref), nst
        for k in ("c", "n", "pbar", "nbar", "U", "J", "Ueff", "status"):
            assert torch.equal(bufs[k], ref[k]), (nst, k)
        assert torch.count_nonzero(h).item() > 0


def test_noalloc_allocates_nothing_and_refuses_oversized_steps():
    cfg = make_config("nio_afm", small=True)
    psi, f = states_and_occupations(cfg)
    f_d = torch.from_numpy(f).cuda()
    fresh = make_hub(cfg, "f64", chunk=256)
    for i in range(fresh.nsites):
        fresh.set_fixed_ueff(i, 0.2)
    psi_d, _ = device_states(fresh, psi)
    S = cfg.nstates
    bufs = fresh.step_buffers(S)
    h = torch.zeros_like(psi_d)
    n0 = fresh.query(15)
    fresh.step_noalloc(psi_d, f_d, h, bufs)
    torch.cuda.synchronize()
    assert fresh.query(15) == n0
    other = make_hub(cfg, "f64", chunk=256)
    for i in range(other.nsites):
        other.set_fixed_ueff(i, 0.2)
    m0 = other.query(15)
    h2 = torch.zeros_like(psi_d)
    b2 = other.step(psi_d, f_d, h2, mode="batched")
    torch.cuda.synchronize()
    assert other.query(15) > m0
    assert torch.equal(h, h2) and torch.equal(bufs["n"], b2["n"])
    # a workspace past the scratch size: refused before any launch (the
    # pointers are never dereferenced)
    big = 1 << 22
    io = _io(psi_d, big, big, f_d, h, big, bufs)
    assert H.lib().hub_step_noalloc(fresh._ctx, ctypes.byref(io)) == H.HUB_ESCRATCH
    assert H.lib().hub_strerror(H.HUB_ESCRATCH) == b"workspace larger than the static scratch buffer"
    assert H.lib().hub_step_noalloc(fresh._ctx, None) == H.HUB_EINVAL
    np.testing.assert_equal(fresh.query(15), n0)
