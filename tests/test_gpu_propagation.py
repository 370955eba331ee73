"""Real-time propagation through the captured step (Sec. V, adiabatic
approximation: the Hubbard potential of each time step is built from that
step's states).  The step graph is captured once and replayed after each
in-place update of the states, a Givens rotation of state pairs standing in
for the propagator.  Every replay must read the updated states: it equals an
eager batched step on the same states bitwise, and after the last update
its projections and V_U psi match the FP64 oracle (U_eff fixed, so the
comparison covers the projection, occupations and apply of the replay).
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import occupations as OO  # noqa: E402
from oracle import potential as OPOT  # noqa: E402
from oracle import projection as OP  # noqa: E402
from oracle import step as OS  # noqa: E402
from synth import make_config  # noqa: E402
from tests.gpu_common import device_states, make_hub, states_and_occupations  # noqa: E402
from tests.helpers import normwise, to_system  # noqa: E402

UEFF = 0.2


@pytest.mark.parametrize("name", ["rt_batched", "nio_afm"])
def test_graph_replays_follow_the_states(name):
    print(f"\n[propagation] {name} f32", flush=True)
    cfg = make_config(name, small=True)
    psi, f = states_and_occupations(cfg)
    hub = make_hub(cfg, "f32", chunk=256)
    for i in range(hub.nsites):
        hub.set_fixed_ueff(i, UEFF)
    psi_d, _ = device_states(hub, psi)
    master = psi_d.to(torch.complex128 if psi_d.is_complex() else torch.float64)
    f_d = torch.from_numpy(f).cuda()
    S = cfg.nstates
    half = S // 2
    rng = np.random.default_rng(7)
    theta = torch.from_numpy(0.05 * rng.uniform(0.5, 1.0, size=half) * rng.choice([-1.0, 1.0], size=half)).cuda()
    cth, sth = torch.cos(theta), torch.sin(theta)
    bufs = hub.step_buffers(S)
    hg = torch.zeros_like(psi_d)
    hub.step(psi_d, f_d, hg, mode="graph", bufs=bufs)              # captured here, replayed below
    c_prev = bufs["c"].clone()
    for r in range(4):
        a = master[..., :half].clone()
        b = master[..., half:2 * half]
        master[..., :half] = cth * a - sth * b
        master[..., half:2 * half] = sth * a + cth * b
        psi_d.copy_(master)
        hg.zero_()
        hub.step(psi_d, f_d, hg, mode="graph", bufs=bufs)
        he = torch.zeros_like(psi_d)
        be = hub.step(psi_d, f_d, he, mode="batched")
        torch.cuda.synchronize()
        assert not torch.equal(bufs["c"], c_prev), r                  # the replay saw the new states
        c_prev = bufs["c"].clone()
        assert torch.equal(hg, he), r
        for k in ("c", "n", "Ueff"):
            assert torch.equal(bufs[k], be[k]), (r, k)
    used = psi_d.cpu().numpy()
    used = used.astype(np.complex128 if np.iscomplexobj(used) else np.float64)
    sys_ = to_system(cfg)
    sps = OP.all_spheres(sys_)
    c = OP.project_sphere(sys_, used, sps)
    if not cfg.is_complex:
        c = c.real
    assert normwise(bufs["c"].cpu().numpy(), c) < 1e-12
    n, _, _ = OO.occupations(sys_, c, f, with_pbar=False)
    V = [OPOT.potential_matrix(sys_, UEFF, nn) for nn in n]
    h_ref = OS.apply_sphere(sys_, c, V, sps)
    if not cfg.is_complex:
        h_ref = h_ref.real
    assert normwise(hg.cpu().numpy(), h_ref) < 2e-7
