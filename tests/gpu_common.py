"""Shared helpers of the GPU parity tests: build a context and its inputs from
a synthetic workload, run the oracle on exactly the same inputs, and convert
between the library's layouts and the oracle's.  Holds no arithmetic of the
method (the oracle and the HIP path each do their own)."""

import numpy as np
import torch

import paper_1711_08935_amd as H
from oracle import projection as OP
from oracle import step as OS
from synth import make_occupations, make_states
from tests.helpers import to_system


def make_hub(cfg, precision, chunk=None):
    return H.Hubbard(cfg.cell, cfg.ngrid, cfg.sites, kpts=cfg.kpts, kweights=cfg.kweights, spin=cfg.spin,
                     is_complex=cfg.is_complex, precision=precision, chunk=chunk)


def device_states(hub, psi_np):
    """Library-layout device tensor from an oracle-layout numpy array, and the
    FP64 numpy copy of what the device holds (FP32-rounded in 'f32')."""
    t = torch.from_numpy(np.ascontiguousarray(psi_np)).to(hub.state_dtype).cuda()
    used = t.cpu().numpy()
    used = used.astype(np.complex128 if np.iscomplexobj(used) else np.float64)
    return t, used


def c_to_oracle(hub, c):
    a = c.cpu().numpy()
    if hub.spin == "spinor":
        a = a.reshape(a.shape[0], a.shape[1], -1, 2)
    return a


def n_site(hub, n, I, L):
    a = n.cpu().numpy()[I]
    if hub.spin == "spinor":
        return np.array([[a[2 * s + t, :L, :L] for t in range(2)] for s in range(2)])
    return a[:, :L, :L]


def oracle_case(cfg, psi_used, f, method="fft"):
    sys_ = to_system(cfg)
    sps = OP.all_spheres(sys_)
    tens = OS.site_tensors(sys_, sps, method=method)
    ref = OS.hubbard_step(sys_, psi_used, f, sps, tens, form="fullgrid")
    return sys_, sps, tens, ref


def states_and_occupations(cfg):
    psi = make_states(cfg).numpy()
    f = make_occupations(cfg)
    return psi, f
