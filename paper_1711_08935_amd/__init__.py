"""MI355X (gfx950) DFT+U / ACBN0 Hubbard kernel: Python binding of libhub.so.

This module only marshals arguments: every step of the Hubbard path runs in
the HIP kernels of ``libhub.so`` (see ``include/hub.h`` for the C ABI, the
layouts and the error codes).  PyTorch provides device memory and streams.
Importing fails loudly when the library has not been built
(``python -m paper_1711_08935_amd.build`` or ``__graft_entry__.build()``).
"""

import ctypes
import hashlib
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# HUB_LIBRARY names another build of the same library (the host-sanitizer
# build of the CPU tests); by default the in-tree libhub.so
LIB_PATH = os.environ.get("HUB_LIBRARY") or os.path.join(_HERE, "libhub.so")

HUB_OK, HUB_EINVAL, HUB_ENOMEM, HUB_EDEVICE, HUB_ESTATE = 0, -1, -2, -3, -4
HUB_WDEGENERATE = 1
HUB_ENONFINITE = -5
HUB_ESCRATCH = -6
SPIN_MODES = {"unpolarized": 1, "collinear": 2, "spinor": 4}
PRECISIONS = {"f64": 0, "f32": 1}
STEP_MODES = {"batched": 0, "graph": 1, "persite": 2}
LMAX = 7


class HubError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {lib().hub_strerror(code).decode()} ({code})")
        self.code = code


class StepIO(ctypes.Structure):
    _fields_ = [("psi", ctypes.c_void_p), ("ld", ctypes.c_int64), ("nstates", ctypes.c_int),
                ("f", ctypes.c_void_p), ("hpsi", ctypes.c_void_p), ("ldh", ctypes.c_int64),
                ("alpha", ctypes.c_double), ("c", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("pbar", ctypes.c_void_p), ("nbar", ctypes.c_void_p), ("U", ctypes.c_void_p),
                ("J", ctypes.c_void_p), ("Ueff", ctypes.c_void_p), ("status", ctypes.c_void_p)]


_LIB = None
EXPORTS = ["hub_create", "hub_set_kpoints", "hub_add_site", "hub_set_fixed_ueff", "hub_set_chunk",
           "hub_set_tuning", "hub_finalize_host", "hub_finalize", "hub_set_stream", "hub_query",
           "hub_site_info", "hub_site_points", "hub_project", "hub_occupations", "hub_coulomb",
           "hub_acbn0_uj", "hub_apply", "hub_energy", "hub_forces", "hub_step", "hub_destroy",
           "hub_strerror", "hub_profile", "hub_profile_read", "hub_set_worklist", "hub_set_class_launch",
           "hub_set_vector_potential", "hub_current", "hub_forces_state_gradient", "hub_sphere_radius",
           "hub_energy_fll", "hub_set_site_spin_orbital", "hub_project_sets", "hub_apply_sets",
           "hub_energy_gradient", "hub_step_noalloc", "hub_step_current", "hub_get_coulomb",
           "hub_set_coulomb"]
STAGES = ["project", "reduce", "nbar", "occupations", "acbn0", "apply", "gradproject", "forces"]


def lib():
    """Load libhub.so (once) and declare the C prototypes."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "hub_create": [ctypes.POINTER(P), DP, ctypes.POINTER(I), I, I, I],
        "hub_set_kpoints": [P, I, DP, DP],
        "hub_add_site": [P, DP, I, D, D, I, ctypes.POINTER(I)],
        "hub_set_fixed_ueff": [P, I, D],
        "hub_set_chunk": [P, I],
        "hub_set_tuning": [P, I, I, I, I],
        "hub_finalize_host": [P],
        "hub_finalize": [P, P],
        "hub_set_stream": [P, P],
        "hub_query": [P, I, ctypes.POINTER(I64)],
        "hub_site_info": [P, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I64), ctypes.POINTER(I)],
        "hub_site_points": [P, I, P, P, P, P],
        "hub_project": [P, P, I64, I, P],
        "hub_occupations": [P, P, I, P, P, P, P],
        "hub_coulomb": [P, I, P],
        "hub_acbn0_uj": [P, P, P, P, P, P, P],
        "hub_apply": [P, P, P, P, I, P, D, P, I64],
        "hub_energy": [P, P, P, P],
        "hub_forces": [P, P, I64, I, P, P, P, P, P],
        "hub_current": [P, P, I64, I, P, P, P, P, P],
        "hub_forces_state_gradient": [P, P, I64, I, P, P, P, P, P],
        "hub_sphere_radius": [I, I, D, DP, D, DP],
        "hub_energy_fll": [P, P, P, P, P],
        "hub_set_site_spin_orbital": [P, I, D],
        "hub_project_sets": [P, P, I64, I, I, I, P],
        "hub_apply_sets": [P, P, P, P, I, P, D, P, I64, I, I],
        "hub_step": [P, ctypes.POINTER(StepIO), I],
        "hub_step_noalloc": [P, ctypes.POINTER(StepIO)],
        "hub_step_current": [P, ctypes.POINTER(StepIO), P, I],
        "hub_get_coulomb": [P, I, P],
        "hub_set_coulomb": [P, I, P],
        "hub_energy_gradient": [P, P, I64, I, P, P, P, P, D, P, I64, P],
        "hub_destroy": [P],
        "hub_strerror": [I],
        "hub_profile": [P, I],
        "hub_profile_read": [P, P, P],
        "hub_set_worklist": [P, I],
        "hub_set_class_launch": [P, I],
        "hub_set_vector_potential": [P, P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "hub_strerror" else I
    _LIB = L
    return L


def _check(code, where):
    if code < 0:
        raise HubError(code, where)
    return code


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _darr(vals):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


HUB_RADIUS_CELL, HUB_RADIUS_THRESHOLD = 1, 2


def sphere_radius(method, l=0, zeta=1.0, cell=None, threshold=0.0):
    """Sphere radius (bohr) by one of the selection methods of Sec. II:
    "cell" (the shortest cell edge) or "threshold" (where the normalized
    Slater radial part drops below ``threshold``).  Host only."""
    m = {"cell": HUB_RADIUS_CELL, "threshold": HUB_RADIUS_THRESHOLD}.get(method)
    if m is None:
        raise ValueError(f"method must be 'cell' or 'threshold', not {method!r}")
    rc = ctypes.c_double(0.0)
    cl = _darr(cell) if cell is not None else None
    _check(lib().hub_sphere_radius(m, int(l), float(zeta), cl, float(threshold), ctypes.byref(rc)),
           "hub_sphere_radius")
    return rc.value


class Hubbard:
    """One Hubbard context: geometry, k-points, shells, tables on the GPU.

    ``sites``: iterable of dicts with keys R (3,), l, zeta, rc, species.
    ``spin``: 'unpolarized' | 'collinear' | 'spinor'; ``precision``: 'f64'
    (FP64 states) or 'f32' (FP32 states; orbital table, sums and all results
    FP64).  Construction builds the host tables; ``finalize()`` uploads them.
    """

    def __init__(self, cell, ngrid, sites, kpts=None, kweights=None, spin="unpolarized",
                 is_complex=False, precision="f64", chunk=None, finalize=True):
        L = lib()
        self._ctx = ctypes.c_void_p()
        cell_a = _darr(cell)
        ng = (ctypes.c_int * 3)(*[int(v) for v in ngrid])
        _check(L.hub_create(ctypes.byref(self._ctx), cell_a, ng, SPIN_MODES[spin], int(bool(is_complex)),
                            PRECISIONS[precision]), "hub_create")
        self.cell = [float(v) for v in cell]
        self.ngrid = [int(v) for v in ngrid]
        self.spin = spin
        self.is_complex = bool(is_complex)
        self.precision = precision
        if kpts is not None:
            kp = [float(v) for row in kpts for v in row]
            kw = [float(v) for v in kweights]
            _check(L.hub_set_kpoints(self._ctx, len(kw), _darr(kp), _darr(kw)), "hub_set_kpoints")
            self.kweights = kw
        else:
            self.kweights = [1.0]
        self._sphere_keys = []
        for s in sites:
            # what a site's Coulomb tensor depends on: the grid, its centre,
            # shell and sphere (exact float images)
            self._sphere_keys.append(hashlib.sha256(repr((
                [float(v).hex() for v in cell], [int(v) for v in ngrid], [float(v).hex() for v in s["R"]],
                int(s["l"]), float(s["zeta"]).hex(), float(s["rc"]).hex())).encode()).hexdigest()
                if s.get("zeta_dn") is None else None)
            sid = ctypes.c_int()
            _check(L.hub_add_site(self._ctx, _darr(s["R"]), int(s["l"]), float(s["zeta"]), float(s["rc"]),
                                  int(s.get("species", 0)), ctypes.byref(sid)), "hub_add_site")
            if s.get("zeta_dn") is not None:
                # spin-dependent orbitals (spinor contexts): spin-down Slater exponent
                _check(L.hub_set_site_spin_orbital(self._ctx, sid.value, float(s["zeta_dn"])),
                       "hub_set_site_spin_orbital")
        if chunk is not None:
            _check(L.hub_set_chunk(self._ctx, int(chunk)), "hub_set_chunk")
        _check(L.hub_finalize_host(self._ctx), "hub_finalize_host")
        self.nsites = self.query(0)
        self.J = self.query(1)
        self.nsets = self.query(2)
        self.nlayers = self.query(3)
        self.nentries = self.query(4)
        self.nchunks = self.query(5)
        self.nspecies = self.query(6)
        self.nk = self.query(7)
        self.nblk = self.query(8)
        self.ngrouped = self.query(11)
        self.nfmax = self.query(12)
        self.site_L, self.site_orb0, self.site_npts, self.site_species = [], [], [], []
        for s in range(self.nsites):
            Lm, o, npts, sp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64(), ctypes.c_int()
            _check(L.hub_site_info(self._ctx, s, ctypes.byref(Lm), ctypes.byref(o), ctypes.byref(npts),
                                   ctypes.byref(sp)), "hub_site_info")
            self.site_L.append(Lm.value)
            self.site_orb0.append(o.value)
            self.site_npts.append(npts.value)
            self.site_species.append(sp.value)
        self.dV = math.prod(c / n for c, n in zip(self.cell, self.ngrid))
        self.G = math.prod(self.ngrid)
        self.finalized = False
        self._kw_dev = None
        if finalize:
            self.finalize()

    # ------------------------------------------------------------ plumbing
    def query(self, what):
        v = ctypes.c_int64()
        _check(lib().hub_query(self._ctx, what, ctypes.byref(v)), "hub_query")
        return v.value

    def finalize(self):
        if not torch.cuda.is_available():
            raise RuntimeError("the Hubbard kernels need a ROCm GPU")
        _check(lib().hub_finalize(self._ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "hub_finalize")
        self.finalized = True
        self.table_bytes = self.query(9)

    def _stream(self):
        _check(lib().hub_set_stream(self._ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "hub_set_stream")

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().hub_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fixed_ueff(self, site, ueff):
        _check(lib().hub_set_fixed_ueff(self._ctx, int(site), float(ueff)), "hub_set_fixed_ueff")

    def set_worklist(self, grouped=True):
        """Batched launches over the grouped (cover-signature) work list, or
        over per-site chunks applied in layers."""
        _check(lib().hub_set_worklist(self._ctx, int(bool(grouped))), "hub_set_worklist")

    CLASS_POLICIES = {"merged": 0, "sequential": 1, "concurrent": 2}

    def set_class_launch(self, policy="merged"):
        """Launch policy of the grouped work list's function-count classes:
        'merged' (one launch), 'sequential' or 'concurrent' (side streams)."""
        _check(lib().hub_set_class_launch(self._ctx, self.CLASS_POLICIES[policy]), "hub_set_class_launch")

    def set_tuning(self, which, cols_per_lane, waves, layout=-1):
        """Kernel shape of the projection (which=0) or apply (1); layout 1 =
        one state set per wave, 0 = sets packed across lanes, -1 = automatic."""
        _check(lib().hub_set_tuning(self._ctx, int(which), int(cols_per_lane), int(waves), int(layout)),
               "hub_set_tuning")

    def site_points(self, site):
        """Host copy of one site's sphere: (g, image3, phi, grad) numpy arrays."""
        import numpy as np
        n = self.site_npts[site]
        Lm = self.site_L[site]
        g = np.zeros(n, np.int32)
        im = np.zeros((n, 3), np.int32)
        phi = np.zeros((n, Lm))
        grad = np.zeros((n, Lm, 3))
        _check(lib().hub_site_points(self._ctx, int(site), g.ctypes.data, im.ctypes.data, phi.ctypes.data,
                                     grad.ctypes.data), "hub_site_points")
        return g, im, phi, grad

    # --------------------------------------------------------- tensor help
    @property
    def state_dtype(self):
        if self.precision == "f64":
            return torch.complex128 if self.is_complex else torch.float64
        return torch.complex64 if self.is_complex else torch.float32

    @property
    def coef_dtype(self):
        return torch.complex128 if self.is_complex else torch.float64

    def ncol(self, nstates):
        return 2 * nstates if self.spin == "spinor" else nstates

    def _states(self, psi, nstates=None, nq=None):
        """Validate a state tensor of nq state sets (default: all); returns
        (ld, nstates)."""
        if psi.dtype != self.state_dtype:
            raise TypeError(f"states must be {self.state_dtype}, got {psi.dtype}")
        if not psi.is_cuda:
            raise TypeError("states must live on the GPU")
        if self.spin == "spinor" and psi.dim() == 4:
            if psi.shape[3] != 2 or not psi[0, 0].is_contiguous():
                raise ValueError("spinor states must be [nk][G][S][2] with contiguous (S, 2)")
            S = psi.shape[2]
            ld = psi.stride(1)
        else:
            if psi.dim() != 3 or psi.stride(2) != 1:
                raise ValueError("states must be [nsets][G][ld-major columns] with unit column stride")
            ld = psi.stride(1)
            S = psi.shape[2] // (2 if self.spin == "spinor" else 1)
        want = self.nsets if nq is None else nq
        if psi.shape[0] != want or psi.shape[1] != self.G:
            raise ValueError(f"states must have {want} sets of {self.G} grid points")
        if psi.stride(0) != self.G * ld:
            raise ValueError("state sets must be consecutive ([q][g][ld])")
        return ld, (nstates if nstates is not None else S)

    def _dev(self, t, dtype=torch.float64):
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"expected a contiguous {dtype} GPU tensor")
        return t

    def empty_c(self, nstates, grad=False):
        rows = self.J * (3 if grad else 1)
        return torch.empty((self.nsets, rows, self.ncol(nstates)), dtype=self.coef_dtype, device="cuda")

    def empty_n(self):
        return torch.empty((self.nsites, self.nblk, LMAX, LMAX), dtype=torch.complex128, device="cuda")

    # ---------------------------------------------------------- entry points
    def project(self, psi, nstates=None, out=None, sets=None):
        """Projections of every state set, or of sets = (first, count) only
        (psi and the result then hold those sets)."""
        ld, S = self._states(psi, nstates, None if sets is None else int(sets[1]))
        if sets is None:
            c = out if out is not None else self.empty_c(S)
            self._stream()
            _check(lib().hub_project(self._ctx, _dptr(psi), ld, S, _dptr(c)), "hub_project")
            return c
        q0, nq = int(sets[0]), int(sets[1])
        c = out if out is not None else self.empty_c(S)[:nq].contiguous()
        self._stream()
        _check(lib().hub_project_sets(self._ctx, _dptr(psi), ld, S, q0, nq, _dptr(c)), "hub_project_sets")
        return c

    def occupations(self, c, f, with_pbar=True, nbar=True):
        S = c.shape[2] // (2 if self.spin == "spinor" else 1)
        f = self._dev(f)
        n = self.empty_n()
        pbar = self.empty_n() if with_pbar else None
        nb = torch.empty((self.nsets, self.nspecies, S), dtype=torch.float64, device="cuda") if nbar else None
        self._stream()
        _check(lib().hub_occupations(self._ctx, _dptr(c), S, _dptr(f), _dptr(n), _dptr(pbar), _dptr(nb)),
               "hub_occupations")
        return n, pbar, nb

    def coulomb(self, site=-1):
        self._stream()
        if site < 0:
            _check(lib().hub_coulomb(self._ctx, -1, ctypes.c_void_p(0)), "hub_coulomb")
            return None
        Lm = self.site_L[site]
        T = torch.empty((Lm, Lm, Lm, Lm), dtype=torch.float64, device="cuda")
        _check(lib().hub_coulomb(self._ctx, int(site), _dptr(T)), "hub_coulomb")
        return T

    def get_coulomb(self, site):
        """The context's Coulomb tensor of one site (L, L, L, L), FP64."""
        Lm = self.site_L[site]
        T = torch.empty((Lm, Lm, Lm, Lm), dtype=torch.float64, device="cuda")
        self._stream()
        _check(lib().hub_get_coulomb(self._ctx, int(site), _dptr(T)), "hub_get_coulomb")
        return T

    def set_coulomb(self, site, tensor):
        """Install a Coulomb tensor computed earlier for this site's sphere."""
        Lm = self.site_L[site]
        t = self._dev(tensor)
        if tuple(t.shape) != (Lm, Lm, Lm, Lm):
            raise ValueError(f"site {site} takes an ({Lm},)*4 tensor")
        self._stream()
        _check(lib().hub_set_coulomb(self._ctx, int(site), _dptr(t)), "hub_set_coulomb")

    def save_coulomb(self, path):
        """Write the context's Coulomb tensors (the costly part of the
        set-up) to an .npz file, each under the key of its sphere."""
        keys, tens = [], []
        for site, key in enumerate(self._sphere_keys):
            if key is None:
                continue
            try:
                t = self.get_coulomb(site)
            except HubError as e:
                if e.code != HUB_ESTATE:
                    raise
                continue
            keys.append(key)
            tens.append(t.cpu().numpy().ravel())
        np.savez(path, keys=np.array(keys), **{f"t{i}": t for i, t in enumerate(tens)})
        return len(keys)

    def load_coulomb(self, path):
        """Install the tensors of an .npz file from save_coulomb for every
        site whose sphere key matches; returns how many were installed (the
        other sites still need hub_coulomb)."""
        with np.load(path, allow_pickle=False) as z:
            have = {str(k): i for i, k in enumerate(z["keys"])}
            done = 0
            for site, key in enumerate(self._sphere_keys):
                if key is None or key not in have:
                    continue
                Lm = self.site_L[site]
                t = torch.from_numpy(z[f"t{have[key]}"].reshape(Lm, Lm, Lm, Lm)).cuda()
                self.set_coulomb(site, t)
                done += 1
        torch.cuda.synchronize()
        return done

    def acbn0(self, n, pbar):
        U = torch.empty(self.nsites, dtype=torch.float64, device="cuda")
        J = torch.empty_like(U)
        Ueff = torch.empty_like(U)
        st = torch.empty(self.nsites, dtype=torch.int32, device="cuda")
        self._stream()
        _check(lib().hub_acbn0_uj(self._ctx, _dptr(n), _dptr(pbar), _dptr(U), _dptr(J), _dptr(Ueff), _dptr(st)),
               "hub_acbn0_uj")
        return U, J, Ueff, st

    def apply(self, Ueff, n, c, hpsi, alpha=1.0, colscale=None, nstates=None, sets=None):
        """hpsi += alpha V_U psi for every state set, or for sets = (first,
        count) only (c, hpsi and colscale then hold those sets)."""
        ld, S = self._states(hpsi, nstates, None if sets is None else int(sets[1]))
        self._stream()
        if sets is None:
            _check(lib().hub_apply(self._ctx, _dptr(Ueff), _dptr(n), _dptr(c), S, _dptr(colscale), float(alpha),
                                   _dptr(hpsi), ld), "hub_apply")
        else:
            _check(lib().hub_apply_sets(self._ctx, _dptr(Ueff), _dptr(n), _dptr(c), S, _dptr(colscale),
                                        float(alpha), _dptr(hpsi), ld, int(sets[0]), int(sets[1])), "hub_apply_sets")
        return hpsi

    def energy(self, Ueff, n):
        EU = torch.empty(self.nsites, dtype=torch.float64, device="cuda")
        self._stream()
        _check(lib().hub_energy(self._ctx, _dptr(Ueff), _dptr(n), _dptr(EU)), "hub_energy")
        return EU

    def energy_fll(self, U, J, n):
        """(n_sites, 6) per site: N, m_x, m_y, m_z, E_DC, E_ee (App. A)."""
        out = torch.empty((self.nsites, 6), dtype=torch.float64, device="cuda")
        self._stream()
        _check(lib().hub_energy_fll(self._ctx, _dptr(self._dev(U)), _dptr(self._dev(J)), _dptr(n), _dptr(out)),
               "hub_energy_fll")
        return out

    def set_vector_potential(self, A=None):
        """Uniform vector potential A (3 floats, bohr^-1) of the velocity
        gauge for later projections, applies and steps; None switches the
        field off."""
        if A is None:
            self._stream()
            _check(lib().hub_set_vector_potential(self._ctx, None), "hub_set_vector_potential")
            return
        arr = (ctypes.c_double * 3)(*[float(x) for x in A])
        self._stream()
        _check(lib().hub_set_vector_potential(self._ctx, arr), "hub_set_vector_potential")

    def current(self, psi, c, f, Ueff, n, nstates=None):
        """Velocity-gauge DFT+U current correction per site, (n_sites, 3) FP64."""
        ld, S = self._states(psi, nstates)
        J = torch.empty((self.nsites, 3), dtype=torch.float64, device="cuda")
        self._stream()
        _check(lib().hub_current(self._ctx, _dptr(psi), ld, S, _dptr(c), _dptr(self._dev(f)), _dptr(Ueff),
                                 _dptr(n), _dptr(J)), "hub_current")
        return J

    def forces(self, psi, c, f, Ueff, n, nstates=None, form="orbital"):
        """Hubbard forces (n_sites, 3).  form="orbital": through the orbital
        gradients <grad phi|psi>; form="state": through the 4th-order
        differences of the states <phi|D psi> (hub_forces_state_gradient)."""
        if form not in ("orbital", "state"):
            raise ValueError(f"form must be 'orbital' or 'state', not {form!r}")
        name = "hub_forces" if form == "orbital" else "hub_forces_state_gradient"
        ld, S = self._states(psi, nstates)
        F = torch.empty((self.nsites, 3), dtype=torch.float64, device="cuda")
        self._stream()
        _check(getattr(lib(), name)(self._ctx, _dptr(psi), ld, S, _dptr(c), _dptr(self._dev(f)), _dptr(Ueff),
                                    _dptr(n), _dptr(F)), name)
        return F

    def energy_gradient(self, psi, c, f, Ueff, n, scale=1.0, want_psi=True, want_R=True, nstates=None):
        """scale times the gradients of sum_I E_U[I] at fixed U_eff
        (hub_energy_gradient): (grad_psi, grad_R).  grad_psi has psi's shape
        and PyTorch's convention for complex tensors (2 dE/dpsi*); grad_R is
        dE/dR, (n_sites, 3).  Either may be skipped (None returned)."""
        ld, S = self._states(psi, nstates)
        gpsi = None
        ldg = 0
        if want_psi:
            gpsi = torch.empty(psi.shape, dtype=psi.dtype, device=psi.device)
            ldg, _ = self._states(gpsi, S)
        gR = torch.empty((self.nsites, 3), dtype=torch.float64, device="cuda") if want_R else None
        self._stream()
        _check(lib().hub_energy_gradient(self._ctx, _dptr(psi), ld, S, _dptr(c), _dptr(self._dev(f)),
                                         _dptr(self._dev(Ueff)), _dptr(n), float(scale), _dptr(gpsi), ldg,
                                         _dptr(gR)), "hub_energy_gradient")
        return gpsi, gR

    def profile(self, enable=True):
        _check(lib().hub_profile(self._ctx, int(bool(enable))), "hub_profile")

    def profile_read(self):
        """{stage: (milliseconds, launches)} accumulated since the last read."""
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int64 * 8)()
        _check(lib().hub_profile_read(self._ctx, ms, cnt), "hub_profile_read")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}

    def step_buffers(self, nstates):
        return dict(c=self.empty_c(nstates), n=self.empty_n(), pbar=self.empty_n(),
                    nbar=torch.empty((self.nsets, self.nspecies, nstates), dtype=torch.float64, device="cuda"),
                    U=torch.empty(self.nsites, dtype=torch.float64, device="cuda"),
                    J=torch.empty(self.nsites, dtype=torch.float64, device="cuda"),
                    Ueff=torch.empty(self.nsites, dtype=torch.float64, device="cuda"),
                    status=torch.empty(self.nsites, dtype=torch.int32, device="cuda"))

    def step(self, psi, f, hpsi, alpha=1.0, mode="graph", bufs=None, nstates=None, current=None):
        """One Hubbard step; returns the dict of device buffers it filled.
        ``current``: an (n_sites, 3) FP64 device tensor that receives the
        velocity-gauge current of the step (hub_step_current)."""
        ld, S = self._states(psi, nstates)
        ldh, S2 = self._states(hpsi, nstates)
        if S2 != S:
            raise ValueError("psi and hpsi hold different state counts")
        b = bufs if bufs is not None else self.step_buffers(S)
        io = StepIO(psi.data_ptr(), ld, S, self._dev(f).data_ptr(), hpsi.data_ptr(), ldh, float(alpha),
                    b["c"].data_ptr(), b["n"].data_ptr(), b["pbar"].data_ptr(), b["nbar"].data_ptr(),
                    b["U"].data_ptr(), b["J"].data_ptr(), b["Ueff"].data_ptr(), b["status"].data_ptr())
        self._stream()
        if current is None:
            _check(lib().hub_step(self._ctx, ctypes.byref(io), STEP_MODES[mode]), "hub_step")
        else:
            if current.dtype != torch.float64 or not current.is_cuda or tuple(current.shape) != (self.nsites, 3) \
                    or not current.is_contiguous():
                raise ValueError("current must be a contiguous (n_sites, 3) float64 CUDA tensor")
            _check(lib().hub_step_current(self._ctx, ctypes.byref(io), current.data_ptr(), STEP_MODES[mode]),
                   "hub_step_current")
        return b

    def step_noalloc(self, psi, f, hpsi, bufs, alpha=1.0, nstates=None):
        """The batched step with its workspaces in the library's static
        scratch array (hub_step_noalloc): no device allocation.  ``bufs``
        (from step_buffers) must be given, so nothing is allocated here."""
        ld, S = self._states(psi, nstates)
        ldh, S2 = self._states(hpsi, nstates)
        if S2 != S:
            raise ValueError("psi and hpsi hold different state counts")
        b = bufs
        io = StepIO(psi.data_ptr(), ld, S, self._dev(f).data_ptr(), hpsi.data_ptr(), ldh, float(alpha),
                    b["c"].data_ptr(), b["n"].data_ptr(), b["pbar"].data_ptr(), b["nbar"].data_ptr(),
                    b["U"].data_ptr(), b["J"].data_ptr(), b["Ueff"].data_ptr(), b["status"].data_ptr())
        self._stream()
        _check(lib().hub_step_noalloc(self._ctx, ctypes.byref(io)), "hub_step_noalloc")
        return b


from .autograd import HubbardEnergy  # noqa: E402,F401
